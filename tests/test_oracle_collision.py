"""Pins of the oracle's per-node collision.

* exact rational agreement with the paper's printed cascade (Sec. 7, Sec. 8,
  Appendices B-E, G), with each misprint shown to matter;
* conservation of mass and of momentum up to the force (Appendix F first rows);
* Galilean invariance of the post-collision central moments (the paper's
  central claim, Sec. 1 and Sec. 5);
* the equilibrium is a fixed point at rho = 1 (factorized attractors equal the
  Maxwellian's there);
* with every rate equal to one the post-collision central moments are the
  attractors.
"""
from fractions import Fraction

import numpy as np
import pytest

from golden_io import load_int_table
from oracle import collision
from oracle.lattice import D3Q15, D3Q27
import paper_cascade as pc

K27 = load_int_table("K27_appendix_A.txt").tolist()
K15 = load_int_table("K15_appendix_G.txt").tolist()


def _rat(rng, lo, hi, den):
    return Fraction(int(rng.integers(int(lo * den), int(hi * den))), den)


def _random_node(lat, rng, umax=0.25, force=0.01):
    rho = _rat(rng, 0.8, 1.2, 97)
    u = [_rat(rng, -umax, umax, 89) for _ in range(3)]
    feq = collision.equilibrium(lat, np.array(rho, dtype=object), np.array(u, dtype=object))
    f = np.array([feq[a] + _rat(rng, -0.01, 0.01, 1009) for a in range(lat.Q)], dtype=object)
    F = np.array([_rat(rng, -force, force, 991) for _ in range(3)], dtype=object)
    om = [_rat(rng, 0.1, 1.95, 41) for _ in range(lat.Q - 4)]
    return f, F, om


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_d3q27_equals_printed_cascade_exactly(seed):
    rng = np.random.default_rng(seed)
    f, F, om = _random_node(D3Q27, rng)
    ours = collision.collide(D3Q27, f, F, om)
    theirs = pc.cascade_d3q27(K27, list(f), list(F), om)
    assert list(ours) == theirs


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_d3q15_equals_printed_cascade_exactly(seed):
    rng = np.random.default_rng(100 + seed)
    f, F, om = _random_node(D3Q15, rng)
    ours = collision.collide(D3Q15, f, F, om)
    theirs = pc.cascade_d3q15(K15, list(f), list(F), om)
    assert list(ours) == theirs


@pytest.mark.parametrize("name", sorted(pc.CORRECTIONS))
def test_each_misprint_changes_the_result(name):
    # Evaluated as printed, each of the seven terms breaks the agreement: the
    # corrections are not cosmetic.
    rng = np.random.default_rng(11)
    f, F, om = _random_node(D3Q27, rng)
    ours = collision.collide(D3Q27, f, F, om)
    as_printed = pc.cascade_d3q27(K27, list(f), list(F), om, printed=(name,))
    assert list(ours) != as_printed


@pytest.mark.parametrize("lat", [D3Q27, D3Q15], ids=str)
def test_float64_matches_exact(lat):
    rng = np.random.default_rng(21)
    f, F, om = _random_node(lat, rng)
    exact = np.array([float(v) for v in collision.collide(lat, f, F, om)])
    fl = collision.collide(lat, f.astype(float), F.astype(float), [float(w) for w in om])
    assert np.abs(fl - exact).max() <= 1e-14 * np.abs(exact).max()


@pytest.mark.parametrize("lat", [D3Q27, D3Q15], ids=str)
def test_conservation_exact(lat):
    rng = np.random.default_rng(31)
    f, F, om = _random_node(lat, rng)
    post = collision.collide(lat, f, F, om)
    E = lat.E.astype(object)
    assert post.sum() == f.sum()
    assert list(post @ E - f @ E) == list(F)            # momentum gains exactly F


def _central(lat, f, u):
    return (lat.Phi.astype(object) @ (collision.central_moment_matrix(lat, u) @ f[:, None]))[:, 0]


def test_galilean_invariance_d3q27():
    # A state with the same central moments about a shifted velocity has the
    # same post-collision central moments (exact, with forcing).
    rng = np.random.default_rng(41)
    f, F, om = _random_node(D3Q27, rng)
    rho, u = collision.macroscopic(D3Q27, f, F)
    U = np.array([Fraction(3, 17), Fraction(-2, 13), Fraction(1, 9)], dtype=object)
    cm = collision.central_moment_matrix(D3Q27, u) @ f
    f_shift = collision._solve(collision.central_moment_matrix(D3Q27, u + U), cm)
    rho2, u2 = collision.macroscopic(D3Q27, f_shift, F)
    assert rho2 == rho and list(u2) == list(u + U)
    post = collision.collide(D3Q27, f, F, om)
    post_shift = collision.collide(D3Q27, f_shift, F, om)
    assert list(_central(D3Q27, post, u)) == list(_central(D3Q27, post_shift, u + U))


def test_galilean_invariance_d3q15_unforced():
    # D3Q15: exact without force (its printed source is not de-aliased at third
    # order, so the forced case is not frame independent).
    rng = np.random.default_rng(42)
    f, F, om = _random_node(D3Q15, rng)
    F = np.array([Fraction(0)] * 3, dtype=object)
    rho, u = collision.macroscopic(D3Q15, f, F)
    U = np.array([Fraction(1, 7), Fraction(-1, 11), Fraction(2, 19)], dtype=object)
    cm = collision.central_moment_matrix(D3Q15, u) @ f
    f_shift = collision._solve(collision.central_moment_matrix(D3Q15, u + U), cm)
    post = collision.collide(D3Q15, f, F, om)
    post_shift = collision.collide(D3Q15, f_shift, F, om)
    assert list(_central(D3Q15, post, u)) == list(_central(D3Q15, post_shift, u + U))


@pytest.mark.parametrize("lat", [D3Q27, D3Q15], ids=str)
def test_equilibrium_fixed_point_unit_density(lat):
    rng = np.random.default_rng(51)
    u = np.array([_rat(rng, -0.3, 0.3, 37) for _ in range(3)], dtype=object)
    feq = collision.equilibrium(lat, np.array(Fraction(1), dtype=object), u)
    zero = np.array([Fraction(0)] * 3, dtype=object)
    om = [_rat(rng, 0.1, 1.95, 41) for _ in range(lat.Q - 4)]
    assert list(collision.collide(lat, feq, zero, om)) == list(feq)


def test_factorized_attractor_is_literal():
    # The attractor is kxx*kyy without a 1/rho: at rho != 1 the equilibrium
    # moves under omega_17 (reading of Eq. transformedcentralmomentattractors).
    u = np.array([Fraction(1, 10), Fraction(0), Fraction(-1, 20)], dtype=object)
    rho = Fraction(6, 5)
    feq = collision.equilibrium(D3Q27, np.array(rho, dtype=object), u)
    zero = np.array([Fraction(0)] * 3, dtype=object)
    om = [Fraction(1)] * 23
    post = collision.collide(D3Q27, feq, zero, om)
    cm = _central(D3Q27, post, u)
    # combination 17 = xxyy + xxzz + yyzz relaxes to 3 (rho/3)^2, not 3 rho/9
    assert cm[17] == 3 * (rho / 3) ** 2


@pytest.mark.parametrize("lat", [D3Q27, D3Q15], ids=str)
def test_unit_rates_reach_attractors(lat):
    rng = np.random.default_rng(61)
    f, F, _ = _random_node(lat, rng)
    om = [Fraction(1)] * (lat.Q - 4)
    post = collision.collide(lat, f, F, om)
    rho, u = collision.macroscopic(lat, f, F)
    cm = _central(lat, post, u)
    assert cm[0] == rho and list(cm[1:4]) == list(F / 2)
    kxx = (2 * cm[9] + 3 * cm[7] + cm[8]) / 6          # xx from (xx-yy, xx+yy-2zz, xx+yy+zz)
    # second-order diagonal combinations reach (0, 0, rho), off-diagonals 0
    assert list(cm[4:9]) == [0, 0, 0, 0, 0] and cm[9] == rho
    assert kxx == rho / 3
    higher = {17: 3 * (rho / 3) ** 2, 18: 0, 19: 0, 26: (rho / 3) ** 3} if lat.Q == 27 else {14: (rho / 3) ** 2}
    for b in range(10, lat.Q):
        assert cm[b] == higher.get(b, 0), b


# ----------------------------------------------------------------------------
# Per-unit-mass factorized attractors (the alternative reading of Sec. 3)
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("lat", [D3Q27, D3Q15], ids=str)
def test_per_mass_equilibrium_fixed_point_any_density(lat):
    # rho (kxx/rho)(kyy/rho) equals the Maxwellian c_s^4 rho at equilibrium for
    # every rho, so f^eq is a fixed point at any density; the literal form
    # moves it when rho != 1.
    rng = np.random.default_rng(52)
    u = np.array([_rat(rng, -0.3, 0.3, 37) for _ in range(3)], dtype=object)
    rho = Fraction(7, 5)
    feq = collision.equilibrium(lat, np.array(rho, dtype=object), u)
    zero = np.array([Fraction(0)] * 3, dtype=object)
    om = [_rat(rng, 0.1, 1.95, 41) for _ in range(lat.Q - 4)]
    assert list(collision.collide(lat, feq, zero, om, per_mass=True)) == list(feq)
    assert list(collision.collide(lat, feq, zero, om)) != list(feq)


@pytest.mark.parametrize("lat", [D3Q27, D3Q15], ids=str)
def test_per_mass_equals_literal_at_unit_density(lat):
    rng = np.random.default_rng(53)
    f, F, om = _random_node(lat, rng)
    f = f / f.sum()                                         # rho = 1 exactly
    assert f.sum() == 1
    assert list(collision.collide(lat, f, F, om, per_mass=True)) == list(collision.collide(lat, f, F, om))


@pytest.mark.parametrize("lat", [D3Q27, D3Q15], ids=str)
def test_per_mass_conservation_and_frame_independence(lat):
    rng = np.random.default_rng(54)
    f, F, om = _random_node(lat, rng)
    if lat.Q == 15:
        F = np.array([Fraction(0)] * 3, dtype=object)
    post = collision.collide(lat, f, F, om, per_mass=True)
    E = lat.E.astype(object)
    assert post.sum() == f.sum()
    assert list(post @ E - f @ E) == list(F)
    rho, u = collision.macroscopic(lat, f, F)
    U = np.array([Fraction(2, 17), Fraction(-1, 13), Fraction(1, 11)], dtype=object)
    cm = collision.central_moment_matrix(lat, u) @ f
    f_shift = collision._solve(collision.central_moment_matrix(lat, u + U), cm)
    post_shift = collision.collide(lat, f_shift, F, om, per_mass=True)
    assert list(_central(lat, post, u)) == list(_central(lat, post_shift, u + U))


def test_per_mass_attractor_value():
    # combination 17 = xxyy + xxzz + yyzz relaxes to 3 rho (1/3)^2 = rho/3 at
    # equilibrium second moments, for any rho.
    u = np.array([Fraction(1, 10), Fraction(0), Fraction(-1, 20)], dtype=object)
    rho = Fraction(6, 5)
    feq = collision.equilibrium(D3Q27, np.array(rho, dtype=object), u)
    zero = np.array([Fraction(0)] * 3, dtype=object)
    post = collision.collide(D3Q27, feq, zero, [Fraction(1)] * 23, per_mass=True)
    assert _central(D3Q27, post, u)[17] == rho / 3
