"""Pins of the oracle's lattice tables against what the paper prints."""
from fractions import Fraction

import numpy as np
import pytest

from golden_io import load_int_table
from oracle import collision
from oracle.lattice import D3Q15, D3Q27
import paper_cascade as pc


def _mono_values(E, word):
    return E[:, 0] ** word.count("x") * E[:, 1] ** word.count("y") * E[:, 2] ** word.count("z")


def test_K27_matches_appendix_A():
    # K built from the Gram-Schmidt definitions of Sec. 2 equals the printed matrix.
    assert (D3Q27.K == load_int_table("K27_appendix_A.txt")).all()


def test_K15_matches_appendix_G():
    assert (D3Q15.K == load_int_table("K15_appendix_G.txt")).all()


@pytest.mark.parametrize("lat", [D3Q27, D3Q15], ids=str)
def test_basis_orthogonal(lat):
    G = lat.K.T @ lat.K
    assert (G == np.diag(lat.D)).all()


@pytest.mark.parametrize("lat", [D3Q27, D3Q15], ids=str)
def test_velocity_columns_and_opposites(lat):
    # Columns 1-3 of the printed K are e_x, e_y, e_z (Sec. 2, Appendix G).
    name = "K27_appendix_A.txt" if lat.Q == 27 else "K15_appendix_G.txt"
    assert (load_int_table(name)[:, 1:4] == lat.E).all()
    assert (lat.E[lat.opp] == -lat.E).all()


def test_ab_sets_are_sign_patterns_d3q27():
    # Appendix B: each printed A/B pair lists the +1 / -1 entries of the monomial.
    for word, (A, B) in pc.AB27.items():
        v = _mono_values(D3Q27.E, word)
        assert set(np.where(v == 1)[0]) == A and set(np.where(v == -1)[0]) == B, word
        assert set(np.where(v == 0)[0]) == set(range(27)) - A - B, word


def test_ab_sets_are_sign_patterns_d3q15():
    for word, (A, B) in pc.AB15.items():
        v = _mono_values(D3Q15.E, word)
        assert set(np.where(v == 1)[0]) == A and set(np.where(v == -1)[0]) == B, word


# Appendix F (D3Q27) and Appendix G (D3Q15): sum_a (K g)_a e^mnp as linear
# forms in g_4.. (g_0..g_3 are zero).
KERNEL_MOMENTS_27 = {
    "xy": {4: 12}, "xz": {5: 12}, "yz": {6: 12},
    "xx": {7: 6, 8: 6, 9: 6}, "yy": {7: -6, 8: 6, 9: 6}, "zz": {8: -12, 9: 6},
    "xyy": {10: 12, 13: 4}, "xzz": {10: 12, 13: -4}, "xxy": {11: 12, 14: 4}, "yzz": {11: 12, 14: -4},
    "xxz": {12: 12, 15: 4}, "yyz": {12: 12, 15: -4}, "xyz": {16: 8},
    "xxyy": {8: 8, 9: 8, 17: 4, 18: 4, 19: 4}, "xxzz": {7: 4, 8: -4, 9: 8, 17: 4, 18: 4, 19: -4},
    "yyzz": {7: -4, 8: -4, 9: 8, 17: 4, 18: -8},
    "xxyz": {6: 8, 20: 8}, "xyyz": {5: 8, 21: 8}, "xyzz": {4: 8, 22: 8},
    "xyyzz": {10: 16, 23: 8}, "xxyzz": {11: 16, 24: 8}, "xxyyz": {12: 16, 25: 8},
    "xxyyzz": {9: 8, 17: 8, 26: 8},
    "1": {}, "x": {}, "y": {}, "z": {},
}
KERNEL_MOMENTS_15 = {
    "xy": {4: 8}, "xz": {5: 8}, "yz": {6: 8},
    "xx": {7: 2, 8: 2, 9: 6}, "yy": {7: -2, 8: 2, 9: 6}, "zz": {8: -4, 9: 6},
    "xyy": {10: 16}, "xzz": {10: 16}, "xxy": {11: 16}, "yzz": {11: 16}, "xxz": {12: 16}, "yyz": {12: 16},
    "xyz": {13: 8}, "xxyy": {9: 8, 14: 16}, "xxzz": {9: 8, 14: 16}, "yyzz": {9: 8, 14: 16},
    "1": {}, "x": {}, "y": {}, "z": {},
}


@pytest.mark.parametrize("lat,table", [(D3Q27, KERNEL_MOMENTS_27), (D3Q15, KERNEL_MOMENTS_15)], ids=["D3Q27", "D3Q15"])
def test_kernel_moment_tables(lat, table):
    for word, coeffs in table.items():
        v = np.ones(lat.Q, dtype=np.int64) if word == "1" else _mono_values(lat.E, word)
        got = v @ lat.K                                        # <K_b | e^mnp>
        want = np.zeros(lat.Q, dtype=np.int64)
        for b, c in coeffs.items():
            want[b] = c
        assert (got[4:] == want[4:]).all(), word


def test_rest_equilibrium_weights():
    # Textbook lattice weights: D3Q27 8/27, 2/27, 1/54, 1/216; D3Q15 2/9, 1/9, 1/72.
    one = np.array(Fraction(1), dtype=object)
    zero_u = np.array([Fraction(0)] * 3, dtype=object)
    w27 = collision.equilibrium(D3Q27, one, zero_u)
    n27 = np.abs(D3Q27.E).sum(axis=1)
    for k, w in zip(range(4), [Fraction(8, 27), Fraction(2, 27), Fraction(1, 54), Fraction(1, 216)]):
        assert all(w27[a] == w for a in np.where(n27 == k)[0])
    w15 = collision.equilibrium(D3Q15, one, zero_u)
    n15 = np.abs(D3Q15.E).sum(axis=1)
    for k, w in [(0, Fraction(2, 9)), (1, Fraction(1, 9)), (3, Fraction(1, 72))]:
        assert all(w15[a] == w for a in np.where(n15 == k)[0])


def test_d3q27_equilibrium_product_form():
    # The D3Q27 equilibrium matching the Maxwellian central moments factorizes
    # per axis: f_a = rho prod_i w1(e_ai; u_i), w1(0) = 2/3 - u^2,
    # w1(+-1) = (1/3 + u^2 +- u)/2.
    rng = np.random.default_rng(0)
    rho = np.array(Fraction(int(rng.integers(90, 110)), 100), dtype=object)
    u = np.array([Fraction(int(v), 200) for v in rng.integers(-20, 20, 3)], dtype=object)
    feq = collision.equilibrium(D3Q27, rho, u)

    def w1(e, ui):
        return Fraction(2, 3) - ui**2 if e == 0 else (Fraction(1, 3) + ui**2 + e * ui) / 2

    for a, e in enumerate(D3Q27.E):
        assert feq[a] == rho * w1(e[0], u[0]) * w1(e[1], u[1]) * w1(e[2], u[2])


def _rational(rng, lo, hi, den):
    return Fraction(int(rng.integers(int(lo * den), int(hi * den))), den)


def test_d3q27_source_equals_appendix_D_E():
    # The oracle solves the matching principle (central moments of S = F on
    # first order, 0 elsewhere); the paper prints S = K D^-1 m^s with m^s of
    # Appendix D.  Exact equality on random rational (F, u).
    rng = np.random.default_rng(5)
    K = load_int_table("K27_appendix_A.txt").tolist()
    for _ in range(4):
        F = [_rational(rng, -0.01, 0.01, 997) for _ in range(3)]
        u = [_rational(rng, -0.3, 0.3, 101) for _ in range(3)]
        S = collision.source(D3Q27, np.array(F, dtype=object), np.array(u, dtype=object))
        printed = pc._source(K, pc.source_projections_d3q27(F, u))
        assert list(S) == printed


def test_d3q27_raw_source_moments_appendix_C():
    # Appendix C: raw source moments, e.g. sigma'_xx = 2 F_x u_x,
    # sigma'_xyy = F_x u_y^2 + 2 F_y u_y u_x, sigma'_xxyyzz = 2 ux uy uz (Fx uy uz + ...).
    rng = np.random.default_rng(6)
    F = [_rational(rng, -0.01, 0.01, 997) for _ in range(3)]
    u = [_rational(rng, -0.3, 0.3, 101) for _ in range(3)]
    S = collision.source(D3Q27, np.array(F, dtype=object), np.array(u, dtype=object))
    Fx, Fy, Fz = F
    ux, uy, uz = u
    m = pc.raw_moments(list(S), pc.AB27, (pc.X27, pc.Y27, pc.Z27))
    assert m["1"] == 0 and (m["x"], m["y"], m["z"]) == (Fx, Fy, Fz)
    assert m["xx"] == 2 * Fx * ux and m["yy"] == 2 * Fy * uy and m["zz"] == 2 * Fz * uz
    assert m["xy"] == Fx * uy + Fy * ux
    assert m["xyy"] == Fx * uy**2 + 2 * Fy * uy * ux
    assert m["xxz"] == Fz * ux**2 + 2 * Fx * ux * uz
    assert m["xyz"] == Fx * uy * uz + Fy * ux * uz + Fz * ux * uy
    assert m["xxyy"] == 2 * Fx * ux * uy**2 + 2 * Fy * uy * ux**2
    assert m["xxyz"] == ux**2 * (Fy * uz + Fz * uy) + 2 * Fx * ux * uy * uz
    assert m["xyyzz"] == Fx * uy**2 * uz**2 + 2 * ux * uy * uz * (Fy * uz + Fz * uy)
    assert m["xxyyzz"] == 2 * ux * uy * uz * (Fx * uy * uz + Fy * uz * ux + Fz * ux * uy)


def test_d3q15_source_low_moments():
    # The printed D3Q15 source has zero mass, first moments F and second
    # moments equal to the continuous ones (2 F_i u_i, F_i u_j + F_j u_i).
    rng = np.random.default_rng(7)
    F = [_rational(rng, -0.01, 0.01, 997) for _ in range(3)]
    u = [_rational(rng, -0.3, 0.3, 101) for _ in range(3)]
    S = list(collision.source(D3Q15, np.array(F, dtype=object), np.array(u, dtype=object)))
    m = pc.raw_moments(S, pc.AB15, (pc.X15, pc.Y15, pc.Z15))
    assert m["1"] == 0 and (m["x"], m["y"], m["z"]) == tuple(F)
    assert m["xx"] == 2 * F[0] * u[0] and m["zz"] == 2 * F[2] * u[2]
    assert m["xz"] == F[0] * u[2] + F[2] * u[0]
    assert m["xyz"] == F[0] * u[1] * u[2] + F[1] * u[0] * u[2] + F[2] * u[0] * u[1]
