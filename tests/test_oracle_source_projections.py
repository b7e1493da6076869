"""Pins of the oracle's source projections m^s_b = <K_b|S> by a second route.

Appendix G prints the D3Q15 projections m^s_0..m^s_14 and says that the raw
source moments behind them follow "analogously" to the D3Q27 ones of Appendix
C.  Those raw moments come from the continuous source (Sec. 3, Eq.
forcingaliased, with the discrete central source moments of Eq.
discretecentralsources): every central moment of the source vanishes except
the first-order ones, which equal F.  The binomial theorem then gives each raw
moment of the monomial x^a y^b z^c as the directional derivative of
u_x^a u_y^b u_z^c along F:

    sigma'_abc = a F_x u_x^(a-1) u_y^b u_z^c + b F_y u_x^a u_y^(b-1) u_z^c
                 + c F_z u_x^a u_y^b u_z^(c-1).

Projecting onto K_b written as a polynomial in (e_x, e_y, e_z) (the Gram-Schmidt
forms listed in Sec. 2 for D3Q27 and Appendix G for D3Q15), monomial by
monomial, reproduces the printed projections.  The polynomials are typed here
from the paper, independently of the oracle's tables, and checked against the
printed integer matrices.  The comparison is exact on random rational (F, u),
so changing any coefficient of any row of the oracle's m^s fails it.
"""
from fractions import Fraction

import numpy as np
import pytest

from golden_io import load_int_table
from oracle import collision
from oracle.lattice import D3Q15, D3Q27


def _poly(*terms):
    """{(a, b, c): coefficient} from (coefficient, word) pairs, word in x/y/z letters ('1' = constant)."""
    out = {}
    for coef, word in terms:
        mono = (0, 0, 0) if word == "1" else (word.count("x"), word.count("y"), word.count("z"))
        out[mono] = out.get(mono, 0) + coef
    return out


# Appendix G, the orthogonal D3Q15 basis K_0 .. K_14 as polynomials.
K15_FORMS = [
    _poly((1, "1")),
    _poly((1, "x")), _poly((1, "y")), _poly((1, "z")),
    _poly((1, "xy")), _poly((1, "xz")), _poly((1, "yz")),
    _poly((1, "xx"), (-1, "yy")),
    _poly((1, "xx"), (1, "yy"), (1, "zz"), (-3, "zz")),
    _poly((1, "xx"), (1, "yy"), (1, "zz"), (-2, "1")),
    _poly((5, "xxx"), (5, "xyy"), (5, "xzz"), (-13, "x")),
    _poly((5, "xxy"), (5, "yyy"), (5, "yzz"), (-13, "y")),
    _poly((5, "xxz"), (5, "yyz"), (5, "zzz"), (-13, "z")),
    _poly((1, "xyz")),
    _poly((30, "xxyy"), (30, "xxzz"), (30, "yyzz"), (-40, "xx"), (-40, "yy"), (-40, "zz"), (32, "1")),
]

# Sec. 2, the orthogonal D3Q27 basis K_0 .. K_26 as polynomials (used to show
# that the same projection reproduces the printed Appendix D).
K27_FORMS = [
    _poly((1, "1")),
    _poly((1, "x")), _poly((1, "y")), _poly((1, "z")),
    _poly((1, "xy")), _poly((1, "xz")), _poly((1, "yz")),
    _poly((1, "xx"), (-1, "yy")),
    _poly((1, "xx"), (1, "yy"), (-2, "zz")),
    _poly((1, "xx"), (1, "yy"), (1, "zz"), (-2, "1")),
    _poly((3, "xyy"), (3, "xzz"), (-4, "x")),
    _poly((3, "xxy"), (3, "yzz"), (-4, "y")),
    _poly((3, "xxz"), (3, "yyz"), (-4, "z")),
    _poly((1, "xyy"), (-1, "xzz")),
    _poly((1, "xxy"), (-1, "yzz")),
    _poly((1, "xxz"), (-1, "yyz")),
    _poly((1, "xyz")),
    _poly((3, "xxyy"), (3, "xxzz"), (3, "yyzz"), (-4, "xx"), (-4, "yy"), (-4, "zz"), (4, "1")),
    _poly((3, "xxyy"), (3, "xxzz"), (-6, "yyzz"), (-4, "xx"), (2, "yy"), (2, "zz")),
    _poly((3, "xxyy"), (-3, "xxzz"), (-2, "yy"), (2, "zz")),
    _poly((3, "xxyz"), (-2, "yz")),
    _poly((3, "xyyz"), (-2, "xz")),
    _poly((3, "xyzz"), (-2, "xy")),
    _poly((9, "xyyzz"), (-6, "xyy"), (-6, "xzz"), (4, "x")),
    _poly((9, "xxyzz"), (-6, "xxy"), (-6, "yzz"), (4, "y")),
    _poly((9, "xxyyz"), (-6, "xxz"), (-6, "yyz"), (4, "z")),
    _poly((27, "xxyyzz"), (-18, "xxyy"), (-18, "xxzz"), (-18, "yyzz"), (12, "xx"), (12, "yy"), (12, "zz"),
          (-8, "1")),
]


def _continuous_raw_source_moment(mono, F, u):
    """Raw moment of the continuous source: the derivative of u^mono along F."""
    a, b, c = mono
    total = Fraction(0)
    for axis, k in enumerate(mono):
        if k == 0:
            continue
        powers = [a, b, c]
        powers[axis] -= 1
        total += k * F[axis] * u[0] ** powers[0] * u[1] ** powers[1] * u[2] ** powers[2]
    return total


def _projections(forms, F, u):
    return [sum(coef * _continuous_raw_source_moment(mono, F, u) for mono, coef in form.items())
            for form in forms]


def _on_lattice(forms, E):
    return [[sum(coef * int(e[0]) ** m[0] * int(e[1]) ** m[1] * int(e[2]) ** m[2] for m, coef in form.items())
             for form in forms] for e in E]


def _random_fu(rng):
    F = [Fraction(int(rng.integers(-997, 998)), 997 * 100) for _ in range(3)]
    u = [Fraction(int(rng.integers(-30, 31)), 101) for _ in range(3)]
    return F, u


def test_typed_forms_match_printed_matrices():
    # The polynomials above, evaluated on the lattice directions, are the
    # printed integer matrices (Appendix A, Appendix G).
    assert _on_lattice(K15_FORMS, D3Q15.E) == load_int_table("K15_appendix_G.txt").tolist()
    assert _on_lattice(K27_FORMS, D3Q27.E) == load_int_table("K27_appendix_A.txt").tolist()


def test_projection_route_reproduces_printed_d3q27_appendix_D():
    # Appendix C -> Appendix D by the projection above, on D3Q27, where the
    # oracle does not use m^s (it solves the matching principle): the printed
    # S_a of Appendix E is K D^-1 m^s, so the oracle's S must project onto K
    # exactly to the derived m^s.
    rng = np.random.default_rng(31)
    K = load_int_table("K27_appendix_A.txt")
    for _ in range(4):
        F, u = _random_fu(rng)
        derived = _projections(K27_FORMS, F, u)
        S = collision.source(D3Q27, np.array(F, dtype=object), np.array(u, dtype=object))
        projected = [sum(int(K[a, b]) * S[a] for a in range(27)) for b in range(27)]
        assert projected == derived


@pytest.mark.parametrize("seed", range(6))
def test_d3q15_projections_from_continuous_raw_moments(seed):
    # Every row of the oracle's D3Q15 m^s, including the third-order rows
    # 10-12 and the fourth-order row 14, equals the K_b projection of the
    # continuous raw source moments.
    rng = np.random.default_rng(200 + seed)
    F, u = _random_fu(rng)
    derived = _projections(K15_FORMS, F, u)
    oracle_ms = collision.source_projections_d3q15(np.array(F, dtype=object), np.array(u, dtype=object))
    assert list(oracle_ms) == derived
    # rows 10, 11, 12 and 14 depend on F and u at every order they carry
    assert all(derived[b] != 0 for b in (10, 11, 12, 14))


def test_d3q15_source_is_K_D_inverse_of_derived_projections():
    # S = K D^-1 m^s (inversion through K^T K = D, Sec. 6): the oracle's S
    # projects back onto the derived m^s row by row.
    rng = np.random.default_rng(77)
    K = load_int_table("K15_appendix_G.txt")
    for _ in range(3):
        F, u = _random_fu(rng)
        S = collision.source(D3Q15, np.array(F, dtype=object), np.array(u, dtype=object))
        projected = [sum(int(K[a, b]) * S[a] for a in range(15)) for b in range(15)]
        assert projected == _projections(K15_FORMS, F, u)


def test_third_order_lattice_moments_alias_on_d3q15():
    # Why the derived m^s_10 differs from a plain raw-moment reading: on D3Q15
    # e_x^3 = e_x, so the lattice third moments of S are not the continuous
    # ones.  <S| e_x e_y^2> of the printed S differs from F_x u_y^2 + 2 F_y u_x u_y
    # by a term of order F (reading recorded for eta').
    rng = np.random.default_rng(5)
    F, u = _random_fu(rng)
    S = collision.source(D3Q15, np.array(F, dtype=object), np.array(u, dtype=object))
    lattice_xyy = sum(S[a] * int(e[0]) * int(e[1]) ** 2 for a, e in enumerate(D3Q15.E))
    continuous_xyy = F[0] * u[1] ** 2 + 2 * F[1] * u[0] * u[1]
    assert lattice_xyy != continuous_xyy
    # the difference is linear in F with no u-free part cancelled: at u = 0 it is -F_x/2
    S0 = collision.source(D3Q15, np.array(F, dtype=object), np.array([Fraction(0)] * 3, dtype=object))
    assert sum(S0[a] * int(e[0]) * int(e[1]) ** 2 for a, e in enumerate(D3Q15.E)) == -F[0] / 2
