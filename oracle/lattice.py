"""Lattice tables of the D3Q27 and D3Q15 central-moment LBM (test infrastructure).

Sources in the paper:
* D3Q27 velocity set: Eq. (velocityd3qq27), Sec. 2; the order of the 27
  directions is the row order of the matrix K in Appendix A (its columns 1-3
  are e_x, e_y, e_z).
* D3Q27 orthogonal basis K_0..K_26: Sec. 2 (Gram-Schmidt result, Eq.
  collisionmatrix1); D = diag(<K_b|K_b>): Sec. 6, after Eq. sourceformulation1.
* D3Q15 velocity set and basis: Appendix G (Eq. velocityd3q15 and the K list).
* Which central-moment combination each collision kernel g_b relaxes: the
  bracket of Eqs. (collisionkernelg4)-(collisionkernelg26) for D3Q27 and the
  collision kernel list of Appendix G for D3Q15.
* Attractors per central moment: Eq. (transformedcentralmomentattractors),
  Sec. 5 (order >= 2 entries) and Appendix G (g_14 bracket) for D3Q15.
* Maxwellian central moments: Sec. 3 list after Eq. (centralmomentfeqdefinition).

A monomial (a, b, c) stands for e_x^a e_y^b e_z^c, or, for a central moment,
(e_x-u_x)^a (e_y-u_y)^b (e_z-u_z)^c.
"""
from fractions import Fraction

import numpy as np

# ----------------------------------------------------------------------------
# Velocity sets
# ----------------------------------------------------------------------------
E27 = np.array([
    (0, 0, 0),
    (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1),
    (1, 1, 0), (-1, 1, 0), (1, -1, 0), (-1, -1, 0),
    (1, 0, 1), (-1, 0, 1), (1, 0, -1), (-1, 0, -1),
    (0, 1, 1), (0, -1, 1), (0, 1, -1), (0, -1, -1),
    (1, 1, 1), (-1, 1, 1), (1, -1, 1), (-1, -1, 1),
    (1, 1, -1), (-1, 1, -1), (1, -1, -1), (-1, -1, -1),
], dtype=np.int64)

# D3Q15: rest, six axis links, eight corners (same order as D3Q27's 19..26).
E15 = np.concatenate([E27[:7], E27[19:]], axis=0)


def opposite_map(E):
    """Index of -e_a for every direction a."""
    out = np.empty(len(E), dtype=np.int64)
    for a, e in enumerate(E):
        hits = np.where((E == -e).all(axis=1))[0]
        assert len(hits) == 1
        out[a] = hits[0]
    return out


# ----------------------------------------------------------------------------
# Polynomials in (e_x, e_y, e_z): dict {(a, b, c): integer coefficient}
# ----------------------------------------------------------------------------
def _p(*terms):
    """Build a polynomial from (coef, 'xyz-word') pairs; '1' is the constant."""
    poly = {}
    for coef, word in terms:
        mono = (0, 0, 0) if word == "1" else (word.count("x"), word.count("y"), word.count("z"))
        poly[mono] = poly.get(mono, 0) + coef
    return {m: c for m, c in poly.items() if c != 0}


SUM2 = ((1, "xx"), (1, "yy"), (1, "zz"))                       # e_x^2+e_y^2+e_z^2
SUM4 = ((1, "xxyy"), (1, "xxzz"), (1, "yyzz"))


def _scaled(k, terms):
    return tuple((k * c, w) for c, w in terms)


# Sec. 2: orthogonal basis vectors K_0..K_26 of the D3Q27 lattice, as written.
K27_POLY = [
    _p((1, "1")),
    _p((1, "x")), _p((1, "y")), _p((1, "z")),
    _p((1, "xy")), _p((1, "xz")), _p((1, "yz")),
    _p((1, "xx"), (-1, "yy")),
    _p(*SUM2, (-3, "zz")),
    _p(*SUM2, (-2, "1")),
    _p((3, "xyy"), (3, "xzz"), (-4, "x")),
    _p((3, "xxy"), (3, "yzz"), (-4, "y")),
    _p((3, "xxz"), (3, "yyz"), (-4, "z")),
    _p((1, "xyy"), (-1, "xzz")),
    _p((1, "xxy"), (-1, "yzz")),
    _p((1, "xxz"), (-1, "yyz")),
    _p((1, "xyz")),
    _p(*_scaled(3, SUM4), *_scaled(-4, SUM2), (4, "1")),
    _p((3, "xxyy"), (3, "xxzz"), (-6, "yyzz"), (-4, "xx"), (2, "yy"), (2, "zz")),
    _p((3, "xxyy"), (-3, "xxzz"), (-2, "yy"), (2, "zz")),
    _p((3, "xxyz"), (-2, "yz")),
    _p((3, "xyyz"), (-2, "xz")),
    _p((3, "xyzz"), (-2, "xy")),
    _p((9, "xyyzz"), (-6, "xyy"), (-6, "xzz"), (4, "x")),
    _p((9, "xxyzz"), (-6, "xxy"), (-6, "yzz"), (4, "y")),
    _p((9, "xxyyz"), (-6, "xxz"), (-6, "yyz"), (4, "z")),
    _p((27, "xxyyzz"), *_scaled(-18, SUM4), *_scaled(12, SUM2), (-8, "1")),
]

# Appendix G: orthogonal basis K_0..K_14 of the D3Q15 lattice, as written.
K15_POLY = K27_POLY[:10] + [
    _p((5, "xxx"), (5, "xyy"), (5, "xzz"), (-13, "x")),
    _p((5, "xxy"), (5, "yyy"), (5, "yzz"), (-13, "y")),
    _p((5, "xxz"), (5, "yyz"), (5, "zzz"), (-13, "z")),
    _p((1, "xyz")),
    _p(*_scaled(30, SUM4), *_scaled(-40, SUM2), (32, "1")),
]


def eval_poly(poly, E):
    """Values of a polynomial on each lattice direction (integer vector)."""
    out = np.zeros(len(E), dtype=np.int64)
    for (a, b, c), coef in poly.items():
        out += coef * E[:, 0] ** a * E[:, 1] ** b * E[:, 2] ** c
    return out


# ----------------------------------------------------------------------------
# Central moments: monomial sets and relaxed combinations
# ----------------------------------------------------------------------------
# D3Q27 supports every e_x^a e_y^b e_z^c with a, b, c <= 2 (Sec. 2).  Listed by
# order so that the combination matrix below is block diagonal by order.
MONO27 = sorted([(a, b, c) for a in range(3) for b in range(3) for c in range(3)],
                key=lambda m: (sum(m), -m[0], -m[1]))
# D3Q15: the fifteen monomials its basis and collision kernel use (Appendix G).
MONO15 = [(0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1),
          (1, 1, 0), (1, 0, 1), (0, 1, 1), (2, 0, 0), (0, 2, 0), (0, 0, 2),
          (1, 2, 0), (2, 1, 0), (2, 0, 1), (1, 1, 1), (2, 2, 0)]

# Central-moment combination relaxed by each kernel g_b (b >= 4), read off the
# bracket of the paper's g_b: e.g. g_10 relaxes (xyy + xzz), g_18 relaxes
# (xxyy + xxzz - 2 yyzz).  Rows 0..3 are the conserved rho and first moments.
COMBO27 = [
    _p((1, "1")), _p((1, "x")), _p((1, "y")), _p((1, "z")),
    _p((1, "xy")), _p((1, "xz")), _p((1, "yz")),                     # g4 g5 g6
    _p((1, "xx"), (-1, "yy")),                                         # g7
    _p((1, "xx"), (1, "yy"), (-2, "zz")),                              # g8
    _p(*SUM2),                                                         # g9
    _p((1, "xyy"), (1, "xzz")), _p((1, "xxy"), (1, "yzz")),            # g10 g11
    _p((1, "xxz"), (1, "yyz")),                                        # g12
    _p((1, "xyy"), (-1, "xzz")), _p((1, "xxy"), (-1, "yzz")),          # g13 g14
    _p((1, "xxz"), (-1, "yyz")),                                       # g15
    _p((1, "xyz")),                                                    # g16
    _p(*SUM4),                                                         # g17
    _p((1, "xxyy"), (1, "xxzz"), (-2, "yyzz")),                        # g18
    _p((1, "xxyy"), (-1, "xxzz")),                                     # g19
    _p((1, "xxyz")), _p((1, "xyyz")), _p((1, "xyzz")),                 # g20 g21 g22
    _p((1, "xyyzz")), _p((1, "xxyzz")), _p((1, "xxyyz")),              # g23 g24 g25
    _p((1, "xxyyzz")),                                                 # g26
]
COMBO15 = COMBO27[:10] + [
    _p((1, "xyy")), _p((1, "xxy")), _p((1, "xxz")),                    # g10 g11 g12
    _p((1, "xyz")),                                                    # g13
    _p((1, "xxyy")),                                                   # g14
]


def combo_matrix(combos, monos):
    """Phi[b, m]: coefficient of central monomial m in combination b."""
    index = {m: i for i, m in enumerate(monos)}
    phi = np.zeros((len(combos), len(monos)), dtype=np.int64)
    for b, poly in enumerate(combos):
        for mono, coef in poly.items():
            phi[b, index[mono]] = coef
    return phi


# Attractor of each central monomial of order >= 2 (Eq.
# transformedcentralmomentattractors): 'cs2' -> c_s^2 rho, a tuple of axes ->
# product of the post-collision second-order central moments on those axes,
# anything unlisted -> 0.  Orders 0 and 1 are conserved and never relaxed.
ATTRACTOR27 = {(2, 0, 0): "cs2", (0, 2, 0): "cs2", (0, 0, 2): "cs2",
               (2, 2, 0): (0, 1), (2, 0, 2): (0, 2), (0, 2, 2): (1, 2),
               (2, 2, 2): (0, 1, 2)}
ATTRACTOR15 = {(2, 0, 0): "cs2", (0, 2, 0): "cs2", (0, 0, 2): "cs2",
               (2, 2, 0): (0, 1)}

# Maxwellian central moments (Sec. 3): rho, c_s^2 rho, c_s^4 rho, c_s^6 rho on
# the even monomials, zero elsewhere.  Value = power of c_s^2 multiplying rho.
MAXWELL27 = {(0, 0, 0): 0, (2, 0, 0): 1, (0, 2, 0): 1, (0, 0, 2): 1,
             (2, 2, 0): 2, (2, 0, 2): 2, (0, 2, 2): 2, (2, 2, 2): 3}
MAXWELL15 = {(0, 0, 0): 0, (2, 0, 0): 1, (0, 2, 0): 1, (0, 0, 2): 1, (2, 2, 0): 2}

CS2 = Fraction(1, 3)          # c_s^2, Sec. 3 (after Eq. Maxwellian)


class Lattice:
    """All tables of one lattice model."""

    def __init__(self, name, E, K_poly, monos, combos, attractor, maxwell):
        self.name = name
        self.E = E
        self.Q = len(E)
        self.opp = opposite_map(E)
        self.K_poly = K_poly
        self.K = np.stack([eval_poly(p, E) for p in K_poly], axis=1)   # K[a, b]
        self.D = (self.K * self.K).sum(axis=0)                          # <K_b|K_b>
        self.monos = monos
        self.combos = combos
        self.Phi = combo_matrix(combos, monos)
        self.order = np.array([max(sum(m) for m in poly) for poly in combos])
        self.attractor = attractor
        self.maxwell = maxwell

    def __repr__(self):
        return f"Lattice({self.name})"


D3Q27 = Lattice("D3Q27", E27, K27_POLY, MONO27, COMBO27, ATTRACTOR27, MAXWELL27)
D3Q15 = Lattice("D3Q15", E15, K15_POLY, MONO15, COMBO15, ATTRACTOR15, MAXWELL15)
LATTICES = {27: D3Q27, 15: D3Q15}
