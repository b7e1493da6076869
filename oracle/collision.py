"""Per-node central-moment collision with forcing, as its plain definition.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper reaches, through its cascaded kernels g_4..g_26 (Sec. 7) and the
post-collision rows of Sec. 8, a result with a short plain definition, which is
what this module writes out (all arrays carry the node batch in the leading
axes and the lattice direction / moment index in the last axis):

1.  rho = sum_a fbar_a,  rho u = sum_a fbar_a e_a + F/2
    (Eqs. densitycalculation, velocitycalculation).
2.  Source S.  D3Q27: the populations whose discrete central moments equal the
    de-aliased continuous ones, F on the three first-order moments and zero on
    every other moment (matching principle, Sec. 5, Eqs. forcingaliased and
    discretecentralsources).  D3Q15: S = K D^-1 m^s with the projections m^s
    printed in Appendix G.
3.  h = fbar + S.  Its central moments about u are formed for every
    combination that a kernel g_b relaxes (raw moments eta' = kappabar' +
    sigma' of Sec. 7 are exactly the raw moments of h).
4.  Each combination relaxes toward its attractor, lowest order first:
    C~_b = C_b + omega_b (A_b - C_b).  The attractors are c_s^2 rho on the
    diagonal second moments and the factorized products of the post-collision
    second-order central moments on xxyy-type and xxyyzz moments (Eq.
    transformedcentralmomentattractors); all others are zero.  Density and the
    first central moments (= F/2) are collision invariants.
5.  The post-collision populations are the unique populations with the
    central moments C~, i.e. fbar~ = (Phi M(u))^-1 C~, which the paper writes
    as fbar + K g + S.

A library linear solve is the only numerical primitive.  The functions accept
float64, complex128 (complex-step derivatives) and object arrays of
fractions.Fraction (exact rational checks).
"""
from fractions import Fraction

import numpy as np

from .lattice import CS2


# ----------------------------------------------------------------------------
# dtype-generic helpers
# ----------------------------------------------------------------------------
def _is_exact(a):
    return np.asarray(a).dtype == object


def _num(value, like):
    """A constant in the arithmetic of ``like`` (Fraction for exact arrays)."""
    if _is_exact(like):
        return Fraction(value)
    return float(value)


def _solve(A, b):
    """Solve A x = b over the last axes; batched.  Exact Gauss-Jordan for
    Fraction arrays, LAPACK otherwise."""
    if not _is_exact(A):
        return np.linalg.solve(A, b[..., None])[..., 0]
    A = np.asarray(A, dtype=object)
    b = np.asarray(b, dtype=object)
    batch = np.broadcast_shapes(A.shape[:-2], b.shape[:-1])
    A = np.broadcast_to(A, batch + A.shape[-2:])
    b = np.broadcast_to(b, batch + b.shape[-1:])
    out = np.empty(batch + b.shape[-1:], dtype=object)
    n = A.shape[-1]
    for idx in np.ndindex(*batch):
        M = [[Fraction(A[idx][i, j]) for j in range(n)] + [Fraction(b[idx][i])] for i in range(n)]
        for col in range(n):
            piv = next(r for r in range(col, n) if M[r][col] != 0)
            M[col], M[piv] = M[piv], M[col]
            p = M[col][col]
            M[col] = [v / p for v in M[col]]
            for r in range(n):
                if r != col and M[r][col] != 0:
                    k = M[r][col]
                    M[r] = [vr - k * vc for vr, vc in zip(M[r], M[col])]
        out[idx] = np.array([M[i][n] for i in range(n)], dtype=object)
    return out


# ----------------------------------------------------------------------------
# Building blocks
# ----------------------------------------------------------------------------
def macroscopic(lat, fbar, F):
    """rho and u from transformed populations (Eqs. densitycalculation,
    velocitycalculation): rho u = sum fbar e + F/2."""
    E = lat.E.astype(object) if _is_exact(fbar) else lat.E
    rho = np.asarray(fbar.sum(axis=-1))
    j = fbar @ E + F * _num(Fraction(1, 2), fbar)
    return rho, j / rho[..., None]


def central_moment_matrix(lat, u):
    """M[..., m, a] = prod_i (e_ai - u_i)^(exponent_i of monomial m)."""
    E = lat.E.astype(object) if _is_exact(u) else lat.E
    c = E - u[..., None, :]                        # (..., Q, 3): e_a - u
    rows = []
    for (p, q, r) in lat.monos:
        rows.append(c[..., 0] ** p * c[..., 1] ** q * c[..., 2] ** r)
    return np.stack(rows, axis=-2)


def _first_order_vector(lat, values3, like):
    """Vector over lat.monos with the three given values on x, y, z."""
    shape = values3.shape[:-1] + (len(lat.monos),)
    out = np.zeros(shape, dtype=object) if _is_exact(like) else np.zeros(shape, dtype=np.result_type(values3, like))
    if _is_exact(like):
        out[...] = Fraction(0)
    for axis, mono in enumerate([(1, 0, 0), (0, 1, 0), (0, 0, 1)]):
        out[..., lat.monos.index(mono)] = values3[..., axis]
    return out


def source_projections_d3q15(F, u):
    """m^s_b = <K_b|S> for D3Q15, as printed in Appendix G."""
    Fx, Fy, Fz = F[..., 0], F[..., 1], F[..., 2]
    ux, uy, uz = u[..., 0], u[..., 1], u[..., 2]
    zero = Fx * 0
    return np.stack([
        zero,
        Fx, Fy, Fz,
        Fx * uy + Fy * ux,
        Fx * uz + Fz * ux,
        Fy * uz + Fz * uy,
        2 * (Fx * ux - Fy * uy),
        2 * (Fx * ux + Fy * uy - 2 * Fz * uz),
        2 * (Fx * ux + Fy * uy + Fz * uz),
        5 * (Fx * (3 * ux**2 + uy**2 + uz**2) + 2 * ux * (Fy * uy + Fz * uz)) - 13 * Fx,
        5 * (Fy * (ux**2 + 3 * uy**2 + uz**2) + 2 * uy * (Fx * ux + Fz * uz)) - 13 * Fy,
        5 * (Fz * (ux**2 + uy**2 + 3 * uz**2) + 2 * uz * (Fx * ux + Fy * uy)) - 13 * Fz,
        Fx * uy * uz + Fy * ux * uz + Fz * ux * uy,
        20 * (Fx * ux * (3 * (uy**2 + uz**2) - 4) + Fy * uy * (3 * (ux**2 + uz**2) - 4)
              + Fz * uz * (3 * (ux**2 + uy**2) - 4)),
    ], axis=-1)


def source(lat, F, u):
    """Source term S_a in velocity space.

    D3Q27: solve M(u) S = sigma, sigma = (0; F_x, F_y, F_z; 0, ..., 0) on the
    central monomials (matching principle, Sec. 5).  D3Q15: S = K D^-1 m^s with
    the printed m^s (Appendix G); inverting m = K^T S uses K^T K = D (Sec. 6).
    """
    if lat.Q == 27:
        sigma = _first_order_vector(lat, F, u)
        return _solve(central_moment_matrix(lat, u), sigma)
    m = source_projections_d3q15(F, u)
    if _is_exact(u):
        inv_d = np.array([Fraction(1, int(d)) for d in lat.D], dtype=object)
        K = lat.K.astype(object)
    else:
        inv_d = 1.0 / lat.D
        K = lat.K
    return (m * inv_d) @ K.T


def attractors(lat, rho, kt_diag, per_mass=False):
    """Attractor of every central monomial (order >= 2) given the
    post-collision diagonal second moments kt_diag[..., 0:3] = (kxx, kyy, kzz).

    The factorized attractors (Sec. 3, the list after Eq.
    centralmomentfdefinitionpostcollision; Eq. transformedcentralmomentattractors)
    are the literal products kxx kyy, kxx kyy kzz by default.  per_mass=True
    factorizes the moments per unit mass instead: rho (kxx/rho)(kyy/rho) and
    rho (kxx/rho)(kyy/rho)(kzz/rho)."""
    like = rho
    zero = rho * 0
    cs2 = _num(CS2, like)
    out = []
    for mono in lat.monos:
        spec = lat.attractor.get(mono)
        if spec is None:
            out.append(zero)
        elif spec == "cs2":
            out.append(cs2 * rho)
        else:
            val = kt_diag[..., spec[0]]
            for axis in spec[1:]:
                val = val * kt_diag[..., axis]
                if per_mass:
                    val = val / rho
            out.append(val)
    return np.stack(out, axis=-1)


def _rates_vector(lat, omega, like):
    """Relaxation rate per combination row (0 for the conserved rows 0..3)."""
    omega = list(omega)
    assert len(omega) == lat.Q - 4, "omega_4 .. omega_(Q-1)"
    if _is_exact(like):
        return np.array([Fraction(0)] * 4 + [Fraction(w) for w in omega], dtype=object)
    return np.array([0.0] * 4 + omega, dtype=np.result_type(float, *[np.asarray(w).dtype for w in omega]))


# ----------------------------------------------------------------------------
# The collision
# ----------------------------------------------------------------------------
def collide(lat, fbar, F, omega, per_mass=False):
    """Post-collision transformed populations fbar~ = fbar + Omega + S (Eq.
    cascadedcollision1), for pre-collision fbar[..., Q], force F[..., 3] and
    rates omega = (omega_4, ..., omega_(Q-1)); per_mass selects the
    per-unit-mass factorized attractors (see attractors)."""
    exact = _is_exact(fbar)
    Phi = lat.Phi.astype(object) if exact else lat.Phi
    rho, u = macroscopic(lat, fbar, F)
    h = fbar + source(lat, F, u)
    M = central_moment_matrix(lat, u)
    C = (Phi @ (M @ h[..., None]))[..., 0]
    w = _rates_vector(lat, omega, fbar)
    Ct = C.copy()

    # Second order first: the attractors need only rho.
    second = lat.order == 2
    A = attractors(lat, rho, np.zeros(rho.shape + (3,), dtype=Ct.dtype)) @ Phi.T
    Ct[..., second] = C[..., second] + w[second] * (A[..., second] - C[..., second])

    # Post-collision diagonal second-order central moments (Phi is block
    # diagonal by order, so these depend on the relaxed second-order rows only).
    kt = _solve(Phi, Ct)
    diag = [lat.monos.index(m) for m in [(2, 0, 0), (0, 2, 0), (0, 0, 2)]]
    kt_diag = np.stack([kt[..., i] for i in diag], axis=-1)

    # Orders three and up, toward the factorized attractors.
    higher = lat.order >= 3
    A = attractors(lat, rho, kt_diag, per_mass) @ Phi.T
    Ct[..., higher] = C[..., higher] + w[higher] * (A[..., higher] - C[..., higher])

    PM = Phi @ M
    return _solve(PM, Ct)


def equilibrium(lat, rho, u):
    """Discrete equilibrium whose central moments match the Maxwellian's
    (Sec. 3 list after Eq. centralmomentfeqdefinition; matching principle of
    Sec. 5): solve M(u) f = Pi^M."""
    cs2 = _num(CS2, rho)
    vals = []
    for mono in lat.monos:
        power = lat.maxwell.get(mono)
        vals.append(rho * 0 if power is None else rho * cs2 ** power)
    return _solve(central_moment_matrix(lat, u), np.stack(vals, axis=-1))
