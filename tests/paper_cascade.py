"""The paper's printed operational scheme, transcribed formula by formula, as an
independent check on the oracle's plain moment-matrix definition.

This module is a test pin, not a second oracle: it restates, in exact rational
arithmetic, the cascaded collision kernels and source terms exactly as printed
(D3Q27: Eqs. collisionkernelg4-g26 of Sec. 7, the post-collision kappa~ of
Sec. 7, raw moments from the A/B sets of Appendix B, source projections of
Appendix D; D3Q15: the corresponding lists of Appendix G).  The post-collision
populations are fbar + K g + S (Eq. cascadedcollision1 with Eq.
cascadecollision1), with K the printed matrix of Appendix A / Appendix G.

Six D3Q27 kernels and one kappa~ line carry misprinted coefficients (listed in
``CORRECTIONS``); the corrected form is used unless a name is passed in
``printed``, in which case that one term is evaluated as printed.  All
relaxation brackets are used as printed.
"""
from fractions import Fraction as Fr

H = Fr(1, 2)
Q4 = Fr(1, 4)
T4 = Fr(3, 4)
T2 = Fr(3, 2)

# name -> (where, printed term, corrected term)
CORRECTIONS = {
    "g16": ("Eq. collisionkernelg16", "3/2 (uz g4 + uy g5 + uz g6)", "3/2 (uz g4 + uy g5 + ux g6)"),
    "g17": ("Eq. collisionkernelg17", "1/2 (-2ux^2 - 2uy^2 - uz^2 - 4) g9", "(-ux^2 - uy^2 - uz^2 - 2) g9"),
    "g18": ("Eq. collisionkernelg18", "1/4 (-2ux^2 + uy^2 + 2uz^2) g9", "1/4 (-2ux^2 + uy^2 + uz^2) g9"),
    "g19": ("Eq. collisionkernelg19", "1/4 (-3uy^2 - 8) g9", "3/4 (uz^2 - uy^2) g9"),
    "g23": ("Eq. collisionkernelg23", "(3/4 ux uz^2 - 1/4 ux) g7", "-(3/4 ux uz^2 + 1/2 ux) g7"),
    "g25": ("Eq. collisionkernelg25", "-6 ux uy g16", "-4 ux uy g16"),
    "kzz": ("Sec. 7, post-collision kappa~_zz", "[eta'_xx - 12 g8 + 6 g9]", "[eta'_zz - 12 g8 + 6 g9]"),
}


def _sets_moment(f, A, B=()):
    return sum(f[a] for a in A) - sum(f[b] for b in B)


# Appendix B: the A/B index sets of the non-conserved raw moments (D3Q27).
AB27 = {
    "xy": ({7, 10, 19, 22, 23, 26}, {8, 9, 20, 21, 24, 25}),
    "xz": ({11, 14, 19, 21, 24, 26}, {12, 13, 20, 22, 23, 25}),
    "yz": ({15, 18, 19, 20, 25, 26}, {16, 17, 21, 22, 23, 24}),
    "xx": ({1, 2, 7, 8, 9, 10, 11, 12, 13, 14, 19, 20, 21, 22, 23, 24, 25, 26}, set()),
    "yy": ({3, 4, 7, 8, 9, 10, 15, 16, 17, 18, 19, 20, 21, 22, 23, 24, 25, 26}, set()),
    "zz": ({5, 6, 11, 12, 13, 14, 15, 16, 17, 18, 19, 20, 21, 22, 23, 24, 25, 26}, set()),
    "xyy": ({7, 9, 19, 21, 23, 25}, {8, 10, 20, 22, 24, 26}),
    "xzz": ({11, 13, 19, 21, 23, 25}, {12, 14, 20, 22, 24, 26}),
    "xxy": ({7, 8, 19, 20, 23, 24}, {9, 10, 21, 22, 25, 26}),
    "yzz": ({15, 17, 19, 20, 23, 24}, {16, 18, 21, 22, 25, 26}),
    "xxz": ({11, 12, 19, 20, 21, 22}, {13, 14, 23, 24, 25, 26}),
    "yyz": ({15, 16, 19, 20, 21, 22}, {17, 18, 23, 24, 25, 26}),
    "xyz": ({19, 22, 24, 25}, {20, 21, 23, 26}),
    "xxyy": ({7, 8, 9, 10, 19, 20, 21, 22, 23, 24, 25, 26}, set()),
    "xxzz": ({11, 12, 13, 14, 19, 20, 21, 22, 23, 24, 25, 26}, set()),
    "yyzz": ({15, 16, 17, 18, 19, 20, 21, 22, 23, 24, 25, 26}, set()),
    "xxyz": ({19, 20, 25, 26}, {21, 22, 23, 24}),
    "xyyz": ({19, 21, 24, 26}, {20, 22, 23, 25}),
    "xyzz": ({19, 22, 23, 26}, {20, 21, 24, 25}),
    "xyyzz": ({19, 21, 23, 25}, {20, 22, 24, 26}),
    "xxyzz": ({19, 20, 23, 24}, {21, 22, 25, 26}),
    "xxyyz": ({19, 20, 21, 22}, {23, 24, 25, 26}),
    "xxyyzz": ({19, 20, 21, 22, 23, 24, 25, 26}, set()),
}

# Appendix G: the A/B index sets of the D3Q15 non-conserved raw moments.
AB15 = {
    "xy": ({7, 10, 11, 14}, {8, 9, 12, 13}),
    "xz": ({7, 9, 12, 14}, {8, 10, 11, 13}),
    "yz": ({7, 8, 13, 14}, {9, 10, 11, 12}),
    "xx": ({1, 2, 7, 8, 9, 10, 11, 12, 13, 14}, set()),
    "yy": ({3, 4, 7, 8, 9, 10, 11, 12, 13, 14}, set()),
    "zz": ({5, 6, 7, 8, 9, 10, 11, 12, 13, 14}, set()),
    "xyy": ({7, 9, 11, 13}, {8, 10, 12, 14}),
    "xxy": ({7, 8, 11, 12}, {9, 10, 13, 14}),
    "xxz": ({7, 8, 9, 10}, {11, 12, 13, 14}),
    "xyz": ({7, 10, 12, 13}, {8, 9, 11, 14}),
    "xxyy": ({7, 8, 9, 10, 11, 12, 13, 14}, set()),
}

# Conserved raw moments from the velocity list (the sets for x, y, z are the
# +1 / -1 components of e_x, e_y, e_z printed in Sec. 2).
X27 = ({1, 7, 9, 11, 13, 19, 21, 23, 25}, {2, 8, 10, 12, 14, 20, 22, 24, 26})
Y27 = ({3, 7, 8, 15, 17, 19, 20, 23, 24}, {4, 9, 10, 16, 18, 21, 22, 25, 26})
Z27 = ({5, 11, 12, 15, 16, 19, 20, 21, 22}, {6, 13, 14, 17, 18, 23, 24, 25, 26})
X15 = ({1, 7, 9, 11, 13}, {2, 8, 10, 12, 14})
Y15 = ({3, 7, 8, 11, 12}, {4, 9, 10, 13, 14})
Z15 = ({5, 7, 8, 9, 10}, {6, 11, 12, 13, 14})


def raw_moments(f, AB, XYZ):
    m = {name: _sets_moment(f, A, B) for name, (A, B) in AB.items()}
    m["1"] = sum(f)
    m["x"], m["y"], m["z"] = (_sets_moment(f, A, B) for A, B in XYZ)
    return m


def source_projections_d3q27(F, u):
    """m^s_b, Appendix D."""
    Fx, Fy, Fz = F
    ux, uy, uz = u
    t = Fr(2, 3)
    return [
        0, Fx, Fy, Fz,
        Fx * uy + Fy * ux, Fx * uz + Fz * ux, Fy * uz + Fz * uy,
        2 * (Fx * ux - Fy * uy), 2 * (Fx * ux + Fy * uy - 2 * Fz * uz), 2 * (Fx * ux + Fy * uy + Fz * uz),
        3 * (Fx * (uy**2 + uz**2) + 2 * ux * (Fy * uy + Fz * uz)) - 4 * Fx,
        3 * (Fy * (ux**2 + uz**2) + 2 * uy * (Fx * ux + Fz * uz)) - 4 * Fy,
        3 * (Fz * (ux**2 + uy**2) + 2 * uz * (Fx * ux + Fy * uy)) - 4 * Fz,
        Fx * (uy**2 - uz**2) + 2 * ux * (Fy * uy - Fz * uz),
        Fy * (ux**2 - uz**2) + 2 * uy * (Fx * ux - Fz * uz),
        Fz * (ux**2 - uy**2) + 2 * uz * (Fx * ux - Fy * uy),
        Fx * uy * uz + Fy * ux * uz + Fz * ux * uy,
        6 * (Fx * ux * (uy**2 + uz**2) + Fy * uy * (ux**2 + uz**2) + Fz * uz * (ux**2 + uy**2))
        - 8 * (Fx * ux + Fy * uy + Fz * uz),
        6 * (Fx * ux * (uy**2 + uz**2) + Fy * uy * (ux**2 - 2 * uz**2) + Fz * uz * (ux**2 - 2 * uy**2))
        - 4 * (2 * Fx * ux - Fy * uy - Fz * uz),
        6 * (Fx * ux * (uy**2 - uz**2) + ux**2 * (Fy * uy - Fz * uz)) - 4 * (Fy * uy - Fz * uz),
        (3 * ux**2 - 2) * (Fy * uz + Fz * uy) + 6 * Fx * ux * uy * uz,
        (3 * uy**2 - 2) * (Fx * uz + Fz * ux) + 6 * Fy * uy * ux * uz,
        (3 * uz**2 - 2) * (Fx * uy + Fy * ux) + 6 * Fz * uz * ux * uy,
        9 * Fx * (uy**2 * uz**2 - t * ((uy**2 + uz**2) - t))
        + 18 * ux * (Fy * uy * uz**2 + Fz * uz * uy**2 - t * (Fy * uy + Fz * uz)),
        9 * Fy * (ux**2 * uz**2 - t * ((ux**2 + uz**2) - t))
        + 18 * uy * (Fx * ux * uz**2 + Fz * uz * ux**2 - t * (Fx * ux + Fz * uz)),
        9 * Fz * (ux**2 * uy**2 - t * ((ux**2 + uy**2) - t))
        + 18 * uz * (Fx * ux * uy**2 + Fy * uy * ux**2 - t * (Fx * ux + Fy * uy)),
        Fx * ux * (54 * uy**2 * uz**2 - 36 * (uy**2 + uz**2) + 24)
        + Fy * uy * (54 * ux**2 * uz**2 - 36 * (ux**2 + uz**2) + 24)
        + Fz * uz * (54 * ux**2 * uy**2 - 36 * (ux**2 + uy**2) + 24),
    ]


def source_projections_d3q15(F, u):
    """m^s_b for D3Q15, Appendix G."""
    Fx, Fy, Fz = F
    ux, uy, uz = u
    return [
        0, Fx, Fy, Fz,
        Fx * uy + Fy * ux, Fx * uz + Fz * ux, Fy * uz + Fz * uy,
        2 * (Fx * ux - Fy * uy), 2 * (Fx * ux + Fy * uy - 2 * Fz * uz), 2 * (Fx * ux + Fy * uy + Fz * uz),
        5 * (Fx * (3 * ux**2 + uy**2 + uz**2) + 2 * ux * (Fy * uy + Fz * uz)) - 13 * Fx,
        5 * (Fy * (ux**2 + 3 * uy**2 + uz**2) + 2 * uy * (Fx * ux + Fz * uz)) - 13 * Fy,
        5 * (Fz * (ux**2 + uy**2 + 3 * uz**2) + 2 * uz * (Fx * ux + Fy * uy)) - 13 * Fz,
        Fx * uy * uz + Fy * ux * uz + Fz * ux * uy,
        20 * (Fx * ux * (3 * (uy**2 + uz**2) - 4) + Fy * uy * (3 * (ux**2 + uz**2) - 4)
              + Fz * uz * (3 * (ux**2 + uy**2) - 4)),
    ]


def _source(K, m):
    """S = K D^-1 m (inversion of Eq. sourceformulation1, D = diag(K^T K))."""
    Q = len(K)
    D = [sum(K[a][b] ** 2 for a in range(Q)) for b in range(Q)]
    return [sum(K[a][b] * Fr(m[b]) / D[b] for b in range(Q)) for a in range(Q)]


def cascade_d3q27(K, f, F, omega, printed=()):
    """Post-collision fbar~ of one node by the printed D3Q27 cascade.

    K: printed 27x27 integer matrix (rows alpha, columns beta), f: 27 Fractions,
    F: 3 Fractions, omega: omega_4..omega_26 (23 Fractions)."""
    w = {b: Fr(omega[b - 4]) for b in range(4, 27)}
    kb = raw_moments(f, AB27, (X27, Y27, Z27))
    rho = kb["1"]
    Fx, Fy, Fz = (Fr(v) for v in F)
    # Eq. rawmomenttransformedconserved / velocitycalculation
    ux = (kb["x"] + Fx / 2) / rho
    uy = (kb["y"] + Fy / 2) / rho
    uz = (kb["z"] + Fz / 2) / rho
    S = _source(K, source_projections_d3q27((Fx, Fy, Fz), (ux, uy, uz)))
    sg = raw_moments(S, AB27, (X27, Y27, Z27))            # sigma' (lattice moments of S)
    sx, sy, sz = sg["x"], sg["y"], sg["z"]
    n = {k: kb[k] + sg[k] for k in kb}                       # eta' = kappabar' + sigma'
    g = [Fr(0)] * 27
    P = set(printed)

    g[4] = w[4] / 12 * (-n["xy"] + rho * ux * uy + H * (sx * uy + sy * ux))
    g[5] = w[5] / 12 * (-n["xz"] + rho * ux * uz + H * (sx * uz + sz * ux))
    g[6] = w[6] / 12 * (-n["yz"] + rho * uy * uz + H * (sy * uz + sz * uy))
    g[7] = w[7] / 12 * (-(n["xx"] - n["yy"]) + rho * (ux**2 - uy**2) + (sx * ux - sy * uy))
    g[8] = w[8] / 36 * (-(n["xx"] + n["yy"] - 2 * n["zz"]) + rho * (ux**2 + uy**2 - 2 * uz**2)
                        + (sx * ux + sy * uy - 2 * sz * uz))
    g[9] = w[9] / 18 * (-(n["xx"] + n["yy"] + n["zz"]) + rho * (ux**2 + uy**2 + uz**2)
                        + (sx * ux + sy * uy + sz * uz) + rho)
    g[10] = (w[10] / 24 * (-(n["xyy"] + n["xzz"]) + 2 * (uy * n["xy"] + uz * n["xz"]) + ux * (n["yy"] + n["zz"])
                           - 2 * rho * ux * (uy**2 + uz**2) - H * sx * (uy**2 + uz**2) - ux * (sy * uy + sz * uz))
             + (uy * g[4] + uz * g[5]) + Q4 * ux * (-g[7] - g[8] + 2 * g[9]))
    g[11] = (w[11] / 24 * (-(n["xxy"] + n["yzz"]) + 2 * (ux * n["xy"] + uz * n["yz"]) + uy * (n["xx"] + n["zz"])
                           - 2 * rho * uy * (ux**2 + uz**2) - H * sy * (ux**2 + uz**2) - uy * (sx * ux + sz * uz))
             + (ux * g[4] + uz * g[6]) + Q4 * uy * (g[7] - g[8] + 2 * g[9]))
    g[12] = (w[12] / 24 * (-(n["xxz"] + n["yyz"]) + 2 * (ux * n["xz"] + uy * n["yz"]) + uz * (n["xx"] + n["yy"])
                           - 2 * rho * uz * (ux**2 + uy**2) - H * sz * (ux**2 + uy**2) - uz * (sx * ux + sy * uy))
             + (ux * g[5] + uy * g[6]) + H * uz * (g[8] + g[9]))
    g[13] = (w[13] / 8 * (-(n["xyy"] - n["xzz"]) + 2 * (uy * n["xy"] - uz * n["xz"]) + ux * (n["yy"] - n["zz"])
                          - 2 * rho * ux * (uy**2 - uz**2) - H * sx * (uy**2 - uz**2) - ux * (sy * uy - sz * uz))
             + 3 * (uy * g[4] - uz * g[5]) + T4 * ux * (-g[7] + 3 * g[8]))
    g[14] = (w[14] / 8 * (-(n["xxy"] - n["yzz"]) + 2 * (ux * n["xy"] - uz * n["yz"]) + uy * (n["xx"] - n["zz"])
                          - 2 * rho * uy * (ux**2 - uz**2) - H * sy * (ux**2 - uz**2) - uy * (sx * ux - sz * uz))
             + 3 * (ux * g[4] - uz * g[6]) + T4 * uy * (g[7] + 3 * g[8]))
    g[15] = (w[15] / 8 * (-(n["xxz"] - n["yyz"]) + 2 * (ux * n["xz"] - uy * n["yz"]) + uz * (n["xx"] - n["yy"])
                          - 2 * rho * uz * (ux**2 - uy**2) - H * sz * (ux**2 - uy**2) - uz * (sx * ux - sy * uy))
             + 3 * (ux * g[5] - uy * g[6]) + T2 * uz * g[7])
    g6_partner = uz if "g16" in P else ux
    g[16] = (w[16] / 8 * (-n["xyz"] + ux * n["yz"] + uy * n["xz"] + uz * n["xy"] - 2 * rho * ux * uy * uz
                          - H * (sx * uy * uz + sy * ux * uz + sz * ux * uy))
             + T2 * (uz * g[4] + uy * g[5] + g6_partner * g[6]))

    # Post-collision second-order central moments (Sec. 7, after g_19).
    kxx = (n["xx"] + 6 * g[7] + 6 * g[8] + 6 * g[9]) - rho * ux**2 - Fx * ux
    kyy = (n["yy"] - 6 * g[7] + 6 * g[8] + 6 * g[9]) - rho * uy**2 - Fy * uy
    kzz = ((n["xx"] if "kzz" in P else n["zz"]) - 12 * g[8] + 6 * g[9]) - rho * uz**2 - Fz * uz

    g9c17 = H * (-2 * ux**2 - 2 * uy**2 - uz**2 - 4) if "g17" in P else (-ux**2 - uy**2 - uz**2 - 2)
    g[17] = (w[17] / 12 * (-(n["xxyy"] + n["xxzz"] + n["yyzz"])
                           + 2 * (ux * (n["xyy"] + n["xzz"]) + uy * (n["yzz"] + n["xxy"]) + uz * (n["xxz"] + n["yyz"]))
                           - ux**2 * (n["yy"] + n["zz"]) - uy**2 * (n["xx"] + n["zz"]) - uz**2 * (n["xx"] + n["yy"])
                           - 4 * (ux * uy * n["xy"] + ux * uz * n["xz"] + uy * uz * n["yz"])
                           + (kxx * kyy + kxx * kzz + kyy * kzz)
                           + 3 * rho * (ux**2 * uy**2 + ux**2 * uz**2 + uy**2 * uz**2)
                           + ux**2 * (uy * sy + uz * sz) + uy**2 * (ux * sx + uz * sz) + uz**2 * (ux * sx + uy * sy))
             - 4 * ux * uy * g[4] - 4 * ux * uz * g[5] - 4 * uy * uz * g[6]
             + H * (ux**2 - uy**2) * g[7] + H * (ux**2 + uy**2 - 2 * uz**2) * g[8] + g9c17 * g[9]
             + 4 * ux * g[10] + 4 * uy * g[11] + 4 * uz * g[12])
    g9c18 = Q4 * (-2 * ux**2 + uy**2 + 2 * uz**2) if "g18" in P else Q4 * (-2 * ux**2 + uy**2 + uz**2)
    g[18] = (w[18] / 24 * (-(n["xxyy"] + n["xxzz"] - 2 * n["yyzz"])
                           + 2 * (ux * n["xyy"] + ux * n["xzz"] + uy * n["xxy"] + uz * n["xxz"]
                                  - 2 * (uy * n["yzz"] + uz * n["yyz"]))
                           - ux**2 * n["yy"] - ux**2 * n["zz"] - uy**2 * n["xx"] - uz**2 * n["xx"]
                           + 2 * uy**2 * n["zz"] + 2 * uz**2 * n["yy"]
                           - 4 * (ux * uy * n["xy"] + ux * uz * n["xz"] - 2 * uy * uz * n["yz"])
                           + (kxx * kyy + kxx * kzz - 2 * kyy * kzz)
                           + 3 * rho * (ux**2 * uy**2 + ux**2 * uz**2 - 2 * uy**2 * uz**2)
                           + ux**2 * uy * sy + ux**2 * uz * sz + uy**2 * ux * sx + uz**2 * ux * sx
                           - 2 * uy**2 * uz * sz - 2 * uz**2 * uy * sy)
             - 2 * ux * uy * g[4] - 2 * ux * uz * g[5] + 4 * uy * uz * g[6]
             + Q4 * (ux**2 - uy**2 - 3 * uz**2 - 2) * g[7] + Q4 * (ux**2 - 5 * uy**2 + uz**2 - 2) * g[8]
             + g9c18 * g[9]
             + 2 * ux * g[10] - uy * g[11] - uz * g[12] + uy * g[14] + uz * g[15])
    g9c19 = Q4 * (-3 * uy**2 - 8) if "g19" in P else T4 * (uz**2 - uy**2)
    g[19] = (w[19] / 8 * (-(n["xxyy"] - n["xxzz"])
                          + 2 * (ux * n["xyy"] - ux * n["xzz"] + uy * n["xxy"] - uz * n["xxz"])
                          - (ux**2 * n["yy"] - ux**2 * n["zz"] + uy**2 * n["xx"] - uz**2 * n["xx"])
                          - 4 * (ux * uy * n["xy"] - ux * uz * n["xz"])
                          + (kxx * kyy - kxx * kzz) + 3 * rho * (ux**2 * uy**2 - ux**2 * uz**2)
                          + (ux**2 * uy * sy - ux**2 * uz * sz + uy**2 * ux * sx - uz**2 * ux * sx))
             - 6 * ux * uy * g[4] + 6 * ux * uz * g[5]
             + Q4 * (3 * ux**2 - 3 * uy**2 + 3 * uz**2 + 2) * g[7]
             + Q4 * (-9 * ux**2 - 3 * uy**2 + 3 * uz**2 - 6) * g[8]
             + g9c19 * g[9]
             + 3 * uy * g[11] - 3 * uz * g[12] + 2 * ux * g[13] + uy * g[14] - uz * g[15])
    g[20] = (w[20] / 8 * (-n["xxyz"] + uz * n["xxy"] + uy * n["xxz"] + 2 * ux * n["xyz"] - uy * uz * n["xx"]
                          - 2 * ux * uz * n["xy"] - 2 * ux * uy * n["xz"] - ux**2 * n["yz"] + 3 * rho * ux**2 * uy * uz
                          + sx * ux * uy * uz + H * ux**2 * (sy * uz + sz * uy))
             - 3 * ux * uz * g[4] - 3 * ux * uy * g[5] - (T2 * ux**2 + 1) * g[6] - T4 * uy * uz * g[7]
             - T4 * uy * uz * g[8] - T4 * uy * uz * g[9] + T2 * uz * g[11] + T2 * uy * g[12]
             + H * uz * g[14] + H * uy * g[15] + 2 * ux * g[16])
    g[21] = (w[21] / 8 * (-n["xyyz"] + 2 * uy * n["xyz"] + uz * n["xyy"] + ux * n["yyz"] - uy**2 * n["xz"]
                          - 2 * uy * uz * n["xy"] - 2 * ux * uy * n["yz"] - ux * uz * n["yy"] + 3 * rho * ux * uy**2 * uz
                          + sy * ux * uy * uz + H * uy**2 * (sx * uz + sz * ux))
             - 3 * uy * uz * g[4] - (T2 * uy**2 + 1) * g[5] - 3 * ux * uy * g[6] + T4 * ux * uz * g[7]
             - T4 * ux * uz * g[8] - T4 * ux * uz * g[9] + T2 * uz * g[10] + T2 * ux * g[12]
             + H * uz * g[13] - H * ux * g[15] + 2 * uy * g[16])
    g[22] = (w[22] / 8 * (-n["xyzz"] + 2 * uz * n["xyz"] + uy * n["xzz"] + ux * n["yzz"] - uz**2 * n["xy"]
                          - 2 * uy * uz * n["xz"] - 2 * ux * uz * n["yz"] - ux * uy * n["zz"] + 3 * rho * ux * uy * uz**2
                          + sz * ux * uy * uz + H * uz**2 * (sx * uy + sy * ux))
             - (T2 * uz**2 + 1) * g[4] - 3 * uy * uz * g[5] - 3 * ux * uz * g[6] + T2 * ux * uy * g[8]
             - T4 * ux * uy * g[9] + T2 * uy * g[10] + T2 * ux * g[11]
             - H * uy * g[13] - H * ux * g[14] + 2 * uz * g[16])
    g7c23 = (T4 * ux * uz**2 - Q4 * ux) if "g23" in P else -(T4 * ux * uz**2 + H * ux)
    g[23] = (w[23] / 8 * (-n["xyyzz"] + ux * n["yyzz"] + 2 * uy * n["xyzz"] + 2 * uz * n["xyyz"]
                          - uy**2 * n["xzz"] - uz**2 * n["xyy"] - 2 * ux * uy * n["yzz"] - 2 * ux * uz * n["yyz"]
                          - 4 * uy * uz * n["xyz"] + ux * uz**2 * n["yy"] + ux * uy**2 * n["zz"]
                          + 2 * uy * uz**2 * n["xy"] + 2 * uy**2 * uz * n["xz"] + 4 * ux * uy * uz * n["yz"]
                          - 4 * rho * ux * uy**2 * uz**2 - H * uy**2 * uz**2 * sx
                          - ux * (uz**2 * uy * sy + uy**2 * uz * sz))
             + (3 * uy * uz**2 + 2 * uy) * g[4] + (3 * uy**2 * uz + 2 * uz) * g[5] + 6 * ux * uy * uz * g[6]
             + g7c23 * g[7] + (T4 * ux * uz**2 - T2 * ux * uy**2 - H * ux) * g[8]
             + (T4 * ux * uz**2 + T4 * ux * uy**2 + ux) * g[9] + (-T2 * uy**2 - T2 * uz**2 - 2) * g[10]
             - 3 * ux * uy * g[11] - 3 * ux * uz * g[12] + (H * uy**2 - H * uz**2) * g[13]
             + ux * uy * g[14] + ux * uz * g[15] - 4 * uy * uz * g[16]
             + H * ux * g[17] - ux * g[18] + 2 * uz * g[21] + 2 * uy * g[22])
    g[24] = (w[24] / 8 * (-n["xxyzz"] + 2 * ux * n["xyzz"] + 2 * uz * n["xxyz"] + uy * n["xxzz"]
                          - ux**2 * n["yzz"] - uz**2 * n["xxy"] - 2 * ux * uy * n["xzz"] - 2 * uy * uz * n["xxz"]
                          - 4 * ux * uz * n["xyz"] + uy * uz**2 * n["xx"] + ux**2 * uy * n["zz"]
                          + 2 * ux * uz**2 * n["xy"] + 2 * ux**2 * uz * n["yz"] + 4 * ux * uy * uz * n["xz"]
                          - 4 * rho * ux**2 * uy * uz**2 - H * ux**2 * uz**2 * sy
                          - uy * (ux * uz**2 * sx + ux**2 * uz * sz))
             + (3 * ux * uz**2 + 2 * ux) * g[4] + 6 * ux * uy * uz * g[5] + (3 * ux**2 * uz + 2 * uz) * g[6]
             + (T4 * uy * uz**2 + H * uy) * g[7] + (T4 * uy * uz**2 - T2 * ux**2 * uy - H * uy) * g[8]
             + (T4 * uy * uz**2 + T4 * ux**2 * uy + uy) * g[9] - 3 * ux * uy * g[10]
             + (-T2 * ux**2 - T2 * uz**2 - 2) * g[11] - 3 * uy * uz * g[12] + ux * uy * g[13]
             + (H * ux**2 - H * uz**2) * g[14] - uy * uz * g[15] - 4 * ux * uz * g[16]
             + H * uy * g[17] + H * uy * g[18] - H * uy * g[19] + 2 * uz * g[20] + 2 * ux * g[22])
    g16c25 = -6 if "g25" in P else -4
    g[25] = (w[25] / 8 * (-n["xxyyz"] + 2 * ux * n["xyyz"] + 2 * uy * n["xxyz"] + uz * n["xxyy"]
                          - ux**2 * n["yyz"] - uy**2 * n["xxz"] - 2 * ux * uz * n["xyy"] - 2 * uy * uz * n["xxy"]
                          - 4 * ux * uy * n["xyz"] + uy**2 * uz * n["xx"] + ux**2 * uz * n["yy"]
                          + 2 * ux * uy**2 * n["xz"] + 2 * ux**2 * uy * n["yz"] + 4 * ux * uy * uz * n["xy"]
                          - 4 * rho * ux**2 * uy**2 * uz - H * ux**2 * uy**2 * sz
                          - uz * (ux * uy**2 * sx + ux**2 * uy * sy))
             + 6 * ux * uy * uz * g[4] + (3 * ux * uy**2 + 2 * ux) * g[5] + (3 * ux**2 * uy + 2 * uy) * g[6]
             + (T4 * uy**2 * uz - T4 * ux**2 * uz) * g[7] + (T4 * uy**2 * uz + T4 * ux**2 * uz + uz) * g[8]
             + (T4 * uy**2 * uz + T4 * ux**2 * uz + uz) * g[9] - 3 * ux * uz * g[10] - 3 * uy * uz * g[11]
             + (-T2 * ux**2 - T2 * uy**2 - 2) * g[12] - ux * uz * g[13] - uy * uz * g[14]
             + (H * ux**2 - H * uy**2) * g[15] + g16c25 * ux * uy * g[16]
             + H * uz * g[17] + H * uz * g[18] + H * uz * g[19] + 2 * uy * g[20] + 2 * ux * g[21])
    g[26] = (w[26] / 8 * (-n["xxyyzz"] + 2 * (ux * n["xyyzz"] + uy * n["xxyzz"] + uz * n["xxyyz"])
                          - (ux**2 * n["yyzz"] + uy**2 * n["xxzz"] + uz**2 * n["xxyy"])
                          - 4 * (ux * uy * n["xyzz"] + ux * uz * n["xyyz"] + uy * uz * n["xxyz"])
                          + 2 * (ux**2 * uy * n["yzz"] + ux * uy**2 * n["xzz"] + ux**2 * uz * n["yyz"]
                                 + ux * uz**2 * n["xyy"] + uy**2 * uz * n["xxz"] + uy * uz**2 * n["xxy"])
                          + 8 * ux * uy * uz * n["xyz"]
                          - (uy**2 * uz**2 * n["xx"] + ux**2 * uz**2 * n["yy"] + ux**2 * uy**2 * n["zz"])
                          - 4 * ux * uy * uz * (uz * n["xy"] + uy * n["xz"] + ux * n["yz"])
                          + 5 * rho * ux**2 * uy**2 * uz**2 + kxx * kyy * kzz
                          + ux * uy * uz * (ux * uy * sz + ux * uz * sy + uy * uz * sx))
             + (-4 * ux * uy - 6 * ux * uy * uz**2) * g[4] + (-4 * ux * uz - 6 * ux * uy**2 * uz) * g[5]
             + (-4 * uy * uz - 6 * ux**2 * uy * uz) * g[6]
             + (H * ux**2 - H * uy**2 + T4 * ux**2 * uz**2 - T4 * uy**2 * uz**2) * g[7]
             + (H * ux**2 + H * uy**2 - uz**2 - T4 * uy**2 * uz**2 - T4 * ux**2 * uz**2 + T2 * ux**2 * uy**2) * g[8]
             + (-ux**2 - uy**2 - uz**2 - T4 * ux**2 * uy**2 - T4 * ux**2 * uz**2 - T4 * uy**2 * uz**2 - 1) * g[9]
             + (3 * ux * uy**2 + 3 * ux * uz**2 + 4 * ux) * g[10] + (3 * ux**2 * uy + 3 * uy * uz**2 + 4 * uy) * g[11]
             + (3 * ux**2 * uz + 3 * uy**2 * uz + 4 * uz) * g[12] + (ux * uz**2 - ux * uy**2) * g[13]
             + (uy * uz**2 - ux**2 * uy) * g[14] + (uy**2 * uz - ux**2 * uz) * g[15] + 8 * ux * uy * uz * g[16]
             + (-H * ux**2 - H * uy**2 - H * uz**2 - 1) * g[17] + (ux**2 - H * uy**2 - H * uz**2) * g[18]
             + (H * uy**2 - H * uz**2) * g[19] - 4 * uy * uz * g[20] - 4 * ux * uz * g[21]
             - 4 * ux * uy * g[22] + 2 * ux * g[23] + 2 * uy * g[24] + 2 * uz * g[25])
    return [f[a] + sum(K[a][b] * g[b] for b in range(27)) + S[a] for a in range(27)]


def cascade_d3q15(K, f, F, omega):
    """Post-collision fbar~ of one node by the printed D3Q15 scheme (Appendix G)."""
    w = {b: Fr(omega[b - 4]) for b in range(4, 15)}
    kb = raw_moments(f, AB15, (X15, Y15, Z15))
    rho = kb["1"]
    Fx, Fy, Fz = (Fr(v) for v in F)
    ux = (kb["x"] + Fx / 2) / rho
    uy = (kb["y"] + Fy / 2) / rho
    uz = (kb["z"] + Fz / 2) / rho
    S = _source(K, source_projections_d3q15((Fx, Fy, Fz), (ux, uy, uz)))
    sg = raw_moments(S, AB15, (X15, Y15, Z15))
    sx, sy, sz = sg["x"], sg["y"], sg["z"]
    n = {k: kb[k] + sg[k] for k in kb}
    g = [Fr(0)] * 15
    g[4] = w[4] / 8 * (-n["xy"] + rho * ux * uy + H * (sx * uy + sy * ux))
    g[5] = w[5] / 8 * (-n["xz"] + rho * ux * uz + H * (sx * uz + sz * ux))
    g[6] = w[6] / 8 * (-n["yz"] + rho * uy * uz + H * (sy * uz + sz * uy))
    g[7] = w[7] / 4 * (-(n["xx"] - n["yy"]) + rho * (ux**2 - uy**2) + (sx * ux - sy * uy))
    g[8] = w[8] / 12 * (-(n["xx"] + n["yy"] - 2 * n["zz"]) + rho * (ux**2 + uy**2 - 2 * uz**2)
                        + (sx * ux + sy * uy - 2 * sz * uz))
    g[9] = w[9] / 18 * (-(n["xx"] + n["yy"] + n["zz"]) + rho * (ux**2 + uy**2 + uz**2)
                        + (sx * ux + sy * uy + sz * uz) + rho)
    E8 = Fr(1, 8)
    g[10] = (w[10] / 16 * (-n["xyy"] + 2 * uy * n["xy"] + ux * n["yy"] - 2 * rho * ux * uy**2
                           - H * sx * uy**2 - sy * uy * ux)
             + uy * g[4] + E8 * ux * (-g[7] + g[8] + 3 * g[9]))
    g[11] = (w[11] / 16 * (-n["xxy"] + 2 * ux * n["xy"] + uy * n["xx"] - 2 * rho * ux**2 * uy
                           - H * sy * ux**2 - sx * ux * uy)
             + ux * g[4] + E8 * uy * (g[7] + g[8] + 3 * g[9]))
    g[12] = (w[12] / 16 * (-n["xxz"] + 2 * ux * n["xz"] + uz * n["xx"] - 2 * rho * ux**2 * uz
                           - H * sz * ux**2 - sx * ux * uz)
             + ux * g[5] + E8 * uz * (g[7] + g[8] + 3 * g[9]))
    g[13] = (w[13] / 8 * (-n["xyz"] + ux * n["yz"] + uy * n["xz"] + uz * n["xy"] - 2 * rho * ux * uy * uz
                          - H * (sx * uy * uz + sy * ux * uz + sz * ux * uy))
             + uz * g[4] + uy * g[5] + ux * g[6])
    # Post-collision second-order central moments, from the D3Q15 kernel
    # moments of Appendix G (<K g|e_x^2> = 2 g7 + 2 g8 + 6 g9, ...).
    kxx = (n["xx"] + 2 * g[7] + 2 * g[8] + 6 * g[9]) - rho * ux**2 - Fx * ux
    kyy = (n["yy"] - 2 * g[7] + 2 * g[8] + 6 * g[9]) - rho * uy**2 - Fy * uy
    g[14] = (w[14] / 16 * (-n["xxyy"] + 2 * ux * n["xyy"] + 2 * uy * n["xxy"] - ux**2 * n["yy"]
                           - uy**2 * n["xx"] - 4 * ux * uy * n["xy"] + kxx * kyy + 3 * rho * ux**2 * uy**2
                           + sx * ux * uy**2 + sy * uy * ux**2)
             - 2 * ux * uy * g[4] + E8 * (ux**2 - uy**2) * g[7] + E8 * (-ux**2 - uy**2) * g[8]
             + (Fr(3, 8) * (-ux**2 - uy**2) - H) * g[9] + 2 * ux * g[10] + 2 * uy * g[11])
    return [f[a] + sum(K[a][b] * g[b] for b in range(15)) + S[a] for a in range(15)]
