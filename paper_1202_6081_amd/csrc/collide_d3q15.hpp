// D3Q15 central-moment collision with forcing (Premnath & Banerjee,
// arXiv:1202.6081, Appendix G).
//
// Steps, per node:
//  1. rho, u from the transformed populations, u including F/2.
//  2. Source S = K D^-1 m^s with the projections m^s printed in Appendix G and
//     the D3Q15 basis K_0..K_14 of Appendix G (inversion as in Eq.
//     sourceformulation1).
//  3. Raw moments of h = fbar + S for the fifteen monomials the D3Q15 kernels
//     use (1, x, y, z, xy, xz, yz, xx, yy, zz, xyy, xxy, xxz, xyz, xxyy); on this
//     lattice they are signed sums over the rest, axis and corner links (the
//     corners by a Walsh-Hadamard transform).
//  4. Binomial shift to central moments, one axis at a time, relaxation of xy, xz, yz (g4..g6),
//     xx-yy, xx+yy-2zz, xx+yy+zz (g7..g9), xyy, xxy, xxz, xyz (g10..g13) toward
//     zero (rho for g9) and xxyy (g14) toward kxx~ kyy~; rho and the first central
//     moments (F/2) are conserved.
//  5. Inverse shift to raw moments and exact inversion of the fifteen raw
//     moments to populations (the K g + S rows of Appendix G), the corners by the
//     inverse transform.
#pragma once

#include <type_traits>
#include <utility>

#include "collide_d3q27.hpp"   // Rates<R>
#include "lattice.hpp"

namespace cmlbm {

// Basis vector K_b of Appendix G evaluated at direction e.
CMLBM_HDC int k15_basis(int b, Vel e) {
  const int x = e.x, y = e.y, z = e.z;
  const int s2 = x * x + y * y + z * z;
  switch (b) {
    case 0: return 1;
    case 1: return x;
    case 2: return y;
    case 3: return z;
    case 4: return x * y;
    case 5: return x * z;
    case 6: return y * z;
    case 7: return x * x - y * y;
    case 8: return s2 - 3 * z * z;
    case 9: return s2 - 2;
    case 10: return 5 * x * s2 - 13 * x;
    case 11: return 5 * y * s2 - 13 * y;
    case 12: return 5 * z * s2 - 13 * z;
    case 13: return x * y * z;
    default: return 30 * (x * x * y * y + x * x * z * z + y * y * z * z) - 40 * s2 + 32;
  }
}

CMLBM_HDC int k15_norm(int b) {
  int d = 0;
  for (int a = 0; a < 15; ++a) d += k15_basis(b, kE15[a]) * k15_basis(b, kE15[a]);
  return d;
}

// Compile-time tables: kB15.v[b][a] = K_b(e_a), kM15.v[m][a] = the monomial m
// (order below) at e_a, kD15[b] = D_b.  Loops over them run through
// static_for so that every entry is a literal constant in the generated code.
struct Tab15 {
  int v[15][15];
};

CMLBM_HDC Vel mono15(int m) {
  constexpr Vel t[15] = {{0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {0, 0, 1}, {1, 1, 0}, {1, 0, 1}, {0, 1, 1}, {2, 0, 0},
                         {0, 2, 0}, {0, 0, 2}, {1, 2, 0}, {2, 1, 0}, {2, 0, 1}, {1, 1, 1}, {2, 2, 0}};
  return t[m];
}

CMLBM_HDC int ipow(int v, int n) { return n == 0 ? 1 : (n == 1 ? v : v * v); }

CMLBM_HDC Tab15 make_basis15() {
  Tab15 t{};
  for (int b = 0; b < 15; ++b)
    for (int a = 0; a < 15; ++a) t.v[b][a] = k15_basis(b, kE15[a]);
  return t;
}

CMLBM_HDC Tab15 make_mono15() {
  Tab15 t{};
  for (int m = 0; m < 15; ++m)
    for (int a = 0; a < 15; ++a)
      t.v[m][a] = ipow(kE15[a].x, mono15(m).x) * ipow(kE15[a].y, mono15(m).y) * ipow(kE15[a].z, mono15(m).z);
  return t;
}

constexpr Tab15 kB15 = make_basis15();
constexpr Tab15 kM15 = make_mono15();

template <int I>
using Ic = std::integral_constant<int, I>;

template <class Fn, int... I>
CMLBM_HD void static_for_impl(Fn&& fn, std::integer_sequence<int, I...>) {
  (fn(Ic<I>{}), ...);
}

// fn(Ic<0>{}), ..., fn(Ic<N-1>{}): the index is a compile-time constant.
template <int N, class Fn>
CMLBM_HD void static_for(Fn&& fn) {
  static_for_impl(fn, std::make_integer_sequence<int, N>{});
}

// Source S_a = sum_b K_b(e_a) m^s_b / D_b with the printed m^s (Appendix G).
template <typename R>
CMLBM_HD void source15(R Fx, R Fy, R Fz, R ux, R uy, R uz, R (&S)[15]) {
  const R ux2 = ux * ux, uy2 = uy * uy, uz2 = uz * uz;
  R ms[15];
  ms[0] = R(0);
  ms[1] = Fx;
  ms[2] = Fy;
  ms[3] = Fz;
  ms[4] = Fx * uy + Fy * ux;
  ms[5] = Fx * uz + Fz * ux;
  ms[6] = Fy * uz + Fz * uy;
  ms[7] = R(2) * (Fx * ux - Fy * uy);
  ms[8] = R(2) * (Fx * ux + Fy * uy - R(2) * Fz * uz);
  ms[9] = R(2) * (Fx * ux + Fy * uy + Fz * uz);
  ms[10] = R(5) * (Fx * (R(3) * ux2 + uy2 + uz2) + R(2) * ux * (Fy * uy + Fz * uz)) - R(13) * Fx;
  ms[11] = R(5) * (Fy * (ux2 + R(3) * uy2 + uz2) + R(2) * uy * (Fx * ux + Fz * uz)) - R(13) * Fy;
  ms[12] = R(5) * (Fz * (ux2 + uy2 + R(3) * uz2) + R(2) * uz * (Fx * ux + Fy * uy)) - R(13) * Fz;
  ms[13] = Fx * uy * uz + Fy * ux * uz + Fz * ux * uy;
  ms[14] = R(20) * (Fx * ux * (R(3) * (uy2 + uz2) - R(4)) + Fy * uy * (R(3) * (ux2 + uz2) - R(4)) +
                    Fz * uz * (R(3) * (ux2 + uy2) - R(4)));
  static_for<15>([&](auto b) {
    constexpr int d = k15_norm(decltype(b)::value);
    ms[b] *= R(1.0 / d);
  });
  static_for<15>([&](auto a) {
    R acc = R(0);
    static_for<14>([&](auto b1) {
      constexpr int k = kB15.v[decltype(b1)::value + 1][decltype(a)::value];
      if constexpr (k != 0) acc += R(k) * ms[decltype(b1)::value + 1];
    });
    S[a] = acc;
  });
}

// The fifteen moments the D3Q15 kernels use, in this order.
enum : int { M0 = 0, MX, MY, MZ, MXY, MXZ, MYZ, MXX, MYY, MZZ, MXYY, MXXY, MXXZ, MXYZ, MXXYY };

// The binomial shift between raw and central moments factors into one shift
// per axis, because this set is closed under lowering any one exponent: along
// an axis the moments form triples (exponent 0, 1, 2), pairs (0, 1) and
// singles, and a triple (m0, m1, m2) shifts by u as
// (m0, m1 - u m0, m2 - 2 u m1 + u^2 m0) (raw to central) or
// (m0, m1 + u m0, m2 + 2 u m1 + u^2 m0) (central to raw).
struct Groups15 {
  int t[4][3];   // triples
  int nt;
  int p[4][2];   // pairs
  int np;
};

template <int AX>
CMLBM_HDC Groups15 groups15() {
  if constexpr (AX == 0)
    return {{{0, 1, 7}, {2, 4, 11}, {3, 5, 12}, {8, 10, 14}}, 4, {{6, 13}, {0, 0}, {0, 0}, {0, 0}}, 1};
  else if constexpr (AX == 1)
    return {{{0, 2, 8}, {1, 4, 10}, {7, 11, 14}, {0, 0, 0}}, 3, {{3, 6}, {5, 13}, {0, 0}, {0, 0}}, 2};
  else
    return {{{0, 3, 9}, {0, 0, 0}, {0, 0, 0}, {0, 0, 0}}, 1, {{1, 5}, {2, 6}, {4, 13}, {7, 12}}, 4};
}

// Shift of moments m by u along axis AX (sg = -1: raw to central, +1: back).
template <int AX, typename R>
CMLBM_HD void shift15(R (&m)[15], R u, R sg) {
  constexpr Groups15 G = groups15<AX>();
  const R v = sg * u;
  static_for<G.nt>([&](auto i) {
    constexpr int a = G.t[decltype(i)::value][0], b = G.t[decltype(i)::value][1], c = G.t[decltype(i)::value][2];
    const R nb = m[b] + v * m[a];           // m2 + 2 v m1 + v^2 m0 = m2 + v (m1 + nb)
    m[c] = m[c] + v * (m[b] + nb);
    m[b] = nb;
  });
  static_for<G.np>([&](auto i) {
    constexpr int a = G.p[decltype(i)::value][0], b = G.p[decltype(i)::value][1];
    m[b] += v * m[a];
  });
}

// Raw moments r of populations f (paper order).  The eight corner links' sign
// patterns are the moments 1, x, y, z, xy, xz, yz, xyz, so the corner sums come
// from a three-stage Walsh-Hadamard transform (24 additions); on the corners
// xyy = x, xxy = y, xxz = z and xx = yy = zz = xxyy = 1, and the axis links
// carry only 1, x, y, z, xx, yy, zz.  Corner 7 + i has e_x = -1 when bit 0 of i
// is set, e_y = -1 for bit 1, e_z = -1 for bit 2.
template <typename R>
CMLBM_HD void raw_moments15(const R (&f)[15], R (&r)[15]) {
  const R s0 = f[7] + f[8], d0 = f[7] - f[8];       // (y, z) = (+, +): sum and x-weighted sum
  const R s1 = f[9] + f[10], d1 = f[9] - f[10];     // (-, +)
  const R s2 = f[11] + f[12], d2 = f[11] - f[12];   // (+, -)
  const R s3 = f[13] + f[14], d3 = f[13] - f[14];   // (-, -)
  const R a_p = s0 + s1, y_p = s0 - s1, x_p = d0 + d1, xy_p = d0 - d1;   // z = +1
  const R a_m = s2 + s3, y_m = s2 - s3, x_m = d2 + d3, xy_m = d2 - d3;   // z = -1
  const R c1 = a_p + a_m, cz = a_p - a_m, cy = y_p + y_m, cyz = y_p - y_m;
  const R cx = x_p + x_m, cxz = x_p - x_m, cxy = xy_p + xy_m, cxyz = xy_p - xy_m;
  const R lxx = f[1] + f[2], lyy = f[3] + f[4], lzz = f[5] + f[6];
  r[M0] = ((f[0] + c1) + (lxx + lyy)) + lzz;
  r[MX] = (f[1] - f[2]) + cx;
  r[MY] = (f[3] - f[4]) + cy;
  r[MZ] = (f[5] - f[6]) + cz;
  r[MXY] = cxy;
  r[MXZ] = cxz;
  r[MYZ] = cyz;
  r[MXX] = lxx + c1;
  r[MYY] = lyy + c1;
  r[MZZ] = lzz + c1;
  r[MXYY] = cx;
  r[MXXY] = cy;
  r[MXXZ] = cz;
  r[MXYZ] = cxyz;
  r[MXXYY] = c1;
}

// Populations with raw moments r: the inverse of raw_moments15.  The corner
// moments (1, x, y, z, xy, xz, yz, xyz) = (xxyy, xyy, xxy, xxz, xy, xz, yz, xyz)
// give the eight corners by the inverse transform (the same three stages and
// a factor 1/8); the axis links follow from the xx, x (etc.) moments less the
// corners' parts, the rest population from the density.
template <typename R>
CMLBM_HD void populations_from_raw15(const R (&r)[15], R (&f)[15]) {
  const R c1 = r[MXXYY];
  const R a1p = r[MXXYY] + r[MXXZ], a1m = r[MXXYY] - r[MXXZ];   // 1 + z, 1 - z
  const R axp = r[MXYY] + r[MXZ], axm = r[MXYY] - r[MXZ];       // x + xz, x - xz
  const R ayp = r[MXXY] + r[MYZ], aym = r[MXXY] - r[MYZ];       // y + yz, y - yz
  const R bxyp = r[MXY] + r[MXYZ], bxym = r[MXY] - r[MXYZ];     // xy + xyz, xy - xyz
  // (y, z) corner pairs: the x-even part b and the x-odd part c
  const R b_pp = a1p + ayp, b_mp = a1p - ayp, b_pm = a1m + aym, b_mm = a1m - aym;
  const R c_pp = axp + bxyp, c_mp = axp - bxyp, c_pm = axm + bxym, c_mm = axm - bxym;
  const R h = R(0.125);
  f[7] = h * (b_pp + c_pp);
  f[8] = h * (b_pp - c_pp);
  f[9] = h * (b_mp + c_mp);
  f[10] = h * (b_mp - c_mp);
  f[11] = h * (b_pm + c_pm);
  f[12] = h * (b_pm - c_pm);
  f[13] = h * (b_mm + c_mm);
  f[14] = h * (b_mm - c_mm);
  const R lxx = r[MXX] - c1, lyy = r[MYY] - c1, lzz = r[MZZ] - c1;
  const R lx = r[MX] - r[MXYY], ly = r[MY] - r[MXXY], lz = r[MZ] - r[MXXZ];
  f[1] = R(0.5) * (lxx + lx);
  f[2] = R(0.5) * (lxx - lx);
  f[3] = R(0.5) * (lyy + ly);
  f[4] = R(0.5) * (lyy - ly);
  f[5] = R(0.5) * (lzz + lz);
  f[6] = R(0.5) * (lzz - lz);
  f[0] = ((r[M0] - c1) - lxx) - (lyy + lzz);
}

// Populations with central moments m about u (m is overwritten by the raw
// moments): shift back along z, y, x, then invert.
template <typename R>
CMLBM_HD void populations_from_central15(R (&m)[15], R ux, R uy, R uz, R (&f)[15]) {
  shift15<2>(m, uz, R(1));
  shift15<1>(m, uy, R(1));
  shift15<0>(m, ux, R(1));
  populations_from_raw15(m, f);
}

// Density and velocity (Eqs. densitycalculation, velocitycalculation).
template <typename R>
CMLBM_HD void moments0_15(const R (&f)[15], R Fx, R Fy, R Fz, R& rho, R& ux, R& uy, R& uz, R& inv_rho) {
  rho = R(0);
#pragma unroll
  for (int a = 0; a < 15; ++a) rho += f[a];
  R cx = R(0), cy = R(0), cz = R(0);
#pragma unroll
  for (int a = 7; a < 15; ++a) {
    cx += R(kE15[a].x) * f[a];
    cy += R(kE15[a].y) * f[a];
    cz += R(kE15[a].z) * f[a];
  }
  const R inv = recip(rho);
  inv_rho = inv;
  ux = (f[1] - f[2] + cx + R(0.5) * Fx) * inv;
  uy = (f[3] - f[4] + cy + R(0.5) * Fy) * inv;
  uz = (f[5] - f[6] + cz + R(0.5) * Fz) * inv;
}

// Raw moments of the source S = K D^-1 m^s (Appendix G), in the moment order
// 1, x, y, z, xy, xz, yz, xx, yy, zz, xyy, xxy, xxz, xyz, xxyy.  With K^T K = D
// they follow from the printed projections m^s alone: e.g. the xx moment is
// m^s_7/2 + m^s_8/6 + m^s_9/3 = 2 F_x u_x and the xyy moment is
// (4/5) m^s_1 + m^s_10/10.
template <typename R>
CMLBM_HD void source_raw15(R Fx, R Fy, R Fz, R ux, R uy, R uz, R (&r)[15]) {
  const R ux2 = ux * ux, uy2 = uy * uy, uz2 = uz * uz;
  const R Fu = Fx * ux, Fv = Fy * uy, Fw = Fz * uz;
  r[0] = R(0);
  r[1] = Fx;
  r[2] = Fy;
  r[3] = Fz;
  r[4] = Fx * uy + Fy * ux;
  r[5] = Fx * uz + Fz * ux;
  r[6] = Fy * uz + Fz * uy;
  r[7] = R(2) * Fu;
  r[8] = R(2) * Fv;
  r[9] = R(2) * Fw;
  r[10] = R(0.5) * (Fx * (R(3) * ux2 + uy2 + uz2 - R(1)) + R(2) * ux * (Fv + Fw));
  r[11] = R(0.5) * (Fy * (ux2 + R(3) * uy2 + uz2 - R(1)) + R(2) * uy * (Fu + Fw));
  r[12] = R(0.5) * (Fz * (ux2 + uy2 + R(3) * uz2 - R(1)) + R(2) * uz * (Fu + Fv));
  r[13] = Fx * uy * uz + Fy * ux * uz + Fz * ux * uy;
  r[14] = R(2.0 / 3.0) * (Fu * (uy2 + uz2) + Fv * (ux2 + uz2) + Fw * (ux2 + uy2));
}

// Adjoint of source_raw15 with respect to F and u (gr: adjoint of r).
template <typename R>
CMLBM_HD void source_raw15_adj(R Fx, R Fy, R Fz, R ux, R uy, R uz, const R (&gr)[15], R& gFx, R& gFy, R& gFz,
                               R& gux, R& guy, R& guz) {
  const R ux2 = ux * ux, uy2 = uy * uy, uz2 = uz * uz;
  const R Fu = Fx * ux, Fv = Fy * uy, Fw = Fz * uz;
  gFx += gr[1] + uy * gr[4] + uz * gr[5] + R(2) * ux * gr[7];
  gFy += gr[2] + ux * gr[4] + uz * gr[6] + R(2) * uy * gr[8];
  gFz += gr[3] + ux * gr[5] + uy * gr[6] + R(2) * uz * gr[9];
  gux += Fy * gr[4] + Fz * gr[5] + R(2) * Fx * gr[7];
  guy += Fx * gr[4] + Fz * gr[6] + R(2) * Fy * gr[8];
  guz += Fx * gr[5] + Fy * gr[6] + R(2) * Fz * gr[9];
  // third order
  gFx += R(0.5) * (R(3) * ux2 + uy2 + uz2 - R(1)) * gr[10] + ux * uy * gr[11] + ux * uz * gr[12];
  gFy += ux * uy * gr[10] + R(0.5) * (ux2 + R(3) * uy2 + uz2 - R(1)) * gr[11] + uy * uz * gr[12];
  gFz += ux * uz * gr[10] + uy * uz * gr[11] + R(0.5) * (ux2 + uy2 + R(3) * uz2 - R(1)) * gr[12];
  gux += (R(3) * Fu + Fv + Fw) * gr[10] + (Fy * ux + Fx * uy) * gr[11] + (Fz * ux + Fx * uz) * gr[12];
  guy += (Fx * uy + Fy * ux) * gr[10] + (R(3) * Fv + Fu + Fw) * gr[11] + (Fz * uy + Fy * uz) * gr[12];
  guz += (Fx * uz + Fz * ux) * gr[10] + (Fy * uz + Fz * uy) * gr[11] + (R(3) * Fw + Fu + Fv) * gr[12];
  gFx += uy * uz * gr[13];
  gFy += ux * uz * gr[13];
  gFz += ux * uy * gr[13];
  gux += (Fy * uz + Fz * uy) * gr[13];
  guy += (Fx * uz + Fz * ux) * gr[13];
  guz += (Fx * uy + Fy * ux) * gr[13];
  // fourth order
  const R c = R(2.0 / 3.0) * gr[14];
  gFx += c * ux * (uy2 + uz2);
  gFy += c * uy * (ux2 + uz2);
  gFz += c * uz * (ux2 + uy2);
  gux += c * (Fx * (uy2 + uz2) + R(2) * ux * (Fv + Fw));
  guy += c * (Fy * (ux2 + uz2) + R(2) * uy * (Fu + Fw));
  guz += c * (Fz * (ux2 + uy2) + R(2) * uz * (Fu + Fv));
}

template <typename R>
CMLBM_HD void collide15(R (&f)[15], R Fx, R Fy, R Fz, const Rates<R>& p) {
  R m[15];
  raw_moments15(f, m);
  const R rho = m[M0];
  const R inv_rho = recip(rho);
  // (explicit fused multiply-adds, as in the D3Q27 collision)
  const R ux = fma_r(R(0.5), Fx, m[MX]) * inv_rho;
  const R uy = fma_r(R(0.5), Fy, m[MY]) * inv_rho;
  const R uz = fma_r(R(0.5), Fz, m[MZ]) * inv_rho;
  // raw moments of h = f + S, then central moments about u
  {
    R rs[15];
    source_raw15(Fx, Fy, Fz, ux, uy, uz, rs);
#pragma unroll
    for (int k = 1; k < 15; ++k) m[k] += rs[k];
  }
  shift15<0>(m, ux, R(-1));
  shift15<1>(m, uy, R(-1));
  shift15<2>(m, uz, R(-1));
  // relaxation; density and the first central moments (F/2) are conserved
  const R d1 = p.wc[7] * (m[MXX] - m[MYY]);
  const R d2 = p.wc[8] * (m[MXX] + m[MYY] - R(2) * m[MZZ]);
  const R t9 = p.wc[9] * (m[MXX] + m[MYY] + m[MZZ]) + p.w[9] * rho;
  const R txx = (R(2) * t9 + d2 + R(3) * d1) * R(1.0 / 6.0);
  const R tyy = (R(2) * t9 + d2 - R(3) * d1) * R(1.0 / 6.0);
  const R tzz = (t9 - d2) * R(1.0 / 3.0);
  m[M0] = rho;
  m[MX] = R(0.5) * Fx;
  m[MY] = R(0.5) * Fy;
  m[MZ] = R(0.5) * Fz;
  m[MXY] *= p.wc[4];
  m[MXZ] *= p.wc[5];
  m[MYZ] *= p.wc[6];
  m[MXX] = txx;
  m[MYY] = tyy;
  m[MZZ] = tzz;
  m[MXYY] *= p.wc[10];
  m[MXXY] *= p.wc[11];
  m[MXXZ] *= p.wc[12];
  m[MXYZ] *= p.wc[13];
  m[MXXYY] = p.wc[14] * m[MXXYY] + p.w[14] * (txx * tyy * (p.per_mass ? inv_rho : R(1)));
  populations_from_central15(m, ux, uy, uz, f);
}

// Initial transformed populations fbar = f^eq(rho, u) - S/2: f^eq has the
// Maxwellian central moments rho, c_s^2 rho (xx, yy, zz), c_s^4 rho (xxyy).
template <typename R>
CMLBM_HD void initial15(R rho, R ux, R uy, R uz, R Fx, R Fy, R Fz, R (&f)[15]) {
  const R c2 = rho * R(1.0 / 3.0);
  R m[15];
#pragma unroll
  for (int k = 0; k < 15; ++k) m[k] = R(0);
  m[M0] = rho;
  m[MXX] = m[MYY] = m[MZZ] = c2;
  m[MXXYY] = rho * R(1.0 / 9.0);
  populations_from_central15(m, ux, uy, uz, f);
  R S[15];
  source15(Fx, Fy, Fz, ux, uy, uz, S);
#pragma unroll
  for (int a = 0; a < 15; ++a) f[a] -= R(0.5) * S[a];
}

// ---------------------------------------------------------------------------
// Adjoint of collide15 (moments in the order of the enum above; the per-axis
// shifts as in the forward collision).
// ---------------------------------------------------------------------------
// Adjoint of shift15: m = its input, g = adjoint of its output (in place ->
// adjoint of its input); adds d/du to gu.
template <int AX, typename R>
CMLBM_HD void shift15_adj(const R (&m)[15], R u, R sg, R (&g)[15], R& gu) {
  constexpr Groups15 G = groups15<AX>();
  const R v = sg * u;
  R gv = R(0);
  static_for<G.nt>([&](auto i) {
    constexpr int a = G.t[decltype(i)::value][0], b = G.t[decltype(i)::value][1], c = G.t[decltype(i)::value][2];
    const R g1 = g[b], g2 = g[c];
    gv += g1 * m[a] + g2 * R(2) * (m[b] + v * m[a]);
    g[a] += v * g1 + v * v * g2;
    g[b] = g1 + R(2) * v * g2;
  });
  static_for<G.np>([&](auto i) {
    constexpr int a = G.p[decltype(i)::value][0], b = G.p[decltype(i)::value][1];
    gv += g[b] * m[a];
    g[a] += v * g[b];
  });
  gu += sg * gv;
}

// Raw moments of h, and the transpose (adjoint) of that linear map.
template <typename R>
CMLBM_HD void raw15(const R (&h)[15], R (&r)[15]) {
  static_for<15>([&](auto m) {
    R acc = R(0);
    static_for<15>([&](auto a) {
      constexpr int k = kM15.v[decltype(m)::value][decltype(a)::value];
      if constexpr (k == 1) acc += h[a];
      if constexpr (k == -1) acc -= h[a];
    });
    r[m] = acc;
  });
}

template <typename R>
CMLBM_HD void raw15_adj(const R (&gr)[15], R (&gh)[15]) {
  static_for<15>([&](auto a) {
    R acc = R(0);
    static_for<15>([&](auto m) {
      constexpr int k = kM15.v[decltype(m)::value][decltype(a)::value];
      if constexpr (k == 1) acc += gr[m];
      if constexpr (k == -1) acc -= gr[m];
    });
    gh[a] = acc;
  });
}

// Transpose of the raw-moment inversion at the end of populations15:
// gs = (d f / d s)^T g.
template <typename R>
CMLBM_HD void inverse15_adj(const R (&g)[15], R (&gs)[15]) {
  R c = R(0), cx = R(0), cy = R(0), cz = R(0), cxy = R(0), cxz = R(0), cyz = R(0), cxyz = R(0);
#pragma unroll
  for (int a = 7; a < 15; ++a) {
    const int x = kE15[a].x, y = kE15[a].y, z = kE15[a].z;
    c += g[a];
    cx += R(x) * g[a];
    cy += R(y) * g[a];
    cz += R(z) * g[a];
    cxy += R(x * y) * g[a];
    cxz += R(x * z) * g[a];
    cyz += R(y * z) * g[a];
    cxyz += R(x * y * z) * g[a];
  }
  const R p1 = R(0.5) * (g[1] + g[2]), m1 = R(0.5) * (g[1] - g[2]);
  const R p2 = R(0.5) * (g[3] + g[4]), m2 = R(0.5) * (g[3] - g[4]);
  const R p3 = R(0.5) * (g[5] + g[6]), m3 = R(0.5) * (g[5] - g[6]);
  gs[0] = g[0];
  gs[1] = m1;
  gs[2] = m2;
  gs[3] = m3;
  gs[4] = R(0.125) * cxy;
  gs[5] = R(0.125) * cxz;
  gs[6] = R(0.125) * cyz;
  gs[7] = p1 - g[0];
  gs[8] = p2 - g[0];
  gs[9] = p3 - g[0];
  gs[10] = R(0.125) * cx - m1;
  gs[11] = R(0.125) * cy - m2;
  gs[12] = R(0.125) * cz - m3;
  gs[13] = R(0.125) * cxyz;
  gs[14] = R(0.125) * c - (p1 + p2 + p3) + R(2) * g[0];
}

// Adjoint of source15 with respect to F and u: gS = adjoint of S.
template <typename R>
CMLBM_HD void source15_adj(R Fx, R Fy, R Fz, R ux, R uy, R uz, const R (&gS)[15], R& gFx, R& gFy, R& gFz,
                           R& gux, R& guy, R& guz) {
  R G[15];
  static_for<14>([&](auto b1) {
    constexpr int b = decltype(b1)::value + 1;
    R acc = R(0);
    static_for<15>([&](auto a) {
      constexpr int k = kB15.v[b][decltype(a)::value];
      if constexpr (k != 0) acc += R(k) * gS[a];
    });
    constexpr int d = k15_norm(b);
    G[b] = acc * R(1.0 / d);
  });
  const R ux2 = ux * ux, uy2 = uy * uy, uz2 = uz * uz;
  gFx += G[1];
  gFy += G[2];
  gFz += G[3];
  // ms4..ms6
  gFx += uy * G[4] + uz * G[5];
  gFy += ux * G[4] + uz * G[6];
  gFz += ux * G[5] + uy * G[6];
  gux += Fy * G[4] + Fz * G[5];
  guy += Fx * G[4] + Fz * G[6];
  guz += Fx * G[5] + Fy * G[6];
  // ms7..ms9
  gFx += R(2) * ux * (G[7] + G[8] + G[9]);
  gFy += R(2) * uy * (-G[7] + G[8] + G[9]);
  gFz += R(2) * uz * (G[9] - R(2) * G[8]);
  gux += R(2) * Fx * (G[7] + G[8] + G[9]);
  guy += R(2) * Fy * (-G[7] + G[8] + G[9]);
  guz += R(2) * Fz * (G[9] - R(2) * G[8]);
  // ms10..ms12
  gFx += (R(5) * (R(3) * ux2 + uy2 + uz2) - R(13)) * G[10] + R(10) * ux * (uy * G[11] + uz * G[12]);
  gFy += (R(5) * (ux2 + R(3) * uy2 + uz2) - R(13)) * G[11] + R(10) * uy * (ux * G[10] + uz * G[12]);
  gFz += (R(5) * (ux2 + uy2 + R(3) * uz2) - R(13)) * G[12] + R(10) * uz * (ux * G[10] + uy * G[11]);
  gux += (R(30) * Fx * ux + R(10) * (Fy * uy + Fz * uz)) * G[10] + R(10) * (Fy * ux + Fx * uy) * G[11] +
         R(10) * (Fz * ux + Fx * uz) * G[12];
  guy += R(10) * (Fx * uy + Fy * ux) * G[10] + (R(30) * Fy * uy + R(10) * (Fx * ux + Fz * uz)) * G[11] +
         R(10) * (Fz * uy + Fy * uz) * G[12];
  guz += R(10) * (Fx * uz + Fz * ux) * G[10] + R(10) * (Fy * uz + Fz * uy) * G[11] +
         (R(30) * Fz * uz + R(10) * (Fx * ux + Fy * uy)) * G[12];
  // ms13
  gFx += uy * uz * G[13];
  gFy += ux * uz * G[13];
  gFz += ux * uy * G[13];
  gux += (Fy * uz + Fz * uy) * G[13];
  guy += (Fx * uz + Fz * ux) * G[13];
  guz += (Fx * uy + Fy * ux) * G[13];
  // ms14
  const R ax = R(3) * (uy2 + uz2) - R(4), ay = R(3) * (ux2 + uz2) - R(4), az = R(3) * (ux2 + uy2) - R(4);
  gFx += R(20) * ux * ax * G[14];
  gFy += R(20) * uy * ay * G[14];
  gFz += R(20) * uz * az * G[14];
  gux += R(20) * (Fx * ax + R(6) * ux * (Fy * uy + Fz * uz)) * G[14];
  guy += R(20) * (Fy * ay + R(6) * uy * (Fx * ux + Fz * uz)) * G[14];
  guz += R(20) * (Fz * az + R(6) * uz * (Fx * ux + Fy * uy)) * G[14];
}

// Adjoint of collide15.  f: pre-collision populations.  g: on entry the
// adjoint of the post-collision populations, on exit the adjoint of f.  Adds
// the force adjoint and gw[b] (adjoint of omega_b, b = 4..14).
template <int PM = -1, typename R, typename W>
CMLBM_HD void collide15_adj(const R (&f)[15], R Fx, R Fy, R Fz, const Rates<R>& p, R (&g)[15], R& gFx, R& gFy,
                            R& gFz, W& gw) {
  const bool pm = PM < 0 ? p.per_mass != 0 : PM != 0;
  R rho, ux, uy, uz, inv_rho;
  moments0_15(f, Fx, Fy, Fz, rho, ux, uy, uz, inv_rho);
  R gux = R(0), guy = R(0), guz = R(0), grho = R(0);
  const R sm = pm ? inv_rho : R(1);

  // forward: central moments c of h = f + S (raw moments of f plus those of S)
  R c[15];
  {
    R rs[15];
    raw15(f, c);
    source_raw15(Fx, Fy, Fz, ux, uy, uz, rs);
#pragma unroll
    for (int m = 0; m < 15; ++m) c[m] += rs[m];
  }
  shift15<0>(c, ux, R(-1));
  shift15<1>(c, uy, R(-1));
  shift15<2>(c, uz, R(-1));
  // relaxed central moments t (conserved rows: rho and F/2)
  const R d1 = p.wc[7] * (c[7] - c[8]);
  const R d2 = p.wc[8] * (c[7] + c[8] - R(2) * c[9]);
  const R t9 = p.wc[9] * (c[7] + c[8] + c[9]) + p.w[9] * rho;
  const R txx = (R(2) * t9 + d2 + R(3) * d1) * R(1.0 / 6.0);
  const R tyy = (R(2) * t9 + d2 - R(3) * d1) * R(1.0 / 6.0);
  const R tzz = (t9 - d2) * R(1.0 / 3.0);
  R t[15];
  t[0] = rho;
  t[1] = R(0.5) * Fx;
  t[2] = R(0.5) * Fy;
  t[3] = R(0.5) * Fz;
#pragma unroll
  for (int m = 4; m < 7; ++m) t[m] = p.wc[m] * c[m];
  t[7] = txx;
  t[8] = tyy;
  t[9] = tzz;
#pragma unroll
  for (int m = 10; m < 14; ++m) t[m] = p.wc[m] * c[m];
  t[14] = p.wc[14] * c[14] + p.w[14] * (txx * tyy * sm);

  // back through the inversion and the shifts central -> raw (z, y, x order
  // reversed: the forward applies z, then y, then x)
  R gt[15];
  inverse15_adj(g, gt);
  {
    R v[15];   // input of the x shift = t shifted along z and y
#pragma unroll
    for (int m = 0; m < 15; ++m) v[m] = t[m];
    shift15<2>(v, uz, R(1));
    shift15<1>(v, uy, R(1));
    shift15_adj<0>(v, ux, R(1), gt, gux);
    shift15<1>(v, uy, R(-1));   // undo: v = input of the y shift
    shift15_adj<1>(v, uy, R(1), gt, guy);
    shift15_adj<2>(t, uz, R(1), gt, guz);
  }
  // relaxation
  grho += gt[0];
  gFx += R(0.5) * gt[1];
  gFy += R(0.5) * gt[2];
  gFz += R(0.5) * gt[3];
  R gc[15];
  gc[0] = gc[1] = gc[2] = gc[3] = R(0);
#pragma unroll
  for (int m = 4; m < 7; ++m) {
    gc[m] = p.wc[m] * gt[m];
    gw[m] -= c[m] * gt[m];
  }
#pragma unroll
  for (int m = 10; m < 14; ++m) {
    gc[m] = p.wc[m] * gt[m];
    gw[m] -= c[m] * gt[m];
  }
  R gtxx = gt[7], gtyy = gt[8];
  const R gtzz = gt[9];
  {
    const R G = gt[14];
    const R A = txx * tyy * sm;
    gc[14] = p.wc[14] * G;
    gw[14] += (A - c[14]) * G;
    const R gA = p.w[14] * G;
    if (pm) grho -= sm * A * gA;
    gtxx += gA * tyy * sm;
    gtyy += gA * txx * sm;
  }
  {
    const R gt9 = (gtxx + gtyy) * R(1.0 / 3.0) + gtzz * R(1.0 / 3.0);
    const R gd2 = (gtxx + gtyy) * R(1.0 / 6.0) - gtzz * R(1.0 / 3.0);
    const R gd1 = R(0.5) * (gtxx - gtyy);
    gw[7] -= (c[7] - c[8]) * gd1;
    gw[8] -= (c[7] + c[8] - R(2) * c[9]) * gd2;
    gw[9] += (rho - (c[7] + c[8] + c[9])) * gt9;
    grho += p.w[9] * gt9;
    const R gD1 = p.wc[7] * gd1, gD2 = p.wc[8] * gd2, gT = p.wc[9] * gt9;
    gc[7] = gD1 + gD2 + gT;
    gc[8] = -gD1 + gD2 + gT;
    gc[9] = R(-2) * gD2 + gT;
  }
  // back through the shifts raw -> central (forward order x, y, z)
  {
    R v[15];   // input of the z shift: c unshifted along z
#pragma unroll
    for (int m = 0; m < 15; ++m) v[m] = c[m];
    shift15<2>(v, uz, R(1));
    shift15_adj<2>(v, uz, R(-1), gc, guz);
    shift15<1>(v, uy, R(1));   // input of the y shift
    shift15_adj<1>(v, uy, R(-1), gc, guy);
    shift15<0>(v, ux, R(1));   // raw moments of h
    shift15_adj<0>(v, ux, R(-1), gc, gux);
  }
  // raw moments (of f and of the source), density and velocity
  R gh[15];
  raw15_adj(gc, gh);
  source_raw15_adj(Fx, Fy, Fz, ux, uy, uz, gc, gFx, gFy, gFz, gux, guy, guz);
  const R inv = inv_rho;
  const R gjx = gux * inv, gjy = guy * inv, gjz = guz * inv;
  grho -= (ux * gux + uy * guy + uz * guz) * inv;
  gFx += R(0.5) * gjx;
  gFy += R(0.5) * gjy;
  gFz += R(0.5) * gjz;
#pragma unroll
  for (int a = 0; a < 15; ++a)
    g[a] = gh[a] + grho + R(kE15[a].x) * gjx + R(kE15[a].y) * gjy + R(kE15[a].z) * gjz;
}

// Adjoint of the force dependence of initial15 (u0 fixed): fbar = f^eq - S/2.
template <typename R>
CMLBM_HD void initial15_adj_force(R ux, R uy, R uz, const R (&lam)[15], R& gFx, R& gFy, R& gFz) {
  R gS[15];
#pragma unroll
  for (int a = 0; a < 15; ++a) gS[a] = R(-0.5) * lam[a];
  R gux = R(0), guy = R(0), guz = R(0);
  source15_adj(R(0), R(0), R(0), ux, uy, uz, gS, gFx, gFy, gFz, gux, guy, guz);
}

}  // namespace cmlbm
