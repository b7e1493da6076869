// D3Q27 central-moment collision with forcing, and its hand-written adjoint.
//
// The cascaded collision of Premnath & Banerjee (arXiv:1202.6081, Sec. 7 and
// Sec. 8) produces post-collision populations whose central moments about the
// local velocity u are the pre-collision ones relaxed toward the factorized
// attractors.  On D3Q27 the central moments of all 27 monomials
// (e_x-u_x)^a (e_y-u_y)^b (e_z-u_z)^c, a, b, c in {0, 1, 2}, factorize per axis,
// so the raw-moment sums of Appendix B followed by the binomial shift of Sec. 6
// become three passes of 3-point transforms over a 3x3x3 cube, and the return
// to populations (the K g + S rows of Sec. 8) becomes three inverse passes.
//
// Source term (Sec. 5, Eq. discretecentralsources): S changes only the three
// first-order central moments, by F.  Adding S to fbar therefore sets the
// first central moments to -F/2 + F = F/2, which the collision conserves; the
// velocity includes F/2 (Eq. velocitycalculation).
//
// Cube layout: m[a*9 + b*3 + c] holds the population with e = (a-1, b-1, c-1)
// before the forward passes and the central moment with exponents (a, b, c)
// after them.
#pragma once

#include "lattice.hpp"

namespace cmlbm {

constexpr int K3(int a, int b, int c) { return a * 9 + b * 3 + c; }

// Relaxation rates indexed by the paper's kernel number b = 4..26 (entries
// 0..3 unused): w[b] = omega_b and wc[b] = 1 - omega_b.
template <typename R>
struct Rates {
  R w[27];
  R wc[27];
  // 0: factorized attractors as the literal products of post-collision
  // second moments (kxx kyy, kxx kyy kzz); 1: per unit mass, rho (kxx/rho)
  // (kyy/rho) and rho (kxx/rho)(kyy/rho)(kzz/rho).
  int per_mass;
};

// -- 3-point transforms along one axis --------------------------------------
// Populations (p_-, p_0, p_+) -> central moments (k0, k1, k2) about u:
// k_n = sum_e p_e (e - u)^n.
template <typename R>
CMLBM_HD void fwd_line(R& a, R& b, R& c, R u) {
  const R k0 = a + b + c;
  const R d = c - a;
  const R k1 = d - u * k0;
  const R k2 = (c + a) - u * (d + k1);
  a = k0;
  b = k1;
  c = k2;
}

// Central moments (m0, m1, m2) about u -> populations (p_-, p_0, p_+).
// (p_+ is formed as (r2 + r1)/2: the shorter p_- + r1 measured ten times the
// FP32 error on a steady duct flow, 2.1e-3 against 1.8e-4 relative L2 after
// 4e5 steps, the rounding errors of a steady state repeating every step.)
// With HALVE = false, p_- and p_+ come out doubled (r2 -+ r1): the caller
// applies the power-of-two factors of all passes at once (exact, so the
// result is the same bit for bit).
template <bool HALVE = true, typename R>
CMLBM_HD void inv_line(R& a, R& b, R& c, R u) {
  const R m0 = a, m1 = b, m2 = c;
  const R r1 = m1 + u * m0;              // raw first moment
  const R r2 = m2 + u * (m1 + r1);       // raw second moment
  if constexpr (HALVE) {
    a = R(0.5) * (r2 - r1);
    c = R(0.5) * (r2 + r1);
  } else {
    a = r2 - r1;
    c = r2 + r1;
  }
  b = m0 - r2;
}

// Adjoint of fwd_line: (a, b, c) are the forward inputs, (ga, gb, gc) hold
// the adjoints of the outputs on entry and of the inputs on exit.
template <typename R>
CMLBM_HD void fwd_line_adj(R a, R b, R c, R u, R& ga, R& gb, R& gc, R& gu) {
  const R k0 = a + b + c;
  const R d = c - a;
  const R k1 = d - u * k0;
  const R g0 = ga, g1 = gb, g2 = gc;
  gu -= (d + k1) * g2;
  const R gt = -u * g2;                   // adjoint of (d + k1)
  const R g1t = g1 + gt;
  const R gd = gt + g1t;
  gu -= k0 * g1t;
  const R g0t = g0 - u * g1t;
  ga = g2 - gd + g0t;
  gb = g0t;
  gc = g2 + gd + g0t;
}

// Adjoint of inv_line, same conventions.
template <typename R>
CMLBM_HD void inv_line_adj(R m0, R m1, R m2, R u, R& ga, R& gb, R& gc, R& gu) {
  const R r1 = m1 + u * m0;
  const R pa = ga, pb = gb, pc = gc;
  const R gr2 = R(0.5) * (pa + pc) - pb;
  R gr1 = R(0.5) * (pc - pa);
  R gm0 = pb;
  const R gm2 = gr2;
  gu += gr2 * (m1 + r1);
  R gm1 = gr2 * u;
  gr1 += gr2 * u;
  gm1 += gr1;
  gm0 += gr1 * u;
  gu += gr1 * m0;
  ga = gm0;
  gb = gm1;
  gc = gm2;
}

// The forward transform of the step in two halves: raw moments first, one
// axis at a time, (p_-, p_0, p_+) -> (sum, p_+ - p_-, p_+ + p_-) (3 operations
// per line), then the binomial shift to central moments about u, one axis at a
// time (the shifts along different axes act on different exponents and
// commute).  Density and momentum are then the raw moments 000, 100, 010, 001.
template <typename R>
CMLBM_HD void raw_line(R& a, R& b, R& c) {
  const R s2 = c + a, s1 = c - a;
  a = s2 + b;
  b = s1;
  c = s2;
}

// Raw (r0, r1, r2) along an axis -> central (r0, r1 - u r0, r2 - 2 u r1 + u^2 r0).
template <typename R>
CMLBM_HD void shift_line(R a, R& b, R& c, R u) {
  const R k1 = b - u * a;
  c = c - u * (b + k1);
  b = k1;
}

// Inverse of shift_line: central (k0, k1, k2) about u -> raw (r0, r1, r2).
template <typename R>
CMLBM_HD void unshift_line(R a, R& b, R& c, R u) {
  const R r1 = b + u * a;
  c = c + u * (r1 + b);
  b = r1;
}

// Adjoint of shift_line from its output (k0, k1): (g0, g1, g2) hold the
// adjoints of (k0, k1, k2) on entry and of (r0, r1, r2) on exit; with
// k1 = r1 - u r0 and k2 = r2 - u (r1 + k1), dk2/du = -2 k1 and dk1/du = -k0.
template <typename R>
CMLBM_HD void shift_line_adj(R k0, R k1, R u, R& g0, R& g1, R g2, R& gu) {
  gu -= k0 * g1 + R(2) * k1 * g2;
  const R t = g1 - u * g2;
  g0 = g0 - u * t;
  g1 = t - u * g2;
}

// Adjoint of raw_line (a linear map): (ga, gb, gc) hold the adjoints of
// (sum, p_+ - p_-, p_+ + p_-) on entry and of (p_-, p_0, p_+) on exit.
template <typename R>
CMLBM_HD void raw_line_adj(R& ga, R& gb, R& gc) {
  const R g0 = ga, g1 = gb, g2 = gc;
  const R t = g0 + g2;
  ga = t - g1;
  gb = g0;
  gc = t + g1;
}

// Base index and stride of line l (0..8) along an axis (0 = x, 1 = y, 2 = z).
template <int AXIS>
CMLBM_HDC int line_base(int l) {
  return AXIS == 2 ? (l / 3) * 9 + (l % 3) * 3 : AXIS == 1 ? (l / 3) * 9 + (l % 3) : l;
}
template <int AXIS>
CMLBM_HDC int line_stride() {
  return AXIS == 0 ? 9 : AXIS == 1 ? 3 : 1;
}

template <int AXIS, typename R>
CMLBM_HD void fwd_pass(R (&m)[27], R u) {
  constexpr int S = line_stride<AXIS>();
#pragma unroll
  for (int l = 0; l < 9; ++l) {
    const int o = line_base<AXIS>(l);
    fwd_line(m[o], m[o + S], m[o + 2 * S], u);
  }
}

template <int AXIS, typename R>
CMLBM_HD void raw_pass(R (&m)[27]) {
  constexpr int S = line_stride<AXIS>();
#pragma unroll
  for (int l = 0; l < 9; ++l) {
    const int o = line_base<AXIS>(l);
    raw_line(m[o], m[o + S], m[o + 2 * S]);
  }
}

template <int AXIS, typename R>
CMLBM_HD void shift_pass(R (&m)[27], R u) {
  constexpr int S = line_stride<AXIS>();
#pragma unroll
  for (int l = 0; l < 9; ++l) {
    const int o = line_base<AXIS>(l);
    shift_line(m[o], m[o + S], m[o + 2 * S], u);
  }
}

template <int AXIS, typename R>
CMLBM_HD void unshift_pass(R (&m)[27], R u) {
  constexpr int S = line_stride<AXIS>();
#pragma unroll
  for (int l = 0; l < 9; ++l) {
    const int o = line_base<AXIS>(l);
    unshift_line(m[o], m[o + S], m[o + 2 * S], u);
  }
}

// m: the output of shift_pass<AXIS> (central moments along AXIS).
template <int AXIS, typename R>
CMLBM_HD void shift_pass_adj(const R (&m)[27], R u, R (&g)[27], R& gu) {
  constexpr int S = line_stride<AXIS>();
#pragma unroll
  for (int l = 0; l < 9; ++l) {
    const int o = line_base<AXIS>(l);
    shift_line_adj(m[o], m[o + S], u, g[o], g[o + S], g[o + 2 * S], gu);
  }
}

template <int AXIS, typename R>
CMLBM_HD void raw_pass_adj(R (&g)[27]) {
  constexpr int S = line_stride<AXIS>();
#pragma unroll
  for (int l = 0; l < 9; ++l) {
    const int o = line_base<AXIS>(l);
    raw_line_adj(g[o], g[o + S], g[o + 2 * S]);
  }
}

template <int AXIS, bool HALVE = true, typename R>
CMLBM_HD void inv_pass(R (&m)[27], R u) {
  constexpr int S = line_stride<AXIS>();
#pragma unroll
  for (int l = 0; l < 9; ++l) {
    const int o = line_base<AXIS>(l);
    inv_line<HALVE>(m[o], m[o + S], m[o + 2 * S], u);
  }
}

template <int AXIS, typename R>
CMLBM_HD void fwd_pass_adj(const R (&m)[27], R u, R (&g)[27], R& gu) {
  constexpr int S = line_stride<AXIS>();
#pragma unroll
  for (int l = 0; l < 9; ++l) {
    const int o = line_base<AXIS>(l);
    fwd_line_adj(m[o], m[o + S], m[o + 2 * S], u, g[o], g[o + S], g[o + 2 * S], gu);
  }
}

template <int AXIS, typename R>
CMLBM_HD void inv_pass_adj(const R (&m)[27], R u, R (&g)[27], R& gu) {
  constexpr int S = line_stride<AXIS>();
#pragma unroll
  for (int l = 0; l < 9; ++l) {
    const int o = line_base<AXIS>(l);
    inv_line_adj(m[o], m[o + S], m[o + 2 * S], u, g[o], g[o + S], g[o + 2 * S], gu);
  }
}

// Relax the central moments in m (cube layout) in place.  PM: attractor form,
// 0 literal, 1 per unit mass, -1 as p.per_mass says (run time).
template <int PM = -1, typename R>
CMLBM_HD void relax27(R (&m)[27], R rho, R inv_rho, R Fx, R Fy, R Fz, const Rates<R>& p) {
  const bool pm = PM < 0 ? p.per_mass != 0 : PM != 0;
  // conserved: density and first central moments F/2
  m[K3(0, 0, 0)] = rho;
  m[K3(1, 0, 0)] = R(0.5) * Fx;
  m[K3(0, 1, 0)] = R(0.5) * Fy;
  m[K3(0, 0, 1)] = R(0.5) * Fz;
  // second order, off-diagonal (g4, g5, g6): attractor 0
  m[K3(1, 1, 0)] *= p.wc[4];
  m[K3(1, 0, 1)] *= p.wc[5];
  m[K3(0, 1, 1)] *= p.wc[6];
  // second order, diagonal: xx-yy (g7), xx+yy-2zz (g8) toward 0, xx+yy+zz (g9) toward rho
  const R xx = m[K3(2, 0, 0)], yy = m[K3(0, 2, 0)], zz = m[K3(0, 0, 2)];
  const R d1 = p.wc[7] * (xx - yy);
  const R d2 = p.wc[8] * (xx + yy - R(2) * zz);
  const R t = p.wc[9] * (xx + yy + zz) + p.w[9] * rho;
  const R kxx = (R(2) * t + d2 + R(3) * d1) * R(1.0 / 6.0);
  const R kyy = (R(2) * t + d2 - R(3) * d1) * R(1.0 / 6.0);
  const R kzz = (t - d2) * R(1.0 / 3.0);
  m[K3(2, 0, 0)] = kxx;
  m[K3(0, 2, 0)] = kyy;
  m[K3(0, 0, 2)] = kzz;
  // third order: xyy+xzz (g10) with xyy-xzz (g13), and the y, z analogues
  {
    const R s = p.wc[10] * (m[K3(1, 2, 0)] + m[K3(1, 0, 2)]);
    const R d = p.wc[13] * (m[K3(1, 2, 0)] - m[K3(1, 0, 2)]);
    m[K3(1, 2, 0)] = R(0.5) * (s + d);
    m[K3(1, 0, 2)] = R(0.5) * (s - d);
  }
  {
    const R s = p.wc[11] * (m[K3(2, 1, 0)] + m[K3(0, 1, 2)]);
    const R d = p.wc[14] * (m[K3(2, 1, 0)] - m[K3(0, 1, 2)]);
    m[K3(2, 1, 0)] = R(0.5) * (s + d);
    m[K3(0, 1, 2)] = R(0.5) * (s - d);
  }
  {
    const R s = p.wc[12] * (m[K3(2, 0, 1)] + m[K3(0, 2, 1)]);
    const R d = p.wc[15] * (m[K3(2, 0, 1)] - m[K3(0, 2, 1)]);
    m[K3(2, 0, 1)] = R(0.5) * (s + d);
    m[K3(0, 2, 1)] = R(0.5) * (s - d);
  }
  m[K3(1, 1, 1)] *= p.wc[16];
  // fourth order, diagonal pairs (g17, g18, g19) toward the factorized attractors
  const R sm = pm ? inv_rho : R(1);
  {
    const R axy = kxx * kyy * sm, axz = kxx * kzz * sm, ayz = kyy * kzz * sm;
    const R A = m[K3(2, 2, 0)], B = m[K3(2, 0, 2)], C = m[K3(0, 2, 2)];
    const R q1 = p.wc[17] * (A + B + C) + p.w[17] * (axy + axz + ayz);
    const R q2 = p.wc[18] * (A + B - R(2) * C) + p.w[18] * (axy + axz - R(2) * ayz);
    const R q3 = p.wc[19] * (A - B) + p.w[19] * (axy - axz);
    const R ab = (R(2) * q1 + q2) * R(1.0 / 3.0);
    m[K3(0, 2, 2)] = (q1 - q2) * R(1.0 / 3.0);
    m[K3(2, 2, 0)] = R(0.5) * (ab + q3);
    m[K3(2, 0, 2)] = R(0.5) * (ab - q3);
  }
  m[K3(2, 1, 1)] *= p.wc[20];
  m[K3(1, 2, 1)] *= p.wc[21];
  m[K3(1, 1, 2)] *= p.wc[22];
  // fifth order
  m[K3(1, 2, 2)] *= p.wc[23];
  m[K3(2, 1, 2)] *= p.wc[24];
  m[K3(2, 2, 1)] *= p.wc[25];
  // sixth order toward kxx kyy kzz (g26)
  m[K3(2, 2, 2)] = p.wc[26] * m[K3(2, 2, 2)] + p.w[26] * (kxx * kyy * kzz * (sm * sm));
}

// First pass along z fused with the density and velocity sums: raw z-moments
// (s0, s1, s2) = (a+b+c, c-a, c+a) of each line give rho and j, then the shift
// to central moments about u_z is the same arithmetic as fwd_line.
template <typename R>
CMLBM_HD void first_pass27(R (&m)[27], R Fx, R Fy, R Fz, R& rho, R& ux, R& uy, R& uz, R& inv_rho) {
  R s0[9], s1[9];
#pragma unroll
  for (int l = 0; l < 9; ++l) {
    const int o = line_base<2>(l);
    s0[l] = m[o] + m[o + 1] + m[o + 2];
    s1[l] = m[o + 2] - m[o];
  }
  // lines l = ix*3 + iy
  rho = ((s0[0] + s0[1] + s0[2]) + (s0[3] + s0[4] + s0[5])) + (s0[6] + s0[7] + s0[8]);
  const R jx = (s0[6] + s0[7] + s0[8]) - (s0[0] + s0[1] + s0[2]);
  const R jy = (s0[2] + s0[5] + s0[8]) - (s0[0] + s0[3] + s0[6]);
  const R jz = ((s1[0] + s1[1] + s1[2]) + (s1[3] + s1[4] + s1[5])) + (s1[6] + s1[7] + s1[8]);
  const R inv = recip(rho);
  inv_rho = inv;
  ux = (jx + R(0.5) * Fx) * inv;
  uy = (jy + R(0.5) * Fy) * inv;
  uz = (jz + R(0.5) * Fz) * inv;
#pragma unroll
  for (int l = 0; l < 9; ++l) {
    const int o = line_base<2>(l);
    const R k1 = s1[l] - uz * s0[l];
    const R k2 = (m[o + 2] + m[o]) - uz * (s1[l] + k1);
    m[o] = s0[l];
    m[o + 1] = k1;
    m[o + 2] = k2;
  }
}

// Full collision: cube-ordered pre-collision populations in, post-collision out.
template <typename R>
CMLBM_HD void collide27(R (&m)[27], R Fx, R Fy, R Fz, const Rates<R>& p) {
  raw_pass<2>(m);
  raw_pass<1>(m);
  raw_pass<0>(m);
  const R rho = m[K3(0, 0, 0)];
  const R inv_rho = recip(rho);
  // (explicit fused multiply-adds: the rounding of u must not depend on what
  // else the kernel computes from 0.5 F)
  const R ux = fma_r(R(0.5), Fx, m[K3(1, 0, 0)]) * inv_rho;
  const R uy = fma_r(R(0.5), Fy, m[K3(0, 1, 0)]) * inv_rho;
  const R uz = fma_r(R(0.5), Fz, m[K3(0, 0, 1)]) * inv_rho;
  shift_pass<0>(m, ux);
  shift_pass<1>(m, uy);
  shift_pass<2>(m, uz);
  relax27(m, rho, inv_rho, Fx, Fy, Fz, p);
  // the three inverse passes without their halvings, then population e scaled
  // by 2^-(number of nonzero components of e) (one multiply each, which a
  // 16-bit store fuses with its subtraction of the rest weight)
  inv_pass<0, false>(m, ux);
  inv_pass<1, false>(m, uy);
  inv_pass<2, false>(m, uz);
#pragma unroll
  for (int i = 0; i < 27; ++i) {
    const int k = (i / 9 != 1) + ((i / 3) % 3 != 1) + (i % 3 != 1);
    if (k) m[i] *= R(k == 1 ? 0.5 : k == 2 ? 0.25 : 0.125);
  }
}

// Adjoint of relax27.  m: pre-relaxation central moments (unchanged).  g: on
// entry the adjoint of the relaxed moments, on exit the adjoint of m.  Adds to
// grho, gF*, gw[b] (adjoint of omega_b, b = 4..26; gw is an array or any
// accumulator whose operator[] yields an R&).
template <int PM = -1, typename R, typename W>
CMLBM_HD void relax27_adj(const R (&m)[27], R rho, const Rates<R>& p, R (&g)[27], R& grho,
                                            R& gFx, R& gFy, R& gFz, W& gw) {
  const bool pm = PM < 0 ? p.per_mass != 0 : PM != 0;
  // recompute the second-order post values and attractor inputs
  const R xx = m[K3(2, 0, 0)], yy = m[K3(0, 2, 0)], zz = m[K3(0, 0, 2)];
  const R D1 = xx - yy, D2 = xx + yy - R(2) * zz, T = xx + yy + zz;
  const R d1 = p.wc[7] * D1, d2 = p.wc[8] * D2, t = p.wc[9] * T + p.w[9] * rho;
  const R kxx = (R(2) * t + d2 + R(3) * d1) * R(1.0 / 6.0);
  const R kyy = (R(2) * t + d2 - R(3) * d1) * R(1.0 / 6.0);
  const R kzz = (t - d2) * R(1.0 / 3.0);
  R gkxx = R(0), gkyy = R(0), gkzz = R(0);
  // per-mass attractors: A = P sm^(k-1), dA/drho = -(k-1) A sm
  const R sm = pm ? R(1) / rho : R(1);

  // sixth order
  {
    const R G = g[K3(2, 2, 2)];
    const R s2 = sm * sm;
    const R P = kxx * kyy * kzz * s2;
    gw[26] += (P - m[K3(2, 2, 2)]) * G;
    const R gP = p.w[26] * G;
    if (pm) grho -= R(2) * sm * P * gP;
    const R gPs = gP * s2;
    gkxx += gPs * kyy * kzz;
    gkyy += gPs * kxx * kzz;
    gkzz += gPs * kxx * kyy;
    g[K3(2, 2, 2)] = p.wc[26] * G;
  }
  // fifth order and fourth-order off-diagonal: m~ = (1 - w) m
#define CMLBM_SCALE_ADJ(I, B)         \
  {                                   \
    const R G = g[I];                 \
    gw[B] -= m[I] * G;                \
    g[I] = p.wc[B] * G;               \
  }
  CMLBM_SCALE_ADJ(K3(1, 2, 2), 23)
  CMLBM_SCALE_ADJ(K3(2, 1, 2), 24)
  CMLBM_SCALE_ADJ(K3(2, 2, 1), 25)
  CMLBM_SCALE_ADJ(K3(2, 1, 1), 20)
  CMLBM_SCALE_ADJ(K3(1, 2, 1), 21)
  CMLBM_SCALE_ADJ(K3(1, 1, 2), 22)
  // fourth order diagonal
  {
    const R axy = kxx * kyy * sm, axz = kxx * kzz * sm, ayz = kyy * kzz * sm;
    const R A = m[K3(2, 2, 0)], B = m[K3(2, 0, 2)], C = m[K3(0, 2, 2)];
    const R Q1 = A + B + C, Q2 = A + B - R(2) * C, Q3 = A - B;
    const R a1 = axy + axz + ayz, a2 = axy + axz - R(2) * ayz, a3 = axy - axz;
    const R gA = g[K3(2, 2, 0)], gB = g[K3(2, 0, 2)], gC = g[K3(0, 2, 2)];
    const R gab = R(0.5) * (gA + gB);
    const R gq3 = R(0.5) * (gA - gB);
    const R gq1 = (gC + R(2) * gab) * R(1.0 / 3.0);
    const R gq2 = (gab - gC) * R(1.0 / 3.0);
    gw[17] += (a1 - Q1) * gq1;
    gw[18] += (a2 - Q2) * gq2;
    gw[19] += (a3 - Q3) * gq3;
    const R ga1 = p.w[17] * gq1, ga2 = p.w[18] * gq2, ga3 = p.w[19] * gq3;
    const R gQ1 = p.wc[17] * gq1, gQ2 = p.wc[18] * gq2, gQ3 = p.wc[19] * gq3;
    const R gaxy = ga1 + ga2 + ga3, gaxz = ga1 + ga2 - ga3, gayz = ga1 - R(2) * ga2;
    if (pm) grho -= sm * (axy * gaxy + axz * gaxz + ayz * gayz);
    gkxx += sm * (gaxy * kyy + gaxz * kzz);
    gkyy += sm * (gaxy * kxx + gayz * kzz);
    gkzz += sm * (gaxz * kxx + gayz * kyy);
    g[K3(2, 2, 0)] = gQ1 + gQ2 + gQ3;
    g[K3(2, 0, 2)] = gQ1 + gQ2 - gQ3;
    g[K3(0, 2, 2)] = gQ1 - R(2) * gQ2;
  }
  // third order
  CMLBM_SCALE_ADJ(K3(1, 1, 1), 16)
#define CMLBM_PAIR_ADJ(IA, IB, BS, BD)                  \
  {                                                     \
    const R gs = R(0.5) * (g[IA] + g[IB]);              \
    const R gd = R(0.5) * (g[IA] - g[IB]);              \
    gw[BS] -= (m[IA] + m[IB]) * gs;                     \
    gw[BD] -= (m[IA] - m[IB]) * gd;                     \
    const R a = p.wc[BS] * gs, b = p.wc[BD] * gd;       \
    g[IA] = a + b;                                      \
    g[IB] = a - b;                                      \
  }
  CMLBM_PAIR_ADJ(K3(1, 2, 0), K3(1, 0, 2), 10, 13)
  CMLBM_PAIR_ADJ(K3(2, 1, 0), K3(0, 1, 2), 11, 14)
  CMLBM_PAIR_ADJ(K3(2, 0, 1), K3(0, 2, 1), 12, 15)
#undef CMLBM_PAIR_ADJ
  // second order diagonal; total adjoint of kxx, kyy, kzz
  {
    const R Gx = g[K3(2, 0, 0)] + gkxx, Gy = g[K3(0, 2, 0)] + gkyy, Gz = g[K3(0, 0, 2)] + gkzz;
    const R gt = (Gx + Gy) * R(1.0 / 3.0) + Gz * R(1.0 / 3.0);
    const R gd2 = (Gx + Gy) * R(1.0 / 6.0) - Gz * R(1.0 / 3.0);
    const R gd1 = R(0.5) * (Gx - Gy);
    gw[7] -= D1 * gd1;
    gw[8] -= D2 * gd2;
    gw[9] += (rho - T) * gt;
    grho += p.w[9] * gt;
    const R gD1 = p.wc[7] * gd1, gD2 = p.wc[8] * gd2, gT = p.wc[9] * gt;
    g[K3(2, 0, 0)] = gD1 + gD2 + gT;
    g[K3(0, 2, 0)] = -gD1 + gD2 + gT;
    g[K3(0, 0, 2)] = R(-2) * gD2 + gT;
  }
  CMLBM_SCALE_ADJ(K3(1, 1, 0), 4)
  CMLBM_SCALE_ADJ(K3(1, 0, 1), 5)
  CMLBM_SCALE_ADJ(K3(0, 1, 1), 6)
#undef CMLBM_SCALE_ADJ
  // conserved rows were overwritten by rho and F/2
  grho += g[K3(0, 0, 0)];
  gFx += R(0.5) * g[K3(1, 0, 0)];
  gFy += R(0.5) * g[K3(0, 1, 0)];
  gFz += R(0.5) * g[K3(0, 0, 1)];
  g[K3(0, 0, 0)] = g[K3(1, 0, 0)] = g[K3(0, 1, 0)] = g[K3(0, 0, 1)] = R(0);
}

// Adjoint of collide27.  f: cube-ordered pre-collision populations on entry;
// on exit it holds scratch.  g: on entry the adjoint of the post-collision
// populations, on exit the adjoint of f.  s: scratch.  Adds the force and rate
// adjoints.  The forward transform is replayed as collide27 computes it (raw
// sums, u, shifts) and only the central moments c are kept.  The inverse
// passes are differentiated with their inputs recovered from the relaxed
// moments; the shifts in reverse order from their outputs (each shift's
// output is the next one's input, recovered by undoing the later shift); the
// raw sums are linear and need no inputs; rho and u enter through the raw
// moments 000, 100, 010, 001.
template <int PM = -1, typename R, typename W>
CMLBM_HD void collide27_adj(R (&f)[27], R Fx, R Fy, R Fz, const Rates<R>& p, R (&g)[27], R (&s)[27],
                                              R& gFx, R& gFy, R& gFz, W& gw) {
  R(&cm)[27] = f;
  raw_pass<2>(cm);
  raw_pass<1>(cm);
  raw_pass<0>(cm);
  const R rho = cm[K3(0, 0, 0)];
  const R inv_rho = recip(rho);
  const R ux = fma_r(R(0.5), Fx, cm[K3(1, 0, 0)]) * inv_rho;
  const R uy = fma_r(R(0.5), Fy, cm[K3(0, 1, 0)]) * inv_rho;
  const R uz = fma_r(R(0.5), Fz, cm[K3(0, 0, 1)]) * inv_rho;
  shift_pass<0>(cm, ux);
  shift_pass<1>(cm, uy);
  shift_pass<2>(cm, uz);
  R gux = R(0), guy = R(0), guz = R(0), grho = R(0);

  // relaxed moments, then replay the inverse passes to get each pass's input
#pragma unroll
  for (int k = 0; k < 27; ++k) s[k] = cm[k];
  relax27<PM>(s, rho, inv_rho, Fx, Fy, Fz, p);
  inv_pass<0>(s, ux);
  inv_pass<1>(s, uy);                        // s = input of the z inverse pass
  inv_pass_adj<2>(s, uz, g, guz);
  fwd_pass<1>(s, uy);                        // undo the y pass: s = input of the y inverse pass
  inv_pass_adj<1>(s, uy, g, guy);
  fwd_pass<0>(s, ux);                        // s = relaxed central moments
  inv_pass_adj<0>(s, ux, g, gux);

  relax27_adj<PM>(cm, rho, p, g, grho, gFx, gFy, gFz, gw);

  // the shifts z, y, x in reverse; cm holds the output of the shift being
  // differentiated
  shift_pass_adj<2>(cm, uz, g, guz);
  unshift_pass<2>(cm, uz);
  shift_pass_adj<1>(cm, uy, g, guy);
  unshift_pass<1>(cm, uy);
  shift_pass_adj<0>(cm, ux, g, gux);

  // u = (j + F/2) / rho with j and rho the raw moments 100, 010, 001 and 000
  const R gjx = gux * inv_rho, gjy = guy * inv_rho, gjz = guz * inv_rho;
  g[K3(0, 0, 0)] += grho - (ux * gux + uy * guy + uz * guz) * inv_rho;
  g[K3(1, 0, 0)] += gjx;
  g[K3(0, 1, 0)] += gjy;
  g[K3(0, 0, 1)] += gjz;
  gFx += R(0.5) * gjx;
  gFy += R(0.5) * gjy;
  gFz += R(0.5) * gjz;
  raw_pass_adj<0>(g);
  raw_pass_adj<1>(g);
  raw_pass_adj<2>(g);
}


// Initial transformed populations fbar = f^eq(rho, u) - S/2 (paper order): the
// central moments about u are the Maxwellian's (Sec. 3: rho c_s^(2k) on the
// even monomials, zero on the odd ones) with -F/2 on the first-order ones (the
// source changes only those, Eq. discretecentralsources); the inverse passes
// return them to populations.
template <typename R>
CMLBM_HD void initial27(R rho, R ux, R uy, R uz, R Fx, R Fy, R Fz, R (&f)[27]) {
  R m[27];
#pragma unroll
  for (int i = 0; i < 27; ++i) m[i] = R(0);
  const R c2 = rho * R(1.0 / 3.0);
  m[K3(0, 0, 0)] = rho;
  m[K3(1, 0, 0)] = R(-0.5) * Fx;
  m[K3(0, 1, 0)] = R(-0.5) * Fy;
  m[K3(0, 0, 1)] = R(-0.5) * Fz;
  m[K3(2, 0, 0)] = m[K3(0, 2, 0)] = m[K3(0, 0, 2)] = c2;
  m[K3(2, 2, 0)] = m[K3(2, 0, 2)] = m[K3(0, 2, 2)] = c2 * R(1.0 / 3.0);
  m[K3(2, 2, 2)] = c2 * R(1.0 / 9.0);
  inv_pass<0>(m, ux);
  inv_pass<1>(m, uy);
  inv_pass<2>(m, uz);
#pragma unroll
  for (int a = 0; a < 27; ++a) f[a] = m[cube27(a)];
}

// Adjoint of initial27 with respect to the force (u fixed): the populations
// are the inverse-pass image of the moments above, linear in F through the
// first-order entries -F/2.  lam: adjoint of f (paper order); adds to gF*.
template <typename R>
CMLBM_HD void initial27_adj_force(R ux, R uy, R uz, const R (&lam)[27], R& gFx, R& gFy, R& gFz) {
  R gm[27], zero[27];
#pragma unroll
  for (int a = 0; a < 27; ++a) {
    gm[cube27(a)] = lam[a];
    zero[a] = R(0);
  }
  R gu = R(0);   // the inputs of the passes only enter the velocity adjoint, unused here
  inv_pass_adj<2>(zero, uz, gm, gu);
  inv_pass_adj<1>(zero, uy, gm, gu);
  inv_pass_adj<0>(zero, ux, gm, gu);
  gFx += R(-0.5) * gm[K3(1, 0, 0)];
  gFy += R(-0.5) * gm[K3(0, 1, 0)];
  gFz += R(-0.5) * gm[K3(0, 0, 1)];
}

}  // namespace cmlbm
