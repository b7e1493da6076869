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
//     lattice they are signed sums over the rest, axis and corner links.
//  4. Binomial shift to central moments, relaxation of xy, xz, yz (g4..g6),
//     xx-yy, xx+yy-2zz, xx+yy+zz (g7..g9), xyy, xxy, xxz, xyz (g10..g13) toward
//     zero (rho for g9) and xxyy (g14) toward kxx~ kyy~; rho and the first central
//     moments (F/2) are conserved.
//  5. Inverse shift to raw moments and exact inversion of the fifteen raw
//     moments to populations (the K g + S rows of Appendix G).
#pragma once

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
#pragma unroll
  for (int b = 0; b < 15; ++b) ms[b] *= R(1.0 / k15_norm(b));
#pragma unroll
  for (int a = 0; a < 15; ++a) {
    R acc = R(0);
#pragma unroll
    for (int b = 1; b < 15; ++b) {
      const int k = k15_basis(b, kE15[a]);
      if (k != 0) acc += R(k) * ms[b];
    }
    S[a] = acc;
  }
}

// Populations with the given central moments about u: rho; first order
// (hx, hy, hz); second order t..; third order txyy, txxy, txxz, txyz; fourth
// order txxyy.  Binomial shift back to raw moments, then the exact inversion of
// the fifteen raw moments on D3Q15.
template <typename R>
CMLBM_HD void populations15(R rho, R ux, R uy, R uz, R hx, R hy, R hz, R txy, R txz, R tyz, R txx, R tyy, R tzz,
                            R txyy, R txxy, R txxz, R txyz, R txxyy, R (&f)[15]) {
  const R ux2 = ux * ux, uy2 = uy * uy, uz2 = uz * uz;
  const R sx = hx + ux * rho, sy = hy + uy * rho, sz = hz + uz * rho;
  const R sxy = txy + ux * hy + uy * hx + ux * uy * rho;
  const R sxz = txz + ux * hz + uz * hx + ux * uz * rho;
  const R syz = tyz + uy * hz + uz * hy + uy * uz * rho;
  const R sxx = txx + R(2) * ux * hx + ux2 * rho;
  const R syy = tyy + R(2) * uy * hy + uy2 * rho;
  const R szz = tzz + R(2) * uz * hz + uz2 * rho;
  const R sxyy = txyy + R(2) * uy * txy + ux * tyy + uy2 * hx + R(2) * ux * uy * hy + ux * uy2 * rho;
  const R sxxy = txxy + R(2) * ux * txy + uy * txx + ux2 * hy + R(2) * ux * uy * hx + ux2 * uy * rho;
  const R sxxz = txxz + R(2) * ux * txz + uz * txx + ux2 * hz + R(2) * ux * uz * hx + ux2 * uz * rho;
  const R sxyz = txyz + ux * tyz + uy * txz + uz * txy + ux * uy * hz + ux * uz * hy + uy * uz * hx +
                 ux * uy * uz * rho;
  const R sxxyy = txxyy + R(2) * ux * txyy + R(2) * uy * txxy + ux2 * tyy + uy2 * txx + R(4) * ux * uy * txy +
                  R(2) * ux * uy2 * hx + R(2) * ux2 * uy * hy + ux2 * uy2 * rho;
  // corners: the eight corner moments determine the eight corner populations
#pragma unroll
  for (int a = 7; a < 15; ++a) {
    const R x = R(kE15[a].x), y = R(kE15[a].y), z = R(kE15[a].z);
    f[a] = R(0.125) * (sxxyy + x * sxyy + y * sxxy + z * sxxz + x * y * sxy + x * z * sxz + y * z * syz +
                       x * y * z * sxyz);
  }
  f[1] = R(0.5) * ((sxx - sxxyy) + (sx - sxyy));
  f[2] = R(0.5) * ((sxx - sxxyy) - (sx - sxyy));
  f[3] = R(0.5) * ((syy - sxxyy) + (sy - sxxy));
  f[4] = R(0.5) * ((syy - sxxyy) - (sy - sxxy));
  f[5] = R(0.5) * ((szz - sxxyy) + (sz - sxxz));
  f[6] = R(0.5) * ((szz - sxxyy) - (sz - sxxz));
  f[0] = rho - (sxx + syy + szz) + R(2) * sxxyy;
}

// Density and velocity (Eqs. densitycalculation, velocitycalculation).
template <typename R>
CMLBM_HD void moments0_15(const R (&f)[15], R Fx, R Fy, R Fz, R& rho, R& ux, R& uy, R& uz) {
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
  const R inv = R(1) / rho;
  ux = (f[1] - f[2] + cx + R(0.5) * Fx) * inv;
  uy = (f[3] - f[4] + cy + R(0.5) * Fy) * inv;
  uz = (f[5] - f[6] + cz + R(0.5) * Fz) * inv;
}

template <typename R>
CMLBM_HD void collide15(R (&f)[15], R Fx, R Fy, R Fz, const Rates<R>& p) {
  R rho, ux, uy, uz;
  moments0_15(f, Fx, Fy, Fz, rho, ux, uy, uz);
  R h[15];
  source15(Fx, Fy, Fz, ux, uy, uz, h);
#pragma unroll
  for (int a = 0; a < 15; ++a) h[a] += f[a];

  // raw moments of h (corner links 7..14 carry all mixed monomials)
  R c0 = R(0), rxy = R(0), rxz = R(0), ryz = R(0), rxyz = R(0), rcx = R(0), rcy = R(0), rcz = R(0);
#pragma unroll
  for (int a = 7; a < 15; ++a) {
    const int x = kE15[a].x, y = kE15[a].y, z = kE15[a].z;
    c0 += h[a];
    rcx += R(x) * h[a];
    rcy += R(y) * h[a];
    rcz += R(z) * h[a];
    rxy += R(x * y) * h[a];
    rxz += R(x * z) * h[a];
    ryz += R(y * z) * h[a];
    rxyz += R(x * y * z) * h[a];
  }
  const R rx = h[1] - h[2] + rcx, ry = h[3] - h[4] + rcy, rz = h[5] - h[6] + rcz;
  const R rxx = h[1] + h[2] + c0, ryy = h[3] + h[4] + c0, rzz = h[5] + h[6] + c0;
  const R rxyy = rcx, rxxy = rcy, rxxz = rcz, rxxyy = c0;   // e_x e_y^2 = e_x on corners, ...

  // central moments of h about u (binomial theorem)
  const R ux2 = ux * ux, uy2 = uy * uy, uz2 = uz * uz;
  const R cxy = rxy - ux * ry - uy * rx + ux * uy * rho;
  const R cxz = rxz - ux * rz - uz * rx + ux * uz * rho;
  const R cyz = ryz - uy * rz - uz * ry + uy * uz * rho;
  const R cxx = rxx - R(2) * ux * rx + ux2 * rho;
  const R cyy = ryy - R(2) * uy * ry + uy2 * rho;
  const R czz = rzz - R(2) * uz * rz + uz2 * rho;
  const R cxyy = rxyy - R(2) * uy * rxy - ux * ryy + uy2 * rx + R(2) * ux * uy * ry - ux * uy2 * rho;
  const R cxxy = rxxy - R(2) * ux * rxy - uy * rxx + ux2 * ry + R(2) * ux * uy * rx - ux2 * uy * rho;
  const R cxxz = rxxz - R(2) * ux * rxz - uz * rxx + ux2 * rz + R(2) * ux * uz * rx - ux2 * uz * rho;
  const R cxyz = rxyz - ux * ryz - uy * rxz - uz * rxy + ux * uy * rz + ux * uz * ry + uy * uz * rx -
                 ux * uy * uz * rho;
  const R cxxyy = rxxyy - R(2) * ux * rxyy - R(2) * uy * rxxy + ux2 * ryy + uy2 * rxx + R(4) * ux * uy * rxy -
                  R(2) * ux * uy2 * rx - R(2) * ux2 * uy * ry + ux2 * uy2 * rho;

  // relaxation
  const R d1 = p.wc[7] * (cxx - cyy);
  const R d2 = p.wc[8] * (cxx + cyy - R(2) * czz);
  const R t9 = p.wc[9] * (cxx + cyy + czz) + p.w[9] * rho;
  const R txx = (R(2) * t9 + d2 + R(3) * d1) * R(1.0 / 6.0);
  const R tyy = (R(2) * t9 + d2 - R(3) * d1) * R(1.0 / 6.0);
  const R tzz = (t9 - d2) * R(1.0 / 3.0);
  populations15(rho, ux, uy, uz, R(0.5) * Fx, R(0.5) * Fy, R(0.5) * Fz, p.wc[4] * cxy, p.wc[5] * cxz,
                p.wc[6] * cyz, txx, tyy, tzz, p.wc[10] * cxyy, p.wc[11] * cxxy, p.wc[12] * cxxz, p.wc[13] * cxyz,
                p.wc[14] * cxxyy + p.w[14] * (txx * tyy), f);
}

// Initial transformed populations fbar = f^eq(rho, u) - S/2: f^eq has the
// Maxwellian central moments rho, c_s^2 rho (xx, yy, zz), c_s^4 rho (xxyy).
template <typename R>
CMLBM_HD void initial15(R rho, R ux, R uy, R uz, R Fx, R Fy, R Fz, R (&f)[15]) {
  const R c2 = rho * R(1.0 / 3.0);
  populations15(rho, ux, uy, uz, R(0), R(0), R(0), R(0), R(0), R(0), c2, c2, c2, R(0), R(0), R(0), R(0),
                rho * R(1.0 / 9.0), f);
  R S[15];
  source15(Fx, Fy, Fz, ux, uy, uz, S);
#pragma unroll
  for (int a = 0; a < 15; ++a) f[a] -= R(0.5) * S[a];
}

}  // namespace cmlbm
