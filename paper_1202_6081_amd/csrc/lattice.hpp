// Lattice velocity sets of the 3D central-moment LBM, for device code.
//
// D3Q27: Eq. (velocityd3qq27) of Premnath & Banerjee (arXiv:1202.6081), in the
// direction order fixed by the rows of the matrix K of Appendix A.
// D3Q15: Appendix G (rest, six axis links, eight corners in the same order as
// D3Q27's 19..26).
#pragma once

#include <cstdint>

// The per-node math in these headers is also compiled for the CPU
// (tests/host/host_collide.cpp), where the CPU tests compare it with the oracle.
#ifndef CMLBM_HD
#define CMLBM_HD __host__ __device__ __forceinline__
#define CMLBM_HDC __host__ __device__ constexpr
#endif

namespace cmlbm {

struct Vel {
  int x, y, z;
};

constexpr Vel kE27[27] = {
    {0, 0, 0},
    {1, 0, 0},   {-1, 0, 0},  {0, 1, 0},   {0, -1, 0},  {0, 0, 1},   {0, 0, -1},
    {1, 1, 0},   {-1, 1, 0},  {1, -1, 0},  {-1, -1, 0},
    {1, 0, 1},   {-1, 0, 1},  {1, 0, -1},  {-1, 0, -1},
    {0, 1, 1},   {0, -1, 1},  {0, 1, -1},  {0, -1, -1},
    {1, 1, 1},   {-1, 1, 1},  {1, -1, 1},  {-1, -1, 1},
    {1, 1, -1},  {-1, 1, -1}, {1, -1, -1}, {-1, -1, -1},
};

constexpr Vel kE15[15] = {
    {0, 0, 0},
    {1, 0, 0},  {-1, 0, 0}, {0, 1, 0},  {0, -1, 0}, {0, 0, 1},   {0, 0, -1},
    {1, 1, 1},  {-1, 1, 1}, {1, -1, 1}, {-1, -1, 1},
    {1, 1, -1}, {-1, 1, -1}, {1, -1, -1}, {-1, -1, -1},
};

template <int Q>
struct Lattice;

template <>
struct Lattice<27> {
  static constexpr int Q = 27;
  __host__ __device__ static constexpr Vel e(int a) { return kE27[a]; }
};

template <>
struct Lattice<15> {
  static constexpr int Q = 15;
  __host__ __device__ static constexpr Vel e(int a) { return kE15[a]; }
};

// Index of -e_a.
template <int Q>
CMLBM_HDC int opposite(int a) {
  for (int b = 0; b < Q; ++b) {
    if (Lattice<Q>::e(b).x == -Lattice<Q>::e(a).x && Lattice<Q>::e(b).y == -Lattice<Q>::e(a).y &&
        Lattice<Q>::e(b).z == -Lattice<Q>::e(a).z)
      return b;
  }
  return -1;
}

// Rest-state populations (unit density): 8/27, 2/27, 1/54, 1/216 for D3Q27 and
// 2/9, 1/9, 1/72 for D3Q15, by the number of nonzero velocity components.
template <int Q>
CMLBM_HDC double weight(int a) {
  const Vel v = Lattice<Q>::e(a);
  const int n = (v.x != 0) + (v.y != 0) + (v.z != 0);
  if (Q == 27) return n == 0 ? 8.0 / 27 : n == 1 ? 2.0 / 27 : n == 2 ? 1.0 / 54 : 1.0 / 216;
  return n == 0 ? 2.0 / 9 : n == 1 ? 1.0 / 9 : 1.0 / 72;
}

// Division of a 32-bit index n < 2^31 by a fixed d >= 1 without a divide:
// with l = ceil(log2 d) and m = floor(2^(31+l) / d) + 1 (which fits 32 bits),
// n / d = floor(n m / 2^(31+l)) for every n < 2^31 (Granlund and Montgomery,
// 1994, Thm. 4.2), i.e. the high word of n m shifted right by l - 1.  d = 1 is
// kept as m = 0.  For a wave-uniform n this is two scalar instructions.
struct Divider {
  uint32_t m, s;
  static Divider of(uint32_t d) {
    if (d <= 1) return {0u, 0u};
    uint32_t l = 0;
    while ((uint64_t(1) << l) < d) ++l;
    return {uint32_t((uint64_t(1) << (31 + l)) / d + 1), l - 1};
  }
  CMLBM_HD uint32_t div(uint32_t n) const {
    return m ? uint32_t((uint64_t(n) * m) >> 32) >> s : n;
  }
};

// a * b + c with one rounding.
CMLBM_HD float fma_r(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
CMLBM_HD double fma_r(double a, double b, double c) { return __builtin_fma(a, b, c); }

// 1/x.  In FP32 device code: the hardware reciprocal (within one ulp) refined
// by one Newton step, r + r (1 - x r), which leaves it within an ulp of the
// correctly rounded quotient in 3 instructions instead of the ~10 of an IEEE
// division.  Elsewhere (FP64, and the CPU build of these headers) the division.
template <typename R>
CMLBM_HD R recip(R x) {
#if defined(__HIP_DEVICE_COMPILE__)
  if constexpr (sizeof(R) == 4) {
    const float r = __builtin_amdgcn_rcpf(x);
    return __builtin_fmaf(r, __builtin_fmaf(-x, r, 1.0f), r);
  }
#endif
  return R(1) / x;
}

// D3Q27 directions as a 3x3x3 cube: index (e_x+1)*9 + (e_y+1)*3 + (e_z+1).
CMLBM_HDC int cube27(int a) {
  return (kE27[a].x + 1) * 9 + (kE27[a].y + 1) * 3 + (kE27[a].z + 1);
}

}  // namespace cmlbm
