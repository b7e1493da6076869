// HIP kernels of the central-moment LBM step for CDNA4 (gfx950).
//
// Data layout in HBM: populations as structure of arrays f[a][z][y][x]
// (x fastest), directions a in the paper's order (Eq. velocityd3qq27 /
// Appendix G).  The stored state is the post-collision, not yet streamed
// fbar~; a step pulls fbar_a(x) = fbar~_a(x - e_a) (Eq. cascadedstreaming1 read
// backwards), with half-way bounce-back fbar_a(x) = fbar~_abar(x) when x - e_a is
// a solid node, collides in registers and writes fbar~(x) at x.  Each wavefront
// covers 64 consecutive x of one row, so every load and store of one direction
// is a contiguous 256 B (FP32) stream; the +-1 shifts in x only straddle one
// extra cache line that the neighbouring wave also touches.
//
// Storage variants: FP64, FP32, and FP32 compute with the deviation
// fbar - w_a stored as FP16 or BF16 (round to nearest even).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "collide_d3q15.hpp"
#include "collide_d3q27.hpp"
#include "kernels.hpp"

namespace cmlbm {

// ---------------------------------------------------------------------------
// Storage policies
// ---------------------------------------------------------------------------
struct StF64 {
  using T = double;
  using R = double;
  static constexpr bool dev = false;
};
struct StF32 {
  using T = float;
  using R = float;
  static constexpr bool dev = false;
};
struct StF16 {
  using T = _Float16;
  using R = float;
  static constexpr bool dev = true;
};
struct StBF16 {
  using T = __bf16;
  using R = float;
  static constexpr bool dev = true;
};

template <class ST, int Q>
__device__ __forceinline__ typename ST::R decode(typename ST::T v, int a) {
  using R = typename ST::R;
  if constexpr (ST::dev)
    return R(weight<Q>(a)) + static_cast<R>(v);
  else
    return v;
}

template <class ST, int Q>
__device__ __forceinline__ typename ST::T encode(typename ST::R v, int a) {
  using R = typename ST::R;
  if constexpr (ST::dev)
    return static_cast<typename ST::T>(v - R(weight<Q>(a)));
  else
    return v;
}

// ---------------------------------------------------------------------------
// Geometry helpers
// ---------------------------------------------------------------------------
struct Coord {
  int x, y, z;
};

// Node index of (x - s*ex, y - s*ey, z - s*ez) with periodic wrap, s = +-1.
struct Neigh {
  int xs[3];       // x - s*e for e = -1, 0, +1
  uint32_t row[3][3];   // ((z - s*ez) * ny + (y - s*ey)) * nx for ey, ez = -1, 0, +1
  __device__ __forceinline__ Neigh(const Geom& g, Coord c, int s) {
    const int xm = c.x == 0 ? g.nx - 1 : c.x - 1, xp = c.x == g.nx - 1 ? 0 : c.x + 1;
    const int ym = c.y == 0 ? g.ny - 1 : c.y - 1, yp = c.y == g.ny - 1 ? 0 : c.y + 1;
    const int zm = c.z == 0 ? g.nz - 1 : c.z - 1, zp = c.z == g.nz - 1 ? 0 : c.z + 1;
    const int X[3] = {s > 0 ? xp : xm, c.x, s > 0 ? xm : xp};
    const int Y[3] = {s > 0 ? yp : ym, c.y, s > 0 ? ym : yp};
    const int Z[3] = {s > 0 ? zp : zm, c.z, s > 0 ? zm : zp};
#pragma unroll
    for (int i = 0; i < 3; ++i) xs[i] = X[i];
#pragma unroll
    for (int j = 0; j < 3; ++j)
#pragma unroll
      for (int k = 0; k < 3; ++k) row[j][k] = (uint32_t(Z[k]) * uint32_t(g.ny) + uint32_t(Y[j])) * uint32_t(g.nx);
  }
  __device__ __forceinline__ uint32_t at(Vel e) const { return row[e.y + 1][e.z + 1] + uint32_t(xs[e.x + 1]); }
};

__device__ __forceinline__ Coord coord_of(const Geom& g, uint32_t n) {
  const uint32_t z = n / g.nxy;
  const uint32_t r = n - z * g.nxy;
  const uint32_t y = r / uint32_t(g.nx);
  return {int(r - y * uint32_t(g.nx)), int(y), int(z)};
}

// Pull the pre-collision populations of node `node` from the post-collision
// array `fin` (s = +1: from x - e_a).  With MASK, a link whose source is solid
// is replaced by the node's own reversed population (half-way bounce-back).
template <int Q, class ST, bool MASK>
__device__ __forceinline__ void pull(const typename ST::T* __restrict__ fin, uint64_t N, const uint8_t* mask,
                                     const Neigh& nb, uint32_t node, typename ST::R (&f)[Q]) {
#pragma unroll
  for (int a = 0; a < Q; ++a) {
    const Vel e = Lattice<Q>::e(a);
    const uint32_t src = nb.at(e);
    typename ST::T v;
    if constexpr (MASK) {
      if (mask[src])
        v = fin[uint64_t(opposite<Q>(a)) * N + node];
      else
        v = fin[uint64_t(a) * N + src];
    } else {
      v = fin[uint64_t(a) * N + src];
    }
    f[a] = decode<ST, Q>(v, a);
  }
}

template <typename R, typename FT>
__device__ __forceinline__ void force_at(const ForceArgs<FT>& F, uint64_t N, uint32_t node, R& Fx, R& Fy, R& Fz) {
  if (F.field) {
    Fx = R(F.scale) * R(F.field[node]);
    Fy = R(F.scale) * R(F.field[N + node]);
    Fz = R(F.scale) * R(F.field[2 * N + node]);
  } else {
    Fx = R(F.uni[0]);
    Fy = R(F.uni[1]);
    Fz = R(F.uni[2]);
  }
}

template <int Q, typename R>
__device__ __forceinline__ void collide(R (&f)[Q], R Fx, R Fy, R Fz, const Rates<R>& p) {
  if constexpr (Q == 27) {
    R m[27];
#pragma unroll
    for (int a = 0; a < 27; ++a) m[cube27(a)] = f[a];
    collide27(m, Fx, Fy, Fz, p);
#pragma unroll
    for (int a = 0; a < 27; ++a) f[a] = m[cube27(a)];
  } else {
    collide15(f, Fx, Fy, Fz, p);
  }
}

// ---------------------------------------------------------------------------
// The fused pull-stream + collide + force step
// ---------------------------------------------------------------------------
template <int Q, class ST, bool MASK>
__global__ __launch_bounds__(256) void k_step(StepArgs<typename ST::R> args) {
  using R = typename ST::R;
  using T = typename ST::T;
  const Geom g = args.g;
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= g.nx) return;
  const Coord c{x, int(blockIdx.y), int(blockIdx.z)};
  const uint32_t node = (uint32_t(c.z) * uint32_t(g.ny) + uint32_t(c.y)) * uint32_t(g.nx) + uint32_t(x);
  if constexpr (MASK) {
    if (args.mask[node]) return;
  }
  const Neigh nb(g, c, +1);
  R f[Q];
  pull<Q, ST, MASK>(static_cast<const T*>(args.fin), g.N, args.mask, nb, node, f);
  R Fx, Fy, Fz;
  force_at(args.force, g.N, node, Fx, Fy, Fz);
  collide<Q>(f, Fx, Fy, Fz, args.rates);
  T* __restrict__ fout = static_cast<T*>(args.fout);
#pragma unroll
  for (int a = 0; a < Q; ++a) fout[uint64_t(a) * g.N + node] = encode<ST, Q>(f[a], a);
}

// Observable pre-collision state fbar(x) (full populations, compute type).
template <int Q, class ST, bool MASK>
__global__ __launch_bounds__(256) void k_gather(AuxArgs<typename ST::R> args) {
  using R = typename ST::R;
  const Geom g = args.g;
  for (uint32_t n = blockIdx.x * blockDim.x + threadIdx.x; n < g.N; n += gridDim.x * blockDim.x) {
    R* out = static_cast<R*>(args.out0);
    if (MASK && args.mask[n]) {
#pragma unroll
      for (int a = 0; a < Q; ++a) out[uint64_t(a) * g.N + n] = R(0);
      continue;
    }
    const Neigh nb(g, coord_of(g, n), +1);
    R f[Q];
    pull<Q, ST, MASK>(static_cast<const typename ST::T*>(args.in0), g.N, args.mask, nb, n, f);
#pragma unroll
    for (int a = 0; a < Q; ++a) out[uint64_t(a) * g.N + n] = f[a];
  }
}

// rho and u (Eqs. densitycalculation, velocitycalculation), zero at solid nodes.
template <int Q, class ST, bool MASK>
__global__ __launch_bounds__(256) void k_macro(AuxArgs<typename ST::R> args) {
  using R = typename ST::R;
  const Geom g = args.g;
  R* rho_out = static_cast<R*>(args.out0);
  R* u_out = static_cast<R*>(args.out1);
  for (uint32_t n = blockIdx.x * blockDim.x + threadIdx.x; n < g.N; n += gridDim.x * blockDim.x) {
    if (MASK && args.mask[n]) {
      rho_out[n] = R(0);
      u_out[n] = u_out[g.N + n] = u_out[2 * g.N + n] = R(0);
      continue;
    }
    const Neigh nb(g, coord_of(g, n), +1);
    R f[Q];
    pull<Q, ST, MASK>(static_cast<const typename ST::T*>(args.in0), g.N, args.mask, nb, n, f);
    R Fx, Fy, Fz;
    force_at(args.force, g.N, n, Fx, Fy, Fz);
    R rho = R(0), jx = R(0), jy = R(0), jz = R(0);
#pragma unroll
    for (int a = 0; a < Q; ++a) {
      const Vel e = Lattice<Q>::e(a);
      rho += f[a];
      jx += R(e.x) * f[a];
      jy += R(e.y) * f[a];
      jz += R(e.z) * f[a];
    }
    rho_out[n] = rho;
    u_out[n] = (jx + R(0.5) * Fx) / rho;
    u_out[g.N + n] = (jy + R(0.5) * Fy) / rho;
    u_out[2 * g.N + n] = (jz + R(0.5) * Fz) / rho;
  }
}

// Block sum of NV doubles held one set per thread; thread 0 gets the result.
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double* sh /* [NV][8] */) {
#pragma unroll
  for (int i = 0; i < NV; ++i) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v[i] += __shfl_xor(v[i], off, 64);
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) {
#pragma unroll
    for (int i = 0; i < NV; ++i) sh[i * 8 + wave] = v[i];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const int nw = (blockDim.x + 63) >> 6;
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      double s = 0;
      for (int w = 0; w < nw; ++w) s += sh[i * 8 + w];
      v[i] = s;
    }
  }
}

// FP64 partial sums of (rho, j_x, j_y, j_z), j = sum fbar e + F/2, per block.
template <int Q, class ST, bool MASK>
__global__ __launch_bounds__(256) void k_totals(AuxArgs<typename ST::R> args, double* partials) {
  using R = typename ST::R;
  const Geom g = args.g;
  double acc[4] = {0, 0, 0, 0};
  for (uint32_t n = blockIdx.x * blockDim.x + threadIdx.x; n < g.N; n += gridDim.x * blockDim.x) {
    if (MASK && args.mask[n]) continue;
    const Neigh nb(g, coord_of(g, n), +1);
    R f[Q];
    pull<Q, ST, MASK>(static_cast<const typename ST::T*>(args.in0), g.N, args.mask, nb, n, f);
    R Fx, Fy, Fz;
    force_at(args.force, g.N, n, Fx, Fy, Fz);
#pragma unroll
    for (int a = 0; a < Q; ++a) {
      const Vel e = Lattice<Q>::e(a);
      const double v = double(f[a]);
      acc[0] += v;
      acc[1] += e.x * v;
      acc[2] += e.y * v;
      acc[3] += e.z * v;
    }
    acc[1] += 0.5 * double(Fx);
    acc[2] += 0.5 * double(Fy);
    acc[3] += 0.5 * double(Fz);
  }
  __shared__ double sh[4 * 8];
  block_sum<4>(acc, sh);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < 4; ++i) partials[uint64_t(blockIdx.x) * 4 + i] = acc[i];
  }
}

// Sum nblk rows of `width` partials into out[0..width) (out += sum when accumulate).
__global__ __launch_bounds__(256) void k_reduce_rows(const double* partials, int nblk, int width, double* out,
                                                     int accumulate) {
  const int col = blockIdx.x;
  double s = 0;
  for (int b = threadIdx.x; b < nblk; b += blockDim.x) s += partials[uint64_t(b) * width + col];
  double v[1] = {s};
  __shared__ double sh[8];
  block_sum<1>(v, sh);
  if (threadIdx.x == 0) out[col] = accumulate ? out[col] + v[0] : v[0];
}

// ---------------------------------------------------------------------------
// Initial condition: fbar(x, 0) = f^eq(rho0, u0) - S/2, then the inverse pull
// into the post-collision array so that the first step's pull reproduces it.
// ---------------------------------------------------------------------------
template <int Q, typename R, typename FT>
__global__ __launch_bounds__(256) void k_initial_pre(Geom g, const R* rho0, const R* u0, ForceArgs<FT> force,
                                                     const uint8_t* mask, R* fpre) {
  for (uint32_t n = blockIdx.x * blockDim.x + threadIdx.x; n < g.N; n += gridDim.x * blockDim.x) {
    R f[Q];
    if (mask && mask[n]) {
#pragma unroll
      for (int a = 0; a < Q; ++a) f[a] = R(0);
    } else {
      const R rho = rho0[n], ux = u0[n], uy = u0[g.N + n], uz = u0[2 * g.N + n];
      R Fx, Fy, Fz;
      force_at(force, g.N, n, Fx, Fy, Fz);
      if constexpr (Q == 27) {
        // central moments of f^eq - S/2 about u: Maxwellian values rho c_s^(2k)
        // on even monomials and -F/2 on the first-order ones; then the inverse passes.
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
      } else {
        initial15(rho, ux, uy, uz, Fx, Fy, Fz, f);
      }
    }
#pragma unroll
    for (int a = 0; a < Q; ++a) fpre[uint64_t(a) * g.N + n] = f[a];
  }
}

// fbar~(y)_a = fbar(y + e_a)_a if y + e_a is fluid, else fbar(y)_abar.
template <int Q, class ST, bool MASK>
__global__ __launch_bounds__(256) void k_scatter_post(Geom g, const typename ST::R* fpre, const uint8_t* mask,
                                                      typename ST::T* fpost) {
  using R = typename ST::R;
  for (uint32_t n = blockIdx.x * blockDim.x + threadIdx.x; n < g.N; n += gridDim.x * blockDim.x) {
    if (MASK && mask[n]) {
#pragma unroll
      for (int a = 0; a < Q; ++a) fpost[uint64_t(a) * g.N + n] = typename ST::T(0);
      continue;
    }
    const Neigh nb(g, coord_of(g, n), -1);    // x + e_a
#pragma unroll
    for (int a = 0; a < Q; ++a) {
      const uint32_t dst = nb.at(Lattice<Q>::e(a));
      R v;
      if (MASK && mask[dst])
        v = fpre[uint64_t(opposite<Q>(a)) * g.N + n];
      else
        v = fpre[uint64_t(a) * g.N + dst];
      fpost[uint64_t(a) * g.N + n] = encode<ST, Q>(v, a);
    }
  }
}

// ---------------------------------------------------------------------------
// Adjoint step (D3Q27).  Forward step n maps the pre-collision state
// fbar^n(x) (pulled from f_post_prev) to fbar~(x) = C(fbar^n(x)), and
// fbar^{n+1}(x)_a = fbar~(x - e_a)_a (or bounce-back).  Given
// lam_next = dL/dfbar^{n+1}, the adjoint of the stored fbar~(x)_a is
// mu_a = lam_next(x + e_a)_a, or lam_next(x)_abar when x + e_a is solid, and
// lam(x) = J_C(fbar^n(x))^T mu.  dL/dF(x) and dL/domega accumulate in FP64.
// ---------------------------------------------------------------------------
template <class ST, bool MASK>
__global__ __launch_bounds__(256) void k_adjoint27(AdjArgs<typename ST::R> args, double* partials) {
  using R = typename ST::R;
  using T = typename ST::T;
  const Geom g = args.g;
  // Per-thread running sums over the (few) nodes this thread visits:
  // wacc[b] = dL/domega_b for b = 4..26, uF = dL/dF for a uniform force.
  R wacc[27];
#pragma unroll
  for (int b = 0; b < 27; ++b) wacc[b] = R(0);
  R uF[3] = {R(0), R(0), R(0)};
  const uint32_t nseg = (uint32_t(g.nx) + blockDim.x - 1) / blockDim.x;
  const uint32_t items = nseg * uint32_t(g.ny) * uint32_t(g.nz);
  for (uint32_t it = blockIdx.x; it < items; it += gridDim.x) {
    const uint32_t row = it / nseg;
    const int x = int((it - row * nseg) * blockDim.x + threadIdx.x);
    if (x >= g.nx) continue;
    const Coord c{x, int(row % uint32_t(g.ny)), int(row / uint32_t(g.ny))};
    const uint32_t node = row * uint32_t(g.nx) + uint32_t(x);
    if (MASK && args.mask[node]) continue;
    // forward pre-collision populations
    R f[27];
    {
      const Neigh nb(g, c, +1);
      R fa[27];
      pull<27, ST, MASK>(static_cast<const T*>(args.fpost), g.N, args.mask, nb, node, fa);
#pragma unroll
      for (int a = 0; a < 27; ++a) f[cube27(a)] = fa[a];
    }
    // adjoint of this node's post-collision populations (reverse streaming)
    R gm[27];
    {
      const Neigh nb(g, c, -1);
      const R* lam = args.lam_next;
#pragma unroll
      for (int a = 0; a < 27; ++a) {
        const uint32_t dst = nb.at(kE27[a]);
        R v;
        if (MASK && args.mask[dst])
          v = lam[uint64_t(opposite<27>(a)) * g.N + node];
        else
          v = lam[uint64_t(a) * g.N + dst];
        gm[cube27(a)] = v;
      }
    }
    R Fx, Fy, Fz;
    force_at(args.force, g.N, node, Fx, Fy, Fz);
    R s[27];
    R gFx = R(0), gFy = R(0), gFz = R(0);
    collide27_adj(f, Fx, Fy, Fz, args.rates, gm, s, gFx, gFy, gFz, wacc);
    R* lam_out = args.lam;
#pragma unroll
    for (int a = 0; a < 27; ++a) lam_out[uint64_t(a) * g.N + node] = gm[cube27(a)];
    if (args.force.field) {
      const double sc = double(args.force.scale);
      args.dLdF[node] += sc * double(gFx);
      args.dLdF[g.N + node] += sc * double(gFy);
      args.dLdF[2 * g.N + node] += sc * double(gFz);
    } else {
      uF[0] += gFx;
      uF[1] += gFy;
      uF[2] += gFz;
    }
  }
  double v[26];
#pragma unroll
  for (int b = 4; b < 27; ++b) v[b - 4] = double(wacc[b]);
  v[23] = double(uF[0]) * double(args.force.scale);
  v[24] = double(uF[1]) * double(args.force.scale);
  v[25] = double(uF[2]) * double(args.force.scale);
  __shared__ double sh[26 * 8];
  block_sum<26>(v, sh);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < 26; ++i) partials[uint64_t(blockIdx.x) * 26 + i] = v[i];
  }
}

// ---------------------------------------------------------------------------
// Host-side launchers
// ---------------------------------------------------------------------------
namespace {

template <class ST>
struct StorageFor;

constexpr int kBlock = 256;

inline dim3 step_grid(const Geom& g, int bx) {
  return dim3((g.nx + bx - 1) / bx, g.ny, g.nz);
}

inline int step_block(const Geom& g) {
  int bx = kBlock;
  if (g.nx < kBlock) bx = ((g.nx + 63) / 64) * 64;
  return bx;
}

inline unsigned aux_grid(const Geom& g) {
  const uint64_t need = (g.N + kBlock - 1) / kBlock;
  return unsigned(need < 8192 ? (need == 0 ? 1 : need) : 8192);
}

template <int Q, class ST>
hipError_t step_impl(const StepArgs<typename ST::R>& a, hipStream_t st) {
  const int bx = step_block(a.g);
  if (a.mask)
    hipLaunchKernelGGL((k_step<Q, ST, true>), step_grid(a.g, bx), dim3(bx), 0, st, a);
  else
    hipLaunchKernelGGL((k_step<Q, ST, false>), step_grid(a.g, bx), dim3(bx), 0, st, a);
  return hipGetLastError();
}

template <int Q, class ST>
hipError_t gather_impl(const AuxArgs<typename ST::R>& a, hipStream_t st) {
  if (a.mask)
    hipLaunchKernelGGL((k_gather<Q, ST, true>), dim3(aux_grid(a.g)), dim3(kBlock), 0, st, a);
  else
    hipLaunchKernelGGL((k_gather<Q, ST, false>), dim3(aux_grid(a.g)), dim3(kBlock), 0, st, a);
  return hipGetLastError();
}

template <int Q, class ST>
hipError_t macro_impl(const AuxArgs<typename ST::R>& a, hipStream_t st) {
  if (a.mask)
    hipLaunchKernelGGL((k_macro<Q, ST, true>), dim3(aux_grid(a.g)), dim3(kBlock), 0, st, a);
  else
    hipLaunchKernelGGL((k_macro<Q, ST, false>), dim3(aux_grid(a.g)), dim3(kBlock), 0, st, a);
  return hipGetLastError();
}

template <int Q, class ST>
hipError_t totals_impl(const AuxArgs<typename ST::R>& a, double* partials, int nblk, double* out4,
                       hipStream_t st) {
  if (a.mask)
    hipLaunchKernelGGL((k_totals<Q, ST, true>), dim3(nblk), dim3(kBlock), 0, st, a, partials);
  else
    hipLaunchKernelGGL((k_totals<Q, ST, false>), dim3(nblk), dim3(kBlock), 0, st, a, partials);
  hipLaunchKernelGGL(k_reduce_rows, dim3(4), dim3(kBlock), 0, st, partials, nblk, 4, out4, 0);
  return hipGetLastError();
}

template <int Q, class ST>
hipError_t init_impl(const Geom& g, const void* rho0, const void* u0, const ForceArgs<typename ST::R>& force,
                     const uint8_t* mask, void* fpre, void* fpost, hipStream_t st) {
  using R = typename ST::R;
  hipLaunchKernelGGL((k_initial_pre<Q, R, R>), dim3(aux_grid(g)), dim3(kBlock), 0, st, g,
                     static_cast<const R*>(rho0), static_cast<const R*>(u0), force, mask, static_cast<R*>(fpre));
  if (mask)
    hipLaunchKernelGGL((k_scatter_post<Q, ST, true>), dim3(aux_grid(g)), dim3(kBlock), 0, st, g,
                       static_cast<const R*>(fpre), mask, static_cast<typename ST::T*>(fpost));
  else
    hipLaunchKernelGGL((k_scatter_post<Q, ST, false>), dim3(aux_grid(g)), dim3(kBlock), 0, st, g,
                       static_cast<const R*>(fpre), mask, static_cast<typename ST::T*>(fpost));
  return hipGetLastError();
}

template <class ST>
hipError_t adjoint_impl(const AdjArgs<typename ST::R>& a, double* partials, int nblk, double* dLdomega,
                        double* dLdF_uniform, hipStream_t st) {
  if (a.mask)
    hipLaunchKernelGGL((k_adjoint27<ST, true>), dim3(nblk), dim3(step_block(a.g)), 0, st, a, partials);
  else
    hipLaunchKernelGGL((k_adjoint27<ST, false>), dim3(nblk), dim3(step_block(a.g)), 0, st, a, partials);
  hipLaunchKernelGGL(k_reduce_rows, dim3(23), dim3(kBlock), 0, st, partials, nblk, 26, dLdomega, 1);
  if (dLdF_uniform)
    hipLaunchKernelGGL(k_reduce_rows, dim3(3), dim3(kBlock), 0, st, partials + 23, nblk, 26, dLdF_uniform, 1);
  return hipGetLastError();
}

}  // namespace

// Dispatch on (Q, precision).
#define CMLBM_DISPATCH(Q, PREC, CALL_F64, CALL_F32, CALL_F16, CALL_BF16) \
  switch (PREC) {                                                        \
    case 0: return CALL_F64;                                             \
    case 1: return CALL_F32;                                             \
    case 2: return CALL_F16;                                             \
    default: return CALL_BF16;                                           \
  }

hipError_t launch_step(int q, int prec, const StepArgs<double>& a64, const StepArgs<float>& a32, hipStream_t st) {
  if (q == 27) {
    CMLBM_DISPATCH(q, prec, (step_impl<27, StF64>(a64, st)), (step_impl<27, StF32>(a32, st)),
                   (step_impl<27, StF16>(a32, st)), (step_impl<27, StBF16>(a32, st)))
  }
  CMLBM_DISPATCH(q, prec, (step_impl<15, StF64>(a64, st)), (step_impl<15, StF32>(a32, st)),
                 (step_impl<15, StF16>(a32, st)), (step_impl<15, StBF16>(a32, st)))
}

hipError_t launch_gather(int q, int prec, const AuxArgs<double>& a64, const AuxArgs<float>& a32, hipStream_t st) {
  if (q == 27) {
    CMLBM_DISPATCH(q, prec, (gather_impl<27, StF64>(a64, st)), (gather_impl<27, StF32>(a32, st)),
                   (gather_impl<27, StF16>(a32, st)), (gather_impl<27, StBF16>(a32, st)))
  }
  CMLBM_DISPATCH(q, prec, (gather_impl<15, StF64>(a64, st)), (gather_impl<15, StF32>(a32, st)),
                 (gather_impl<15, StF16>(a32, st)), (gather_impl<15, StBF16>(a32, st)))
}

hipError_t launch_macro(int q, int prec, const AuxArgs<double>& a64, const AuxArgs<float>& a32, hipStream_t st) {
  if (q == 27) {
    CMLBM_DISPATCH(q, prec, (macro_impl<27, StF64>(a64, st)), (macro_impl<27, StF32>(a32, st)),
                   (macro_impl<27, StF16>(a32, st)), (macro_impl<27, StBF16>(a32, st)))
  }
  CMLBM_DISPATCH(q, prec, (macro_impl<15, StF64>(a64, st)), (macro_impl<15, StF32>(a32, st)),
                 (macro_impl<15, StF16>(a32, st)), (macro_impl<15, StBF16>(a32, st)))
}

hipError_t launch_totals(int q, int prec, const AuxArgs<double>& a64, const AuxArgs<float>& a32, double* partials,
                         int nblk, double* out4, hipStream_t st) {
  if (q == 27) {
    CMLBM_DISPATCH(q, prec, (totals_impl<27, StF64>(a64, partials, nblk, out4, st)),
                   (totals_impl<27, StF32>(a32, partials, nblk, out4, st)),
                   (totals_impl<27, StF16>(a32, partials, nblk, out4, st)),
                   (totals_impl<27, StBF16>(a32, partials, nblk, out4, st)))
  }
  CMLBM_DISPATCH(q, prec, (totals_impl<15, StF64>(a64, partials, nblk, out4, st)),
                 (totals_impl<15, StF32>(a32, partials, nblk, out4, st)),
                 (totals_impl<15, StF16>(a32, partials, nblk, out4, st)),
                 (totals_impl<15, StBF16>(a32, partials, nblk, out4, st)))
}

hipError_t launch_init(int q, int prec, const Geom& g, const void* rho0, const void* u0, const ForceArgs<double>& f64,
                       const ForceArgs<float>& f32, const uint8_t* mask, void* fpre, void* fpost, hipStream_t st) {
  if (q == 27) {
    CMLBM_DISPATCH(q, prec, (init_impl<27, StF64>(g, rho0, u0, f64, mask, fpre, fpost, st)),
                   (init_impl<27, StF32>(g, rho0, u0, f32, mask, fpre, fpost, st)),
                   (init_impl<27, StF16>(g, rho0, u0, f32, mask, fpre, fpost, st)),
                   (init_impl<27, StBF16>(g, rho0, u0, f32, mask, fpre, fpost, st)))
  }
  CMLBM_DISPATCH(q, prec, (init_impl<15, StF64>(g, rho0, u0, f64, mask, fpre, fpost, st)),
                 (init_impl<15, StF32>(g, rho0, u0, f32, mask, fpre, fpost, st)),
                 (init_impl<15, StF16>(g, rho0, u0, f32, mask, fpre, fpost, st)),
                 (init_impl<15, StBF16>(g, rho0, u0, f32, mask, fpre, fpost, st)))
}

hipError_t launch_adjoint(int prec, const AdjArgs<double>& a64, const AdjArgs<float>& a32, double* partials,
                          int nblk, double* dLdomega, double* dLdF_uniform, hipStream_t st) {
  CMLBM_DISPATCH(27, prec, (adjoint_impl<StF64>(a64, partials, nblk, dLdomega, dLdF_uniform, st)),
                 (adjoint_impl<StF32>(a32, partials, nblk, dLdomega, dLdF_uniform, st)),
                 (adjoint_impl<StF16>(a32, partials, nblk, dLdomega, dLdF_uniform, st)),
                 (adjoint_impl<StBF16>(a32, partials, nblk, dLdomega, dLdF_uniform, st)))
}

#undef CMLBM_DISPATCH

}  // namespace cmlbm
