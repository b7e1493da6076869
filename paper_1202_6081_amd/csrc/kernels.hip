// HIP kernels of the central-moment LBM step for CDNA4 (gfx950).
//
// Population buffers (the post-collision, not yet streamed fbar~ of Eq.
// cascadedcollision1) use a blocked row layout.  Row r = z*ny + y holds Q*nx
// values; inside a row, x is cut into blocks of 64 consecutive nodes (the last
// block may be shorter) and each block stores its Q directions one after the
// other, 64 values each:
//     element(a, r, x) = r*nx*Q + b*64*Q + a*len(b) + (x - 64 b),  b = x/64,
//     len(b) = min(64, nx - 64 b).
// A wavefront covers one block, so the 27 direction streams of one wavefront's
// stores fall in one contiguous 27*256 B (FP32) region and its loads in nine
// such regions (one per source row), which keeps DRAM page locality with 55
// concurrent streams.  Directions are in the paper's order (Eq.
// velocityd3qq27 / Appendix G).  Fields (force, velocity, mask, adjoints) stay
// structure of arrays [c][z][y][x].
//
// A step pulls fbar_a(x) = fbar~_a(x - e_a) (Eq. cascadedstreaming1 read
// backwards), with half-way bounce-back fbar_a(x) = fbar~_abar(x) when x - e_a
// is a solid node, collides in registers and writes fbar~(x).
//
// Storage variants: FP64, FP32, and FP32 compute with the deviation
// fbar - w_a stored as FP16 or BF16 (round to nearest even).
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>
#include <type_traits>

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

// All Q stored values of one node (the hot paths): as encode, with FP16
// deviations converted two at a time by the packed conversion (the same
// round-to-nearest-even of each FP32 value; measured as fast as or faster than
// the mixed-precision multiply-add-and-round the compiler otherwise forms).
template <class ST, int Q>
__device__ __forceinline__ void encode_all(const typename ST::R (&f)[Q], typename ST::T (&v)[Q]) {
  using R = typename ST::R;
  if constexpr (ST::dev && __is_same(typename ST::T, _Float16)) {
    typedef float f32x2 __attribute__((ext_vector_type(2)));
    typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));
#pragma unroll
    for (int a = 0; a + 1 < Q; a += 2) {
      const f16x2 h = __builtin_convertvector((f32x2){f[a] - R(weight<Q>(a)), f[a + 1] - R(weight<Q>(a + 1))}, f16x2);
      v[a] = h.x;
      v[a + 1] = h.y;
    }
    if constexpr (Q & 1) v[Q - 1] = encode<ST, Q>(f[Q - 1], Q - 1);
  } else {
#pragma unroll
    for (int a = 0; a < Q; ++a) v[a] = encode<ST, Q>(f[a], a);
  }
}

// Marks the encoded populations as computed here (an empty statement per
// register: no instruction is emitted), so that the compiler does not sink the
// end of the collision into later branches, where it would fuse its multiplies
// and adds differently.  FP16 deviations are pinned in the pairs that the
// packed conversion writes, so that they stay packed.
template <class ST, int Q>
__device__ __forceinline__ void pin_all(typename ST::T (&v)[Q]) {
  using T = typename ST::T;
  if constexpr (ST::dev && __is_same(T, _Float16)) {
#pragma unroll
    for (int a = 0; a + 1 < Q; a += 2) {
      uint32_t p = uint32_t(__builtin_bit_cast(uint16_t, v[a])) | (uint32_t(__builtin_bit_cast(uint16_t, v[a + 1])) << 16);
      asm volatile("" : "+v"(p));
      v[a] = __builtin_bit_cast(T, uint16_t(p));
      v[a + 1] = __builtin_bit_cast(T, uint16_t(p >> 16));
    }
    if constexpr (Q & 1) asm volatile("" : "+v"(v[Q - 1]));
  } else {
#pragma unroll
    for (int a = 0; a < Q; ++a) asm volatile("" : "+v"(v[a]));
  }
}

// Element idx of an array whose byte size fits in 32 bits: a uniform base
// pointer plus a 32-bit byte offset, which maps onto the scalar-base form of
// the global load instructions.
template <typename T>
__device__ __forceinline__ T ld32(const T* base, uint32_t idx) {
  return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + idx * uint32_t(sizeof(T)));
}

// ---------------------------------------------------------------------------
// Geometry
// ---------------------------------------------------------------------------
struct Coord {
  int x, y, z;
};

// Node x of row `row` (row = z*ny + y).
__device__ __forceinline__ Coord row_coord(const RowMap& rm, const Geom& g, uint32_t row, uint32_t x) {
  const uint32_t z = rm.ny.div(row);
  return {int(x), int(row - z * uint32_t(g.ny)), int(z)};
}

__device__ __forceinline__ Coord coord_of(const Geom& g, uint32_t n) {
  const uint32_t z = n / g.nxy;
  const uint32_t r = n - z * g.nxy;
  const uint32_t y = r / uint32_t(g.nx);
  return {int(r - y * uint32_t(g.nx)), int(y), int(z)};
}

// Offset of (a, x) inside a row of the blocked population layout.
template <int Q>
__device__ __forceinline__ uint32_t in_row(uint32_t nx, int a, uint32_t x) {
  const uint32_t b0 = x & ~63u;
  const uint32_t len = min(64u, nx - b0);
  return b0 * uint32_t(Q) + uint32_t(a) * len + (x - b0);
}

// Source rows and x positions of the pull (s = +1: x - e) or of the reverse
// gather (s = -1: x + e), periodic.
struct Stencil {
  uint32_t row[3][3];   // row index (z - s*ez)*ny + (y - s*ey), indexed [ey+1][ez+1]
  uint32_t xs[3];       // x - s*ex, indexed [ex+1]
  __device__ __forceinline__ Stencil(const Geom& g, Coord c, int s) {
    const int xm = c.x == 0 ? g.nx - 1 : c.x - 1, xp = c.x == g.nx - 1 ? 0 : c.x + 1;
    const int ym = c.y == 0 ? g.ny - 1 : c.y - 1, yp = c.y == g.ny - 1 ? 0 : c.y + 1;
    const int zm = c.z == 0 ? g.nz - 1 : c.z - 1, zp = c.z == g.nz - 1 ? 0 : c.z + 1;
    const int X[3] = {s > 0 ? xp : xm, c.x, s > 0 ? xm : xp};
    const int Y[3] = {s > 0 ? yp : ym, c.y, s > 0 ? ym : yp};
    const int Z[3] = {s > 0 ? zp : zm, c.z, s > 0 ? zm : zp};
#pragma unroll
    for (int i = 0; i < 3; ++i) xs[i] = uint32_t(X[i]);
#pragma unroll
    for (int j = 0; j < 3; ++j)
#pragma unroll
      for (int k = 0; k < 3; ++k) row[j][k] = uint32_t(Z[k]) * uint32_t(g.ny) + uint32_t(Y[j]);
  }
  __device__ __forceinline__ uint32_t node(Vel e, uint32_t nx) const {
    return row[e.y + 1][e.z + 1] * nx + xs[e.x + 1];
  }
};

// Raw buffer access: a resource over one row (base in SGPRs, size bound) plus a
// 32-bit byte offset.  Stores past the bound are dropped by the hardware.
// Word 3 = 0x00020000 is the raw-buffer descriptor of the gfx9 family.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t array_rsrc(const void* base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, int(bytes), 0x00020000);
}

// Load through a buffer resource: base in scalar registers, 32-bit per-lane
// and wave-uniform byte offsets, so that no 64-bit per-lane address is formed
// (with plain pointers the compiler factors the per-lane offset out of a group
// of loads and adds each uniform part back with a 64-bit vector add).
template <typename T>
__device__ __forceinline__ T buf_load(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
  if constexpr (sizeof(T) == 4) {
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
  } else if constexpr (sizeof(T) == 8) {
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
  } else {
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b16(r, voff, soff, 0));
  }
}

// Element of a byte offset from a uniform base (scalar-base load form).
template <typename T>
__device__ __forceinline__ T ldb(const void* base, uint32_t byte_off) {
  return *reinterpret_cast<const T*>(static_cast<const char*>(base) + byte_off);
}

// Pull the pre-collision populations of node (row0, x) from the blocked
// post-collision buffer `fin`.  With MASK, a link whose source is solid takes
// the node's own reversed population (half-way bounce-back).
//
// WAVE: the caller guarantees that a wavefront covers one 64-node block of
// one row (block size a multiple of 64, one row per block).  Then the block
// start and length of the node's own x are wave-uniform, and the byte offset
// of direction a splits into a per-lane part and a scalar part a*len, folded
// into the base pointer; only the x-neighbour directions keep a per-lane
// multiply-add.  BUF: load through buffer resources over the source rows
// (where the caller's register pressure makes the compiler rebuild 64-bit
// per-lane addresses for the plain loads).
template <int Q, class ST, bool MASK, bool WAVE = false, bool BUF = false>
__device__ __forceinline__ void pull(const typename ST::T* __restrict__ fin, const Geom& g, const uint8_t* mask,
                                     const Stencil& st, uint32_t row0, uint32_t x, typename ST::R (&f)[Q]) {
  using T = typename ST::T;
  const uint64_t rowQ = uint64_t(g.nx) * Q;
  if constexpr (WAVE) {
    constexpr uint32_t sz = uint32_t(sizeof(T));
    const uint32_t nx = uint32_t(g.nx);
    const uint32_t b0 = __builtin_amdgcn_readfirstlane(x & ~63u);
    const uint32_t lenB = min(64u, nx - b0) * sz;            // wave-uniform
    const uint32_t cbase = (b0 * uint32_t(Q) + (x - b0)) * sz;
    uint32_t nbase[3], nlen[3];
#pragma unroll
    for (int i = 0; i < 3; i += 2) {
      const uint32_t xs = st.xs[i];
      const uint32_t bb = xs & ~63u;
      nbase[i] = (bb * uint32_t(Q) + (xs - bb)) * sz;
      nlen[i] = min(64u, nx - bb) * sz;
    }
    const T* own = fin + uint64_t(row0) * rowQ;
    // bit a: x - e_a solid.  One round of mask loads ahead of the population
    // loads, which then issue back to back (a mask byte tested per direction
    // made each population load wait for its own mask load).  Direction 0
    // reads the node's own slot 0 either way.
    uint32_t solid = 0;
    if constexpr (MASK) {
#pragma unroll
      for (int a = 1; a < Q; ++a) solid |= uint32_t(mask[st.node(Lattice<Q>::e(a), nx)] != 0) << a;
    }
    // When every block of a row is full (nx a multiple of 64), the blocks of
    // the x-neighbours have the same direction stride lenB, and that part of
    // their offsets is wave-uniform too.
    auto gather = [&](auto full) {
#pragma unroll
      for (int a = 0; a < Q; ++a) {
        const Vel e = Lattice<Q>::e(a);
        const T* rp = fin + uint64_t(st.row[e.y + 1][e.z + 1]) * rowQ;
        T v;
        if constexpr (BUF) {
          static_assert(!MASK, "a per-lane choice of row must not select the descriptor");
          const uint32_t rowB = uint32_t(rowQ) * sz;
          if (e.x == 0)
            v = buf_load<T>(array_rsrc(rp, rowB), cbase, uint32_t(a) * lenB);
          else if constexpr (decltype(full)::value)
            v = buf_load<T>(array_rsrc(rp, rowB), nbase[e.x + 1], uint32_t(a) * lenB);
          else
            v = buf_load<T>(array_rsrc(rp, rowB), nbase[e.x + 1] + uint32_t(a) * nlen[e.x + 1], 0u);
        } else {
          if (MASK && ((solid >> a) & 1u))
            v = ldb<T>(reinterpret_cast<const char*>(own) + uint32_t(opposite<Q>(a)) * lenB, cbase);
          else if (e.x == 0)
            v = ldb<T>(reinterpret_cast<const char*>(rp) + uint32_t(a) * lenB, cbase);
          else if constexpr (decltype(full)::value)
            v = ldb<T>(reinterpret_cast<const char*>(rp) + uint32_t(a) * lenB, nbase[e.x + 1]);
          else
            v = ldb<T>(rp, nbase[e.x + 1] + uint32_t(a) * nlen[e.x + 1]);
        }
        f[a] = decode<ST, Q>(v, a);
      }
    };
    if ((nx & 63u) == 0)
      gather(std::true_type{});
    else
      gather(std::false_type{});
  } else {
    uint32_t solid = 0;   // bit a: x - e_a solid, as above
    if constexpr (MASK) {
#pragma unroll
      for (int a = 1; a < Q; ++a) solid |= uint32_t(mask[st.node(Lattice<Q>::e(a), uint32_t(g.nx))] != 0) << a;
    }
#pragma unroll
    for (int a = 0; a < Q; ++a) {
      const Vel e = Lattice<Q>::e(a);
      const T* rp = fin + uint64_t(st.row[e.y + 1][e.z + 1]) * rowQ;
      T v;
      if constexpr (MASK) {
        if ((solid >> a) & 1u)
          v = ld32(fin + uint64_t(row0) * rowQ, in_row<Q>(uint32_t(g.nx), opposite<Q>(a), x));
        else
          v = ld32(rp, in_row<Q>(uint32_t(g.nx), a, st.xs[e.x + 1]));
      } else {
        v = ld32(rp, in_row<Q>(uint32_t(g.nx), a, st.xs[e.x + 1]));
      }
      f[a] = decode<ST, Q>(v, a);
    }
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
// Launch shape: one block covers CMLBM_STEP_BLOCK consecutive x of one row, so
// every row base is uniform across the block.  Hardware hands consecutive
// block ids to the eight XCDs in turn; with CMLBM_XCD_REMAP the block id is
// permuted so that each XCD receives a contiguous run of rows, keeping a row's
// segments and their shared edge cache lines in one XCD's L2.
#ifndef CMLBM_STEP_BLOCK
#define CMLBM_STEP_BLOCK 256
#endif
#ifndef CMLBM_XCD_REMAP
#define CMLBM_XCD_REMAP 1
#endif
#ifndef CMLBM_NT_STORE
#define CMLBM_NT_STORE 1
#endif
// In-place scatter phase without walls: 0 = shifted stores, 1 = aligned stores
// for 16-bit storage only (measured: 16-bit 2-5% faster aligned, FP32 2% slower
// from the block barrier, FP64 even), 2 = aligned stores always.
#ifndef CMLBM_ALIGNED_SCATTER
#define CMLBM_ALIGNED_SCATTER 1
#endif

__device__ __forceinline__ uint32_t step_block_id() {
  uint32_t L = blockIdx.x;
#if CMLBM_XCD_REMAP
  const uint32_t G = gridDim.x, per = G >> 3;
  if (L < (per << 3)) L = (L & 7u) * per + (L >> 3);
#endif
  return L;
}

constexpr int kStoreAux = CMLBM_NT_STORE ? 2 : 0;   // 2: nontemporal (streaming) store
// A per-lane byte offset past every row's bound: the raw buffer store drops it.
constexpr uint32_t kDropOffset = 0x80000000u;

// voff: per-lane byte offset; soff: wave-uniform byte offset; AUX: cache
// policy bits (kStoreAux streams past the caches; 0 keeps the line).
template <int AUX = kStoreAux, typename T>
__device__ __forceinline__ void buf_store(T v, __amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
  if constexpr (sizeof(T) == 4) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, voff, soff, AUX);
  } else if constexpr (sizeof(T) == 8) {
    typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, voff, soff, AUX);
  } else {
    __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(uint16_t, v), r, voff, soff, AUX);
  }
}

// FP64 mass and momentum of one node's pre-collision populations, rho u
// including F/2 (Eqs. densitycalculation, velocitycalculation).
template <int Q, typename R>
__device__ __forceinline__ void add_node_totals(const R (&f)[Q], R Fx, R Fy, R Fz, double (&acc)[4]) {
  double rho = 0, jx = 0.5 * double(Fx), jy = 0.5 * double(Fy), jz = 0.5 * double(Fz);
#pragma unroll
  for (int a = 0; a < Q; ++a) {
    const Vel e = Lattice<Q>::e(a);
    const double v = double(f[a]);
    rho += v;
    if (e.x > 0) jx += v;
    if (e.x < 0) jx -= v;
    if (e.y > 0) jy += v;
    if (e.y < 0) jy -= v;
    if (e.z > 0) jz += v;
    if (e.z < 0) jz -= v;
  }
  acc[0] += rho;
  acc[1] += jx;
  acc[2] += jy;
  acc[3] += jz;
}

template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double* sh /* [NV][8] */);

// Body force at node (row, x), row = z*ny + y uniform across the wavefront.
template <typename R>
__device__ __forceinline__ void force_row(const StepArgs<R>& args, const Geom& g, uint32_t row, uint32_t x, R& Fx,
                                          R& Fy, R& Fz) {
  if (args.force.field) {
    const R* Ff = args.force.field + uint64_t(row) * uint32_t(g.nx);
    const R sc = R(args.force.scale);
    Fx = sc * ld32(Ff, x);
    Fy = sc * ld32(Ff + g.N, x);
    Fz = sc * ld32(Ff + 2 * g.N, x);
  } else {
    Fx = R(args.force.uni[0]);
    Fy = R(args.force.uni[1]);
    Fz = R(args.force.uni[2]);
  }
}

// The two ends of one node's update: pull + force, and the store.
template <int Q, class ST, bool MASK>
__device__ __forceinline__ void load_node(const StepArgs<typename ST::R>& args, const Geom& g, uint32_t row,
                                          uint32_t x, typename ST::R (&f)[Q], typename ST::R& Fx,
                                          typename ST::R& Fy, typename ST::R& Fz) {
  const Coord c = row_coord(args.rm, g, row, x);
  const Stencil st(g, c, +1);
  pull<Q, ST, MASK, true>(static_cast<const typename ST::T*>(args.fin), g, args.mask, st, row, x, f);
  force_row(args, g, row, x, Fx, Fy, Fz);
}

// Store of node (row, x); a wavefront covers one 64-node block of the row, so
// the direction stride of the blocked layout is wave-uniform (scalar offset).
template <int Q, class ST>
__device__ __forceinline__ void store_node(const StepArgs<typename ST::R>& args, const Geom& g, uint32_t row,
                                           uint32_t x, const typename ST::R (&f)[Q]) {
  using T = typename ST::T;
  constexpr uint32_t sz = uint32_t(sizeof(T));
  const uint32_t nx = uint32_t(g.nx);
  const uint32_t rowQ = nx * uint32_t(Q);
  const __amdgpu_buffer_rsrc_t rs = array_rsrc(static_cast<T*>(args.fout) + uint64_t(row) * rowQ, rowQ * sz);
  const uint32_t b0 = __builtin_amdgcn_readfirstlane(x & ~63u);
  const uint32_t lenB = min(64u, nx - b0) * sz;
  const uint32_t cbase = (b0 * uint32_t(Q) + (x - b0)) * sz;
  T v[Q];
  encode_all<ST, Q>(f, v);
#pragma unroll
  for (int a = 0; a < Q; ++a) buf_store(v[a], rs, cbase, uint32_t(a) * lenB);
}

// With TOT, the step also writes its block's FP64 totals of the input state to
// args.partials[blockIdx.x][0..3].
template <int Q, class ST, bool MASK, bool TOT>
__global__ __launch_bounds__(CMLBM_STEP_BLOCK) void k_step(StepArgs<typename ST::R> args) {
  using R = typename ST::R;
  const Geom g = args.g;
  const uint32_t L = step_block_id();
  const uint32_t row = args.rm.seg.div(L);        // row = z * ny + y, uniform over the block
  const uint32_t x = (L - row * args.rm.nseg) * blockDim.x + threadIdx.x;
  const bool active = x < uint32_t(g.nx) && !(MASK && args.mask[row * uint32_t(g.nx) + x]);
  double acc[4] = {0, 0, 0, 0};
  if constexpr (!TOT) {
    if (!active) return;
  }
  if (active) {
    R f[Q];
    R Fx, Fy, Fz;
    load_node<Q, ST, MASK>(args, g, row, x, f, Fx, Fy, Fz);
    if constexpr (TOT) add_node_totals<Q>(f, Fx, Fy, Fz, acc);
    collide<Q>(f, Fx, Fy, Fz, args.rates);
    store_node<Q, ST>(args, g, row, x, f);
  }
  if constexpr (TOT) {
    __shared__ double sh[4 * 8];
    block_sum<4>(acc, sh);
    if (threadIdx.x == 0) {
#pragma unroll
      for (int i = 0; i < 4; ++i) args.partials[uint64_t(blockIdx.x) * 4 + i] = acc[i];
    }
  }
}

// ---------------------------------------------------------------------------
// In-place step: one population buffer (the AA pattern of Bailey, Myre, Walsh,
// Lilja and Saar, 2009)
// ---------------------------------------------------------------------------
// The buffer alternates between two phases of the same blocked rows:
//   phase 0: slot a of node x holds the pre-collision fbar_a(x);
//   phase 1: slot abar of node x holds the post-collision fbar~_a(x).
// Phase 0 -> 1 (ODD = false) reads and writes only the node's own slots.
// Phase 1 -> 0 (ODD = true) takes fbar_a(x) = fbar~_a(x - e_a) from slot abar
// of x - e_a (when x - e_a is solid, bounce-back gives fbar~_abar(x), which is
// slot a of x), collides, and moves fbar~_a(x), the next fbar_a(x + e_a), into
// slot a of x + e_a (when x + e_a is solid, it returns as fbar_abar(x) into
// slot abar of x).  Writing b = abar in the second list shows that the slots a
// node writes are exactly the slots it read, and a slot (y, c) of a fluid node
// y is read by y - e_c alone (or by y itself when y - e_c is solid), so no two
// nodes touch one slot: the update is race-free in place.  Solid nodes' slots
// are never touched.
// Its stores keep the written lines in the caches (measured faster here than
// streaming stores: the lines were just read, and the scattered phase writes
// each line in two parts).
constexpr int kInplaceAux = 0;

// With TOT, the block's FP64 totals of the pre-collision state it collides go
// to args.partials[blockIdx.x][0..3] (as in k_step).
template <int Q, class ST, bool MASK, bool ODD, bool TOT>
__global__ __launch_bounds__(CMLBM_STEP_BLOCK) void k_step_inplace(StepArgs<typename ST::R> args) {
  using R = typename ST::R;
  using T = typename ST::T;
  constexpr uint32_t sz = uint32_t(sizeof(T));
  const Geom g = args.g;
  const uint32_t nx = uint32_t(g.nx);
  const uint32_t L = step_block_id();
  const uint32_t row = args.rm.seg.div(L);        // uniform over the block
  const uint32_t x = (L - row * args.rm.nseg) * blockDim.x + threadIdx.x;
  const bool active = x < nx && !(MASK && args.mask[row * nx + x]);
  double acc[4] = {0, 0, 0, 0};
  if constexpr (!TOT) {
    if (!active) return;
  }
  if (active) {
    T* const buf = static_cast<T*>(args.fout);
    const uint32_t rowQ = nx * uint32_t(Q);
    const uint32_t b0 = __builtin_amdgcn_readfirstlane(x & ~63u);
    const uint32_t lenB = min(64u, nx - b0) * sz;            // wave-uniform direction stride
    const uint32_t cbase = (b0 * uint32_t(Q) + (x - b0)) * sz;
    // the node's own row (plain loads measured faster here than buffer loads)
    const char* own = reinterpret_cast<const char*>(buf + uint64_t(row) * rowQ);
    const __amdgpu_buffer_rsrc_t rs = array_rsrc(own, rowQ * sz);
    R f[Q];
    if constexpr (!ODD) {
#pragma unroll
      for (int a = 0; a < Q; ++a) f[a] = decode<ST, Q>(ldb<T>(own + uint32_t(a) * lenB, cbase), a);
      R Fx, Fy, Fz;
      force_row(args, g, row, x, Fx, Fy, Fz);
      if constexpr (TOT) add_node_totals<Q>(f, Fx, Fy, Fz, acc);
      collide<Q>(f, Fx, Fy, Fz, args.rates);
      T v[Q];
      encode_all<ST, Q>(f, v);
#pragma unroll
      for (int a = 0; a < Q; ++a) buf_store<kInplaceAux>(v[a], rs, cbase, uint32_t(opposite<Q>(a)) * lenB);
    } else {
      const Coord c = row_coord(args.rm, g, row, x);
      const Stencil st(g, c, +1);      // row[ey+1][ez+1], xs[ex+1]: x - e; index with -e for x + e
      uint32_t nbase[3], nlen[3];      // blocked offsets of x - 1 ([2]) and x + 1 ([0]), and their block strides
#pragma unroll
      for (int i = 0; i < 3; i += 2) {
        const uint32_t xs = st.xs[i];
        const uint32_t bb = xs & ~63u;
        nbase[i] = (bb * uint32_t(Q) + (xs - bb)) * sz;
        nlen[i] = min(64u, nx - bb) * sz;
      }
      uint32_t solid = 0;              // bit a: x - e_a is solid
      if constexpr (MASK) {
#pragma unroll
        for (int a = 0; a < Q; ++a) solid |= uint32_t(args.mask[st.node(Lattice<Q>::e(a), nx)] != 0) << a;
      }
      // (full rows: the x-neighbours' direction stride is lenB, as in pull)
      const bool full = (nx & 63u) == 0;
      auto gather = [&](auto fullrow) {
#pragma unroll
        for (int a = 0; a < Q; ++a) {
          const Vel e = Lattice<Q>::e(a);
          const __amdgpu_buffer_rsrc_t rr = array_rsrc(buf + uint64_t(st.row[e.y + 1][e.z + 1]) * rowQ, rowQ * sz);
          const uint32_t ab = uint32_t(opposite<Q>(a));
          T v;
          if constexpr (MASK) {
            // plain loads: a per-lane choice of row must not pick the descriptor
            const char* rp = reinterpret_cast<const char*>(buf + uint64_t(st.row[e.y + 1][e.z + 1]) * rowQ);
            if ((solid >> a) & 1u)
              v = ldb<T>(own + uint32_t(a) * lenB, cbase);
            else if (e.x == 0)
              v = ldb<T>(rp + ab * lenB, cbase);
            else if constexpr (decltype(fullrow)::value)
              v = ldb<T>(rp + ab * lenB, nbase[e.x + 1]);
            else
              v = ldb<T>(rp, nbase[e.x + 1] + ab * nlen[e.x + 1]);
          } else if (e.x == 0) {
            v = buf_load<T>(rr, cbase, ab * lenB);
          } else if constexpr (decltype(fullrow)::value) {
            v = buf_load<T>(rr, nbase[e.x + 1], ab * lenB);
          } else {
            v = buf_load<T>(rr, nbase[e.x + 1] + ab * nlen[e.x + 1], 0u);
          }
          f[a] = decode<ST, Q>(v, a);
        }
      };
      if (full)
        gather(std::true_type{});
      else
        gather(std::false_type{});
      R Fx, Fy, Fz;
      force_row(args, g, row, x, Fx, Fy, Fz);
      if constexpr (TOT) add_node_totals<Q>(f, Fx, Fy, Fz, acc);
      collide<Q>(f, Fx, Fy, Fz, args.rates);
      T v[Q];
      encode_all<ST, Q>(f, v);
      // Finish the collision before the per-lane store branches: otherwise the
      // compiler sinks its last operations into them, and the rounding departs
      // from the two-buffer step's.
      if constexpr (MASK) pin_all<ST, Q>(v);
      auto scatter = [&](auto fullrow) {
#pragma unroll
        for (int a = 0; a < Q; ++a) {
          const Vel e = Lattice<Q>::e(a);
          const int ab = opposite<Q>(a);
          const __amdgpu_buffer_rsrc_t rt = array_rsrc(buf + uint64_t(st.row[1 - e.y][1 - e.z]) * rowQ, rowQ * sz);
          uint32_t off, soff;
          if (e.x == 0) {
            off = cbase;
            soff = uint32_t(a) * lenB;
          } else if constexpr (decltype(fullrow)::value) {
            off = nbase[1 - e.x];
            soff = uint32_t(a) * lenB;
          } else {
            off = nbase[1 - e.x] + uint32_t(a) * nlen[1 - e.x];
            soff = 0u;
          }
          if constexpr (MASK) {
            // x + e_a = x - e_abar solid: the population returns into slot abar
            // of x.  The neighbour store is issued for every lane, the lanes
            // that bounce dropping theirs (offset past the bound); the bounce
            // store only by wavefronts with a bouncing lane (a wave-uniform
            // branch), the other lanes dropping it.  Neither the descriptor nor
            // the uniform offset ever becomes a per-lane choice.
            const bool back = (solid >> ab) & 1u;
            buf_store<kInplaceAux>(v[a], rt, back ? kDropOffset : off, soff);
            if (__builtin_amdgcn_ballot_w64(back))
              buf_store<kInplaceAux>(v[a], rs, back ? cbase : kDropOffset, uint32_t(ab) * lenB);
          } else {
            buf_store<kInplaceAux>(v[a], rt, off, soff);
          }
        }
      };
      if (full)
        scatter(std::true_type{});
      else
        scatter(std::false_type{});
    }
  }
  if constexpr (TOT) {
    __shared__ double sh[4 * 8];
    block_sum<4>(acc, sh);
    if (threadIdx.x == 0) {
#pragma unroll
      for (int i = 0; i < 4; ++i) args.partials[uint64_t(blockIdx.x) * 4 + i] = acc[i];
    }
  }
}

// Whole-wavefront shifts by one lane (DPP wave_shr:1 / wave_shl:1): lane i
// gets v from lane i - 1 (from_lane_below) or i + 1 (from_lane_above); the
// lane with no source (0, resp. 63) gets `edge` instead.
template <int CTRL, typename T>
__device__ __forceinline__ T wave_shift(T v, T edge) {
  if constexpr (sizeof(T) == 8) {
    const uint64_t u = __builtin_bit_cast(uint64_t, v), w = __builtin_bit_cast(uint64_t, edge);
    const uint32_t lo = uint32_t(__builtin_amdgcn_update_dpp(int(uint32_t(w)), int(uint32_t(u)), CTRL, 0xF, 0xF, false));
    const uint32_t hi =
        uint32_t(__builtin_amdgcn_update_dpp(int(uint32_t(w >> 32)), int(uint32_t(u >> 32)), CTRL, 0xF, 0xF, false));
    return __builtin_bit_cast(T, (uint64_t(hi) << 32) | lo);
  } else if constexpr (sizeof(T) == 4) {
    return __builtin_bit_cast(
        T, __builtin_amdgcn_update_dpp(__builtin_bit_cast(int, edge), __builtin_bit_cast(int, v), CTRL, 0xF, 0xF, false));
  } else {
    const int r = __builtin_amdgcn_update_dpp(int(__builtin_bit_cast(uint16_t, edge)), int(__builtin_bit_cast(uint16_t, v)),
                                              CTRL, 0xF, 0xF, false);
    return __builtin_bit_cast(T, uint16_t(r));
  }
}
// Value of v in lane 63 (any lane may ask; EXEC does not matter).
template <typename T>
__device__ __forceinline__ T read_lane63(T v) {
  if constexpr (sizeof(T) == 8) {
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = uint32_t(__builtin_amdgcn_readlane(int(uint32_t(u)), 63));
    const uint32_t hi = uint32_t(__builtin_amdgcn_readlane(int(uint32_t(u >> 32)), 63));
    return __builtin_bit_cast(T, (uint64_t(hi) << 32) | lo);
  } else if constexpr (sizeof(T) == 4) {
    return __builtin_bit_cast(T, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 63));
  } else {
    return __builtin_bit_cast(T, uint16_t(__builtin_amdgcn_readlane(int(__builtin_bit_cast(uint16_t, v)), 63)));
  }
}

template <typename T>
__device__ __forceinline__ T from_lane_below(T v, T edge) {
  return wave_shift<0x138>(v, edge);
}
template <typename T>
__device__ __forceinline__ T from_lane_above(T v, T edge) {
  return wave_shift<0x130>(v, edge);
}

// Scatter phase of the in-place step on a lattice without walls, with aligned
// stores.  The scatter writes fbar~_a(x) one node over in x for the directions
// with e_x = +-1; stored as is, every wavefront store of those directions would
// straddle one more cache line than it fills.  Here the lane of node x writes,
// at its own (aligned) position in the target row, the value of its x -+ 1
// neighbour instead: taken from the neighbouring lane, across a wavefront edge
// from the neighbouring wavefront through LDS, and, at the two ends of the
// block's row segment, written by the end node itself with one shifted store
// (to the next segment's first node or the previous one's last, periodic).  Same
// slots, same values as k_step_inplace<Q, ST, false, true, TOT>.
template <int Q, class ST, bool TOT>
__global__ __launch_bounds__(CMLBM_STEP_BLOCK) void k_scatter_periodic(StepArgs<typename ST::R> args) {
  using R = typename ST::R;
  using T = typename ST::T;
  constexpr uint32_t sz = uint32_t(sizeof(T));
  constexpr int kWaves = CMLBM_STEP_BLOCK / 64;
  __shared__ T edge_up[kWaves][Q];   // lane 63 of each wavefront (e_x = +1 directions)
  __shared__ T edge_dn[kWaves][Q];   // lane 0 of each wavefront (e_x = -1 directions)
  const Geom g = args.g;
  const uint32_t nx = uint32_t(g.nx);
  const uint32_t L = step_block_id();
  const uint32_t row = args.rm.seg.div(L);               // uniform over the block
  const uint32_t x0 = (L - row * args.rm.nseg) * blockDim.x;   // the block's row segment [x0, xend)
  const uint32_t xend = min(x0 + blockDim.x, nx);
  const uint32_t x = x0 + threadIdx.x;
  const bool active = x < nx;
  const int lane = int(threadIdx.x & 63u), wave = int(threadIdx.x >> 6);
  T* const buf = static_cast<T*>(args.fout);
  const uint32_t rowQ = nx * uint32_t(Q);
  const uint32_t b0 = __builtin_amdgcn_readfirstlane(x & ~63u);
  const uint32_t lenB = (b0 < nx ? min(64u, nx - b0) : 64u) * sz;
  const uint32_t cbase = (b0 * uint32_t(Q) + (x - b0)) * sz;
  const Coord c = row_coord(args.rm, g, row, active ? x : nx - 1);
  const Stencil st(g, c, +1);
  uint32_t nbase[3], nlen[3];
#pragma unroll
  for (int i = 0; i < 3; i += 2) {
    const uint32_t xs = st.xs[i];
    const uint32_t bb = xs & ~63u;
    nbase[i] = (bb * uint32_t(Q) + (xs - bb)) * sz;
    nlen[i] = min(64u, nx - bb) * sz;
  }
  T v[Q];
#pragma unroll
  for (int a = 0; a < Q; ++a) v[a] = T(0);
  double acc[4] = {0, 0, 0, 0};
  if (active) {
    R f[Q];
    // (full rows: the x-neighbours' direction stride is lenB, as in pull)
    auto gather = [&](auto fullrow) {
#pragma unroll
      for (int a = 0; a < Q; ++a) {
        const Vel e = Lattice<Q>::e(a);
        const __amdgpu_buffer_rsrc_t rr = array_rsrc(buf + uint64_t(st.row[e.y + 1][e.z + 1]) * rowQ, rowQ * sz);
        const uint32_t ab = uint32_t(opposite<Q>(a));
        T v;
        if (e.x == 0)
          v = buf_load<T>(rr, cbase, ab * lenB);
        else if constexpr (decltype(fullrow)::value)
          v = buf_load<T>(rr, nbase[e.x + 1], ab * lenB);
        else
          v = buf_load<T>(rr, nbase[e.x + 1] + ab * nlen[e.x + 1], 0u);
        f[a] = decode<ST, Q>(v, a);
      }
    };
    if ((nx & 63u) == 0)
      gather(std::true_type{});
    else
      gather(std::false_type{});
    R Fx, Fy, Fz;
    force_row(args, g, row, x, Fx, Fy, Fz);
    if constexpr (TOT) add_node_totals<Q>(f, Fx, Fy, Fz, acc);
    collide<Q>(f, Fx, Fy, Fz, args.rates);
    encode_all<ST, Q>(f, v);
    // Finish the collision here, ahead of the barrier and the edge branch
    // (same contraction as the two-buffer step).
    pin_all<ST, Q>(v);
  }
  // Lane 63's values, read with every lane active: inside the lane-0 branch
  // below, the compiler may finish a value (extract a 16-bit half from a
  // packed register) under that branch's single lane, and the read of lane 63
  // would then see a register that lane never wrote.  The reads are
  // convergent, so the compiler keeps them, and what feeds them, out here.
  T up63[Q];
#pragma unroll
  for (int a = 0; a < Q; ++a) up63[a] = Lattice<Q>::e(a).x > 0 ? read_lane63(v[a]) : T(0);
  // One lane writes both edges.
  if (lane == 0) {
#pragma unroll
    for (int a = 0; a < Q; ++a) {
      if (Lattice<Q>::e(a).x > 0) edge_up[wave][a] = up63[a];
      if (Lattice<Q>::e(a).x < 0) edge_dn[wave][a] = v[a];
    }
  }
  __syncthreads();
  // The stores are predicated without branches: a lane that has nothing to
  // write at a slot gets the byte offset kDrop, past the row's bound, and the
  // raw buffer store drops it.  The one node that writes across the segment's
  // end (to x + 1 after the last node, x - 1 before the first) is the same for
  // the whole block, so that target's offsets are wave-uniform.
  constexpr uint32_t kDrop = kDropOffset;
  const uint32_t xn = xend == nx ? 0u : xend, xp = x0 == 0 ? nx - 1 : x0 - 1;   // periodic
  const uint32_t bn = xn & ~63u, bp = xp & ~63u;
  const uint32_t off_own = active ? cbase : kDrop;
  const uint32_t off_prev = active && x > x0 ? cbase : kDrop;        // e_x = +1: from x - 1
  const uint32_t off_next = active && x + 1 < xend ? cbase : kDrop;  // e_x = -1: from x + 1
  const uint32_t off_after = x == xend - 1 ? (bn * uint32_t(Q) + (xn - bn)) * sz : kDrop;
  const uint32_t off_before = x == x0 ? (bp * uint32_t(Q) + (xp - bp)) * sz : kDrop;
  const uint32_t len_after = min(64u, nx - bn) * sz, len_before = min(64u, nx - bp) * sz;
  const int wprev = wave > 0 ? wave - 1 : 0, wnext = wave + 1 < kWaves ? wave + 1 : wave;
  // Only the wavefront holding the segment's last node (first node) has a
  // store across the segment's end to issue: a wave-uniform branch skips
  // those instructions in the others.
  const uint32_t wv = __builtin_amdgcn_readfirstlane(uint32_t(wave));
  const bool has_last = x0 + 64u * wv <= xend - 1 && xend - 1 < x0 + 64u * (wv + 1);
  const bool has_first = wv == 0;
#pragma unroll
  for (int a = 0; a < Q; ++a) {
    const Vel e = Lattice<Q>::e(a);
    const __amdgpu_buffer_rsrc_t rt = array_rsrc(buf + uint64_t(st.row[1 - e.y][1 - e.z]) * rowQ, rowQ * sz);
    if (e.x == 0) {
      buf_store<kInplaceAux>(v[a], rt, off_own, uint32_t(a) * lenB);
    } else if (e.x > 0) {              // slot a of x receives fbar~_a(x - 1)
      buf_store<kInplaceAux>(from_lane_below(v[a], edge_up[wprev][a]), rt, off_prev, uint32_t(a) * lenB);
      if (has_last) buf_store<kInplaceAux>(v[a], rt, off_after, uint32_t(a) * len_after);      // to x + 1
    } else {                           // slot a of x receives fbar~_a(x + 1)
      buf_store<kInplaceAux>(from_lane_above(v[a], edge_dn[wnext][a]), rt, off_next, uint32_t(a) * lenB);
      if (has_first) buf_store<kInplaceAux>(v[a], rt, off_before, uint32_t(a) * len_before);    // to x - 1
    }
  }
  if constexpr (TOT) {
    __shared__ double sh[4 * 8];
    block_sum<4>(acc, sh);
    if (threadIdx.x == 0) {
#pragma unroll
      for (int i = 0; i < 4; ++i) args.partials[uint64_t(blockIdx.x) * 4 + i] = acc[i];
    }
  }
}

// ---------------------------------------------------------------------------
// Read-out kernels (grid-stride over nodes)
// ---------------------------------------------------------------------------
// Observable pre-collision state fbar(x): full populations, compute type,
// structure of arrays [Q][N].
template <int Q, class ST, bool MASK>
__global__ __launch_bounds__(256) void k_gather(AuxArgs<typename ST::R> args) {
  using R = typename ST::R;
  const Geom g = args.g;
  R* out = static_cast<R*>(args.out0);
  for (uint32_t n = blockIdx.x * blockDim.x + threadIdx.x; n < g.N; n += gridDim.x * blockDim.x) {
    if (MASK && args.mask[n]) {
#pragma unroll
      for (int a = 0; a < Q; ++a) out[uint64_t(a) * g.N + n] = R(0);
      continue;
    }
    const Coord c = coord_of(g, n);
    const Stencil st(g, c, +1);
    R f[Q];
    pull<Q, ST, MASK>(static_cast<const typename ST::T*>(args.in0), g, args.mask, st,
                      n / uint32_t(g.nx), uint32_t(c.x), f);
#pragma unroll
    for (int a = 0; a < Q; ++a) out[uint64_t(a) * g.N + n] = f[a];
  }
}

// Population buffer (blocked layout, storage type) <-> full populations in
// compute type, structure of arrays [Q][N].  EXPORT: buffer -> SoA.
template <int Q, class ST, bool EXPORT>
__global__ __launch_bounds__(256) void k_convert(Geom g, const void* in, void* out) {
  using R = typename ST::R;
  using T = typename ST::T;
  const uint64_t rowQ = uint64_t(g.nx) * Q;
  for (uint32_t n = blockIdx.x * blockDim.x + threadIdx.x; n < g.N; n += gridDim.x * blockDim.x) {
    const uint32_t row = n / uint32_t(g.nx), x = n - row * uint32_t(g.nx);
    // all Q loads first, then the stores: the buffers may alias as far as the
    // compiler knows, so a store between two loads would make the second wait
    if constexpr (EXPORT) {
      R v[Q];
#pragma unroll
      for (int a = 0; a < Q; ++a)
        v[a] = decode<ST, Q>(static_cast<const T*>(in)[uint64_t(row) * rowQ + in_row<Q>(uint32_t(g.nx), a, x)], a);
#pragma unroll
      for (int a = 0; a < Q; ++a) static_cast<R*>(out)[uint64_t(a) * g.N + n] = v[a];
    } else {
      T v[Q];
#pragma unroll
      for (int a = 0; a < Q; ++a) v[a] = encode<ST, Q>(static_cast<const R*>(in)[uint64_t(a) * g.N + n], a);
#pragma unroll
      for (int a = 0; a < Q; ++a) static_cast<T*>(out)[uint64_t(row) * rowQ + in_row<Q>(uint32_t(g.nx), a, x)] = v[a];
    }
  }
}

// Populations of node n read from its own slots: the pre-collision state of a
// buffer in phase 0 of the in-place scheme.
template <int Q, class ST>
__device__ __forceinline__ void load_own(const typename ST::T* buf, const Geom& g, uint32_t n,
                                         typename ST::R (&f)[Q]) {
  const uint32_t row = n / uint32_t(g.nx), x = n - row * uint32_t(g.nx);
  const typename ST::T* rp = buf + uint64_t(row) * uint64_t(g.nx) * Q;
#pragma unroll
  for (int a = 0; a < Q; ++a) f[a] = decode<ST, Q>(ld32(rp, in_row<Q>(uint32_t(g.nx), a, x)), a);
}

// Pre-collision populations of fluid node n: pulled from a post-collision
// buffer, or (PRE) read in place from a pre-collision one.
template <int Q, class ST, bool MASK, bool PRE>
__device__ __forceinline__ void node_state(const AuxArgs<typename ST::R>& args, uint32_t n, Coord c,
                                           typename ST::R (&f)[Q]) {
  const auto* in = static_cast<const typename ST::T*>(args.in0);
  if constexpr (PRE) {
    load_own<Q, ST>(in, args.g, n, f);
  } else {
    const Stencil st(args.g, c, +1);
    pull<Q, ST, MASK>(in, args.g, args.mask, st, n / uint32_t(args.g.nx), uint32_t(c.x), f);
  }
}

// rho and u (Eqs. densitycalculation, velocitycalculation), zero at solid nodes.
template <int Q, class ST, bool MASK, bool PRE>
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
    R f[Q];
    node_state<Q, ST, MASK, PRE>(args, n, coord_of(g, n), f);
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
template <int Q, class ST, bool MASK, bool PRE>
__global__ __launch_bounds__(256) void k_totals(AuxArgs<typename ST::R> args, double* partials) {
  using R = typename ST::R;
  const Geom g = args.g;
  double acc[4] = {0, 0, 0, 0};
  for (uint32_t n = blockIdx.x * blockDim.x + threadIdx.x; n < g.N; n += gridDim.x * blockDim.x) {
    if (MASK && args.mask[n]) continue;
    R f[Q];
    node_state<Q, ST, MASK, PRE>(args, n, coord_of(g, n), f);
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

// First stage of a long reduction: block b sums rows [b*chunk, (b+1)*chunk) of
// a [nrows][NV] array into stage[b][NV].
template <int NV>
__global__ __launch_bounds__(256) void k_reduce_chunks(const double* rows, uint64_t nrows, double* stage) {
  const uint64_t chunk = (nrows + gridDim.x - 1) / gridDim.x;
  const uint64_t r0 = uint64_t(blockIdx.x) * chunk;
  const uint64_t r1 = r0 + chunk < nrows ? r0 + chunk : nrows;
  double v[NV];
#pragma unroll
  for (int i = 0; i < NV; ++i) v[i] = 0;
  for (uint64_t r = r0 + threadIdx.x; r < r1; r += blockDim.x)
#pragma unroll
    for (int i = 0; i < NV; ++i) v[i] += rows[r * NV + i];
  __shared__ double sh[NV * 8];
  block_sum<NV>(v, sh);
  if (threadIdx.x == 0)
#pragma unroll
    for (int i = 0; i < NV; ++i) stage[uint64_t(blockIdx.x) * NV + i] = v[i];
}

// ---------------------------------------------------------------------------
// Initial condition: fbar(x, 0) = f^eq(rho0, u0) - S/2, then the inverse pull
// into the post-collision buffer so that the first step's pull reproduces it.
// ---------------------------------------------------------------------------
// fpre: with BLOCKED, a population buffer (storage type, blocked rows: phase 0
// of the in-place step); otherwise "real" structure of arrays [Q][N].
template <int Q, class ST, bool BLOCKED, typename FT>
__global__ __launch_bounds__(256) void k_initial_pre(Geom g, const typename ST::R* rho0, const typename ST::R* u0,
                                                     ForceArgs<FT> force, const uint8_t* mask, void* fpre) {
  using R = typename ST::R;
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
        initial27(rho, ux, uy, uz, Fx, Fy, Fz, f);
      } else {
        initial15(rho, ux, uy, uz, Fx, Fy, Fz, f);
      }
    }
    if constexpr (BLOCKED) {
      const uint32_t row = n / uint32_t(g.nx), x = n - row * uint32_t(g.nx);
      typename ST::T* rp = static_cast<typename ST::T*>(fpre) + uint64_t(row) * uint64_t(g.nx) * Q;
#pragma unroll
      for (int a = 0; a < Q; ++a) rp[in_row<Q>(uint32_t(g.nx), a, x)] = encode<ST, Q>(f[a], a);
    } else {
#pragma unroll
      for (int a = 0; a < Q; ++a) static_cast<R*>(fpre)[uint64_t(a) * g.N + n] = f[a];
    }
  }
}

// fbar~(y)_a = fbar(y + e_a)_a if y + e_a is fluid, else fbar(y)_abar; fpre is
// structure of arrays, fpost the blocked population buffer.
template <int Q, class ST, bool MASK>
__global__ __launch_bounds__(256) void k_scatter_post(Geom g, const typename ST::R* fpre, const uint8_t* mask,
                                                      typename ST::T* fpost) {
  using R = typename ST::R;
  const uint64_t rowQ = uint64_t(g.nx) * Q;
  for (uint32_t n = blockIdx.x * blockDim.x + threadIdx.x; n < g.N; n += gridDim.x * blockDim.x) {
    const Coord c = coord_of(g, n);
    const uint64_t base = uint64_t(n / uint32_t(g.nx)) * rowQ;
    if (MASK && mask[n]) {
#pragma unroll
      for (int a = 0; a < Q; ++a) fpost[base + in_row<Q>(uint32_t(g.nx), a, uint32_t(c.x))] = typename ST::T(0);
      continue;
    }
    const Stencil st(g, c, -1);    // x + e_a
    // the mask bytes in one round, then every load, then the stores (the
    // buffers may alias as far as the compiler knows)
    uint32_t solid = 0;            // bit a: x + e_a solid
    if constexpr (MASK) {
#pragma unroll
      for (int a = 1; a < Q; ++a) solid |= uint32_t(mask[st.node(Lattice<Q>::e(a), uint32_t(g.nx))] != 0) << a;
    }
    R v[Q];
#pragma unroll
    for (int a = 0; a < Q; ++a) {
      const uint32_t dst = st.node(Lattice<Q>::e(a), uint32_t(g.nx));
      const uint64_t at = ((solid >> a) & 1u) ? uint64_t(opposite<Q>(a)) * g.N + n : uint64_t(a) * g.N + dst;
      v[a] = fpre[at];
    }
#pragma unroll
    for (int a = 0; a < Q; ++a) fpost[base + in_row<Q>(uint32_t(g.nx), a, uint32_t(c.x))] = encode<ST, Q>(v[a], a);
  }
}

// ---------------------------------------------------------------------------
// Adjoint step (D3Q27 and D3Q15).  Forward step n maps the pre-collision state
// fbar^n(x) (pulled from f_post_prev) to fbar~(x) = C(fbar^n(x)), and
// fbar^{n+1}(x)_a = fbar~(x - e_a)_a (or bounce-back).  Given
// lam_next = dL/dfbar^{n+1} (structure of arrays), the adjoint of the stored
// fbar~(x)_a is mu_a = lam_next(x + e_a)_a, or lam_next(x)_abar when x + e_a is
// solid, and lam(x) = J_C(fbar^n(x))^T mu.  dL/dF(x) and dL/domega accumulate
// in FP64.
// ---------------------------------------------------------------------------
// Launch shape: a block walks a contiguous run of row segments (one segment =
// blockDim.x consecutive x of one row), so row bases are uniform and the
// neighbour rows that one segment gathers from are reused by the next ones
// from the same XCD's L2; block ids are permuted per XCD as in the step.
// The adjoint's output stores (lambda, dL/dF): CMLBM_ADJ_NT = 1 streams them
// past the caches, as the step's population stores, so that they do not evict
// the neighbour rows the gathers reuse.
#ifndef CMLBM_ADJ_NT
#define CMLBM_ADJ_NT 1
#endif
template <typename T>
__device__ __forceinline__ void st32_out(T* base, uint32_t idx, T v) {
  T* p = reinterpret_cast<T*>(reinterpret_cast<char*>(base) + idx * uint32_t(sizeof(T)));
  if constexpr (CMLBM_ADJ_NT)
    __builtin_nontemporal_store(v, p);
  else
    *p = v;
}

constexpr int kAdjBlock = 256;   // largest adjoint block (smaller for nx < 256)
constexpr int kAdjAux = CMLBM_ADJ_NT ? 2 : 0;   // cache policy of the adjoint's stores (2: streaming)

// Register slot of direction a in the adjoint's population vectors: cube
// order for D3Q27 (the axis passes), the paper's order for D3Q15.
template <int Q>
__device__ __forceinline__ constexpr int slot(int a) {
  if constexpr (Q == 27)
    return cube27(a);
  else
    return a;
}

// Per-thread column of LDS: element b (4..26) at sh[(b - 4) * kAdjBlock + tid].
template <typename R>
struct LdsColumn {
  R* p;
  __device__ __forceinline__ R& operator[](int b) const { return p[(b - 4) * kAdjBlock]; }
};

// Waves per SIMD the adjoint is compiled for: three 27-vectors and the line
// transforms fit 168 VGPRs in FP32 (3 waves); FP64 needs twice the registers.
#ifndef CMLBM_ADJ_WAVES_F32
#define CMLBM_ADJ_WAVES_F32 3
#endif
#ifndef CMLBM_ADJ_WAVES_F64
#define CMLBM_ADJ_WAVES_F64 1
#endif
template <class ST, bool MASK>
constexpr int adjoint_waves() {
  return sizeof(typename ST::R) == 8 ? CMLBM_ADJ_WAVES_F64 : (MASK ? 3 : CMLBM_ADJ_WAVES_F32);
}

// The node count as a value the compiler must take as new at each use (an
// empty statement: no instruction).  The adjoint addresses 2Q direction planes
// of the [Q][N] adjoint arrays; hoisted out of its loop, their 64-bit bases
// overflow the scalar registers and are spilled and reloaded on every pass.
// Recomputed at the point of use they cost a few scalar instructions instead.
__device__ __forceinline__ uint64_t per_item(uint64_t n) {
  asm volatile("" : "+s"(n));
  return n;
}

// PM: attractor form compiled in (0 literal, 1 per unit mass); the host picks
// the instance that matches the rates' per_mass flag.
template <int Q, class ST, bool MASK, int PM>
__global__ __launch_bounds__(kAdjBlock) __attribute__((amdgpu_waves_per_eu(adjoint_waves<ST, MASK>()))) void k_adjoint(
    AdjArgs<typename ST::R> args, double* partials) {
  using R = typename ST::R;
  using T = typename ST::T;
  const Geom g = args.g;
  const uint32_t nx = uint32_t(g.nx);
  // Per-thread running sums over the (few) nodes this thread visits, in LDS to
  // keep registers for the collision: dL/domega_b for b = 4..26; uF = dL/dF
  // for a uniform force.
  __shared__ R wsh[23 * kAdjBlock];
  LdsColumn<R> wacc{wsh + threadIdx.x};
#pragma unroll
  for (int b = 4; b < 27; ++b) wacc[b] = R(0);   // (b >= Q stays zero)
  R uF[3] = {R(0), R(0), R(0)};
  const uint32_t nseg = (nx + blockDim.x - 1) / blockDim.x;
  const uint32_t items = nseg * uint32_t(g.ny) * uint32_t(g.nz);
  // Row segments are dealt to the eight XCDs in contiguous runs; inside its
  // run, an XCD's blocks take the segments in turn (its block b: b, b + per,
  // b + 2 per, ...), so that the blocks running at one time work on adjacent
  // segments and find the cache lines they share still in the XCD's L2.  (The
  // grid is a multiple of 8; consecutive block ids go to the XCDs in turn.)
  const uint32_t per = gridDim.x >> 3;
  const uint32_t run = (items + 7u) >> 3;
  const uint32_t i0 = (blockIdx.x & 7u) * run;
  const uint32_t i1 = min(items, i0 + run);
  for (uint32_t it = i0 + (blockIdx.x >> 3); it < i1; it += per) {
    const uint32_t row = it / nseg;
    const uint32_t x = (it - row * nseg) * blockDim.x + threadIdx.x;
    if (x >= nx) continue;
    const uint32_t rowB = nx * uint32_t(sizeof(R)), xB = x * uint32_t(sizeof(R));   // one row of a [Q][N] plane
    const Coord c{int(x), int(row % uint32_t(g.ny)), int(row / uint32_t(g.ny))};
    const Stencil up(g, c, +1);    // up.node(e) = x - e
    R f[Q], gm[Q];
    if constexpr (MASK) {
      // bit a: x - e_a is solid (bit 0: x itself).  x + e_a = x - e_abar, so
      // the same bits serve the reverse gather; one round of mask loads, then
      // both gathers' loads together.
      uint32_t solid = 0;
#pragma unroll
      for (int a = 0; a < Q; ++a) solid |= uint32_t(args.mask[up.node(Lattice<Q>::e(a), nx)] != 0) << a;
      if (solid & 1u) continue;
      const T* fin = static_cast<const T*>(args.fpost);
      const uint64_t rowQ = uint64_t(nx) * Q;
      constexpr uint32_t sz = uint32_t(sizeof(T));
      const uint32_t b0 = __builtin_amdgcn_readfirstlane(x & ~63u);
      const uint32_t lenB = min(64u, nx - b0) * sz;
      const uint32_t cbase = (b0 * uint32_t(Q) + (x - b0)) * sz;
      const char* own = reinterpret_cast<const char*>(fin + uint64_t(row) * rowQ);
      const Stencil dn(g, c, -1);  // dn.node(e) = x + e
      const uint64_t N = per_item(g.N);
#pragma unroll
      for (int a = 0; a < Q; ++a) {
        const Vel e = Lattice<Q>::e(a);
        const uint32_t ab = uint32_t(opposite<Q>(a));
        // pull: fbar_a(x) = fbar~_a(x - e_a), or fbar~_abar(x) from x's own slot
        T v;
        if ((solid >> a) & 1u) {
          v = ldb<T>(own + ab * lenB, cbase);
        } else {
          const uint32_t xs = up.xs[e.x + 1], bb = xs & ~63u;
          v = ldb<T>(fin + uint64_t(up.row[e.y + 1][e.z + 1]) * rowQ,
                     (bb * uint32_t(Q) + (xs - bb)) * sz + uint32_t(a) * min(64u, nx - bb) * sz);
        }
        f[slot<Q>(a)] = decode<ST, Q>(v, a);
        // reverse gather: lam_a(x + e_a), or lam_abar(x) where x + e_a is solid
        gm[slot<Q>(a)] = ((solid >> ab) & 1u)
                             ? ld32(args.lam_next + uint64_t(ab) * N + uint64_t(row) * nx, x)
                             : ld32(args.lam_next + uint64_t(a) * N + uint64_t(dn.row[e.y + 1][e.z + 1]) * nx,
                                    dn.xs[e.x + 1]);
      }
    } else {
      // forward pre-collision populations (D3Q27: in cube order)
      R fa[Q];
      pull<Q, ST, false, true, true>(static_cast<const T*>(args.fpost), g, args.mask, up, row, x, fa);
#pragma unroll
      for (int a = 0; a < Q; ++a) f[slot<Q>(a)] = fa[a];
      // adjoint of this node's post-collision populations (reverse streaming)
      const Stencil dn(g, c, -1);
      const uint64_t N = per_item(g.N);
#pragma unroll
      for (int a = 0; a < Q; ++a) {
        const Vel e = Lattice<Q>::e(a);
        gm[slot<Q>(a)] =
            buf_load<R>(array_rsrc(args.lam_next + uint64_t(a) * N + uint64_t(dn.row[e.y + 1][e.z + 1]) * nx, rowB),
                        dn.xs[e.x + 1] * uint32_t(sizeof(R)), 0u);
      }
    }
    R Fx, Fy, Fz;
    if (args.force.field) {
      const R* Ff = args.force.field + uint64_t(row) * nx;
      const R sc = R(args.force.scale);
      Fx = sc * ld32(Ff, x);
      Fy = sc * ld32(Ff + g.N, x);
      Fz = sc * ld32(Ff + 2 * g.N, x);
    } else {
      Fx = R(args.force.uni[0]);
      Fy = R(args.force.uni[1]);
      Fz = R(args.force.uni[2]);
    }
    R gFx = R(0), gFy = R(0), gFz = R(0);
    if constexpr (Q == 27) {
      R s[27];
      collide27_adj<PM>(f, Fx, Fy, Fz, args.rates, gm, s, gFx, gFy, gFz, wacc);
    } else {
      collide15_adj<PM>(f, Fx, Fy, Fz, args.rates, gm, gFx, gFy, gFz, wacc);
    }
    const uint64_t N = per_item(g.N);
#pragma unroll
    for (int a = 0; a < Q; ++a)
      buf_store<kAdjAux>(gm[slot<Q>(a)], array_rsrc(args.lam + uint64_t(a) * N + uint64_t(row) * nx, rowB), xB, 0u);
    if (args.force.field) {
      const double sc = double(args.force.scale);
      const uint32_t xD = x * uint32_t(sizeof(double));
      const double gF[3] = {double(gFx), double(gFy), double(gFz)};
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const __amdgpu_buffer_rsrc_t rd = array_rsrc(args.dLdF + uint64_t(k) * N + uint64_t(row) * nx, nx * 8u);
        buf_store<kAdjAux>(buf_load<double>(rd, xD, 0u) + sc * gF[k], rd, xD, 0u);
      }
    } else {
      uF[0] += gFx;
      uF[1] += gFy;
      uF[2] += gFz;
    }
  }
  double v[26];
#pragma unroll
  for (int b = 4; b < 27; ++b) v[b - 4] = b < Q ? double(wacc[b]) : 0.0;
  __syncthreads();
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
// Wall-layout sensitivity.  Give each node a wall fraction phi(x) in [0, 1] and
// stream by fbar_a(x) = (1 - phi(x)) fbar~_a(x - e_a) + phi(x - e_a) fbar~_abar(x):
// a population leaving s for t = s + e_c arrives with weight 1 - phi(t) and
// returns to s reversed with weight phi(t).  At phi in {0, 1} this is the pull
// with half-way bounce-back (Sec. 9) that the step kernels run.  Its derivative
// at the mask, with lam_next = dL/dfbar^{n+1}:
//   dL/dphi(t) += sum_c fbar~_c(s) [lam_cbar(s) - lam_c(t)],  s = t - e_c fluid
// (solid nodes hold no populations).  Each fluid node s recomputes fbar~(s)
// from the pull of f_post_prev and adds its terms to its fluid targets with
// FP64 atomics; solid targets get nothing (the collision switches off there).
// ---------------------------------------------------------------------------
template <int Q, class ST, bool MASK>
__global__ __launch_bounds__(256) void k_wall_sens(AdjArgs<typename ST::R> args, double* dLdphi) {
  using R = typename ST::R;
  const Geom g = args.g;
  const uint32_t nx = uint32_t(g.nx);
  for (uint32_t n = blockIdx.x * blockDim.x + threadIdx.x; n < g.N; n += gridDim.x * blockDim.x) {
    if (MASK && args.mask[n]) continue;
    const Coord c = coord_of(g, n);
    R f[Q];
    {
      const Stencil up(g, c, +1);
      pull<Q, ST, MASK>(static_cast<const typename ST::T*>(args.fpost), g, args.mask, up, n / nx, uint32_t(c.x), f);
    }
    R Fx, Fy, Fz;
    force_at(args.force, g.N, n, Fx, Fy, Fz);
    collide<Q>(f, Fx, Fy, Fz, args.rates);
    const Stencil dn(g, c, -1);
#pragma unroll
    for (int a = 1; a < Q; ++a) {
      const uint32_t t = dn.node(Lattice<Q>::e(a), nx);
      if (MASK && args.mask[t]) continue;
      const double own = double(args.lam_next[uint64_t(opposite<Q>(a)) * g.N + n]);
      const double arrived = double(args.lam_next[uint64_t(a) * g.N + t]);
      atomicAdd(dLdphi + t, double(f[a]) * (own - arrived));
    }
  }
}

// The same terms from the state the streaming moves: fpost = fbar~ as the
// step stored it, lam_next = dL/dfbar of the pre-collision state that
// streaming fpost produces.  Each fluid node t gathers its own terms, in a
// fixed order and without atomics, and no collision is recomputed:
//   dL/dphi(t) += sum_a fbar~_a(s) (lam_abar(s) - lam_a(t)),  s = t - e_a fluid.
constexpr uint32_t kWallTileZ = 8;   // planes per tile of the wall term's row order

template <int Q, class ST, bool MASK>
__global__ __launch_bounds__(CMLBM_STEP_BLOCK) void k_wall_gather(AdjArgs<typename ST::R> args, double* dLdphi) {
  using R = typename ST::R;
  using T = typename ST::T;
  constexpr uint32_t sz = uint32_t(sizeof(T)), rz = uint32_t(sizeof(R));
  const Geom g = args.g;
  const uint32_t nx = uint32_t(g.nx);
  // one block per row segment, as the step kernels: every source row of a
  // direction is uniform over the block, so each direction's three loads go
  // through buffer descriptors with per-lane x offsets only.  Each lambda
  // value is read twice, by its own node and by the neighbour it feeds; the
  // rows are taken in tiles of kWallTileZ planes, z fastest inside a tile,
  // so that a row's neighbours in the planes above and below are processed
  // within a few blocks of it and its lambda values are still in L2 (in
  // plain row order the planes are a whole plane of rows apart).
  const uint32_t nseg = (nx + blockDim.x - 1) / blockDim.x;
  const uint32_t L = step_block_id();
  const uint32_t q = L / nseg;                       // position in the tiled row order
  const uint32_t x = (L - q * nseg) * blockDim.x + threadIdx.x;
  if (x >= nx) return;
  const uint32_t ny = uint32_t(g.ny), nz = uint32_t(g.nz);
  const uint32_t tile = q / (ny * kWallTileZ);
  const uint32_t z0 = tile * kWallTileZ, h = min(kWallTileZ, nz - z0);
  const uint32_t within = q - z0 * ny;
  const uint32_t yy = within / h, zz = z0 + (within - yy * h);
  const uint32_t row = zz * ny + yy;
  if (MASK && args.mask[uint64_t(row) * nx + x]) return;
  const Coord c{int(x), int(yy), int(zz)};
  const Stencil up(g, c, +1);      // up.node(e) = t - e
  // bit a: t - e_a solid (one round of mask loads; the value loads below do
  // not wait on it, and a solid source's term is dropped by a select: its
  // slots hold no state)
  uint32_t solid = 0;
  if constexpr (MASK) {
#pragma unroll
    for (int a = 1; a < Q; ++a) solid |= uint32_t(args.mask[up.node(Lattice<Q>::e(a), nx)] != 0) << a;
  }
  const T* fin = static_cast<const T*>(args.fpost);
  const uint32_t rowQB = nx * uint32_t(Q) * sz, rowB = nx * rz;
  const uint64_t N = per_item(g.N);
  // all 3 (Q - 1) loads are issued before the first term is formed (the
  // pins below): interleaved with the FP64 sums, the compiler let the loads
  // in flight drain to a handful several times per node
  T v[Q];
  R own[Q], arrived[Q];
  v[0] = T(0);
#pragma unroll
  for (int a = 1; a < Q; ++a) {
    const Vel e = Lattice<Q>::e(a);
    const uint32_t ab = uint32_t(opposite<Q>(a));
    const uint32_t srow = up.row[e.y + 1][e.z + 1], xs = up.xs[e.x + 1];
    v[a] = buf_load<T>(array_rsrc(fin + uint64_t(srow) * nx * Q, rowQB), in_row<Q>(nx, a, xs) * sz, 0u);
    own[a] = buf_load<R>(array_rsrc(args.lam_next + uint64_t(ab) * N + uint64_t(srow) * nx, rowB), xs * rz, 0u);
    arrived[a] = buf_load<R>(array_rsrc(args.lam_next + uint64_t(a) * N + uint64_t(row) * nx, rowB), x * rz, 0u);
  }
  pin_all<ST, Q>(v);
#pragma unroll
  for (int a = 1; a < Q; ++a) {
    asm volatile("" : "+v"(own[a]));
    asm volatile("" : "+v"(arrived[a]));
  }
  double acc = 0.0;
#pragma unroll
  for (int a = 1; a < Q; ++a) {
    const double term = double(decode<ST, Q>(v[a], a)) * (double(own[a]) - double(arrived[a]));
    acc += ((solid >> a) & 1u) ? 0.0 : term;
  }
  dLdphi[uint64_t(row) * nx + x] += acc;
}

// ---------------------------------------------------------------------------
// Kinetic-energy loss and its seed: E = sum over fluid x of |j|^2 / (2 rho),
// j = sum fbar e + F/2, on pre-collision populations (compute type).
// dE/dfbar_a = u.e_a - |u|^2/2, dE/dF = u/2 (times the force scale).
// ---------------------------------------------------------------------------
template <int Q, typename R>
__device__ __forceinline__ void node_moments(const R* fpre, uint64_t N, uint32_t n, R Fx, R Fy, R Fz, R& rho,
                                             R& ux, R& uy, R& uz) {
  R jx = R(0), jy = R(0), jz = R(0);
  rho = R(0);
#pragma unroll
  for (int a = 0; a < Q; ++a) {
    const Vel e = Lattice<Q>::e(a);
    const R v = fpre[uint64_t(a) * N + n];
    rho += v;
    jx += R(e.x) * v;
    jy += R(e.y) * v;
    jz += R(e.z) * v;
  }
  const R inv = R(1) / rho;
  ux = (jx + R(0.5) * Fx) * inv;
  uy = (jy + R(0.5) * Fy) * inv;
  uz = (jz + R(0.5) * Fz) * inv;
}

template <int Q, typename R>
__global__ __launch_bounds__(256) void k_ke_sum(Geom g, const R* fpre, const uint8_t* mask, ForceArgs<R> force,
                                                double* partials) {
  double acc[1] = {0};
  for (uint32_t n = blockIdx.x * blockDim.x + threadIdx.x; n < g.N; n += gridDim.x * blockDim.x) {
    if (mask && mask[n]) continue;
    R Fx, Fy, Fz;
    force_at(force, g.N, n, Fx, Fy, Fz);
    R rho, ux, uy, uz;
    node_moments<Q>(fpre, g.N, n, Fx, Fy, Fz, rho, ux, uy, uz);
    acc[0] += 0.5 * double(rho) * (double(ux) * ux + double(uy) * uy + double(uz) * uz);
  }
  __shared__ double sh[8];
  block_sum<1>(acc, sh);
  if (threadIdx.x == 0) partials[blockIdx.x] = acc[0];
}

template <int Q, typename R>
__global__ __launch_bounds__(256) void k_ke_seed(Geom g, const R* fpre, const uint8_t* mask, ForceArgs<R> force,
                                                 double scale, R* lam, double* dLdF, double* partials) {
  double acc[3] = {0, 0, 0};
  for (uint32_t n = blockIdx.x * blockDim.x + threadIdx.x; n < g.N; n += gridDim.x * blockDim.x) {
    if (mask && mask[n]) {
#pragma unroll
      for (int a = 0; a < Q; ++a) lam[uint64_t(a) * g.N + n] = R(0);
      continue;
    }
    R Fx, Fy, Fz;
    force_at(force, g.N, n, Fx, Fy, Fz);
    R rho, ux, uy, uz;
    node_moments<Q>(fpre, g.N, n, Fx, Fy, Fz, rho, ux, uy, uz);
    const R half_u2 = R(0.5) * (ux * ux + uy * uy + uz * uz);
    const R sc = R(scale);
#pragma unroll
    for (int a = 0; a < Q; ++a) {
      const Vel e = Lattice<Q>::e(a);
      lam[uint64_t(a) * g.N + n] = sc * (R(e.x) * ux + R(e.y) * uy + R(e.z) * uz - half_u2);
    }
    const double c = 0.5 * scale * double(force.scale);
    if (force.field) {
      dLdF[n] += c * double(ux);
      dLdF[g.N + n] += c * double(uy);
      dLdF[2 * g.N + n] += c * double(uz);
    } else {
      acc[0] += c * double(ux);
      acc[1] += c * double(uy);
      acc[2] += c * double(uz);
    }
  }
  __shared__ double sh[3 * 8];
  block_sum<3>(acc, sh);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < 3; ++i) partials[uint64_t(blockIdx.x) * 3 + i] = acc[i];
  }
}

// Adjoint of the initial condition fbar(x, 0) = f^eq(rho0, u0) - S(F, u0)/2
// with respect to F (D3Q27): S is the inverse-pass image of the central moments
// (0; F; 0, ...), so dL/dF = -(scale/2) (first-order rows of P(u0)^T lam0).
template <int Q, typename R>
__global__ __launch_bounds__(256) void k_init_adjoint(Geom g, const R* u0, const R* lam0, const uint8_t* mask,
                                                      ForceArgs<R> force, double* dLdF, double* partials) {
  double acc[3] = {0, 0, 0};
  for (uint32_t n = blockIdx.x * blockDim.x + threadIdx.x; n < g.N; n += gridDim.x * blockDim.x) {
    if (mask && mask[n]) continue;
    const R ux = u0[n], uy = u0[g.N + n], uz = u0[2 * g.N + n];
    R lam[Q];
#pragma unroll
    for (int a = 0; a < Q; ++a) lam[a] = lam0[uint64_t(a) * g.N + n];
    R gx_ = R(0), gy_ = R(0), gz_ = R(0);
    if constexpr (Q == 27)
      initial27_adj_force(ux, uy, uz, lam, gx_, gy_, gz_);
    else
      initial15_adj_force(ux, uy, uz, lam, gx_, gy_, gz_);
    const double c = double(force.scale);
    const double gx = c * double(gx_), gy = c * double(gy_), gz = c * double(gz_);
    if (force.field) {
      dLdF[n] += gx;
      dLdF[g.N + n] += gy;
      dLdF[2 * g.N + n] += gz;
    } else {
      acc[0] += gx;
      acc[1] += gy;
      acc[2] += gz;
    }
  }
  __shared__ double sh[3 * 8];
  block_sum<3>(acc, sh);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < 3; ++i) partials[uint64_t(blockIdx.x) * 3 + i] = acc[i];
  }
}

// ---------------------------------------------------------------------------
// Host-side launchers
// ---------------------------------------------------------------------------
namespace {

constexpr int kBlock = 256;

inline int step_block(const Geom& g) {
  int bx = CMLBM_STEP_BLOCK;
  if (g.nx < bx) bx = ((g.nx + 63) / 64) * 64;
  return bx;
}

inline dim3 step_grid(const Geom& g, int bx) {
  return dim3(unsigned((g.nx + bx - 1) / bx) * unsigned(g.ny) * unsigned(g.nz));
}

}  // namespace

uint64_t step_blocks(const Geom& g) { return step_grid(g, step_block(g)).x; }

// Scratch of the allocation-free fused-totals step (one copy per device).  In
// host code `scratch` names a host-side stand-in, not device memory: kernels
// get the device address that static_scratch() looks up.
static __device__ __align__(256) double scratch[kStaticScratchDoubles];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
double* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t static_scratch(double** out) {
  *out = nullptr;
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = static_cast<double*>(p);
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

namespace {

inline int adjoint_block(const Geom& g) { return g.nx < 256 ? ((g.nx + 63) / 64) * 64 : 256; }

inline unsigned aux_grid(const Geom& g) {
  const uint64_t need = (g.N + kBlock - 1) / kBlock;
  return unsigned(need < 8192 ? (need == 0 ? 1 : need) : 8192);
}

inline RowMap row_map(const Geom& g, int bx) {
  const uint32_t nseg = uint32_t((g.nx + bx - 1) / bx);
  return {nseg, Divider::of(nseg), Divider::of(uint32_t(g.ny))};
}

template <int Q, class ST>
hipError_t step_impl(const StepArgs<typename ST::R>& args, hipStream_t st) {
  const int bx = step_block(args.g);
  const dim3 grid = step_grid(args.g, bx);
  StepArgs<typename ST::R> a = args;
  a.rm = row_map(a.g, bx);
  if (!a.partials) {
    if (a.mask)
      hipLaunchKernelGGL((k_step<Q, ST, true, false>), grid, dim3(bx), 0, st, a);
    else
      hipLaunchKernelGGL((k_step<Q, ST, false, false>), grid, dim3(bx), 0, st, a);
    return hipGetLastError();
  }
  if (a.mask)
    hipLaunchKernelGGL((k_step<Q, ST, true, true>), grid, dim3(bx), 0, st, a);
  else
    hipLaunchKernelGGL((k_step<Q, ST, false, true>), grid, dim3(bx), 0, st, a);
  hipLaunchKernelGGL(k_reduce_chunks<4>, dim3(kReduceChunks), dim3(kBlock), 0, st, a.partials, uint64_t(grid.x),
                     a.stage);
  hipLaunchKernelGGL(k_reduce_rows, dim3(4), dim3(kBlock), 0, st, a.stage, kReduceChunks, 4, a.totals, 0);
  return hipGetLastError();
}

template <int Q, class ST, bool TOT>
void inplace_launch(const StepArgs<typename ST::R>& a, int parity, dim3 grid, int bx, hipStream_t st) {
  if (parity == 0) {
    if (a.mask)
      hipLaunchKernelGGL((k_step_inplace<Q, ST, true, false, TOT>), grid, dim3(bx), 0, st, a);
    else
      hipLaunchKernelGGL((k_step_inplace<Q, ST, false, false, TOT>), grid, dim3(bx), 0, st, a);
  } else {
    if (a.mask)
      hipLaunchKernelGGL((k_step_inplace<Q, ST, true, true, TOT>), grid, dim3(bx), 0, st, a);
    else if (CMLBM_ALIGNED_SCATTER == 2 || (CMLBM_ALIGNED_SCATTER == 1 && sizeof(typename ST::T) == 2))
      hipLaunchKernelGGL((k_scatter_periodic<Q, ST, TOT>), grid, dim3(bx), 0, st, a);
    else
      hipLaunchKernelGGL((k_step_inplace<Q, ST, false, true, TOT>), grid, dim3(bx), 0, st, a);
  }
}

template <int Q, class ST>
hipError_t inplace_impl(const StepArgs<typename ST::R>& args, int parity, hipStream_t st) {
  const int bx = step_block(args.g);
  const dim3 grid = step_grid(args.g, bx);
  StepArgs<typename ST::R> a = args;
  a.rm = row_map(a.g, bx);
  if (!a.partials) {
    inplace_launch<Q, ST, false>(a, parity, grid, bx, st);
    return hipGetLastError();
  }
  inplace_launch<Q, ST, true>(a, parity, grid, bx, st);
  hipLaunchKernelGGL(k_reduce_chunks<4>, dim3(kReduceChunks), dim3(kBlock), 0, st, a.partials, uint64_t(grid.x),
                     a.stage);
  hipLaunchKernelGGL(k_reduce_rows, dim3(4), dim3(kBlock), 0, st, a.stage, kReduceChunks, 4, a.totals, 0);
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
hipError_t convert_impl(const Geom& g, const void* in, void* out, bool to_soa, hipStream_t st) {
  if (to_soa)
    hipLaunchKernelGGL((k_convert<Q, ST, true>), dim3(aux_grid(g)), dim3(kBlock), 0, st, g, in, out);
  else
    hipLaunchKernelGGL((k_convert<Q, ST, false>), dim3(aux_grid(g)), dim3(kBlock), 0, st, g, in, out);
  return hipGetLastError();
}

template <int Q, class ST>
hipError_t macro_impl(const AuxArgs<typename ST::R>& a, bool pre, hipStream_t st) {
  const dim3 grid(aux_grid(a.g)), block(kBlock);
  if (pre && a.mask)
    hipLaunchKernelGGL((k_macro<Q, ST, true, true>), grid, block, 0, st, a);
  else if (pre)
    hipLaunchKernelGGL((k_macro<Q, ST, false, true>), grid, block, 0, st, a);
  else if (a.mask)
    hipLaunchKernelGGL((k_macro<Q, ST, true, false>), grid, block, 0, st, a);
  else
    hipLaunchKernelGGL((k_macro<Q, ST, false, false>), grid, block, 0, st, a);
  return hipGetLastError();
}

template <int Q, class ST>
hipError_t totals_impl(const AuxArgs<typename ST::R>& a, bool pre, double* partials, int nblk, double* out4,
                       hipStream_t st) {
  if (pre && a.mask)
    hipLaunchKernelGGL((k_totals<Q, ST, true, true>), dim3(nblk), dim3(kBlock), 0, st, a, partials);
  else if (pre)
    hipLaunchKernelGGL((k_totals<Q, ST, false, true>), dim3(nblk), dim3(kBlock), 0, st, a, partials);
  else if (a.mask)
    hipLaunchKernelGGL((k_totals<Q, ST, true, false>), dim3(nblk), dim3(kBlock), 0, st, a, partials);
  else
    hipLaunchKernelGGL((k_totals<Q, ST, false, false>), dim3(nblk), dim3(kBlock), 0, st, a, partials);
  hipLaunchKernelGGL(k_reduce_rows, dim3(4), dim3(kBlock), 0, st, partials, nblk, 4, out4, 0);
  return hipGetLastError();
}

template <int Q, class ST>
hipError_t init_impl(const Geom& g, const void* rho0, const void* u0, const ForceArgs<typename ST::R>& force,
                     const uint8_t* mask, void* fpre, void* fpost, hipStream_t st) {
  using R = typename ST::R;
  if (!fpost) {      // phase-0 in-place buffer only
    hipLaunchKernelGGL((k_initial_pre<Q, ST, true, R>), dim3(aux_grid(g)), dim3(kBlock), 0, st, g,
                       static_cast<const R*>(rho0), static_cast<const R*>(u0), force, mask, fpre);
    return hipGetLastError();
  }
  hipLaunchKernelGGL((k_initial_pre<Q, ST, false, R>), dim3(aux_grid(g)), dim3(kBlock), 0, st, g,
                     static_cast<const R*>(rho0), static_cast<const R*>(u0), force, mask, fpre);
  if (mask)
    hipLaunchKernelGGL((k_scatter_post<Q, ST, true>), dim3(aux_grid(g)), dim3(kBlock), 0, st, g,
                       static_cast<const R*>(fpre), mask, static_cast<typename ST::T*>(fpost));
  else
    hipLaunchKernelGGL((k_scatter_post<Q, ST, false>), dim3(aux_grid(g)), dim3(kBlock), 0, st, g,
                       static_cast<const R*>(fpre), mask, static_cast<typename ST::T*>(fpost));
  return hipGetLastError();
}

template <int Q, class ST>
hipError_t adjoint_impl(const AdjArgs<typename ST::R>& args, double* partials, int nblk, double* dLdomega,
                        double* dLdF_uniform, hipStream_t st) {
  const dim3 grid(nblk), block(adjoint_block(args.g));
  const AdjArgs<typename ST::R>& a = args;
  if (a.rates.per_mass) {
    if (a.mask)
      hipLaunchKernelGGL((k_adjoint<Q, ST, true, 1>), grid, block, 0, st, a, partials);
    else
      hipLaunchKernelGGL((k_adjoint<Q, ST, false, 1>), grid, block, 0, st, a, partials);
  } else {
    if (a.mask)
      hipLaunchKernelGGL((k_adjoint<Q, ST, true, 0>), grid, block, 0, st, a, partials);
    else
      hipLaunchKernelGGL((k_adjoint<Q, ST, false, 0>), grid, block, 0, st, a, partials);
  }
  // two stages: kReduceChunks blocks sum contiguous runs of block rows (all 26
  // columns), then one block per column adds the chunk sums into the outputs
  double* stage = partials + uint64_t(26) * uint64_t(nblk);
  hipLaunchKernelGGL(k_reduce_chunks<26>, dim3(kReduceChunks), dim3(kBlock), 0, st, partials, uint64_t(nblk), stage);
  hipLaunchKernelGGL(k_reduce_rows, dim3(Q - 4), dim3(kBlock), 0, st, stage, kReduceChunks, 26, dLdomega, 1);
  if (dLdF_uniform)
    hipLaunchKernelGGL(k_reduce_rows, dim3(3), dim3(kBlock), 0, st, stage + 23, kReduceChunks, 26, dLdF_uniform, 1);
  return hipGetLastError();
}

template <int Q, class ST>
hipError_t wall_sens_impl(const AdjArgs<typename ST::R>& a, double* dLdphi, bool post, hipStream_t st) {
  const dim3 grid(aux_grid(a.g)), block(kBlock);
  if (post) {
    const int bx = step_block(a.g);
    if (a.mask)
      hipLaunchKernelGGL((k_wall_gather<Q, ST, true>), step_grid(a.g, bx), dim3(bx), 0, st, a, dLdphi);
    else
      hipLaunchKernelGGL((k_wall_gather<Q, ST, false>), step_grid(a.g, bx), dim3(bx), 0, st, a, dLdphi);
  } else {
    if (a.mask)
      hipLaunchKernelGGL((k_wall_sens<Q, ST, true>), grid, block, 0, st, a, dLdphi);
    else
      hipLaunchKernelGGL((k_wall_sens<Q, ST, false>), grid, block, 0, st, a, dLdphi);
  }
  return hipGetLastError();
}

}  // namespace

// Dispatch on (Q, precision).
#define CMLBM_DISPATCH(PREC, CALL_F64, CALL_F32, CALL_F16, CALL_BF16) \
  switch (PREC) {                                                     \
    case 0: return CALL_F64;                                          \
    case 1: return CALL_F32;                                          \
    case 2: return CALL_F16;                                          \
    default: return CALL_BF16;                                        \
  }

hipError_t launch_step(int q, int prec, const StepArgs<double>& a64, const StepArgs<float>& a32, hipStream_t st) {
  if (q == 27) {
    CMLBM_DISPATCH(prec, (step_impl<27, StF64>(a64, st)), (step_impl<27, StF32>(a32, st)),
                   (step_impl<27, StF16>(a32, st)), (step_impl<27, StBF16>(a32, st)))
  }
  CMLBM_DISPATCH(prec, (step_impl<15, StF64>(a64, st)), (step_impl<15, StF32>(a32, st)),
                 (step_impl<15, StF16>(a32, st)), (step_impl<15, StBF16>(a32, st)))
}

hipError_t launch_step_inplace(int q, int prec, const StepArgs<double>& a64, const StepArgs<float>& a32, int parity,
                              hipStream_t st) {
  if (q == 27) {
    CMLBM_DISPATCH(prec, (inplace_impl<27, StF64>(a64, parity, st)), (inplace_impl<27, StF32>(a32, parity, st)),
                   (inplace_impl<27, StF16>(a32, parity, st)), (inplace_impl<27, StBF16>(a32, parity, st)))
  }
  CMLBM_DISPATCH(prec, (inplace_impl<15, StF64>(a64, parity, st)), (inplace_impl<15, StF32>(a32, parity, st)),
                 (inplace_impl<15, StF16>(a32, parity, st)), (inplace_impl<15, StBF16>(a32, parity, st)))
}

hipError_t launch_gather(int q, int prec, const AuxArgs<double>& a64, const AuxArgs<float>& a32, hipStream_t st) {
  if (q == 27) {
    CMLBM_DISPATCH(prec, (gather_impl<27, StF64>(a64, st)), (gather_impl<27, StF32>(a32, st)),
                   (gather_impl<27, StF16>(a32, st)), (gather_impl<27, StBF16>(a32, st)))
  }
  CMLBM_DISPATCH(prec, (gather_impl<15, StF64>(a64, st)), (gather_impl<15, StF32>(a32, st)),
                 (gather_impl<15, StF16>(a32, st)), (gather_impl<15, StBF16>(a32, st)))
}

hipError_t launch_convert(int q, int prec, const Geom& g, const void* in, void* out, bool to_soa, hipStream_t st) {
  if (q == 27) {
    CMLBM_DISPATCH(prec, (convert_impl<27, StF64>(g, in, out, to_soa, st)),
                   (convert_impl<27, StF32>(g, in, out, to_soa, st)),
                   (convert_impl<27, StF16>(g, in, out, to_soa, st)),
                   (convert_impl<27, StBF16>(g, in, out, to_soa, st)))
  }
  CMLBM_DISPATCH(prec, (convert_impl<15, StF64>(g, in, out, to_soa, st)),
                 (convert_impl<15, StF32>(g, in, out, to_soa, st)),
                 (convert_impl<15, StF16>(g, in, out, to_soa, st)),
                 (convert_impl<15, StBF16>(g, in, out, to_soa, st)))
}

hipError_t launch_macro(int q, int prec, const AuxArgs<double>& a64, const AuxArgs<float>& a32, bool pre,
                        hipStream_t st) {
  if (q == 27) {
    CMLBM_DISPATCH(prec, (macro_impl<27, StF64>(a64, pre, st)), (macro_impl<27, StF32>(a32, pre, st)),
                   (macro_impl<27, StF16>(a32, pre, st)), (macro_impl<27, StBF16>(a32, pre, st)))
  }
  CMLBM_DISPATCH(prec, (macro_impl<15, StF64>(a64, pre, st)), (macro_impl<15, StF32>(a32, pre, st)),
                 (macro_impl<15, StF16>(a32, pre, st)), (macro_impl<15, StBF16>(a32, pre, st)))
}

hipError_t launch_totals(int q, int prec, const AuxArgs<double>& a64, const AuxArgs<float>& a32, bool pre,
                         double* partials, int nblk, double* out4, hipStream_t st) {
  if (q == 27) {
    CMLBM_DISPATCH(prec, (totals_impl<27, StF64>(a64, pre, partials, nblk, out4, st)),
                   (totals_impl<27, StF32>(a32, pre, partials, nblk, out4, st)),
                   (totals_impl<27, StF16>(a32, pre, partials, nblk, out4, st)),
                   (totals_impl<27, StBF16>(a32, pre, partials, nblk, out4, st)))
  }
  CMLBM_DISPATCH(prec, (totals_impl<15, StF64>(a64, pre, partials, nblk, out4, st)),
                 (totals_impl<15, StF32>(a32, pre, partials, nblk, out4, st)),
                 (totals_impl<15, StF16>(a32, pre, partials, nblk, out4, st)),
                 (totals_impl<15, StBF16>(a32, pre, partials, nblk, out4, st)))
}

hipError_t launch_init(int q, int prec, const Geom& g, const void* rho0, const void* u0, const ForceArgs<double>& f64,
                       const ForceArgs<float>& f32, const uint8_t* mask, void* fpre, void* fpost, hipStream_t st) {
  if (q == 27) {
    CMLBM_DISPATCH(prec, (init_impl<27, StF64>(g, rho0, u0, f64, mask, fpre, fpost, st)),
                   (init_impl<27, StF32>(g, rho0, u0, f32, mask, fpre, fpost, st)),
                   (init_impl<27, StF16>(g, rho0, u0, f32, mask, fpre, fpost, st)),
                   (init_impl<27, StBF16>(g, rho0, u0, f32, mask, fpre, fpost, st)))
  }
  CMLBM_DISPATCH(prec, (init_impl<15, StF64>(g, rho0, u0, f64, mask, fpre, fpost, st)),
                 (init_impl<15, StF32>(g, rho0, u0, f32, mask, fpre, fpost, st)),
                 (init_impl<15, StF16>(g, rho0, u0, f32, mask, fpre, fpost, st)),
                 (init_impl<15, StBF16>(g, rho0, u0, f32, mask, fpre, fpost, st)))
}

hipError_t launch_adjoint(int q, int prec, const AdjArgs<double>& a64, const AdjArgs<float>& a32, double* partials,
                          int nblk, double* dLdomega, double* dLdF_uniform, hipStream_t st) {
  if (q == 27) {
    CMLBM_DISPATCH(prec, (adjoint_impl<27, StF64>(a64, partials, nblk, dLdomega, dLdF_uniform, st)),
                   (adjoint_impl<27, StF32>(a32, partials, nblk, dLdomega, dLdF_uniform, st)),
                   (adjoint_impl<27, StF16>(a32, partials, nblk, dLdomega, dLdF_uniform, st)),
                   (adjoint_impl<27, StBF16>(a32, partials, nblk, dLdomega, dLdF_uniform, st)))
  }
  CMLBM_DISPATCH(prec, (adjoint_impl<15, StF64>(a64, partials, nblk, dLdomega, dLdF_uniform, st)),
                 (adjoint_impl<15, StF32>(a32, partials, nblk, dLdomega, dLdF_uniform, st)),
                 (adjoint_impl<15, StF16>(a32, partials, nblk, dLdomega, dLdF_uniform, st)),
                 (adjoint_impl<15, StBF16>(a32, partials, nblk, dLdomega, dLdF_uniform, st)))
}

hipError_t launch_wall_sensitivity(int q, int prec, const AdjArgs<double>& a64, const AdjArgs<float>& a32,
                                   double* dLdphi, bool post, hipStream_t st) {
  if (q == 27) {
    CMLBM_DISPATCH(prec, (wall_sens_impl<27, StF64>(a64, dLdphi, post, st)),
                   (wall_sens_impl<27, StF32>(a32, dLdphi, post, st)), (wall_sens_impl<27, StF16>(a32, dLdphi, post, st)),
                   (wall_sens_impl<27, StBF16>(a32, dLdphi, post, st)))
  }
  CMLBM_DISPATCH(prec, (wall_sens_impl<15, StF64>(a64, dLdphi, post, st)),
                 (wall_sens_impl<15, StF32>(a32, dLdphi, post, st)), (wall_sens_impl<15, StF16>(a32, dLdphi, post, st)),
                 (wall_sens_impl<15, StBF16>(a32, dLdphi, post, st)))
}

#undef CMLBM_DISPATCH

namespace {
template <int Q, typename R>
hipError_t ke_sum_impl(const Geom& g, const void* fpre, const uint8_t* mask, const ForceArgs<R>& f, double* partials,
                       int nblk, double* out, hipStream_t st) {
  hipLaunchKernelGGL((k_ke_sum<Q, R>), dim3(nblk), dim3(kBlock), 0, st, g, static_cast<const R*>(fpre), mask, f,
                     partials);
  hipLaunchKernelGGL(k_reduce_rows, dim3(1), dim3(kBlock), 0, st, partials, nblk, 1, out, 0);
  return hipGetLastError();
}
template <int Q, typename R>
hipError_t ke_seed_impl(const Geom& g, const void* fpre, const uint8_t* mask, const ForceArgs<R>& f, double scale,
                        void* lam, double* dLdF, double* partials, int nblk, hipStream_t st) {
  hipLaunchKernelGGL((k_ke_seed<Q, R>), dim3(nblk), dim3(kBlock), 0, st, g, static_cast<const R*>(fpre), mask, f,
                     scale, static_cast<R*>(lam), dLdF, partials);
  if (!f.field) hipLaunchKernelGGL(k_reduce_rows, dim3(3), dim3(kBlock), 0, st, partials, nblk, 3, dLdF, 1);
  return hipGetLastError();
}
template <int Q, typename R>
hipError_t init_adj_impl(const Geom& g, const void* u0, const void* lam0, const uint8_t* mask, const ForceArgs<R>& f,
                         double* dLdF, double* partials, int nblk, hipStream_t st) {
  hipLaunchKernelGGL((k_init_adjoint<Q, R>), dim3(nblk), dim3(kBlock), 0, st, g, static_cast<const R*>(u0),
                     static_cast<const R*>(lam0), mask, f, dLdF, partials);
  if (!f.field) hipLaunchKernelGGL(k_reduce_rows, dim3(3), dim3(kBlock), 0, st, partials, nblk, 3, dLdF, 1);
  return hipGetLastError();
}
}  // namespace

hipError_t launch_ke_sum(int q, int prec, const Geom& g, const void* fpre, const uint8_t* mask,
                         const ForceArgs<double>& f64, const ForceArgs<float>& f32, double* partials, int nblk,
                         double* out, hipStream_t st) {
  if (prec == 0)
    return q == 27 ? ke_sum_impl<27>(g, fpre, mask, f64, partials, nblk, out, st)
                   : ke_sum_impl<15>(g, fpre, mask, f64, partials, nblk, out, st);
  return q == 27 ? ke_sum_impl<27>(g, fpre, mask, f32, partials, nblk, out, st)
                 : ke_sum_impl<15>(g, fpre, mask, f32, partials, nblk, out, st);
}

hipError_t launch_ke_seed(int q, int prec, const Geom& g, const void* fpre, const uint8_t* mask,
                          const ForceArgs<double>& f64, const ForceArgs<float>& f32, double scale, void* lam,
                          double* dLdF, double* partials, int nblk, hipStream_t st) {
  if (prec == 0)
    return q == 27 ? ke_seed_impl<27>(g, fpre, mask, f64, scale, lam, dLdF, partials, nblk, st)
                   : ke_seed_impl<15>(g, fpre, mask, f64, scale, lam, dLdF, partials, nblk, st);
  return q == 27 ? ke_seed_impl<27>(g, fpre, mask, f32, scale, lam, dLdF, partials, nblk, st)
                 : ke_seed_impl<15>(g, fpre, mask, f32, scale, lam, dLdF, partials, nblk, st);
}

hipError_t launch_init_adjoint(int q, int prec, const Geom& g, const void* u0, const void* lam0,
                               const uint8_t* mask, const ForceArgs<double>& f64, const ForceArgs<float>& f32,
                               double* dLdF, double* partials, int nblk, hipStream_t st) {
  if (prec == 0)
    return q == 27 ? init_adj_impl<27, double>(g, u0, lam0, mask, f64, dLdF, partials, nblk, st)
                   : init_adj_impl<15, double>(g, u0, lam0, mask, f64, dLdF, partials, nblk, st);
  return q == 27 ? init_adj_impl<27, float>(g, u0, lam0, mask, f32, dLdF, partials, nblk, st)
                 : init_adj_impl<15, float>(g, u0, lam0, mask, f32, dLdF, partials, nblk, st);
}

uint64_t max_work_items(const Geom& g) {
  const uint64_t step = uint64_t(step_grid(g, step_block(g)).x) * uint64_t(step_block(g));
  const uint64_t adj = uint64_t(adjoint_blocks(g)) * uint64_t(adjoint_block(g));
  return step > adj ? step : adj;
}

}  // namespace cmlbm
