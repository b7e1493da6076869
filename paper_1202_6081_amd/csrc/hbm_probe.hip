// HBM rate probes for the roofline: the rates this device sustains for plain
// streams, for streams with exactly the step's memory traffic (27 population
// loads in the blocked row layout, 3 force loads, 27 nontemporal population
// stores per node), and for the adjoint step's (the same pull, 27 adjoint
// loads gathered from the downstream neighbours and 27 adjoint stores in
// structure-of-arrays layout, the force, and a read-modify-write of the FP64
// force gradient), with no arithmetic of the method.  A standalone program;
// prints one JSON line.
//
//   hbm_probe [n]        n^3 nodes for the stencil probes (n a multiple of 256; default 512)
//
// The plain streams come in several flavours (4, 8 and 16 bytes per lane;
// plain, nontemporal and system-coherent cache policies; one pass over the
// buffer, each work-group moving one contiguous chunk, or a grid-stride loop
// of 8192 work-groups); each stream's best flavour is the ceiling reported.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>

namespace {

constexpr int kQ = 27;
constexpr int kBlock = 256;

#define PROBE_CHECK(x)                                                                   \
  do {                                                                                   \
    const hipError_t e_ = (x);                                                           \
    if (e_ != hipSuccess) {                                                              \
      std::fprintf(stderr, "hbm_probe: %s at line %d\n", hipGetErrorString(e_), __LINE__); \
      std::exit(1);                                                                      \
    }                                                                                    \
  } while (0)

typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// Cache-policy bits of gfx950 buffer instructions: 0 plain, 2 nontemporal,
// 16 system coherent (sc1), 17 sc0 + sc1.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t chunk_rsrc(const char* base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<char*>(base), (short)0, int(bytes), 0x00020000);
}

template <int W, int AUX>
__device__ __forceinline__ void st_lane(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t v) {
  if constexpr (W == 4)
    __builtin_amdgcn_raw_buffer_store_b32(v, r, voff, 0, AUX);
  else if constexpr (W == 8)
    __builtin_amdgcn_raw_buffer_store_b64(u32x2{v, v}, r, voff, 0, AUX);
  else
    __builtin_amdgcn_raw_buffer_store_b128(u32x4{v, v, v, v}, r, voff, 0, AUX);
}

template <int W, int AUX>
__device__ __forceinline__ uint32_t ld_lane(__amdgpu_buffer_rsrc_t r, uint32_t voff) {
  if constexpr (W == 4) {
    return __builtin_amdgcn_raw_buffer_load_b32(r, voff, 0, AUX);
  } else if constexpr (W == 8) {
    const u32x2 t = __builtin_amdgcn_raw_buffer_load_b64(r, voff, 0, AUX);
    return t.x ^ t.y;
  } else {
    const u32x4 t = __builtin_amdgcn_raw_buffer_load_b128(r, voff, 0, AUX);
    return (t.x ^ t.y) ^ (t.z ^ t.w);
  }
}

// Plain streams over nchunks chunks of kBlock * W bytes; work-group g moves
// chunks g, g + gridDim.x, ... (one pass when the grid has a work-group per
// chunk).  The read stream's sink store is never taken (the buffer holds
// zeros) but keeps the loads live.
template <int W, int AUX>
__global__ __launch_bounds__(kBlock) void k_read(const char* a, size_t nchunks, uint32_t* sink) {
  uint32_t s = 0;
  for (size_t c = blockIdx.x; c < nchunks; c += gridDim.x)
    s ^= ld_lane<W, AUX>(chunk_rsrc(a + c * (kBlock * W), kBlock * W), threadIdx.x * W);
  if (s == 0x5a5a5a5au) sink[0] = s;
}

template <int W, int AUX>
__global__ __launch_bounds__(kBlock) void k_write(char* b, size_t nchunks) {
  for (size_t c = blockIdx.x; c < nchunks; c += gridDim.x)
    st_lane<W, AUX>(chunk_rsrc(b + c * (kBlock * W), kBlock * W), threadIdx.x * W, uint32_t(c));
}

template <int W, int LAUX, int SAUX>
__global__ __launch_bounds__(kBlock) void k_copy(const char* a, char* b, size_t nchunks) {
  for (size_t c = blockIdx.x; c < nchunks; c += gridDim.x)
    st_lane<W, SAUX>(chunk_rsrc(b + c * (kBlock * W), kBlock * W), threadIdx.x * W,
                     ld_lane<W, LAUX>(chunk_rsrc(a + c * (kBlock * W), kBlock * W), threadIdx.x * W));
}

__device__ __forceinline__ uint32_t wrap(int v, uint32_t n) {
  return v < 0 ? uint32_t(v + int(n)) : (uint32_t(v) >= n ? uint32_t(v) - n : uint32_t(v));
}

// Blocked row layout: row r holds 27 * nx floats; x is cut into 64-node
// blocks, each storing its 27 directions one after the other.
__device__ __forceinline__ uint64_t slot(uint32_t row, uint32_t nx, int a, uint32_t x) {
  return uint64_t(row) * nx * kQ + uint64_t(x >> 6) * (64 * kQ) + uint32_t(a) * 64u + (x & 63u);
}

// One thread per node, 256 nodes of one row per block, rows dealt to the 8
// XCDs in contiguous runs.  PULL: direction a is read from the node at x - e_a
// (periodic), as the pull step reads; otherwise from the node itself, so every
// wavefront load covers whole cache lines.
template <bool PULL>
__global__ __launch_bounds__(kBlock) void k_stencil(const float* fin, const float* force, float* fout,
                                                   uint32_t nx, uint32_t ny, uint32_t nz) {
  uint32_t L = blockIdx.x;
  const uint32_t per = gridDim.x >> 3;
  if (L < (per << 3)) L = (L & 7u) * per + (L >> 3);
  const uint32_t nseg = nx / kBlock;
  const uint32_t row = L / nseg;
  const uint32_t x = (L - row * nseg) * kBlock + threadIdx.x;
  const uint32_t y = row % ny, z = row / ny;
  const uint64_t N = uint64_t(nx) * ny * nz;
  const uint64_t node = uint64_t(row) * nx + x;
  float v[kQ];
  int a = 0;
#pragma unroll
  for (int ez = -1; ez <= 1; ++ez)
#pragma unroll
    for (int ey = -1; ey <= 1; ++ey)
#pragma unroll
      for (int ex = -1; ex <= 1; ++ex, ++a) {
        if (PULL) {
          const uint32_t r = wrap(int(z) - ez, nz) * ny + wrap(int(y) - ey, ny);
          v[a] = fin[slot(r, nx, a, wrap(int(x) - ex, nx))];
        } else {
          v[a] = fin[slot(row, nx, a, x)];
        }
      }
  const float s = force[node] + force[N + node] + force[2 * N + node];
#pragma unroll
  for (int b = 0; b < kQ; ++b) __builtin_nontemporal_store(v[b] + s, &fout[slot(row, nx, b, x)]);
}

// The adjoint step's traffic: fpost pulled as in the step; lam_next[a] read
// at x + e_a (structure of arrays [27][N]); lam[a] and the three FP64
// gradient components written at x, the gradient read first.
__global__ __launch_bounds__(kBlock) void k_adjoint_traffic(const float* fpost, const float* lam_next, float* lam,
                                                           const float* force, double* dLdF, uint32_t nx, uint32_t ny,
                                                           uint32_t nz) {
  uint32_t L = blockIdx.x;
  const uint32_t per = gridDim.x >> 3;
  if (L < (per << 3)) L = (L & 7u) * per + (L >> 3);
  const uint32_t nseg = nx / kBlock;
  const uint32_t row = L / nseg;
  const uint32_t x = (L - row * nseg) * kBlock + threadIdx.x;
  const uint32_t y = row % ny, z = row / ny;
  const uint64_t N = uint64_t(nx) * ny * nz;
  const uint64_t node = uint64_t(row) * nx + x;
  float f[kQ], g[kQ];
  int a = 0;
#pragma unroll
  for (int ez = -1; ez <= 1; ++ez)
#pragma unroll
    for (int ey = -1; ey <= 1; ++ey)
#pragma unroll
      for (int ex = -1; ex <= 1; ++ex, ++a) {
        const uint32_t up = wrap(int(z) - ez, nz) * ny + wrap(int(y) - ey, ny);
        f[a] = fpost[slot(up, nx, a, wrap(int(x) - ex, nx))];
        const uint32_t dn = wrap(int(z) + ez, nz) * ny + wrap(int(y) + ey, ny);
        g[a] = lam_next[uint64_t(a) * N + uint64_t(dn) * nx + wrap(int(x) + ex, nx)];
      }
  const float s = force[node] + force[N + node] + force[2 * N + node];
  float t = 0.f;
#pragma unroll
  for (int b = 0; b < kQ; ++b) t += f[b];
#pragma unroll
  for (int b = 0; b < kQ; ++b) __builtin_nontemporal_store(g[b] + t + s, &lam[uint64_t(b) * N + node]);
#pragma unroll
  for (int c = 0; c < 3; ++c)
    __builtin_nontemporal_store(dLdF[uint64_t(c) * N + node] + double(t), &dLdF[uint64_t(c) * N + node]);
}

template <class Launch>
double time_ms(hipEvent_t e0, hipEvent_t e1, int reps, Launch launch) {
  for (int i = 0; i < 3; ++i) launch();
  PROBE_CHECK(hipGetLastError());
  PROBE_CHECK(hipEventRecord(e0));
  for (int i = 0; i < reps; ++i) launch();
  PROBE_CHECK(hipEventRecord(e1));
  PROBE_CHECK(hipEventSynchronize(e1));
  float ms = 0.f;
  PROBE_CHECK(hipEventElapsedTime(&ms, e0, e1));
  return double(ms) / reps;
}

}  // namespace

int main(int argc, char** argv) {
  const long n = argc > 1 ? std::atol(argv[1]) : 512;
  if (n < kBlock || n % kBlock != 0 || n > 1024) {
    std::fprintf(stderr, "hbm_probe: n must be a multiple of %d in [%d, 1024]\n", kBlock, kBlock);
    return 2;
  }
  const uint32_t nx = uint32_t(n), ny = uint32_t(n), nz = uint32_t(n);
  const uint64_t N = uint64_t(nx) * ny * nz;
  const size_t pop_bytes = size_t(kQ) * N * sizeof(float);
  const size_t force_bytes = size_t(3) * N * sizeof(float);
  float *fin = nullptr, *fout = nullptr, *force = nullptr;
  uint32_t* sink = nullptr;
  PROBE_CHECK(hipMalloc(&fin, pop_bytes));
  PROBE_CHECK(hipMalloc(&fout, pop_bytes));
  PROBE_CHECK(hipMalloc(&force, force_bytes));
  PROBE_CHECK(hipMalloc(&sink, sizeof(uint32_t)));
  PROBE_CHECK(hipMemset(fin, 0, pop_bytes));
  PROBE_CHECK(hipMemset(fout, 0, pop_bytes));
  PROBE_CHECK(hipMemset(force, 0, force_bytes));
  hipEvent_t e0, e1;
  PROBE_CHECK(hipEventCreate(&e0));
  PROBE_CHECK(hipEventCreate(&e1));

  // plain streams over the first 4 GiB (at most) of the population buffers,
  // each in several flavours: "name" -> GB/s, and the best of each stream
  const size_t stream_bytes = (pop_bytes < (size_t(4) << 30) ? pop_bytes : (size_t(4) << 30)) & ~size_t(4095);
  const dim3 block(kBlock);
  const char* ca = reinterpret_cast<const char*>(fin);
  char* cb = reinterpret_cast<char*>(fout);
  std::string flavours;
  double best_read = 0, best_write = 0, best_copy = 0;
  auto flavour = [&](const char* name, double bytes, double ms, double& best) {
    const double g = bytes / (ms * 1e-3) / 1e9;
    if (g > best) best = g;
    char buf[96];
    std::snprintf(buf, sizeof(buf), "%s\"%s\": %.1f", flavours.empty() ? "" : ", ", name, g);
    flavours += buf;
  };
#define PROBE_STREAMS(W, ONEPASS, TAG)                                                                           \
  {                                                                                                              \
    const size_t nc = stream_bytes / (kBlock * W);                                                               \
    const dim3 g(ONEPASS ? unsigned(nc) : 8192u);                                                                \
    const double sb = double(stream_bytes);                                                                      \
    flavour("read_" TAG "_plain", sb, time_ms(e0, e1, 10, [&] {                                                  \
      hipLaunchKernelGGL((k_read<W, 0>), g, block, 0, 0, ca, nc, sink); }), best_read);                           \
    flavour("read_" TAG "_nt", sb, time_ms(e0, e1, 10, [&] {                                                     \
      hipLaunchKernelGGL((k_read<W, 2>), g, block, 0, 0, ca, nc, sink); }), best_read);                           \
    flavour("write_" TAG "_plain", sb, time_ms(e0, e1, 10, [&] {                                                 \
      hipLaunchKernelGGL((k_write<W, 0>), g, block, 0, 0, cb, nc); }), best_write);                               \
    flavour("write_" TAG "_nt", sb, time_ms(e0, e1, 10, [&] {                                                    \
      hipLaunchKernelGGL((k_write<W, 2>), g, block, 0, 0, cb, nc); }), best_write);                               \
    flavour("write_" TAG "_sc1", sb, time_ms(e0, e1, 10, [&] {                                                   \
      hipLaunchKernelGGL((k_write<W, 16>), g, block, 0, 0, cb, nc); }), best_write);                              \
    flavour("copy_" TAG "_plain", 2 * sb, time_ms(e0, e1, 10, [&] {                                              \
      hipLaunchKernelGGL((k_copy<W, 0, 0>), g, block, 0, 0, ca, cb, nc); }), best_copy);                          \
    flavour("copy_" TAG "_nt", 2 * sb, time_ms(e0, e1, 10, [&] {                                                 \
      hipLaunchKernelGGL((k_copy<W, 2, 2>), g, block, 0, 0, ca, cb, nc); }), best_copy);                          \
  }
  PROBE_STREAMS(4, false, "w4_stride")
  PROBE_STREAMS(8, true, "w8_onepass")
  PROBE_STREAMS(8, false, "w8_stride")
  PROBE_STREAMS(16, true, "w16_onepass")
  PROBE_STREAMS(16, false, "w16_stride")
#undef PROBE_STREAMS

  // the step's traffic: 228 bytes per node
  const dim3 grid(unsigned(N / kBlock));
  const double ms_pull = time_ms(e0, e1, 20, [&] {
    hipLaunchKernelGGL(k_stencil<true>, grid, block, 0, 0, fin, force, fout, nx, ny, nz);
  });
  const double ms_own = time_ms(e0, e1, 20, [&] {
    hipLaunchKernelGGL(k_stencil<false>, grid, block, 0, 0, fin, force, fout, nx, ny, nz);
  });
  PROBE_CHECK(hipFree(fout));
  fout = nullptr;

  // the adjoint step's traffic: 384 bytes per node, where its buffers fit
  float *lam_next = nullptr, *lam = nullptr;
  double* dLdF = nullptr;
  const size_t grad_bytes = size_t(3) * N * sizeof(double);
  size_t free_b = 0, total_b = 0;
  PROBE_CHECK(hipMemGetInfo(&free_b, &total_b));
  char adj_json[128];
  std::snprintf(adj_json, sizeof(adj_json), "\"adjoint_traffic_ms\": null, \"adjoint_traffic_GBs\": null");
  if (2 * pop_bytes + grad_bytes + (size_t(1) << 30) < free_b) {
    PROBE_CHECK(hipMalloc(&lam_next, pop_bytes));
    PROBE_CHECK(hipMalloc(&lam, pop_bytes));
    PROBE_CHECK(hipMalloc(&dLdF, grad_bytes));
    PROBE_CHECK(hipMemset(lam_next, 0, pop_bytes));
    PROBE_CHECK(hipMemset(lam, 0, pop_bytes));
    PROBE_CHECK(hipMemset(dLdF, 0, grad_bytes));
    const double ms_adj = time_ms(e0, e1, 20, [&] {
      hipLaunchKernelGGL(k_adjoint_traffic, grid, block, 0, 0, fin, lam_next, lam, force, dLdF, nx, ny, nz);
    });
    const double adj_bytes = double(3 * kQ + 3) * sizeof(float) + 6.0 * sizeof(double);
    std::snprintf(adj_json, sizeof(adj_json), "\"adjoint_traffic_ms\": %.4f, \"adjoint_traffic_GBs\": %.1f", ms_adj,
                  adj_bytes * double(N) / (ms_adj * 1e-3) / 1e9);
    PROBE_CHECK(hipFree(lam_next));
    PROBE_CHECK(hipFree(lam));
    PROBE_CHECK(hipFree(dLdF));
  }

  const double node_bytes = double(2 * kQ + 3) * sizeof(float);
  auto gbs = [](double bytes, double ms) { return bytes / (ms * 1e-3) / 1e9; };
  std::printf(
      "{\"nodes\": %llu, \"read_GBs\": %.1f, \"write_GBs\": %.1f, \"copy_GBs\": %.1f, "
      "\"step_traffic_pull_ms\": %.4f, \"step_traffic_pull_GBs\": %.1f, "
      "\"step_traffic_own_node_ms\": %.4f, \"step_traffic_own_node_GBs\": %.1f, %s, \"stream_flavours_GBs\": {%s}}\n",
      static_cast<unsigned long long>(N), best_read, best_write, best_copy, ms_pull, gbs(node_bytes * double(N), ms_pull),
      ms_own, gbs(node_bytes * double(N), ms_own), adj_json, flavours.c_str());
  PROBE_CHECK(hipFree(fin));
  PROBE_CHECK(hipFree(force));
  PROBE_CHECK(hipFree(sink));
  return 0;
}
