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
//   hbm_probe placement  the step's traffic at 512^3 on buffers placed three ways (one
//                        JSON line each): the process's first allocations, buffers carved
//                        from one 150 GiB allocation, and new allocations made after all of
//                        that memory was released
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>

namespace {

constexpr int kQ = 27;
constexpr int kBlock = 256;
typedef float f4 __attribute__((ext_vector_type(4)));

#define PROBE_CHECK(x)                                                                   \
  do {                                                                                   \
    const hipError_t e_ = (x);                                                           \
    if (e_ != hipSuccess) {                                                              \
      std::fprintf(stderr, "hbm_probe: %s at line %d\n", hipGetErrorString(e_), __LINE__); \
      std::exit(1);                                                                      \
    }                                                                                    \
  } while (0)

__global__ __launch_bounds__(kBlock) void k_read(const f4* a, size_t n4, float* sink) {
  float s = 0.f;
  for (size_t i = size_t(blockIdx.x) * kBlock + threadIdx.x; i < n4; i += size_t(gridDim.x) * kBlock) {
    const f4 v = a[i];
    s += (v.x + v.y) + (v.z + v.w);
  }
  if (s == -1.f) sink[0] = s;   // the buffer holds zeros: never taken, keeps the loads live
}

__global__ __launch_bounds__(kBlock) void k_write(f4* b, size_t n4) {
  for (size_t i = size_t(blockIdx.x) * kBlock + threadIdx.x; i < n4; i += size_t(gridDim.x) * kBlock)
    __builtin_nontemporal_store(f4{0.f, 0.f, 0.f, 0.f}, &b[i]);
}

__global__ __launch_bounds__(kBlock) void k_copy(const f4* a, f4* b, size_t n4) {
  for (size_t i = size_t(blockIdx.x) * kBlock + threadIdx.x; i < n4; i += size_t(gridDim.x) * kBlock)
    __builtin_nontemporal_store(a[i], &b[i]);
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

// The step's traffic at 512^3 (both directions between the two buffers) on
// buffers placed three ways.  The same kernel, the same bytes: only where the
// pages lie differs.
int placement_study() {
  const uint32_t n = 512;
  const uint64_t N = uint64_t(n) * n * n;
  const size_t pop = size_t(kQ) * N * sizeof(float), fb = size_t(3) * N * sizeof(float);
  hipEvent_t e0, e1;
  PROBE_CHECK(hipEventCreate(&e0));
  PROBE_CHECK(hipEventCreate(&e1));
  const dim3 grid(unsigned(N / kBlock)), block(kBlock);
  auto run = [&](const char* name, float* fa, float* fb_, float* force) {
    PROBE_CHECK(hipMemset(fa, 0, pop));
    PROBE_CHECK(hipMemset(fb_, 0, pop));
    PROBE_CHECK(hipMemset(force, 0, fb));
    const double ab = time_ms(e0, e1, 20, [&] {
      hipLaunchKernelGGL(k_stencil<true>, grid, block, 0, 0, fa, force, fb_, n, n, n);
    });
    const double ba = time_ms(e0, e1, 20, [&] {
      hipLaunchKernelGGL(k_stencil<true>, grid, block, 0, 0, fb_, force, fa, n, n, n);
    });
    std::printf("{\"placement\": \"%s\", \"ms_a_to_b\": %.4f, \"ms_b_to_a\": %.4f, \"GBs\": %.1f}\n", name, ab,
                ba, 228.0 * double(N) / (0.5 * (ab + ba) * 1e-3) / 1e9);
    std::fflush(stdout);
  };
  float *a = nullptr, *b = nullptr, *f = nullptr;
  PROBE_CHECK(hipMalloc(&a, pop));
  PROBE_CHECK(hipMalloc(&b, pop));
  PROBE_CHECK(hipMalloc(&f, fb));
  run("first allocations", a, b, f);
  const size_t big = size_t(150) << 30;   // room for the three buffers many times over
  char* pool = nullptr;
  PROBE_CHECK(hipMalloc(&pool, big));
  run("carved from one 150 GiB allocation", reinterpret_cast<float*>(pool), reinterpret_cast<float*>(pool + pop),
      reinterpret_cast<float*>(pool + 2 * pop));
  PROBE_CHECK(hipFree(a));
  PROBE_CHECK(hipFree(b));
  PROBE_CHECK(hipFree(f));
  PROBE_CHECK(hipFree(pool));
  PROBE_CHECK(hipMalloc(&a, pop));
  PROBE_CHECK(hipMalloc(&b, pop));
  PROBE_CHECK(hipMalloc(&f, fb));
  run("allocated after releasing the above", a, b, f);
  PROBE_CHECK(hipFree(a));
  PROBE_CHECK(hipFree(b));
  PROBE_CHECK(hipFree(f));
  return 0;
}

}  // namespace

int main(int argc, char** argv) {
  if (argc > 1 && std::strcmp(argv[1], "placement") == 0) return placement_study();
  const long n = argc > 1 ? std::atol(argv[1]) : 512;
  if (n < kBlock || n % kBlock != 0 || n > 1024) {
    std::fprintf(stderr, "hbm_probe: n must be a multiple of %d in [%d, 1024]\n", kBlock, kBlock);
    return 2;
  }
  const uint32_t nx = uint32_t(n), ny = uint32_t(n), nz = uint32_t(n);
  const uint64_t N = uint64_t(nx) * ny * nz;
  const size_t pop_bytes = size_t(kQ) * N * sizeof(float);
  const size_t force_bytes = size_t(3) * N * sizeof(float);
  float *fin = nullptr, *fout = nullptr, *force = nullptr, *sink = nullptr;
  PROBE_CHECK(hipMalloc(&fin, pop_bytes));
  PROBE_CHECK(hipMalloc(&fout, pop_bytes));
  PROBE_CHECK(hipMalloc(&force, force_bytes));
  PROBE_CHECK(hipMalloc(&sink, sizeof(float)));
  PROBE_CHECK(hipMemset(fin, 0, pop_bytes));
  PROBE_CHECK(hipMemset(fout, 0, pop_bytes));
  PROBE_CHECK(hipMemset(force, 0, force_bytes));
  hipEvent_t e0, e1;
  PROBE_CHECK(hipEventCreate(&e0));
  PROBE_CHECK(hipEventCreate(&e1));

  // plain streams over the first 4 GiB (at most) of the population buffers
  const size_t stream_bytes = (pop_bytes < (size_t(4) << 30) ? pop_bytes : (size_t(4) << 30)) & ~size_t(15);
  const size_t n4 = stream_bytes / sizeof(f4);
  const dim3 sgrid(8192), block(kBlock);
  const auto* a4 = reinterpret_cast<const f4*>(fin);
  auto* b4 = reinterpret_cast<f4*>(fout);
  const double ms_read = time_ms(e0, e1, 20, [&] { hipLaunchKernelGGL(k_read, sgrid, block, 0, 0, a4, n4, sink); });
  const double ms_write = time_ms(e0, e1, 20, [&] { hipLaunchKernelGGL(k_write, sgrid, block, 0, 0, b4, n4); });
  const double ms_copy = time_ms(e0, e1, 20, [&] { hipLaunchKernelGGL(k_copy, sgrid, block, 0, 0, a4, b4, n4); });

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
      "\"step_traffic_own_node_ms\": %.4f, \"step_traffic_own_node_GBs\": %.1f, %s}\n",
      static_cast<unsigned long long>(N), gbs(double(stream_bytes), ms_read), gbs(double(stream_bytes), ms_write),
      gbs(2.0 * double(stream_bytes), ms_copy), ms_pull, gbs(node_bytes * double(N), ms_pull), ms_own,
      gbs(node_bytes * double(N), ms_own), adj_json);
  PROBE_CHECK(hipFree(fin));
  PROBE_CHECK(hipFree(force));
  PROBE_CHECK(hipFree(sink));
  return 0;
}
