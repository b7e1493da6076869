// Count of the non-finite populations a buffer holds: the check for a run that
// has lost stability.  The relaxation rates of Sec. 7 must lie in (0, 2) and
// are tuned for stability rather than guaranteeing it; a single NaN spreads
// to every population of the node that pulls it and from there one node per
// step in every direction, so a periodic check catches a diverging run early.
// The 16-bit deviation formats also overflow: FP16 holds |fbar_a - w_a| up to
// 65504 and rounds beyond that to +-Inf.
#include <hip/hip_runtime.h>

#include "checks.hpp"

namespace cmlbm {
namespace {

constexpr int kCheckBlock = 256;
constexpr uint32_t kCheckMaxBlocks = 8192;

// Offset of direction a of node x inside a row of the population buffer: a row
// holds its nodes in sub-blocks of 64 (the last one shorter when 64 does not
// divide nx), each sub-block storing its nodes' direction 0 first, then 1, ...
// (the layout the step kernels write).
template <int Q>
__device__ __forceinline__ uint32_t row_offset(uint32_t nx, int a, uint32_t x) {
  const uint32_t first = x & ~63u;
  const uint32_t width = min(64u, nx - first);
  return first * uint32_t(Q) + uint32_t(a) * width + (x - first);
}

__global__ void k_count_zero(unsigned long long* count) { *count = 0ull; }

// One node per thread (grid-stride): its Q stored values are checked against
// the exponent mask `ones` (a value is NaN or +-Inf iff all its exponent bits
// are set).  Each wavefront adds its total to the counter once, and only when
// it found something.
template <int Q, typename U>
__global__ __launch_bounds__(kCheckBlock) void k_check_finite(Geom g, const U* buf, const uint8_t* mask, U ones,
                                                              unsigned long long* count) {
  // N < 2^31 (the library's limit), so node indices and rows fit 32 bits
  const uint32_t nx = uint32_t(g.nx), N = uint32_t(g.N);
  const uint64_t rowQ = uint64_t(nx) * Q;
  uint32_t bad = 0;
  for (uint32_t n = blockIdx.x * blockDim.x + threadIdx.x; n < N; n += gridDim.x * blockDim.x) {
    if (mask && mask[n]) continue;
    const uint32_t row = n / nx;
    const uint32_t x = n - row * nx;
    const U* rp = buf + uint64_t(row) * rowQ;
#pragma unroll
    for (int a = 0; a < Q; ++a) bad += (rp[row_offset<Q>(nx, a, x)] & ones) == ones ? 1u : 0u;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) bad += __shfl_xor(bad, off, 64);
  if ((threadIdx.x & 63) == 0 && bad != 0) atomicAdd(count, (unsigned long long)bad);
}

template <int Q, typename U>
hipError_t check_impl(const Geom& g, const void* f_buf, const uint8_t* mask, U ones, unsigned long long* count,
                      hipStream_t st) {
  const uint64_t want = (g.N + kCheckBlock - 1) / kCheckBlock;
  const uint32_t blocks = uint32_t(want < kCheckMaxBlocks ? (want ? want : 1) : kCheckMaxBlocks);
  hipLaunchKernelGGL(k_count_zero, dim3(1), dim3(1), 0, st, count);
  hipLaunchKernelGGL((k_check_finite<Q, U>), dim3(blocks), dim3(kCheckBlock), 0, st, g,
                     static_cast<const U*>(f_buf), mask, ones, count);
  return hipGetLastError();
}

template <int Q>
hipError_t check_q(StoreFormat fmt, const Geom& g, const void* f_buf, const uint8_t* mask,
                   unsigned long long* count, hipStream_t st) {
  switch (fmt) {
    case StoreFormat::F64:
      return check_impl<Q, uint64_t>(g, f_buf, mask, uint64_t(0x7FF0000000000000ull), count, st);
    case StoreFormat::F32:
      return check_impl<Q, uint32_t>(g, f_buf, mask, 0x7F800000u, count, st);
    case StoreFormat::F16:
      return check_impl<Q, uint16_t>(g, f_buf, mask, uint16_t(0x7C00u), count, st);
    case StoreFormat::BF16:
      return check_impl<Q, uint16_t>(g, f_buf, mask, uint16_t(0x7F80u), count, st);
  }
  return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_check_finite(int q, StoreFormat fmt, const Geom& g, const void* f_buf, const uint8_t* mask,
                               unsigned long long* count_dev, hipStream_t st) {
  if (q == 27) return check_q<27>(fmt, g, f_buf, mask, count_dev, st);
  if (q == 15) return check_q<15>(fmt, g, f_buf, mask, count_dev, st);
  return hipErrorInvalidValue;
}

}  // namespace cmlbm
