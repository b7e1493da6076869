// Diagnostics over population buffers, kept apart from the step kernels.
#pragma once

#include <hip/hip_runtime_api.h>

#include <cstdint>

#include "kernels.hpp"

namespace cmlbm {

// Storage formats of a population buffer, by the bits that mark a value that
// is not finite (an exponent field of all ones: NaN or +-Inf).
enum class StoreFormat { F64, F32, F16, BF16 };

// count_dev = number of stored populations of fluid nodes (every node without
// a mask) whose storage bits are NaN or +-Inf.  f_buf has the blocked row
// layout of every population buffer; count_dev is one 64-bit device counter,
// overwritten.  Two launches on `st`, no host synchronization.
hipError_t launch_check_finite(int q, StoreFormat fmt, const Geom& g, const void* f_buf, const uint8_t* mask,
                               unsigned long long* count_dev, hipStream_t st);

}  // namespace cmlbm
