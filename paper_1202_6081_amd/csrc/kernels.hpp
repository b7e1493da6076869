// Internal interface between the C ABI (api.cpp) and the HIP kernels.
#pragma once

#include <hip/hip_runtime_api.h>

#include <cstdint>

#include "collide_d3q27.hpp"   // Rates<R>

namespace cmlbm {

struct Geom {
  int nx, ny, nz;
  uint32_t nxy;
  uint64_t N;   // nodes
};

// The launch's map from a block's linear index to its row segment: rows
// r = z*ny + y of nx nodes are cut into nseg segments of one block each, so
// block L works on row L / nseg, segment L % nseg, and row r is (y, z) =
// (r % ny, r / ny).  The dividers are set up on the host (Divider), which keeps
// these divisions on the scalar unit.  Filled by the launchers.
struct RowMap {
  uint32_t nseg;
  Divider seg, ny;
};

// Body force: a uniform vector (already multiplied by the time scale) or a
// field [3][nz][ny][nx] times `scale`.
template <typename FT>
struct ForceArgs {
  FT uni[3];
  const FT* field;
  FT scale;
};

template <typename R>
struct StepArgs {
  Geom g;
  const void* fin;
  void* fout;
  const uint8_t* mask;
  ForceArgs<R> force;
  Rates<R> rates;
  // Optional FP64 totals of the input state, fused into the step: per-block
  // partials [step_blocks(g)][4], a second-stage buffer [kReduceChunks][4] and
  // the device output [4].  All null for a plain step.
  double* partials;
  double* stage;
  double* totals;
  RowMap rm;
};

template <typename R>
struct AuxArgs {
  Geom g;
  const void* in0;
  void* out0;
  void* out1;
  const uint8_t* mask;
  ForceArgs<R> force;
};

template <typename R>
struct AdjArgs {
  Geom g;
  const void* fpost;      // forward post-collision state of step n (storage type)
  const R* lam_next;      // dL/dfbar^{n+1} (compute type)
  R* lam;                 // dL/dfbar^n (compute type)
  double* dLdF;           // [3][N], accumulated (force field mode)
  const uint8_t* mask;
  ForceArgs<R> force;
  Rates<R> rates;
};

// prec: 0 FP64, 1 FP32, 2 FP32 compute / FP16 deviation storage, 3 BF16 deviations.
hipError_t launch_step(int q, int prec, const StepArgs<double>& a64, const StepArgs<float>& a32, hipStream_t st);
hipError_t launch_gather(int q, int prec, const AuxArgs<double>& a64, const AuxArgs<float>& a32, hipStream_t st);
// Population buffer (blocked layout) <-> full populations in compute type,
// structure of arrays [Q][N]; to_soa selects the direction.
hipError_t launch_convert(int q, int prec, const Geom& g, const void* in, void* out, bool to_soa, hipStream_t st);
// pre: the buffer holds pre-collision populations (phase 0 of the in-place
// step) and is read in place instead of pulled.
hipError_t launch_macro(int q, int prec, const AuxArgs<double>& a64, const AuxArgs<float>& a32, bool pre,
                        hipStream_t st);
hipError_t launch_totals(int q, int prec, const AuxArgs<double>& a64, const AuxArgs<float>& a32, bool pre,
                         double* partials, int nblk, double* out4, hipStream_t st);
// One in-place step on the buffer a.fout (a.fin unused); parity = phase of the
// buffer on entry (0 or 1).
hipError_t launch_step_inplace(int q, int prec, const StepArgs<double>& a64, const StepArgs<float>& a32, int parity,
                               hipStream_t st);
// fpost == nullptr: fpre is an in-place buffer in phase 0 (storage type, blocked rows).
hipError_t launch_init(int q, int prec, const Geom& g, const void* rho0, const void* u0, const ForceArgs<double>& f64,
                       const ForceArgs<float>& f32, const uint8_t* mask, void* fpre, void* fpost, hipStream_t st);
hipError_t launch_adjoint(int q, int prec, const AdjArgs<double>& a64, const AdjArgs<float>& a32, double* partials,
                          int nblk, double* dLdomega, double* dLdF_uniform, hipStream_t st);

// Wall-layout sensitivity of one step (fpost, lam_next, mask, force, rates of
// the AdjArgs; lam and dLdF unused): accumulates into dLdphi[N] (FP64).
// post = false: fpost is the step's input state and the collision is
// recomputed (FP64 atomics); post = true: fpost is the collided state the
// streaming moves, and each node gathers its own terms.
hipError_t launch_wall_sensitivity(int q, int prec, const AdjArgs<double>& a64, const AdjArgs<float>& a32,
                                   double* dLdphi, bool post, hipStream_t st);

hipError_t launch_ke_sum(int q, int prec, const Geom& g, const void* fpre, const uint8_t* mask,
                         const ForceArgs<double>& f64, const ForceArgs<float>& f32, double* partials, int nblk,
                         double* out, hipStream_t st);
hipError_t launch_ke_seed(int q, int prec, const Geom& g, const void* fpre, const uint8_t* mask,
                          const ForceArgs<double>& f64, const ForceArgs<float>& f32, double scale, void* lam,
                          double* dLdF, double* partials, int nblk, hipStream_t st);
hipError_t launch_init_adjoint(int q, int prec, const Geom& g, const void* u0, const void* lam0,
                               const uint8_t* mask, const ForceArgs<double>& f64, const ForceArgs<float>& f32,
                               double* dLdF, double* partials, int nblk, hipStream_t st);

// Blocks of the adjoint launch: a multiple of 8 (one share per XCD), each block
// visiting about CMLBM_ADJ_ITEMS row segments (each thread at most that many
// nodes, plus one).
#ifndef CMLBM_ADJ_ITEMS
#define CMLBM_ADJ_ITEMS 8
#endif
inline int adjoint_blocks(const Geom& g) {
  const int bx = g.nx < 256 ? ((g.nx + 63) / 64) * 64 : 256;
  const uint64_t items = uint64_t((g.nx + bx - 1) / bx) * uint64_t(g.ny) * uint64_t(g.nz);
  uint64_t nb = (items + CMLBM_ADJ_ITEMS - 1) / CMLBM_ADJ_ITEMS;
  nb = ((nb + 7) / 8) * 8;
  return int(nb);
}

constexpr int kTotalsBlocks = 2048;
constexpr int kReduceChunks = 256;

// Blocks of one step launch (one block per CMLBM_STEP_BLOCK-wide row segment).
uint64_t step_blocks(const Geom& g);

// Static device scratch of the allocation-free fused-totals step: room for the
// per-block partials of at most kStaticStepBlocks step blocks and the
// second-stage sums, kStaticScratchDoubles doubles (16 MiB + 8 KiB) per device,
// held until the process ends.
constexpr uint64_t kStaticStepBlocks = uint64_t(1) << 19;
constexpr uint64_t kStaticScratchDoubles = 4 * (kStaticStepBlocks + kReduceChunks);

// Device address of that scratch on the current device, looked up once per
// device (hipGetSymbolAddress) and cached; *out is null on failure.
hipError_t static_scratch(double** out);

// Work-items of the largest grid the lattice's launches use (the step and the
// adjoint cover whole row segments rounded up to 64 lanes); a dispatch counts
// its work-items in 32 bits.
uint64_t max_work_items(const Geom& g);

}  // namespace cmlbm
