// C ABI of the central-moment LBM library (declared in include/cmlbm.h).
// Argument checking, handle state and kernel dispatch; no arithmetic of the
// method lives here.
#include "cmlbm.h"

#include <hip/hip_runtime_api.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <initializer_list>
#include <string>

#include "checks.hpp"
#include "kernels.hpp"

struct cmlbm_sim {
  int q = 27;
  int prec = 1;
  int device = 0;
  cmlbm::Geom g{};
  double omega[23] = {};
  double F[3] = {0, 0, 0};
  const void* Ffield = nullptr;
  double fscale = 1.0;
  int per_mass = 0;
  const uint8_t* mask = nullptr;
  double* totals_partials = nullptr;   // [kTotalsBlocks][4]
  double* totals_out = nullptr;        // [4]
  double* adj_partials = nullptr;      // [adj_nblk][26] + [kReduceChunks][26]: adjoint dL/domega, uniform dL/dF
  int adj_nblk = 0;
  double* step_partials = nullptr;     // [step_blocks][4] + [kReduceChunks][4], fused step totals
  double* static_partials = nullptr;   // this device's static scratch (cmlbm_step_totals_noalloc), not owned
  std::string static_err;              // why static_partials is null
  std::string err;
};

namespace {

thread_local std::string g_create_error;

cmlbm_status fail(cmlbm_sim* s, cmlbm_status code, const std::string& msg) {
  if (s) s->err = msg;
  return code;
}

cmlbm_status ok(cmlbm_sim* s) {
  s->err.clear();
  return CMLBM_OK;
}

cmlbm_status check_hip(cmlbm_sim* s, hipError_t e, const char* what) {
  if (e == hipSuccess) return ok(s);
  return fail(s, CMLBM_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

// Work is launched on the current device: it must be the handle's.
cmlbm_status on_device(cmlbm_sim* s) {
  int cur = -1;
  if (hipGetDevice(&cur) != hipSuccess) return fail(s, CMLBM_EDEVICE, "hipGetDevice failed");
  if (cur != s->device)
    return fail(s, CMLBM_EINVAL, "current HIP device " + std::to_string(cur) + " is not the handle's device " +
                                     std::to_string(s->device));
  return CMLBM_OK;
}

// Element sizes: population buffers hold the storage type, "real" fields the
// arithmetic type.
size_t pop_bytes(const cmlbm_sim* s) { return s->prec == CMLBM_F64 ? 8 : (s->prec == CMLBM_F32 ? 4 : 2); }
size_t real_bytes(const cmlbm_sim* s) { return s->prec == CMLBM_F64 ? 8 : 4; }

struct DevBuf {
  const void* p;
  size_t elem;
};

// Every kernel reads and writes its buffers one element at a time, with loads
// and stores of the element's size: each pointer must be aligned to it.
cmlbm_status check_aligned(cmlbm_sim* s, std::initializer_list<DevBuf> bufs) {
  for (const DevBuf& b : bufs)
    if (reinterpret_cast<uintptr_t>(b.p) % b.elem != 0)
      return fail(s, CMLBM_EINVAL, "device buffer not aligned to its element size (" + std::to_string(b.elem) + " B)");
  return CMLBM_OK;
}

#define CMLBM_CHECK_ALIGNED(s, ...)                          \
  do {                                                       \
    const cmlbm_status al_ = check_aligned(s, {__VA_ARGS__}); \
    if (al_ != CMLBM_OK) return al_;                         \
  } while (0)

#define CMLBM_WORK_ENTRY(s)                   \
  do {                                        \
    if (!(s)) return CMLBM_EINVAL;            \
    const cmlbm_status dev_ = on_device(s);   \
    if (dev_ != CMLBM_OK) return dev_;        \
  } while (0)

template <typename R>
cmlbm::Rates<R> make_rates(const cmlbm_sim* s) {
  cmlbm::Rates<R> r{};
  for (int b = 0; b < 27; ++b) {
    r.w[b] = R(0);
    r.wc[b] = R(1);
  }
  for (int b = 4; b < s->q; ++b) {
    r.w[b] = R(s->omega[b - 4]);
    r.wc[b] = R(1.0 - s->omega[b - 4]);
  }
  r.per_mass = s->per_mass;
  return r;
}

template <typename R>
cmlbm::ForceArgs<R> make_force(const cmlbm_sim* s) {
  cmlbm::ForceArgs<R> f{};
  for (int i = 0; i < 3; ++i) f.uni[i] = R(s->F[i] * s->fscale);
  f.field = static_cast<const R*>(s->Ffield);
  f.scale = R(s->fscale);
  return f;
}

template <typename R>
cmlbm::AuxArgs<R> make_aux(const cmlbm_sim* s, const void* in0, void* out0, void* out1) {
  cmlbm::AuxArgs<R> a{};
  a.g = s->g;
  a.in0 = in0;
  a.out0 = out0;
  a.out1 = out1;
  a.mask = s->mask;
  a.force = make_force<R>(s);
  return a;
}

}  // namespace

extern "C" {

const char* cmlbm_version(void) { return "0.1.0"; }

const char* cmlbm_status_string(cmlbm_status code) {
  switch (code) {
    case CMLBM_OK: return "ok";
    case CMLBM_EINVAL: return "invalid argument";
    case CMLBM_EUNSUPPORTED: return "unsupported";
    case CMLBM_EDEVICE: return "device error";
    case CMLBM_ENOMEM: return "out of device memory";
    case CMLBM_ESTATE: return "invalid call order";
  }
  return "unknown status";
}

const char* cmlbm_last_error(const cmlbm_sim* sim) {
  if (!sim) return g_create_error.c_str();
  return sim->err.c_str();
}

cmlbm_status cmlbm_create(int q, int nx, int ny, int nz, int precision, cmlbm_sim** out) {
  g_create_error.clear();
  if (!out) {
    g_create_error = "out is NULL";
    return CMLBM_EINVAL;
  }
  *out = nullptr;
  if (q != 15 && q != 27) {
    g_create_error = "q must be 15 or 27";
    return CMLBM_EINVAL;
  }
  if (nx < 1 || ny < 1 || nz < 1 || nx > 65535 || ny > 65535 || nz > 65535) {
    g_create_error = "lattice dimensions must be in [1, 65535]";
    return CMLBM_EINVAL;
  }
  const uint64_t N = uint64_t(nx) * uint64_t(ny) * uint64_t(nz);
  if (N >= (uint64_t(1) << 31)) {
    g_create_error = "nx*ny*nz must be below 2^31";
    return CMLBM_EINVAL;
  }
  {
    cmlbm::Geom g{};
    g.nx = nx;
    g.ny = ny;
    g.nz = nz;
    g.nxy = uint32_t(nx) * uint32_t(ny);
    g.N = N;
    if (cmlbm::max_work_items(g) > UINT32_MAX) {
      g_create_error = "too many rows for one launch: the launches give every row a multiple of 64 lanes, "
                       "so a lattice this short in x exceeds 2^32 work-items; make x the longest axis";
      return CMLBM_EINVAL;
    }
  }
  if (precision < CMLBM_F64 || precision > CMLBM_F32_BF16DEV) {
    g_create_error = "unknown precision";
    return CMLBM_EINVAL;
  }
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
    g_create_error = "no HIP device";
    return CMLBM_EDEVICE;
  }
  cmlbm_sim* s = new cmlbm_sim();
  s->q = q;
  s->prec = precision;
  (void)hipGetDevice(&s->device);
  s->g.nx = nx;
  s->g.ny = ny;
  s->g.nz = nz;
  s->g.nxy = uint32_t(nx) * uint32_t(ny);
  s->g.N = N;
  for (double& w : s->omega) w = 1.0;
  const uint64_t step_rows = cmlbm::step_blocks(s->g) + cmlbm::kReduceChunks;
  s->adj_nblk = cmlbm::adjoint_blocks(s->g);
  if (hipMalloc(&s->totals_partials, sizeof(double) * 4 * cmlbm::kTotalsBlocks) != hipSuccess ||
      hipMalloc(&s->totals_out, sizeof(double) * 4) != hipSuccess ||
      hipMalloc(&s->step_partials, sizeof(double) * 4 * step_rows) != hipSuccess ||
      hipMalloc(&s->adj_partials, sizeof(double) * 26 * (size_t(s->adj_nblk) + cmlbm::kReduceChunks)) != hipSuccess) {
    g_create_error = "device scratch allocation failed";
    cmlbm_destroy(s);
    return CMLBM_ENOMEM;
  }
  // the allocation-free step's scratch: looked up once per device, here, with
  // the handle's device current
  const hipError_t se = cmlbm::static_scratch(&s->static_partials);
  if (se != hipSuccess) s->static_err = std::string("static scratch lookup failed: ") + hipGetErrorString(se);
  *out = s;
  return CMLBM_OK;
}

void cmlbm_destroy(cmlbm_sim* sim) {
  if (!sim) return;
  if (sim->totals_partials) (void)hipFree(sim->totals_partials);
  if (sim->totals_out) (void)hipFree(sim->totals_out);
  if (sim->adj_partials) (void)hipFree(sim->adj_partials);
  if (sim->step_partials) (void)hipFree(sim->step_partials);
  delete sim;
}

cmlbm_status cmlbm_set_rates(cmlbm_sim* s, const double* omega, int n) {
  if (!s) return CMLBM_EINVAL;
  if (!omega) return fail(s, CMLBM_EINVAL, "omega is NULL");
  if (n != s->q - 4) return fail(s, CMLBM_EINVAL, "expected q-4 rates (omega_4 .. omega_(q-1))");
  for (int i = 0; i < n; ++i) {
    if (!(omega[i] > 0.0 && omega[i] < 2.0))
      return fail(s, CMLBM_EINVAL, "omega_" + std::to_string(i + 4) + " outside (0, 2)");
  }
  for (int i = 0; i < n; ++i) s->omega[i] = omega[i];
  return ok(s);
}

cmlbm_status cmlbm_set_force_uniform(cmlbm_sim* s, double fx, double fy, double fz) {
  if (!s) return CMLBM_EINVAL;
  if (!std::isfinite(fx) || !std::isfinite(fy) || !std::isfinite(fz))
    return fail(s, CMLBM_EINVAL, "force must be finite");
  s->F[0] = fx;
  s->F[1] = fy;
  s->F[2] = fz;
  s->Ffield = nullptr;
  return ok(s);
}

cmlbm_status cmlbm_set_force_field(cmlbm_sim* s, const void* F_dev) {
  if (!s) return CMLBM_EINVAL;
  CMLBM_CHECK_ALIGNED(s, {F_dev, real_bytes(s)});
  s->Ffield = F_dev;
  if (!F_dev) s->F[0] = s->F[1] = s->F[2] = 0.0;
  return ok(s);
}

cmlbm_status cmlbm_set_attractor_per_mass(cmlbm_sim* s, int per_mass) {
  if (!s) return CMLBM_EINVAL;
  if (per_mass != 0 && per_mass != 1) return fail(s, CMLBM_EINVAL, "per_mass must be 0 or 1");
  s->per_mass = per_mass;
  return ok(s);
}

cmlbm_status cmlbm_set_force_scale(cmlbm_sim* s, double scale) {
  if (!s) return CMLBM_EINVAL;
  if (!std::isfinite(scale)) return fail(s, CMLBM_EINVAL, "scale must be finite");
  s->fscale = scale;
  return ok(s);
}

cmlbm_status cmlbm_set_mask(cmlbm_sim* s, const uint8_t* mask_dev) {
  if (!s) return CMLBM_EINVAL;
  s->mask = mask_dev;
  return ok(s);
}

cmlbm_status cmlbm_init_equilibrium(cmlbm_sim* s, const void* rho_dev, const void* u_dev, void* f_pre_dev,
                                    void* f_post_dev, void* stream) {
  CMLBM_WORK_ENTRY(s);
  if (!rho_dev || !u_dev || !f_pre_dev || !f_post_dev) return fail(s, CMLBM_EINVAL, "NULL buffer");
  if (f_pre_dev == f_post_dev) return fail(s, CMLBM_EINVAL, "f_pre and f_post must differ");
  CMLBM_CHECK_ALIGNED(s, {rho_dev, real_bytes(s)}, {u_dev, real_bytes(s)}, {f_pre_dev, real_bytes(s)},
                      {f_post_dev, pop_bytes(s)});
  hipError_t e = cmlbm::launch_init(s->q, s->prec, s->g, rho_dev, u_dev, make_force<double>(s),
                                    make_force<float>(s), s->mask, f_pre_dev, f_post_dev,
                                    static_cast<hipStream_t>(stream));
  return check_hip(s, e, "init_equilibrium");
}

cmlbm_status cmlbm_init_equilibrium_inplace(cmlbm_sim* s, const void* rho_dev, const void* u_dev, void* f_dev,
                                            void* stream) {
  CMLBM_WORK_ENTRY(s);
  if (!rho_dev || !u_dev || !f_dev) return fail(s, CMLBM_EINVAL, "NULL buffer");
  CMLBM_CHECK_ALIGNED(s, {rho_dev, real_bytes(s)}, {u_dev, real_bytes(s)}, {f_dev, pop_bytes(s)});
  hipError_t e = cmlbm::launch_init(s->q, s->prec, s->g, rho_dev, u_dev, make_force<double>(s),
                                    make_force<float>(s), s->mask, f_dev, nullptr,
                                    static_cast<hipStream_t>(stream));
  return check_hip(s, e, "init_equilibrium_inplace");
}

namespace {

// scratch: [step_blocks][4] partials followed by [kReduceChunks][4] stage sums
// (used only with totals_dev).
cmlbm_status step_common(cmlbm_sim* s, const void* f_in, void* f_out, double* totals_dev, double* scratch,
                         void* stream) {
  if (!f_in || !f_out) return fail(s, CMLBM_EINVAL, "NULL population buffer");
  if (f_in == f_out) return fail(s, CMLBM_EINVAL, "f_in and f_out must differ (pull streaming)");
  CMLBM_CHECK_ALIGNED(s, {f_in, pop_bytes(s)}, {f_out, pop_bytes(s)}, {totals_dev, sizeof(double)});
  double* partials = nullptr;
  double* stage = nullptr;
  if (totals_dev) {
    partials = scratch;
    stage = scratch + 4 * cmlbm::step_blocks(s->g);
  }
  cmlbm::StepArgs<double> a64{};
  cmlbm::StepArgs<float> a32{};
  if (s->prec == CMLBM_F64) {
    a64.g = s->g;
    a64.fin = f_in;
    a64.fout = f_out;
    a64.mask = s->mask;
    a64.force = make_force<double>(s);
    a64.rates = make_rates<double>(s);
    a64.partials = partials;
    a64.stage = stage;
    a64.totals = totals_dev;
  } else {
    a32.g = s->g;
    a32.fin = f_in;
    a32.fout = f_out;
    a32.mask = s->mask;
    a32.force = make_force<float>(s);
    a32.rates = make_rates<float>(s);
    a32.partials = partials;
    a32.stage = stage;
    a32.totals = totals_dev;
  }
  return check_hip(s, cmlbm::launch_step(s->q, s->prec, a64, a32, static_cast<hipStream_t>(stream)), "step");
}

}  // namespace

cmlbm_status cmlbm_step(cmlbm_sim* s, const void* f_in, void* f_out, void* stream) {
  CMLBM_WORK_ENTRY(s);
  return step_common(s, f_in, f_out, nullptr, nullptr, stream);
}

cmlbm_status cmlbm_step_totals(cmlbm_sim* s, const void* f_in, void* f_out, double* totals_dev, void* stream) {
  CMLBM_WORK_ENTRY(s);
  if (!totals_dev) return fail(s, CMLBM_EINVAL, "totals_dev is NULL");
  return step_common(s, f_in, f_out, totals_dev, s->step_partials, stream);
}

cmlbm_status cmlbm_step_totals_noalloc(cmlbm_sim* s, const void* f_in, void* f_out, double* totals_dev,
                                       void* stream) {
  CMLBM_WORK_ENTRY(s);
  if (cmlbm::step_blocks(s->g) > cmlbm::kStaticStepBlocks)
    return fail(s, CMLBM_EINVAL,
                "lattice too large for the static scratch: " + std::to_string(cmlbm::step_blocks(s->g)) +
                    " step blocks (ceil(nx/256)*ny*nz), at most " + std::to_string(cmlbm::kStaticStepBlocks));
  if (!totals_dev) return fail(s, CMLBM_EINVAL, "totals_dev is NULL");
  if (!s->static_partials) return fail(s, CMLBM_EDEVICE, s->static_err);
  return step_common(s, f_in, f_out, totals_dev, s->static_partials, stream);
}

cmlbm_status cmlbm_run(cmlbm_sim* s, void* f_a, void* f_b, int nsteps, void* stream, int* result_in_b) {
  CMLBM_WORK_ENTRY(s);
  if (nsteps < 0) return fail(s, CMLBM_EINVAL, "nsteps < 0");
  if (!f_a || !f_b) return fail(s, CMLBM_EINVAL, "NULL population buffer");
  if (f_a == f_b) return fail(s, CMLBM_EINVAL, "f_a and f_b must differ");
  CMLBM_CHECK_ALIGNED(s, {f_a, pop_bytes(s)}, {f_b, pop_bytes(s)});
  void* bufs[2] = {f_a, f_b};
  for (int n = 0; n < nsteps; ++n) {
    cmlbm_status st = cmlbm_step(s, bufs[n & 1], bufs[(n + 1) & 1], stream);
    if (st != CMLBM_OK) return st;
  }
  if (result_in_b) *result_in_b = nsteps & 1;
  return ok(s);
}

cmlbm_status cmlbm_gather_precollision(cmlbm_sim* s, const void* f_post, void* f_pre, void* stream) {
  CMLBM_WORK_ENTRY(s);
  if (!f_post || !f_pre) return fail(s, CMLBM_EINVAL, "NULL buffer");
  if (f_post == f_pre) return fail(s, CMLBM_EINVAL, "f_post and f_pre must differ");
  CMLBM_CHECK_ALIGNED(s, {f_post, pop_bytes(s)}, {f_pre, real_bytes(s)});
  hipError_t e = cmlbm::launch_gather(s->q, s->prec, make_aux<double>(s, f_post, f_pre, nullptr),
                                      make_aux<float>(s, f_post, f_pre, nullptr), static_cast<hipStream_t>(stream));
  return check_hip(s, e, "gather_precollision");
}

cmlbm_status cmlbm_export_populations(cmlbm_sim* s, const void* f_buf, void* f_soa, void* stream) {
  CMLBM_WORK_ENTRY(s);
  if (!f_buf || !f_soa) return fail(s, CMLBM_EINVAL, "NULL buffer");
  if (f_buf == f_soa) return fail(s, CMLBM_EINVAL, "f_buf and f_soa must differ");
  CMLBM_CHECK_ALIGNED(s, {f_buf, pop_bytes(s)}, {f_soa, real_bytes(s)});
  hipError_t e = cmlbm::launch_convert(s->q, s->prec, s->g, f_buf, f_soa, true, static_cast<hipStream_t>(stream));
  return check_hip(s, e, "export_populations");
}

cmlbm_status cmlbm_import_populations(cmlbm_sim* s, const void* f_soa, void* f_buf, void* stream) {
  CMLBM_WORK_ENTRY(s);
  if (!f_buf || !f_soa) return fail(s, CMLBM_EINVAL, "NULL buffer");
  if (f_buf == f_soa) return fail(s, CMLBM_EINVAL, "f_buf and f_soa must differ");
  CMLBM_CHECK_ALIGNED(s, {f_buf, pop_bytes(s)}, {f_soa, real_bytes(s)});
  hipError_t e = cmlbm::launch_convert(s->q, s->prec, s->g, f_soa, f_buf, false, static_cast<hipStream_t>(stream));
  return check_hip(s, e, "import_populations");
}

namespace {

cmlbm_status macro_common(cmlbm_sim* s, const void* f, void* rho, void* u, bool pre, void* stream) {
  if (!f || !rho || !u) return fail(s, CMLBM_EINVAL, "NULL buffer");
  CMLBM_CHECK_ALIGNED(s, {f, pop_bytes(s)}, {rho, real_bytes(s)}, {u, real_bytes(s)});
  hipError_t e = cmlbm::launch_macro(s->q, s->prec, make_aux<double>(s, f, rho, u), make_aux<float>(s, f, rho, u),
                                     pre, static_cast<hipStream_t>(stream));
  return check_hip(s, e, "macroscopic");
}

cmlbm_status totals_common(cmlbm_sim* s, const void* f, double out4[4], bool pre, void* stream) {
  if (!f || !out4) return fail(s, CMLBM_EINVAL, "NULL buffer");
  CMLBM_CHECK_ALIGNED(s, {f, pop_bytes(s)});
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipError_t e = cmlbm::launch_totals(s->q, s->prec, make_aux<double>(s, f, nullptr, nullptr),
                                      make_aux<float>(s, f, nullptr, nullptr), pre, s->totals_partials,
                                      cmlbm::kTotalsBlocks, s->totals_out, st);
  if (e != hipSuccess) return check_hip(s, e, "totals");
  e = hipMemcpyAsync(out4, s->totals_out, sizeof(double) * 4, hipMemcpyDeviceToHost, st);
  if (e != hipSuccess) return check_hip(s, e, "totals copy");
  return check_hip(s, hipStreamSynchronize(st), "totals sync");
}

}  // namespace

cmlbm_status cmlbm_macroscopic(cmlbm_sim* s, const void* f_post, void* rho, void* u, void* stream) {
  CMLBM_WORK_ENTRY(s);
  return macro_common(s, f_post, rho, u, false, stream);
}

cmlbm_status cmlbm_totals(cmlbm_sim* s, const void* f_post, double out4[4], void* stream) {
  CMLBM_WORK_ENTRY(s);
  return totals_common(s, f_post, out4, false, stream);
}

namespace {

cmlbm_status inplace_common(cmlbm_sim* s, void* f, int parity, double* totals_dev, void* stream) {
  if (!f) return fail(s, CMLBM_EINVAL, "NULL population buffer");
  if (parity != 0 && parity != 1) return fail(s, CMLBM_EINVAL, "parity must be 0 or 1");
  CMLBM_CHECK_ALIGNED(s, {f, pop_bytes(s)}, {totals_dev, sizeof(double)});
  double* partials = nullptr;
  double* stage = nullptr;
  if (totals_dev) {
    partials = s->step_partials;
    stage = s->step_partials + 4 * cmlbm::step_blocks(s->g);
  }
  cmlbm::StepArgs<double> a64{};
  cmlbm::StepArgs<float> a32{};
  if (s->prec == CMLBM_F64) {
    a64.g = s->g;
    a64.fout = f;
    a64.mask = s->mask;
    a64.force = make_force<double>(s);
    a64.rates = make_rates<double>(s);
    a64.partials = partials;
    a64.stage = stage;
    a64.totals = totals_dev;
  } else {
    a32.g = s->g;
    a32.fout = f;
    a32.mask = s->mask;
    a32.force = make_force<float>(s);
    a32.rates = make_rates<float>(s);
    a32.partials = partials;
    a32.stage = stage;
    a32.totals = totals_dev;
  }
  return check_hip(s, cmlbm::launch_step_inplace(s->q, s->prec, a64, a32, parity, static_cast<hipStream_t>(stream)),
                   "step_inplace");
}

}  // namespace

cmlbm_status cmlbm_step_inplace(cmlbm_sim* s, void* f, int parity, void* stream) {
  CMLBM_WORK_ENTRY(s);
  return inplace_common(s, f, parity, nullptr, stream);
}

cmlbm_status cmlbm_step_inplace_totals(cmlbm_sim* s, void* f, int parity, double* totals_dev, void* stream) {
  CMLBM_WORK_ENTRY(s);
  if (!totals_dev) return fail(s, CMLBM_EINVAL, "totals_dev is NULL");
  return inplace_common(s, f, parity, totals_dev, stream);
}

cmlbm_status cmlbm_run_inplace(cmlbm_sim* s, void* f, int nsteps, void* stream) {
  CMLBM_WORK_ENTRY(s);
  if (!f) return fail(s, CMLBM_EINVAL, "NULL population buffer");
  if (nsteps < 0 || (nsteps & 1)) return fail(s, CMLBM_EINVAL, "nsteps must be even and >= 0");
  CMLBM_CHECK_ALIGNED(s, {f, pop_bytes(s)});
  for (int n = 0; n < nsteps; ++n) {
    cmlbm_status st = cmlbm_step_inplace(s, f, n & 1, stream);
    if (st != CMLBM_OK) return st;
  }
  return ok(s);
}

cmlbm_status cmlbm_macroscopic_pre(cmlbm_sim* s, const void* f_pre_buf, void* rho, void* u, void* stream) {
  CMLBM_WORK_ENTRY(s);
  return macro_common(s, f_pre_buf, rho, u, true, stream);
}

cmlbm_status cmlbm_totals_pre(cmlbm_sim* s, const void* f_pre_buf, double out4[4], void* stream) {
  CMLBM_WORK_ENTRY(s);
  return totals_common(s, f_pre_buf, out4, true, stream);
}

cmlbm_status cmlbm_adjoint_step(cmlbm_sim* s, const void* f_post_prev, const void* lam_next, void* lam,
                                double* dLdF_dev, double* dLdomega_dev, void* stream) {
  CMLBM_WORK_ENTRY(s);
  if (!f_post_prev || !lam_next || !lam || !dLdF_dev || !dLdomega_dev) return fail(s, CMLBM_EINVAL, "NULL buffer");
  if (lam == lam_next || lam == f_post_prev || lam_next == f_post_prev)
    return fail(s, CMLBM_EINVAL, "lam, lam_next and f_post_prev must differ");
  CMLBM_CHECK_ALIGNED(s, {f_post_prev, pop_bytes(s)}, {lam_next, real_bytes(s)}, {lam, real_bytes(s)},
                      {dLdF_dev, sizeof(double)}, {dLdomega_dev, sizeof(double)});
  const int nblk = s->adj_nblk;
  cmlbm::AdjArgs<double> a64{};
  cmlbm::AdjArgs<float> a32{};
  if (s->prec == CMLBM_F64) {
    a64.g = s->g;
    a64.fpost = f_post_prev;
    a64.lam_next = static_cast<const double*>(lam_next);
    a64.lam = static_cast<double*>(lam);
    a64.dLdF = dLdF_dev;
    a64.mask = s->mask;
    a64.force = make_force<double>(s);
    a64.rates = make_rates<double>(s);
  } else {
    a32.g = s->g;
    a32.fpost = f_post_prev;
    a32.lam_next = static_cast<const float*>(lam_next);
    a32.lam = static_cast<float*>(lam);
    a32.dLdF = dLdF_dev;
    a32.mask = s->mask;
    a32.force = make_force<float>(s);
    a32.rates = make_rates<float>(s);
  }
  double* dLdF_uniform = s->Ffield ? nullptr : dLdF_dev;
  hipError_t e = cmlbm::launch_adjoint(s->q, s->prec, a64, a32, s->adj_partials, nblk, dLdomega_dev, dLdF_uniform,
                                       static_cast<hipStream_t>(stream));
  return check_hip(s, e, "adjoint_step");
}

static cmlbm_status wall_sensitivity(cmlbm_sim* s, const void* f_post_prev, const void* lam_next, double* dLdphi_dev,
                                     bool post, void* stream) {
  CMLBM_WORK_ENTRY(s);
  if (!f_post_prev || !lam_next || !dLdphi_dev) return fail(s, CMLBM_EINVAL, "NULL buffer");
  if (f_post_prev == lam_next || static_cast<const void*>(dLdphi_dev) == lam_next ||
      static_cast<const void*>(dLdphi_dev) == f_post_prev)
    return fail(s, CMLBM_EINVAL, "f_post_prev, lam_next and dLdphi must differ");
  CMLBM_CHECK_ALIGNED(s, {f_post_prev, pop_bytes(s)}, {lam_next, real_bytes(s)}, {dLdphi_dev, sizeof(double)});
  cmlbm::AdjArgs<double> a64{};
  cmlbm::AdjArgs<float> a32{};
  if (s->prec == CMLBM_F64) {
    a64.g = s->g;
    a64.fpost = f_post_prev;
    a64.lam_next = static_cast<const double*>(lam_next);
    a64.mask = s->mask;
    a64.force = make_force<double>(s);
    a64.rates = make_rates<double>(s);
  } else {
    a32.g = s->g;
    a32.fpost = f_post_prev;
    a32.lam_next = static_cast<const float*>(lam_next);
    a32.mask = s->mask;
    a32.force = make_force<float>(s);
    a32.rates = make_rates<float>(s);
  }
  hipError_t e =
      cmlbm::launch_wall_sensitivity(s->q, s->prec, a64, a32, dLdphi_dev, post, static_cast<hipStream_t>(stream));
  return check_hip(s, e, post ? "wall_sensitivity_post" : "wall_sensitivity");
}

cmlbm_status cmlbm_wall_sensitivity(cmlbm_sim* s, const void* f_post_prev, const void* lam_next, double* dLdphi_dev,
                                    void* stream) {
  return wall_sensitivity(s, f_post_prev, lam_next, dLdphi_dev, false, stream);
}

cmlbm_status cmlbm_wall_sensitivity_post(cmlbm_sim* s, const void* f_post, const void* lam, double* dLdphi_dev,
                                         void* stream) {
  return wall_sensitivity(s, f_post, lam, dLdphi_dev, true, stream);
}

cmlbm_status cmlbm_check_finite(cmlbm_sim* s, const void* f_buf, int64_t* nonfinite, void* stream) {
  CMLBM_WORK_ENTRY(s);
  if (!f_buf || !nonfinite) return fail(s, CMLBM_EINVAL, "NULL buffer");
  CMLBM_CHECK_ALIGNED(s, {f_buf, pop_bytes(s)});
  static const cmlbm::StoreFormat fmt[4] = {cmlbm::StoreFormat::F64, cmlbm::StoreFormat::F32,
                                            cmlbm::StoreFormat::F16, cmlbm::StoreFormat::BF16};
  // The result slot of the synchronous reductions (32 bytes) holds the counter.
  auto* count = reinterpret_cast<unsigned long long*>(s->totals_out);
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipError_t e = cmlbm::launch_check_finite(s->q, fmt[s->prec], s->g, f_buf, s->mask, count, st);
  if (e != hipSuccess) return check_hip(s, e, "check_finite");
  unsigned long long host = 0;
  e = hipMemcpyAsync(&host, count, sizeof(host), hipMemcpyDeviceToHost, st);
  if (e != hipSuccess) return check_hip(s, e, "check_finite copy");
  e = hipStreamSynchronize(st);
  if (e != hipSuccess) return check_hip(s, e, "check_finite sync");
  *nonfinite = int64_t(host);
  return ok(s);
}

cmlbm_status cmlbm_kinetic_energy_sum(cmlbm_sim* s, const void* f_pre, double* out, void* stream) {
  CMLBM_WORK_ENTRY(s);
  if (!f_pre || !out) return fail(s, CMLBM_EINVAL, "NULL buffer");
  CMLBM_CHECK_ALIGNED(s, {f_pre, real_bytes(s)});
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipError_t e = cmlbm::launch_ke_sum(s->q, s->prec, s->g, f_pre, s->mask, make_force<double>(s), make_force<float>(s),
                                      s->totals_partials, cmlbm::kTotalsBlocks, s->totals_out, st);
  if (e != hipSuccess) return check_hip(s, e, "kinetic_energy_sum");
  e = hipMemcpyAsync(out, s->totals_out, sizeof(double), hipMemcpyDeviceToHost, st);
  if (e != hipSuccess) return check_hip(s, e, "kinetic_energy_sum copy");
  return check_hip(s, hipStreamSynchronize(st), "kinetic_energy_sum sync");
}

cmlbm_status cmlbm_kinetic_energy_seed(cmlbm_sim* s, const void* f_pre, double scale, void* lam, double* dLdF_dev,
                                       void* stream) {
  CMLBM_WORK_ENTRY(s);
  if (!f_pre || !lam || !dLdF_dev) return fail(s, CMLBM_EINVAL, "NULL buffer");
  if (f_pre == lam) return fail(s, CMLBM_EINVAL, "f_pre and lam must differ");
  CMLBM_CHECK_ALIGNED(s, {f_pre, real_bytes(s)}, {lam, real_bytes(s)}, {dLdF_dev, sizeof(double)});
  hipError_t e = cmlbm::launch_ke_seed(s->q, s->prec, s->g, f_pre, s->mask, make_force<double>(s),
                                       make_force<float>(s), scale, lam, dLdF_dev, s->totals_partials,
                                       cmlbm::kTotalsBlocks, static_cast<hipStream_t>(stream));
  return check_hip(s, e, "kinetic_energy_seed");
}

cmlbm_status cmlbm_init_adjoint(cmlbm_sim* s, const void* u0_dev, const void* lam0_dev, double* dLdF_dev,
                                void* stream) {
  CMLBM_WORK_ENTRY(s);
  if (!u0_dev || !lam0_dev || !dLdF_dev) return fail(s, CMLBM_EINVAL, "NULL buffer");
  CMLBM_CHECK_ALIGNED(s, {u0_dev, real_bytes(s)}, {lam0_dev, real_bytes(s)}, {dLdF_dev, sizeof(double)});
  hipError_t e = cmlbm::launch_init_adjoint(s->q, s->prec, s->g, u0_dev, lam0_dev, s->mask, make_force<double>(s),
                                            make_force<float>(s), dLdF_dev, s->totals_partials,
                                            cmlbm::kTotalsBlocks, static_cast<hipStream_t>(stream));
  return check_hip(s, e, "init_adjoint");
}

}  // extern "C"
