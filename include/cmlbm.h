/*
 * cmlbm -- C ABI of the 3D central-moment lattice Boltzmann step on MI355X.
 *
 * The method is Premnath & Banerjee, "On the Three-dimensional Central Moment
 * Lattice Boltzmann Method" (arXiv:1202.6081): D3Q27 and D3Q15 lattices,
 * central moments relaxed toward factorized attractors in cascade, and a
 * de-aliased body-force source treated semi-implicitly with the implicitness
 * removed by fbar = f - S/2.
 *
 * Conventions shared by every call
 * --------------------------------
 * Status:     every call returns cmlbm_status; 0 is success, negative values
 *             are errors.  No C++ exception crosses this boundary.  After an
 *             error, cmlbm_last_error(sim) holds a message.
 * Ownership:  the caller allocates and owns every device buffer (populations,
 *             fields, mask, gradients).  The library borrows a pointer for the
 *             duration of a call, except the force field and the mask, which
 *             are borrowed until replaced or until cmlbm_destroy.  The library
 *             owns only the opaque handle and device scratch for reductions
 *             (nx*ny*nz/8 bytes for the fused step totals, about
 *             26*ceil(nx/256)*ny*nz bytes for the adjoint's partial sums, and
 *             about 120 KiB), all allocated by cmlbm_create: no other call
 *             allocates.  cmlbm_step_totals_noalloc uses a static device array
 *             of the library instead (see there).
 *             Device pointers must be aligned to their element size
 *             (hipMalloc and torch allocations are); a call given a
 *             misaligned one returns EINVAL before launching anything.
 * Streams:    `stream` is a hipStream_t (NULL = the default stream).  Work is
 *             enqueued asynchronously; only the calls with host outputs
 *             (cmlbm_totals, cmlbm_totals_pre, cmlbm_kinetic_energy_sum)
 *             synchronize.  The calls that reduce (the *_totals calls, the
 *             adjoint and loss calls) use the handle's device scratch: work
 *             from one handle must not overlap in time across streams (use one
 *             stream per handle, or order the streams).
 * Devices:    a handle belongs to the device current at cmlbm_create; every
 *             call that launches work returns EINVAL when another device is
 *             current.
 * Threads:    a handle must not be used by two host threads at once.
 * Layout:     fields are structure of arrays, x fastest: vector fields
 *             (velocity, force, force gradient) [3][nz][ny][nx], scalars
 *             [nz][ny][nx], and "SoA populations" f[a][nz][ny][nx] with
 *             directions a in the paper's order (Eq. velocityd3qq27 and
 *             Appendix A for D3Q27; Appendix G for D3Q15).
 *             The population *buffers* of cmlbm_step / cmlbm_run (q * nx * ny *
 *             nz values of the storage type) use a blocked row layout: row
 *             r = z*ny + y holds q*nx values; inside a row x is cut into blocks
 *             of 64 consecutive nodes (the last may be shorter) and a block
 *             stores its q directions one after the other:
 *               index(a, r, x) = r*nx*q + b*64*q + a*len + (x - 64*b),
 *               b = x / 64, len = min(64, nx - 64*b).
 *             cmlbm_export_populations / cmlbm_import_populations convert to
 *             and from SoA populations.
 * State:      the population buffers passed to cmlbm_step / cmlbm_run hold the
 *             post-collision, not yet streamed populations fbar~ (Eq.
 *             cascadedcollision1).  The paper's state, the pre-collision
 *             fbar(x, t), is read out by cmlbm_gather_precollision.  The
 *             in-place calls (cmlbm_step_inplace and the calls after it) keep
 *             one buffer of the same layout in two phases, described there.
 * Types:      "real" means double for CMLBM_F64 and float for the other three
 *             precisions.  Population buffers are double (F64), float (F32),
 *             IEEE binary16 (F32_F16DEV) or bfloat16 (F32_BF16DEV); the 16-bit
 *             formats hold fbar - w_a, the deviation from the rest-state weight
 *             w_a (8/27, 2/27, 1/54, 1/216 for D3Q27; 2/9, 1/9, 1/72 for
 *             D3Q15), rounded to nearest even.  Arithmetic is in "real".
 */
#ifndef CMLBM_H
#define CMLBM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  CMLBM_OK = 0,
  CMLBM_EINVAL = -1,       /* bad argument: null pointer, size, rate, aliasing */
  CMLBM_EUNSUPPORTED = -2, /* valid request this library does not provide */
  CMLBM_EDEVICE = -3,      /* HIP runtime error; message in cmlbm_last_error */
  CMLBM_ENOMEM = -4,       /* device scratch allocation failed */
  CMLBM_ESTATE = -5        /* call order violated */
} cmlbm_status;

typedef enum { CMLBM_D3Q15 = 15, CMLBM_D3Q27 = 27 } cmlbm_lattice;

typedef enum {
  CMLBM_F64 = 0,         /* FP64 storage and arithmetic */
  CMLBM_F32 = 1,         /* FP32 storage and arithmetic */
  CMLBM_F32_F16DEV = 2,  /* FP32 arithmetic, FP16 storage of fbar - w */
  CMLBM_F32_BF16DEV = 3  /* FP32 arithmetic, BF16 storage of fbar - w */
} cmlbm_precision;

typedef struct cmlbm_sim cmlbm_sim; /* opaque; host memory owned by the library */

/* Create a handle for a nx * ny * nz lattice, periodic in all directions until
 * a mask is set.  q: 15 or 27 (Eq. velocityd3qq27, Appendix G).  All rates
 * start at 1, the force at zero, the force scale at 1.  Limits: 1 <= nx,
 * ny, nz <= 65535, nx * ny * nz < 2^31, and ny * nz rows of nx rounded up to
 * 64 (to 256 above 256) below 2^32 lanes, which only a lattice short in x with
 * more than 2^26 rows reaches (make x the longest axis).  Errors: EINVAL
 * (sizes, q, precision, out == NULL), EDEVICE (no HIP device), ENOMEM. */
cmlbm_status cmlbm_create(int q, int nx, int ny, int nz, int precision, cmlbm_sim **out);

/* Release the handle and its device scratch.  NULL is allowed. */
void cmlbm_destroy(cmlbm_sim *sim);

/* Relaxation rates omega_4 .. omega_(q-1) of the collision kernels g_4 ..
 * g_(q-1) (Sec. 7; Appendix G for D3Q15), n == q - 4 values, each in the open
 * interval (0, 2) (end of Sec. 7).  The shear viscosity is
 * nu = (1/omega - 1/2)/3 with omega = omega_4 = ... = omega_8.  Host array,
 * copied.  Errors: EINVAL (n, NULL, a rate outside (0, 2)). */
cmlbm_status cmlbm_set_rates(cmlbm_sim *sim, const double *omega, int n);

/* Form of the factorized attractors of the fourth- and sixth-order central
 * moments (Sec. 3, the list after Eq. centralmomentfdefinitionpostcollision;
 * Eq. transformedcentralmomentattractors).  per_mass = 0 (the default): the
 * literal products of the post-collision second moments, kxx~ kyy~ and
 * kxx~ kyy~ kzz~, as printed.  per_mass = 1: the same factorization per unit
 * mass, rho (kxx~/rho)(kyy~/rho) and rho (kxx~/rho)(kyy~/rho)(kzz~/rho), for
 * which the equilibrium is a fixed point at every density.  The two agree at
 * rho = 1.  Applies to the step and to the adjoint.  Errors: EINVAL unless
 * per_mass is 0 or 1. */
cmlbm_status cmlbm_set_attractor_per_mass(cmlbm_sim *sim, int per_mass);

/* Uniform body force F (force per unit volume, Sec. 3 Eq. forcingaliased).
 * Replaces any force field. */
cmlbm_status cmlbm_set_force_uniform(cmlbm_sim *sim, double fx, double fy, double fz);

/* Spatially varying body force, device array [3][nz][ny][nx] of "real",
 * borrowed until replaced.  NULL removes the field and sets the uniform force
 * to zero. */
cmlbm_status cmlbm_set_force_field(cmlbm_sim *sim, const void *F_dev);

/* Multiplier applied to the force (uniform or field) from the next call on,
 * e.g. cos(Omega t) for the time-periodic forcing of Sec. 9.  Default 1. */
cmlbm_status cmlbm_set_force_scale(cmlbm_sim *sim, double scale);

/* Solid mask for half-way bounce-back walls (Sec. 9): device array
 * [nz][ny][nx] of uint8, 0 = fluid, nonzero = solid; borrowed until replaced.
 * Solid nodes are never collided or written by cmlbm_step; a population that
 * would stream into a solid node returns reversed to its source node in the
 * same step.  NULL returns to fully periodic. */
cmlbm_status cmlbm_set_mask(cmlbm_sim *sim, const uint8_t *mask_dev);

/* Initial state.  rho_dev [nz][ny][nx] and u_dev [3][nz][ny][nx] ("real",
 * device) give the macroscopic fields; the pre-collision state is
 * fbar(x, 0) = f^eq(rho, u) - S(F, u)/2 (the transformation of Sec. 4 applied
 * to the equilibrium with the Maxwellian central moments of Sec. 3), so that
 * the velocity read back is u.  It is written, as full "real" populations,
 * into f_pre_dev [q][nz][ny][nx]; f_post_dev (population storage type) receives
 * the post-collision buffer whose first step pulls exactly fbar(x, 0).  Uses
 * the current force and mask.  Errors: EINVAL (NULL, f_pre_dev == f_post_dev). */
cmlbm_status cmlbm_init_equilibrium(cmlbm_sim *sim, const void *rho_dev, const void *u_dev, void *f_pre_dev,
                                    void *f_post_dev, void *stream);

/* One time step (Eqs. cascadedcollision1 and cascadedstreaming1): pull-stream
 * f_in (post-collision of step t-1), collide with forcing, write the
 * post-collision populations of step t into f_out.  f_in != f_out. */
cmlbm_status cmlbm_step(cmlbm_sim *sim, const void *f_in, void *f_out, void *stream);

/* One step exactly as cmlbm_step, which also reduces the FP64 totals of the
 * state it steps from (the pre-collision fbar(x, t) it pulls) inside the same
 * pass: totals_dev[0..3] = (sum rho, sum rho u_x, sum rho u_y, sum rho u_z)
 * over fluid nodes, rho u including F/2 (Eqs. densitycalculation,
 * velocitycalculation); the same quantities as cmlbm_totals(f_in), without a
 * second read of the populations.  totals_dev: 4 doubles of device memory,
 * overwritten, written asynchronously on `stream` (no host synchronization).
 * Errors: as cmlbm_step; EINVAL if totals_dev is NULL. */
cmlbm_status cmlbm_step_totals(cmlbm_sim *sim, const void *f_in, void *f_out, double *totals_dev, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same step
 * and totals as cmlbm_step_totals, bit for bit, with the per-block partial sums
 * kept in a static device array of the library (16 MiB + 8 KiB per device,
 * held until the process ends) instead of the handle's scratch.  This call
 * allocates nothing and clears nothing: every partial it reads was written by
 * the same call.  All handles on one device share that array, so calls that
 * overlap in time on one device race (order them on one stream).  Limit: the
 * lattice may have at most 2^19 step blocks, ceil(nx/256)*ny*nz <= 524288
 * (512^3, for instance).  Errors: as cmlbm_step_totals; EINVAL for a larger
 * lattice (checked before any launch); EDEVICE if the array's device address
 * could not be looked up when the handle was created. */
cmlbm_status cmlbm_step_totals_noalloc(cmlbm_sim *sim, const void *f_in, void *f_out, double *totals_dev,
                                       void *stream);

/* nsteps >= 0 steps ping-ponging between f_a and f_b, starting from f_a.
 * *result_in_b (may be NULL) is set to 1 when the last state is in f_b. */
cmlbm_status cmlbm_run(cmlbm_sim *sim, void *f_a, void *f_b, int nsteps, void *stream, int *result_in_b);

/* Copy a population buffer (blocked layout, storage type) into SoA
 * populations of "real" type [q][nz][ny][nx], decoding the 16-bit deviation
 * formats (the post-collision values themselves, not streamed).  f_buf != f_soa. */
cmlbm_status cmlbm_export_populations(cmlbm_sim *sim, const void *f_buf, void *f_soa, void *stream);

/* The inverse: SoA "real" populations into a population buffer (16-bit
 * formats store the rounded deviation from w_a). */
cmlbm_status cmlbm_import_populations(cmlbm_sim *sim, const void *f_soa, void *f_buf, void *stream);

/* The paper's state: pre-collision fbar(x, t) pulled from the post-collision
 * buffer f_post, as full "real" populations [q][nz][ny][nx] (zeros at solid
 * nodes).  f_post != f_pre. */
cmlbm_status cmlbm_gather_precollision(cmlbm_sim *sim, const void *f_post, void *f_pre, void *stream);

/* Density and velocity (Eqs. densitycalculation, velocitycalculation,
 * rho u = sum fbar e + F/2) of the pre-collision state of f_post; "real"
 * outputs rho [nz][ny][nx], u [3][nz][ny][nx]; zeros at solid nodes. */
cmlbm_status cmlbm_macroscopic(cmlbm_sim *sim, const void *f_post, void *rho, void *u, void *stream);

/* FP64 totals over fluid nodes of the pre-collision state: out4 = (sum rho,
 * sum rho u_x, sum rho u_y, sum rho u_z) with rho u including F/2.  Host
 * output; synchronizes `stream`. */
cmlbm_status cmlbm_totals(cmlbm_sim *sim, const void *f_post, double out4[4], void *stream);

/* In-place stepping: one population buffer instead of two, same bytes moved
 * per step (the AA pattern of Bailey et al., 2009, applied to the step of
 * Eqs. cascadedcollision1 and cascadedstreaming1, with the half-way
 * bounce-back of Sec. 9).  The buffer has the blocked layout and storage type
 * of the other population buffers and is in one of two phases:
 *   phase 0: slot a of node x holds the pre-collision fbar_a(x, t), the
 *            paper's state (cmlbm_import_populations of the f_pre written by
 *            cmlbm_init_equilibrium or cmlbm_gather_precollision gives it;
 *            cmlbm_export_populations reads it back);
 *   phase 1: slot abar of node x holds the post-collision fbar~_a(x, t).
 * parity = the phase of f on entry; each call is one time step (one
 * collision of every fluid node).  parity 0: phase 0 holding fbar(t) ->
 * phase 1 holding fbar~(t), every node reading and writing only its own
 * slots.  parity 1: phase 1 holding fbar~(t) -> phase 0 holding fbar(t + 2):
 * each node gathers fbar(x, t + 1) from its neighbours, collides, and scatters
 * the result to the slots its neighbours pull from next.  Solid nodes' slots
 * are never read or written.  Errors: EINVAL (NULL, parity not 0 or 1).  Calls
 * on one buffer must be ordered (one stream). */
cmlbm_status cmlbm_step_inplace(cmlbm_sim *sim, void *f, int parity, void *stream);

/* One in-place step exactly as cmlbm_step_inplace, which also reduces the FP64
 * totals of the pre-collision state it collides inside the same pass:
 * totals_dev[0..3] = (sum rho, sum rho u_x, sum rho u_y, sum rho u_z) over
 * fluid nodes, rho u including F/2 (Eqs. densitycalculation,
 * velocitycalculation).  Parity 0 totals fbar(t), the state the buffer holds;
 * parity 1 totals fbar(t + 1), the state it gathers.  The same values as
 * cmlbm_step_totals at the same step of a two-buffer run.  totals_dev: 4
 * doubles of device memory, overwritten asynchronously on `stream`.  Errors:
 * as cmlbm_step_inplace; EINVAL if totals_dev is NULL. */
cmlbm_status cmlbm_step_inplace_totals(cmlbm_sim *sim, void *f, int parity, double *totals_dev, void *stream);

/* The initial state of cmlbm_init_equilibrium, fbar(x, 0), written straight
 * into an in-place buffer f_dev in phase 0 (population storage type, blocked
 * rows): the same values as cmlbm_import_populations of its f_pre, without
 * the full-size "real" intermediate.  Solid nodes get zero populations (the
 * 16-bit formats store the rounded deviation -w_a).
 * Errors: EINVAL (NULL). */
cmlbm_status cmlbm_init_equilibrium_inplace(cmlbm_sim *sim, const void *rho_dev, const void *u_dev, void *f_dev,
                                            void *stream);

/* nsteps in-place steps (parities 0, 1, 0, 1, ...): f holds the pre-collision
 * fbar(t) in phase 0 on entry and fbar(t + nsteps) in phase 0 on return, the
 * same populations that cmlbm_run followed by cmlbm_gather_precollision gives.
 * Errors: EINVAL (NULL, nsteps odd or negative). */
cmlbm_status cmlbm_run_inplace(cmlbm_sim *sim, void *f, int nsteps, void *stream);

/* cmlbm_macroscopic and cmlbm_totals of a buffer in phase 0 (pre-collision
 * populations read in place rather than pulled). */
cmlbm_status cmlbm_macroscopic_pre(cmlbm_sim *sim, const void *f_pre_buf, void *rho, void *u, void *stream);
cmlbm_status cmlbm_totals_pre(cmlbm_sim *sim, const void *f_pre_buf, double out4[4], void *stream);

/* Adjoint of one step, D3Q27 or D3Q15 (reverse streaming plus the transposed
 * Jacobian of the central-moment collision and force terms of Sec. 7 and
 * Appendix G).  Forward step n maps the pre-collision state fbar^n, pulled
 * from f_post_prev, to fbar^(n+1).  Given lam_next = dL/dfbar^(n+1) ("real"
 * SoA populations [q][nz][ny][nx]), writes lam = dL/dfbar^n and accumulates
 * (adds) into
 *   dLdF_dev:     FP64 [3][nz][ny][nx] when a force field is set, or FP64 [3]
 *                 (dL/dF of the uniform force) otherwise;
 *   dLdomega_dev: FP64 [q-4], dL/domega_4 .. dL/domega_(q-1).
 * The force, rates and attractor form must be those of the forward step.
 * lam, lam_next and f_post_prev must not overlap. */
cmlbm_status cmlbm_adjoint_step(cmlbm_sim *sim, const void *f_post_prev, const void *lam_next, void *lam,
                                double *dLdF_dev, double *dLdomega_dev, void *stream);

/* Wall-layout sensitivity of one step.  The paper's walls are whole nodes
 * with half-way bounce-back (Sec. 9); to differentiate a loss with respect to
 * where they lie, give every node a wall fraction phi in [0, 1] and stream by
 *   fbar_a(x) = (1 - phi(x)) fbar~_a(x - e_a) + phi(x - e_a) fbar~_abar(x),
 * which is plain streaming at phi = 0 and the half-way bounce-back at phi = 1
 * (the population from s to t = s + e_a arrives with weight 1 - phi(t) and
 * returns reversed with weight phi(t), so mass is conserved).  At phi = the
 * mask, this call adds the step's contribution
 *   dL/dphi(t) += sum_a fbar~_a(t - e_a) (lam_abar(t - e_a) - lam_a(t))
 * over fluid neighbours t - e_a, to dLdphi_dev (FP64 [nz][ny][nx]) at every
 * fluid node t; solid nodes are left unchanged (the collision switches off at
 * phi = 1, so the derivative does not exist there).  f_post_prev and lam_next
 * are those of cmlbm_adjoint_step for the same step (lam_next = dL/dfbar^(n+1),
 * "real" SoA populations); call it before the adjoint step that replaces
 * lam_next.  The additions are FP64 atomics, in no fixed order.  Uses the
 * current force, rates and mask.  Errors: EINVAL (NULL, aliasing). */
cmlbm_status cmlbm_wall_sensitivity(cmlbm_sim *sim, const void *f_post_prev, const void *lam_next,
                                    double *dLdphi_dev, void *stream);

/* The same contribution from the state the streaming moves: f_post = fbar~
 * of the step as cmlbm_step wrote it (storage type, the buffer layout of
 * cmlbm_step's output), lam = dL/dfbar of the pre-collision state that
 * streaming f_post produces ("real" SoA populations; lam_next above).  Each
 * fluid node t gathers its own terms
 *   dL/dphi(t) += sum_a fbar~_a(t - e_a) (lam_abar(t - e_a) - lam_a(t))
 * (fluid neighbours t - e_a) in a fixed order, so the result is deterministic;
 * no collision is recomputed, and with 16-bit storage the terms use the
 * rounded populations the forward run streamed.  Call it with lam = the
 * output of the adjoint step whose f_post_prev is f_post, or with the
 * incoming gradient for the last state of a run.  Uses the current mask.
 * Errors: EINVAL (NULL, aliasing). */
cmlbm_status cmlbm_wall_sensitivity_post(cmlbm_sim *sim, const void *f_post, const void *lam,
                                         double *dLdphi_dev, void *stream);

/* Stability check (no operation of the paper: the relaxation rates of Sec. 7
 * lie in (0, 2) and are tuned for stability, which they do not guarantee):
 * *nonfinite = the number of stored populations of fluid nodes (every node
 * without a mask) in f_buf whose stored value is NaN or +-Inf.  f_buf is any
 * population buffer (blocked layout, storage type): the post-collision buffer
 * of cmlbm_step, or an in-place buffer in either phase.  For the 16-bit
 * deviation formats the stored deviation fbar_a - w_a is checked; FP16 rounds
 * |fbar_a - w_a| > 65504 to +-Inf, so overflow counts too.  One NaN
 * population makes every population of the node that pulls it NaN in the
 * next step, so 0 after a run means no node has diverged.  Reads f_buf once;
 * host output; synchronizes `stream`.  Errors: EINVAL (NULL, misaligned). */
cmlbm_status cmlbm_check_finite(cmlbm_sim *sim, const void *f_buf, int64_t *nonfinite, void *stream);

/* Kinetic-energy loss of a pre-collision state: *out = sum over fluid nodes of
 * |rho u|^2 / (2 rho), rho u = sum fbar e + F/2 (Eqs. densitycalculation,
 * velocitycalculation), accumulated in FP64.  f_pre: "real" [q][nz][ny][nx]
 * (as written by cmlbm_gather_precollision).  Host output; synchronizes. */
cmlbm_status cmlbm_kinetic_energy_sum(cmlbm_sim *sim, const void *f_pre, double *out, void *stream);

/* Seed of the adjoint sweep for the loss L = scale * (the sum above):
 * writes lam = dL/dfbar ("real" [q][nz][ny][nx]; dL/dfbar_a = scale (u.e_a -
 * |u|^2/2), zero at solid nodes) and accumulates dL/dF of the direct F/2 term,
 * scale * u/2, into dLdF_dev (FP64 [3][nz][ny][nx] for a force field, FP64 [3]
 * for a uniform force). */
cmlbm_status cmlbm_kinetic_energy_seed(cmlbm_sim *sim, const void *f_pre, double scale, void *lam,
                                       double *dLdF_dev, void *stream);

/* Adjoint of the initial state of cmlbm_init_equilibrium with respect to the
 * force: fbar(x, 0) = f^eq(rho, u0) - S(F, u0)/2 depends on F through S (Sec. 5
 * matching principle).  Accumulates -(1/2) (dS/dF)^T lam0 into dLdF_dev (same
 * layout as above).  u0_dev: "real" [3][nz][ny][nx]; lam0_dev = dL/dfbar(0)
 * ("real" SoA populations). */
cmlbm_status cmlbm_init_adjoint(cmlbm_sim *sim, const void *u0_dev, const void *lam0_dev, double *dLdF_dev,
                                void *stream);

/* Message for a status code (static string). */
const char *cmlbm_status_string(cmlbm_status code);

/* Message of the last failed call on this handle (valid until the next call);
 * "" when the last call succeeded.  NULL sim returns the message of the last
 * failed cmlbm_create on this thread. */
const char *cmlbm_last_error(const cmlbm_sim *sim);

/* Library version string, "major.minor.patch". */
const char *cmlbm_version(void);

#ifdef __cplusplus
}
#endif

#endif /* CMLBM_H */
