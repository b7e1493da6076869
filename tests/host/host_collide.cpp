// Host build of the library's per-node device math, for CPU tests.
//
// The collision, its adjoint and the initial state are written once, as
// host-and-device functions in the library's headers; this file compiles
// those same functions for the CPU (with the HIP qualifiers defined away) and
// exports them with C linkage so that the CPU tests can compare them, element
// by element, with the oracle.  Populations are in the paper's direction order
// (the kernels reorder D3Q27 into the 3x3x3 cube exactly as done here).
#define __host__
#define __device__
#define __forceinline__ inline __attribute__((always_inline))

#include <cstdint>

#include "collide_d3q15.hpp"
#include "collide_d3q27.hpp"

namespace {

template <typename R>
cmlbm::Rates<R> rates(int q, const double* omega, int per_mass) {
  cmlbm::Rates<R> r{};
  for (int b = 0; b < 27; ++b) {
    r.w[b] = R(0);
    r.wc[b] = R(1);
  }
  for (int b = 4; b < q; ++b) {
    r.w[b] = R(omega[b - 4]);
    r.wc[b] = R(1.0 - omega[b - 4]);
  }
  r.per_mass = per_mass;
  return r;
}

template <typename R>
void collide(int q, const R* f, const R* F, const double* omega, int per_mass, R* out) {
  const cmlbm::Rates<R> p = rates<R>(q, omega, per_mass);
  if (q == 27) {
    R m[27];
    for (int a = 0; a < 27; ++a) m[cmlbm::cube27(a)] = f[a];
    cmlbm::collide27(m, F[0], F[1], F[2], p);
    for (int a = 0; a < 27; ++a) out[a] = m[cmlbm::cube27(a)];
  } else {
    R v[15];
    for (int a = 0; a < 15; ++a) v[a] = f[a];
    cmlbm::collide15(v, F[0], F[1], F[2], p);
    for (int a = 0; a < 15; ++a) out[a] = v[a];
  }
}

// gw[b - 4] accumulates dL/domega_b.
struct RateAcc {
  double* p;
  double& operator[](int b) const { return p[b - 4]; }
};

}  // namespace

extern "C" {

// Post-collision populations of one node (FP64 and FP32 arithmetic).
void hc_collide_f64(int q, const double* f, const double* F, const double* omega, int per_mass, double* out) {
  collide<double>(q, f, F, omega, per_mass, out);
}

void hc_collide_f32(int q, const float* f, const float* F, const double* omega, int per_mass, float* out) {
  collide<float>(q, f, F, omega, per_mass, out);
}

// Transposed Jacobian of the collision at f: g_in = adjoint of the
// post-collision populations, g_out = adjoint of f; adds dL/dF to gF[3] and
// dL/domega_b to gw[b - 4] (FP64).
void hc_collide_adj_f64(int q, const double* f, const double* F, const double* omega, int per_mass,
                        const double* g_in, double* g_out, double* gF, double* gw) {
  const cmlbm::Rates<double> p = rates<double>(q, omega, per_mass);
  double gw_full[27] = {};
  RateAcc acc{gw_full + 4};
  if (q == 27) {
    double m[27], g[27], s[27];
    for (int a = 0; a < 27; ++a) {
      m[cmlbm::cube27(a)] = f[a];
      g[cmlbm::cube27(a)] = g_in[a];
    }
    cmlbm::collide27_adj(m, F[0], F[1], F[2], p, g, s, gF[0], gF[1], gF[2], acc);
    for (int a = 0; a < 27; ++a) g_out[a] = g[cmlbm::cube27(a)];
  } else {
    double v[15], g[15];
    for (int a = 0; a < 15; ++a) {
      v[a] = f[a];
      g[a] = g_in[a];
    }
    cmlbm::collide15_adj(v, F[0], F[1], F[2], p, g, gF[0], gF[1], gF[2], acc);
    for (int a = 0; a < 15; ++a) g_out[a] = g[a];
  }
  for (int b = 4; b < q; ++b) gw[b - 4] += gw_full[b];
}

// Initial state fbar = f^eq(rho, u) - S(F, u)/2 of one node.
void hc_initial_f64(int q, double rho, const double* u, const double* F, double* out) {
  if (q == 27) {
    double f[27];
    cmlbm::initial27(rho, u[0], u[1], u[2], F[0], F[1], F[2], f);
    for (int a = 0; a < 27; ++a) out[a] = f[a];
  } else {
    double f[15];
    cmlbm::initial15(rho, u[0], u[1], u[2], F[0], F[1], F[2], f);
    for (int a = 0; a < 15; ++a) out[a] = f[a];
  }
}

// Adjoint of the initial state with respect to F (u fixed): adds to gF[3].
void hc_initial_adj_force_f64(int q, const double* u, const double* lam, double* gF) {
  if (q == 27) {
    double l[27];
    for (int a = 0; a < 27; ++a) l[a] = lam[a];
    cmlbm::initial27_adj_force(u[0], u[1], u[2], l, gF[0], gF[1], gF[2]);
  } else {
    double l[15];
    for (int a = 0; a < 15; ++a) l[a] = lam[a];
    cmlbm::initial15_adj_force(u[0], u[1], u[2], l, gF[0], gF[1], gF[2]);
  }
}

}  // extern "C"
