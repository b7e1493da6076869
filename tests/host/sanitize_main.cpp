// Driver for the sanitizer build of the host device math: runs every exported
// function of host_collide.cpp on pseudo-random nodes of both lattices, in
// FP64 and FP32, and checks that mass is conserved and every output finite.
// Built with -fsanitize=address,undefined by the CPU tests; any report or a
// nonzero exit status fails them.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <initializer_list>

extern "C" {
void hc_collide_f64(int q, const double* f, const double* F, const double* omega, int per_mass, double* out);
void hc_collide_f32(int q, const float* f, const float* F, const double* omega, int per_mass, float* out);
void hc_collide_adj_f64(int q, const double* f, const double* F, const double* omega, int per_mass,
                        const double* g_in, double* g_out, double* gF, double* gw);
void hc_initial_f64(int q, double rho, const double* u, const double* F, double* out);
void hc_initial_adj_force_f64(int q, const double* u, const double* lam, double* gF);
}

namespace {
uint64_t state = 0x9e3779b97f4a7c15ull;
double uniform(double lo, double hi) {   // xorshift64*
  state ^= state >> 12;
  state ^= state << 25;
  state ^= state >> 27;
  const uint64_t r = state * 0x2545f4914f6cdd1dull;
  return lo + (hi - lo) * double(r >> 11) * (1.0 / 9007199254740992.0);
}
}  // namespace

int main() {
  int bad = 0;
  for (int q : {27, 15}) {
    for (int it = 0; it < 200; ++it) {
      const int pm = it & 1;
      double u[3], F[3], omega[23], f[27], out[27], g[27], gout[27], gF[3] = {0, 0, 0}, gw[23] = {};
      for (int i = 0; i < 3; ++i) {
        u[i] = uniform(-0.1, 0.1);
        F[i] = uniform(-1e-3, 1e-3);
      }
      for (int i = 0; i < q - 4; ++i) omega[i] = uniform(0.2, 1.9);
      const double rho = uniform(0.9, 1.1);
      hc_initial_f64(q, rho, u, F, f);
      for (int a = 0; a < q; ++a) f[a] += uniform(-1e-3, 1e-3);
      hc_collide_f64(q, f, F, omega, pm, out);
      double m0 = 0, m1 = 0;
      for (int a = 0; a < q; ++a) {
        m0 += f[a];
        m1 += out[a];
        g[a] = uniform(-1, 1);
      }
      if (!(std::fabs(m0 - m1) < 1e-12)) ++bad;
      hc_collide_adj_f64(q, f, F, omega, pm, g, gout, gF, gw);
      hc_initial_adj_force_f64(q, u, g, gF);
      float f32[27], F32[3] = {float(F[0]), float(F[1]), float(F[2])}, o32[27];
      for (int a = 0; a < q; ++a) f32[a] = float(f[a]);
      hc_collide_f32(q, f32, F32, omega, pm, o32);
      for (int a = 0; a < q; ++a)
        if (!std::isfinite(out[a]) || !std::isfinite(gout[a]) || !std::isfinite(o32[a])) ++bad;
      for (int i = 0; i < 3; ++i)
        if (!std::isfinite(gF[i])) ++bad;
      for (int i = 0; i < q - 4; ++i)
        if (!std::isfinite(gw[i])) ++bad;
    }
  }
  std::printf("host device math: %d failures\n", bad);
  return bad == 0 ? 0 : 1;
}
