// Test infrastructure: drives every entry point of the FP64 oracle on small 2D and
// 3D grids so that the oracle can be built and run under AddressSanitizer and
// UndefinedBehaviorSanitizer (see tests/test_oracle_sanitized.py).  Compiled together
// with sgp_oracle.cpp; prints "ok" when every result is finite.
#include <cmath>
#include <cstdio>
#include <vector>

extern "C" {
void orc_set_threads(int n);
void orc_fft(int dim, const int* n, double* data, int sign);
void orc_propagator(double Omega, double gamma, double nu_p, double nu_q, double delta, double* out25);
void orc_nl_point(const double* params, double V, double delta, double* psi5);
void orc_linear_step(int dim, const int* n, const double* L, const double* params, double delta, double* psi);
void orc_nl_step(int dim, const int* n, const double* L, const double* params, double delta, double theta,
                 double* psi);
void orc_rotation_map(int dim, const int* n, const double* L, const double* params, double t, int forward,
                      double* psi);
void orc_evolve(int dim, const int* n, const double* L, const double* params, int order, double tau, long nsteps,
                double t0, int mode, double* psi);
void orc_adjoint(int dim, const int* n, const double* L, const double* params, int order, double tau, long nsteps,
                 double t0, const double* psi0, const double* gT, double* g0, double* dpar, long K);
void orc_observables(int dim, const int* n, const double* L, const double* params, double theta, const double* psi,
                     double* out4);
}

namespace {

// deterministic values in [-0.5, 0.5) from a 64-bit linear congruential sequence
struct Lcg {
  unsigned long long s;
  double next() {
    s = s * 6364136223846793005ULL + 1442695040888963407ULL;
    return (double)(s >> 11) * (1.0 / 9007199254740992.0) - 0.5;
  }
};

bool finite(const std::vector<double>& v) {
  for (double x : v)
    if (!std::isfinite(x)) return false;
  return true;
}

bool run(int dim, const int n[3], const double L[3]) {
  const double params[8] = {50.0, -1.5, 3.0, 0.6, 0.7, 1.0, 1.2, 2.0};
  const long npts = (long)n[0] * n[1] * n[2];
  std::vector<double> psi(10 * npts), g(10 * npts), gT(10 * npts);
  Lcg r{(unsigned long long)(dim * 1000 + n[0])};
  for (auto& x : psi) x = 0.1 * r.next();
  for (auto& x : gT) x = r.next();
  bool ok = true;
  std::vector<double> a(psi);
  orc_fft(dim, n, a.data(), -1);
  orc_fft(dim, n, a.data(), +1);
  ok &= finite(a);
  std::vector<double> P(50);
  orc_propagator(0.6, 0.7, 0.3, -0.4, 1e-2, P.data());
  ok &= finite(P);
  std::vector<double> p5(psi.begin(), psi.begin() + 10);
  orc_nl_point(params, 0.5, 1e-2, p5.data());
  ok &= finite(p5);
  a = psi;
  orc_linear_step(dim, n, L, params, 1e-2, a.data());
  orc_nl_step(dim, n, L, params, 1e-2, 0.3, a.data());
  orc_rotation_map(dim, n, L, params, 0.4, 1, a.data());
  orc_rotation_map(dim, n, L, params, 0.4, 0, a.data());
  ok &= finite(a);
  for (int order : {2, 4, 6})
    for (int mode : {0, 1}) {
      a = psi;
      orc_evolve(dim, n, L, params, order, 2e-3, 3, 0.1, mode, a.data());
      ok &= finite(a);
    }
  std::vector<double> dpar(5), obs(4);
  orc_adjoint(dim, n, L, params, 4, 2e-3, 5, 0.0, psi.data(), gT.data(), g.data(), dpar.data(), 2);
  ok &= finite(g) && finite(dpar);
  orc_observables(dim, n, L, params, 0.2, psi.data(), obs.data());
  ok &= finite(obs);
  return ok;
}

}  // namespace

int main() {
  orc_set_threads(2);
  const int n2[3] = {16, 24, 1}, n3[3] = {12, 8, 8};
  const double L2[3] = {4.0, 5.0, 1.0}, L3[3] = {3.0, 3.0, 2.5};
  const bool ok = run(2, n2, L2) && run(3, n3, L3);
  std::printf("%s\n", ok ? "ok" : "non-finite result");
  return ok ? 0 : 1;
}
