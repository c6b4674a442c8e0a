// Runs the MLP kernels (forward, backward, Adam) under the CPU emulation and
// compares them with the FP64 oracle: `emu_mlp N`.
#include <hip/hip_runtime.h>
#include <cmath>
#include <cstdio>
#include <random>
#include <vector>
#include "tileqr.h"
extern "C" {
void oracle_mlp_forward(const double *p, const double *x, int64_t n, double *y);
double oracle_mlp_grad(const double *p, const double *x, const double *y, int64_t n, double *g);
}
int main(int argc, char **argv) {
  const int NP = 8769;
  int n = argc > 1 ? atoi(argv[1]) : 150;
  int nm = 3;
  std::mt19937_64 g(7);
  std::normal_distribution<float> Nd(0.f, 1.f);
  std::vector<float> p((size_t)NP * nm), X((size_t)n * 5), y(n);
  for (auto &v : p) v = 0.2f * Nd(g);
  for (auto &v : X) v = Nd(g);
  for (auto &v : y) v = Nd(g);
  // forward
  std::vector<float> yo((size_t)n * nm);
  int rc = qr_mlp_forward(p.data(), nm, X.data(), n, yo.data(), nullptr);
  double worst = 0;
  for (int m = 0; m < nm; ++m) {
    std::vector<double> pd(p.begin() + (size_t)m * NP, p.begin() + (size_t)(m + 1) * NP), xd(X.begin(), X.end()), yd(n);
    oracle_mlp_forward(pd.data(), xd.data(), n, yd.data());
    for (int r = 0; r < n; ++r) worst = std::max(worst, std::fabs(yd[r] - yo[(size_t)m * n + r]) / (1e-3 + std::fabs(yd[r])));
  }
  printf("forward rc=%d worst rel %.3e\n", rc, worst);
  bool ok = rc == 0 && worst < 1e-3;
  // gradient
  std::vector<float> gr(NP), loss(1);
  rc = qr_mlp_grad(p.data(), X.data(), y.data(), n, gr.data(), loss.data(), nullptr);
  std::vector<double> pd(p.begin(), p.begin() + NP), xd(X.begin(), X.end()), yd(y.begin(), y.end()), gd(NP);
  double lo = oracle_mlp_grad(pd.data(), xd.data(), yd.data(), n, gd.data());
  double num = 0, den = 0;
  for (int e = 0; e < NP; ++e) { num += (gd[e] - gr[e]) * (gd[e] - gr[e]); den += gd[e] * gd[e]; }
  printf("grad rc=%d rel %.3e  loss %.6f vs %.6f\n", rc, std::sqrt(num / den), loss[0], lo);
  ok = ok && rc == 0 && std::sqrt(num / den) < 1e-5 && std::fabs(loss[0] - lo) < 1e-5 * std::fabs(lo);
  // training: loss decreases
  std::vector<double> lo0(nm);
  for (int m = 0; m < nm; ++m) {
    std::vector<double> pm(p.begin() + (size_t)m * NP, p.begin() + (size_t)(m + 1) * NP), gm(NP);
    lo0[m] = oracle_mlp_grad(pm.data(), xd.data(), yd.data(), n, gm.data());
  }
  std::vector<float> adam((size_t)2 * nm * NP, 0.f), lout(nm);
  rc = qr_mlp_train(p.data(), nm, adam.data(), X.data(), y.data(), n, 3, 32, 1e-3f, 11, 0, lout.data(), nullptr);
  printf("train rc=%d loss after 3 epochs: %.4f %.4f %.4f\n", rc, lout[0], lout[1], lout[2]);
  ok = ok && rc == 0;
  for (int m = 0; m < nm; ++m) {
    std::vector<double> pm(p.begin() + (size_t)m * NP, p.begin() + (size_t)(m + 1) * NP), gm(NP);
    const double after = oracle_mlp_grad(pm.data(), xd.data(), yd.data(), n, gm.data());
    printf("  model %d full-batch loss now %.4f\n", m, after);
    ok = ok && after < lo0[m];
  }
  return ok ? 0 : 1;
}
