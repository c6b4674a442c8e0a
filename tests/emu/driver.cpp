// Runs the library's tile-QR kernels under the CPU emulation and compares
// the results with the C oracle: `emu_qr M N NB IB [P]` (factor + Q^T A
// with P row domains) or `emu_qr batch COUNT SEED` (one
// launch over uneven matrices).
#include <hip/hip_runtime.h>
#include <cstdio>
#include <vector>
#include <random>
#include <string>
#include "tq_sched.h"
#include "layout.h"
#include "plan.h"
#include "device_api.h"
extern "C" {
void oracle_geqr2(int64_t m, int64_t n, double *a, int64_t lda, double *tau);
void oracle_apply_qt(int64_t m, int64_t k, const double *v, int64_t ldv, const double *tau, int64_t nrhs, double *b, int64_t ldb);
}

// Tasks decoded on the device from the ticket in program order (the
// allocation-free entry point's launch): no task list.
static bool g_decode = false;

static int run(std::vector<MatDesc> mats, bool apply, int grid) {
  size_t lds = 0; int64_t c = 0;
  for (auto &m : mats) { m.ctr = c; c += apply ? ctr_count_apply(m) : ctr_count_factor(m); lds = std::max(lds, (size_t)lds_plan(m.nb, m.ib).doubles * 8); }
  std::vector<Task> order; int64_t nctr = 0;
  if (build_order(mats, apply, grid, order, &nctr)) { printf("build_order failed\n"); return 1; }
  std::vector<int> ctr(nctr + 64, 0);
  int err = 0;
  std::vector<MatDesc> dm = mats;
  TqLaunch a;
  a.tasks = order.data(); a.ntasks = order.size(); a.single = mats[0]; a.mats = mats.size() > 1 ? dm.data() : nullptr;
  if (g_decode && !apply && mats.size() == 1) a.tasks = nullptr;  // same count: every task once
  a.ctr = ctr.data(); a.ctr_base = ctr.data(); a.nctr_zero = nctr + 1; a.ticket = (unsigned *)(ctr.data() + nctr);
  a.trace = nullptr; a.err = &err; a.use_waits = 1; a.timeout = 1LL << 60; a.lds_bytes = lds; a.grid = grid;
  tq_launch_persistent(a, nullptr);
  if (err) printf("device error %d\n", err);
  return err;
}

// Batched: several matrices of uneven sizes and tilings in one launch (the
// union DAG), each compared with the oracle.
static int batch_main(int count, int seed) {
  std::mt19937_64 g(seed);
  std::uniform_real_distribution<double> U(-1, 1);
  const int nbs[3] = {64, 96, 128}, ibs[3][3] = {{16, 32, 64}, {16, 24, 48}, {16, 32, 128}};
  std::vector<int> Ms, Ns, NBs, IBs;
  for (int b = 0; b < count; ++b) {
    int M = 40 + (int)(g() % 150), N = 20 + (int)(g() % M);
    int c = (int)(g() % 3);
    Ms.push_back(M); Ns.push_back(N); NBs.push_back(nbs[c]); IBs.push_back(ibs[c][g() % 3]);
  }
  std::vector<std::vector<double>> As(count), A0s(count), Ts(count);
  std::vector<MatDesc> mats;
  for (int b = 0; b < count; ++b) {
    int M = Ms[b], N = Ns[b], nb = NBs[b], ib = IBs[b];
    As[b].resize((size_t)M * N);
    for (auto &x : As[b]) x = U(g);
    A0s[b] = As[b];
    MatDesc md; memset(&md, 0, sizeof md);
    LdsPlan lp = lds_plan(nb, ib);
    md_init(md, M, N, nb, ib, strip_width(nb), M);
    md.gmax = lp.gmax;
    md.lda = M;
    Ts[b].assign((size_t)md.KT * md.MT * ib * nb + 1, std::nan(""));
    md.A = As[b].data(); md.T = Ts[b].data();
    mats.push_back(md);
  }
  if (run(mats, false, 1)) return 1;
  double worst = 0;
  for (int b = 0; b < count; ++b) {
    int M = Ms[b], N = Ns[b], K = std::min(M, N);
    std::vector<double> Ao = A0s[b], tau(K);
    oracle_geqr2(M, N, Ao.data(), M, tau.data());
    double num = 0, den = 0;
    for (int i = 0; i < K; ++i) {
      double sg = As[b][i + (size_t)i * M] < 0 ? -1 : 1, so = Ao[i + (size_t)i * M] < 0 ? -1 : 1;
      for (int j = i; j < N; ++j) { double d = sg * As[b][i + (size_t)j * M] - so * Ao[i + (size_t)j * M]; num += d * d; den += Ao[i + (size_t)j * M] * Ao[i + (size_t)j * M]; }
    }
    double r = sqrt(num / den);
    worst = std::max(worst, r);
    printf("  b=%d M=%d N=%d nb=%d ib=%d R_rel=%.3e\n", b, M, N, NBs[b], IBs[b], r);
  }
  printf("batch count=%d seed=%d worst R_rel=%.3e\n", count, seed, worst);
  return worst < 1e-12 ? 0 : 1;
}

int main(int argc, char **argv) {
  if (std::string(argv[1]) == "batch") return batch_main(atoi(argv[2]), atoi(argv[3]));
  if (std::string(argv[1]) == "decode") { g_decode = true; ++argv; }
  int M = atoi(argv[1]), N = atoi(argv[2]), nb = atoi(argv[3]), ib = atoi(argv[4]);
  const int p = argc > 5 && !g_decode ? atoi(argv[5]) : 1;
  int64_t lda = M;
  std::mt19937_64 g(M * 7 + N);
  std::uniform_real_distribution<double> U(-1, 1);
  std::vector<double> A((size_t)lda * N), A0, Ao;
  for (auto &x : A) x = U(g);
  A0 = A; Ao = A;
  MatDesc md; memset(&md, 0, sizeof md);
  md_init(md, M, N, nb, ib, strip_width(nb), M, p);
  md.gmax = lds_plan(nb, ib).gmax;
  md.lda = lda;
  std::vector<double> T((size_t)T_doubles(md) + 1, std::nan(""));
  md.A = A.data(); md.T = T.data();
  if (run({md}, false, 1)) return 1;
  int K = std::min(M, N);
  std::vector<double> tau(K);
  oracle_geqr2(M, N, Ao.data(), lda, tau.data());
  // R comparison after sign normalisation
  double num = 0, den = 0;
  for (int i = 0; i < K; ++i) {
    double sg = A[i + (size_t)i * lda] < 0 ? -1 : 1, so = Ao[i + (size_t)i * lda] < 0 ? -1 : 1;
    for (int j = i; j < N; ++j) { double d = sg * A[i + (size_t)j * lda] - so * Ao[i + (size_t)j * lda]; num += d * d; den += Ao[i + (size_t)j * lda] * Ao[i + (size_t)j * lda]; }
  }
  // Q^T A0 via the emulated apply
  std::vector<double> B = A0;
  md.B = B.data(); md.ldb = lda; md.nrhs = N; md.SB = (N + md.w - 1) / md.w;
  if (run({md}, true, 1)) return 1;
  double rn = 0, an = 0;
  for (int j = 0; j < N; ++j) for (int i = 0; i < M; ++i) {
    double r = (i <= j && i < K) ? A[i + (size_t)j * lda] : 0.0;
    double d = B[i + (size_t)j * lda] - r; rn += d * d; an += A0[i + (size_t)j * lda] * A0[i + (size_t)j * lda];
  }
  // Q (Q^T A0) = A0 via the emulated reverse application
  md.notrans = 1;
  if (run({md}, true, 1)) return 1;
  double qn = 0;
  for (size_t e = 0; e < B.size(); ++e) qn += (B[e] - A0[e]) * (B[e] - A0[e]);
  const double rrel = sqrt(num / den), res = sqrt(rn / an), qres = sqrt(qn / an);
  printf("M=%d N=%d nb=%d ib=%d p=%d (h=%d)  R_rel=%.3e  resid=%.3e  QQt=%.3e\n", M, N, nb, ib, p,
         md.h, rrel, res, qres);
  return (rrel < 1e-12 && res < 1e-13 && qres < 1e-13) ? 0 : 1;
}
