// Host runtime of the tileqr C ABI: argument checking, the cache of
// persistent-launch plans (ticket order + dependency counters), launches,
// graph capture of batched launches, the Step-1 kernel benchmark and the
// run-time (NB, IB) decision.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <list>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/tileqr.h"
#include "device_api.h"
#include "layout.h"
#include "mlp_api.h"
#include "plan.h"

namespace {

std::mutex g_mu;

// ------------------------------------------------------------------ device

struct DevState {
  bool init = false;
  int ncu = 0;
  long long wall_khz = 100000;
  int *err = nullptr;  // sticky device error word
};
// Compute units of the device (taken from the device when its state is set
// up; the decision table's "all" budget stands for this count).
int g_full_cus = 256;

DevState g_dev[64];

int dev_state(DevState **out) {
  int d = 0;
  if (hipGetDevice(&d) != hipSuccess) return TILEQR_ERR_NODEVICE;
  if (d < 0 || d >= 64) return TILEQR_ERR_NODEVICE;
  DevState &s = g_dev[d];
  if (!s.init) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, d) != hipSuccess) return TILEQR_ERR_NODEVICE;
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) return TILEQR_ERR_NODEVICE;
    s.ncu = prop.multiProcessorCount;
    g_full_cus = s.ncu;
    int khz = 0;
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, d) == hipSuccess && khz > 0)
      s.wall_khz = khz;
    if (hipMalloc(&s.err, 256) != hipSuccess) return TILEQR_ERR_NOMEM;
    if (hipMemset(s.err, 0, 256) != hipSuccess) return TILEQR_ERR_HIP;
    if (hipDeviceSynchronize() != hipSuccess) return TILEQR_ERR_HIP;
    s.init = true;
  }
  *out = &s;
  return 0;
}

long long watchdog_ticks(const DevState &s) {
  double sec = 60.0;
  if (const char *e = std::getenv("TILEQR_WATCHDOG_S")) sec = std::atof(e);
  if (sec <= 0) sec = 60.0;
  return (long long)(sec * (double)s.wall_khz * 1000.0);
}

// ------------------------------------------------------------------- plans

struct Plan {
  Task *d_tasks = nullptr;
  int64_t ntasks = 0;
  int *d_ctr = nullptr;  // counters, then the ticket
  int64_t nctr = 0;
  MatDesc *d_mats = nullptr;
  std::vector<MatDesc> mats;  // host copy (pointers filled per call for singles)
  int grid = 1;
  size_t lds = 0;
  hipGraphExec_t graph = nullptr;
  ~Plan() {
    if (graph) hipGraphExecDestroy(graph);
    if (d_tasks) hipFree(d_tasks);
    if (d_ctr) hipFree(d_ctr);
    if (d_mats) hipFree(d_mats);
  }
};

// Device facts of the allocation-free entry point (no error word of its own:
// it lives in the static scratch).
struct NoallocDev {
  bool init = false;
  int ncu = 0;
  long long wall_khz = 100000;
};
NoallocDev g_noalloc[64];

// Compute units the persistent grid and its schedule are sized for (0: all
// of the device); see qr_set_compute_units.
int g_cu_limit = 0;

struct PlanKey {
  int dev, apply, nb, ib;
  int64_t M, N, nrhs;
  uint64_t batch_hash;
  int cus = g_cu_limit;
  int h = 0;  // tile rows per domain of the reduction tree
  bool operator<(const PlanKey &o) const {
    return std::tie(dev, apply, nb, ib, M, N, nrhs, batch_hash, cus, h) <
           std::tie(o.dev, o.apply, o.nb, o.ib, o.M, o.N, o.nrhs, o.batch_hash, o.cus, o.h);
  }
  bool operator==(const PlanKey &o) const { return !(*this < o) && !(o < *this); }
};

std::map<PlanKey, Plan *> g_plans;
std::list<PlanKey> g_lru;
const size_t kMaxPlans = 4096;

void touch(const PlanKey &k) {
  g_lru.remove(k);
  g_lru.push_front(k);
  while (g_lru.size() > kMaxPlans) {
    PlanKey old = g_lru.back();
    g_lru.pop_back();
    auto it = g_plans.find(old);
    if (it != g_plans.end()) {
      hipDeviceSynchronize();
      delete it->second;
      g_plans.erase(it);
    }
  }
}

// Geometry of one matrix: strip width and staged V chunks.
void md_setup(MatDesc &md, int64_t M, int64_t N, int nb, int ib, int64_t nrhs, int p = 1) {
  const LdsPlan lp = lds_plan(nb, ib);
  md_init(md, M, N, nb, ib, strip_width(nb), nrhs, p);
  md.gmax = lp.gmax;
}

// Builds (or fetches) the plan of a set of matrices sharing one kernel class.
int get_plan(const PlanKey &key, std::vector<MatDesc> mats, bool apply, const DevState &ds,
             Plan **out) {
  auto it = g_plans.find(key);
  if (it != g_plans.end()) {
    touch(key);
    *out = it->second;
    return 0;
  }
  size_t lds = 0;
  int64_t ctr = 0;
  for (MatDesc &m : mats) {
    m.ctr = ctr;
    ctr += apply ? ctr_count_apply(m) : ctr_count_factor(m);
    lds = std::max(lds, (size_t)lds_plan(m.nb, m.ib).doubles * 8);
  }
  int occ = tq_occupancy(lds);
  const int cus = (key.cus > 0 && key.cus < ds.ncu) ? key.cus : ds.ncu;
  int grid = std::max(1, cus * occ);
  Plan *p = new Plan();
  p->lds = lds;
  std::vector<Task> order;
  int64_t nctr = 0;
  int rc = build_order(mats, apply, grid, order, &nctr);
  if (rc != 0) {
    delete p;
    return TILEQR_ERR_INTERNAL;
  }
  if ((int64_t)order.size() >= ((int64_t)1 << 31)) {
    delete p;
    return TILEQR_ERR_TOO_LARGE;
  }
  // Host-side bounds check of every task against its matrix's tiling.
  for (const Task &t : order) {
    const MatDesc &m = mats[task_mat(t)];
    bool ok = t.k >= 0 && t.k < m.KT && t.i >= t.k && t.i < m.MT && t.j >= 0 && t.j < m.NT;
    const int s = task_strip(t), ty = task_type(t);
    if (ty == TK_LARFB || ty == TK_SSRFB || ty == TK_TTMQR) ok = ok && t.j > t.k && s < strips_of(m, t.j);
    if (task_on_B(ty)) ok = ok && s < m.SB;
    if (ty == TK_GEQRT || ty == TK_LARFB || ty == TK_LARFB_B) ok = ok && tree_is_head(m, t.i, t.k);
    if (ty == TK_TSQRT || ty == TK_SSRFB || ty == TK_SSRFB_B) ok = ok && !tree_is_head(m, t.i, t.k);
    if (ty == TK_TTQRT || ty == TK_TTMQR || ty == TK_TTMQR_B)
      ok = ok && t.i % m.h == 0 && t.i / m.h > t.k / m.h;
    if (!ok) {
      delete p;
      return TILEQR_ERR_INTERNAL;
    }
  }
  p->ntasks = (int64_t)order.size();
  p->nctr = nctr;
  p->grid = (int)std::min<int64_t>(grid, std::max<int64_t>(1, p->ntasks));
  p->mats = mats;
  if (p->ntasks > 0) {
    if (hipMalloc(&p->d_tasks, sizeof(Task) * p->ntasks) != hipSuccess) {
      delete p;
      return TILEQR_ERR_NOMEM;
    }
    if (hipMemcpy(p->d_tasks, order.data(), sizeof(Task) * p->ntasks, hipMemcpyHostToDevice) !=
        hipSuccess) {
      delete p;
      return TILEQR_ERR_HIP;
    }
  }
  if (hipMalloc(&p->d_ctr, sizeof(int) * (nctr + 64)) != hipSuccess) {
    delete p;
    return TILEQR_ERR_NOMEM;
  }
  if (mats.size() > 1) {
    if (hipMalloc(&p->d_mats, sizeof(MatDesc) * mats.size()) != hipSuccess) {
      delete p;
      return TILEQR_ERR_NOMEM;
    }
    if (hipMemcpy(p->d_mats, mats.data(), sizeof(MatDesc) * mats.size(), hipMemcpyHostToDevice) !=
        hipSuccess) {
      delete p;
      return TILEQR_ERR_HIP;
    }
  }
  g_plans[key] = p;
  touch(key);
  *out = p;
  return 0;
}

TqLaunch make_launch(const Plan &p, const DevState &ds, const MatDesc &single) {
  TqLaunch a;
  a.tasks = p.d_tasks;
  a.ntasks = p.ntasks;
  a.single = single;
  a.mats = p.d_mats;
  a.ctr = p.d_ctr;
  a.ctr_base = p.d_ctr;
  a.nctr_zero = p.nctr + 1;
  a.ticket = (unsigned int *)(p.d_ctr + p.nctr);
  a.err = ds.err;
  a.use_waits = 1;
  a.timeout = watchdog_ticks(ds);
  a.lds_bytes = p.lds;
  a.grid = p.grid;
  a.trace = nullptr;
  return a;
}

// Optional per-task trace of the last traced launch (TILEQR_TRACE=1).
struct TraceState {
  long long *d = nullptr;
  int64_t cap = 0, n = 0;
  std::vector<Task> order;
  int dev = -1;
};
TraceState g_trace;

bool trace_on() {
  const char *e = std::getenv("TILEQR_TRACE");
  return e && e[0] == '1';
}

long long *trace_buffer(int64_t ntasks) {
  int dev = 0;
  hipGetDevice(&dev);
  if (ntasks > g_trace.cap || dev != g_trace.dev) {
    if (g_trace.d) hipFree(g_trace.d);
    g_trace.d = nullptr;
    g_trace.cap = 0;
    if (hipMalloc(&g_trace.d, sizeof(long long) * 4 * ntasks) != hipSuccess) return nullptr;
    g_trace.cap = ntasks;
    g_trace.dev = dev;
  }
  g_trace.n = ntasks;
  return g_trace.d;
}

bool nb_ok(int nb) { return nb >= 16 && nb <= 512; }
bool nb_enabled(int nb) { return nb <= TQ_MAX_ENABLED_NB; }

int resolve_tiling(int64_t M, int64_t N, int64_t batch, int *nb, int *ib) {
  if (*nb == 0 || *ib == 0) {
    int tnb = 0, tib = 0, src = 0;
    int rc = qr_tune(M, N, batch, &tnb, &tib, &src);
    if (rc != 0) return rc;
    if (*nb == 0) *nb = tnb;
    if (*ib == 0) *ib = std::min(tib, *nb);
  }
  return 0;
}

int units_for(int64_t M, int64_t N, int64_t batch);
int domains_for(int64_t M, int64_t N, int nb);

int factor_one(double *A, int64_t M, int64_t N, int64_t lda, int NB, int IB, int p, double *T,
               hipStream_t st, const DevState &ds) {
  if (M == 0 || N == 0) return 0;
  MatDesc md;
  std::memset(&md, 0, sizeof(md));
  md_setup(md, M, N, NB, IB, 0, p);
  md.lda = lda;
  PlanKey key{0, 0, NB, IB, M, N, 0, 0};
  key.cus = units_for(M, N, 1);
  key.h = md.h;
  hipGetDevice(&key.dev);
  Plan *pl = nullptr;
  int rc = get_plan(key, {md}, false, ds, &pl);
  if (rc) return rc;
  md.A = A;
  md.T = T;
  md.B = nullptr;
  md.ctr = 0;
  TqLaunch a = make_launch(*pl, ds, md);
  if (trace_on()) {
    a.trace = trace_buffer(pl->ntasks);
    g_trace.order.resize(pl->ntasks);
    if (pl->ntasks)
      hipMemcpy(g_trace.order.data(), pl->d_tasks, sizeof(Task) * pl->ntasks, hipMemcpyDeviceToHost);
  }
  if (tq_launch_persistent(a, st) != hipSuccess) return TILEQR_ERR_HIP;
  return 0;
}

uint64_t mix(uint64_t h, uint64_t v) {
  h ^= v + 0x9E3779B97F4A7C15ull + (h << 6) + (h >> 2);
  return h;
}

// ------------------------------------------------------------ decision table

struct TableEntry {
  int64_t M, N, batch;
  int nb, ib;
  double gflops;
  int cus;     // compute units the grid is sized for (0: all)
  int p;       // row domains of the reduction tree (1: flat tree)
  int budget;  // compute units of the callers the entry was tuned for (0: all)
};
std::vector<TableEntry> g_table;
int g_default_nb = 128, g_default_ib = 32;

// Nearest benchmarked configuration (Section 6.1): log M, log N, log batch;
// ties go to the larger configuration. nullptr when the table is empty.
// Budget of the table section that serves callers limited to `cus` compute
// units (0: the whole device): the nearest in log scale (Section 6.1's
// interpolation over the core count); -1 when the table is empty.
int table_budget(int cus) {
  const double want = std::log((double)(cus > 0 ? cus : g_full_cus));
  int best = -1;
  double bd = 1e300;
  for (const TableEntry &e : g_table) {
    const int eff = e.budget > 0 ? e.budget : g_full_cus;
    const double d = std::fabs(std::log((double)eff) - want);
    if (d < bd - 1e-12 || (std::fabs(d - bd) <= 1e-12 && e.budget == 0)) {
      bd = d;
      best = e.budget;
    }
  }
  return best;
}

const TableEntry *nearest_entry(int64_t M, int64_t N, int64_t batch) {
  const double lm = std::log((double)std::max<int64_t>(M, 1)),
               ln = std::log((double)std::max<int64_t>(N, 1)), lb = std::log((double)batch);
  const int budget = table_budget(g_cu_limit);
  const TableEntry *best = nullptr;
  double bd = 1e300;
  int64_t bsize = -1;
  for (const TableEntry &e : g_table) {
    if (e.budget != budget) continue;
    const double d = std::pow(std::log((double)e.M) - lm, 2) +
                     std::pow(std::log((double)e.N) - ln, 2) +
                     std::pow(std::log((double)e.batch) - lb, 2);
    const int64_t size = e.M * e.N * e.batch;
    if (d < bd - 1e-12 || (std::fabs(d - bd) <= 1e-12 && size > bsize)) {
      bd = d;
      bsize = size;
      best = &e;
    }
  }
  return best;
}

// Units for one factorization: the explicit setting if any, else the
// decision table's choice for the shape (0: all).
int units_for(int64_t M, int64_t N, int64_t batch) {
  if (g_cu_limit > 0) return g_cu_limit;
  const TableEntry *e = nearest_entry(M, N, batch);
  return e ? e->cus : 0;
}

// Row domains of the reduction tree for one matrix: the nearest entry's
// (tuned with its tile order; 1 without a table). Called with g_mu held.
int domains_for(int64_t M, int64_t N, int nb) {
  (void)nb;
  const TableEntry *e = nearest_entry(M, N, 1);
  return e && e->p > 0 ? e->p : 1;
}

struct ModelState {
  int nmodels = 0;
  std::vector<float> params;
  float fmean[5], fstd[5];
  float ymean = 0, ystd = 1;
  std::vector<int> cand;  // (NB, IB) pairs
};
ModelState g_model;

}  // namespace

// =========================================================================
// C ABI
// =========================================================================

extern "C" {

const char *qr_version(void) { return "tileqr 0.1 (gfx950, FP64 MFMA)"; }

int64_t qr_T_size_ca(int64_t M, int64_t N, int NB, int IB, int p) {
  if (M < 0) return -1;
  if (N < 0) return -2;
  if (!nb_ok(NB)) return -3;
  if (IB < 1 || IB > NB) return -4;
  if (p < 0) return -5;
  if (M > INT32_MAX || N > INT32_MAX) return -1;
  if (p == 0) {
    std::lock_guard<std::mutex> lk(g_mu);
    p = domains_for(M, N, NB);
  }
  MatDesc md;
  std::memset(&md, 0, sizeof(md));
  md_init(md, M, N, NB, IB, strip_width(NB), 0, p);
  return T_doubles(md);
}

int64_t qr_T_size(int64_t M, int64_t N, int NB, int IB) { return qr_T_size_ca(M, N, NB, IB, 1); }

int qr_factor_ca(double *A, int64_t M, int64_t N, int64_t lda, int NB, int IB, int p, double *T,
                 void *stream) {
  if (M < 0) return -2;
  if (N < 0) return -3;
  if (!A && M * N > 0) return -1;
  if (lda < std::max<int64_t>(1, M)) return -4;
  if (NB != 0 && !nb_ok(NB)) return -5;
  if (IB < 0 || (NB != 0 && IB > NB)) return -6;
  if (p < 0) return -7;
  if (M > INT32_MAX || N > INT32_MAX) return TILEQR_ERR_TOO_LARGE;
  int rc = resolve_tiling(M, N, 1, &NB, &IB);
  if (rc) return rc;
  if (!nb_ok(NB)) return -5;
  if (IB < 1 || IB > NB) return -6;
  if (!T && M * N > 0) return -8;
  if (!nb_enabled(NB)) return TILEQR_ERR_DISABLED;
  std::lock_guard<std::mutex> lk(g_mu);
  if (p == 0) p = domains_for(M, N, NB);
  DevState *ds;
  if ((rc = dev_state(&ds))) return rc;
  return factor_one(A, M, N, lda, NB, IB, p, T, (hipStream_t)stream, *ds);
}

int qr_factor(double *A, int64_t M, int64_t N, int64_t lda, int NB, int IB, double *T,
              void *stream) {
  const int rc = qr_factor_ca(A, M, N, lda, NB, IB, 1, T, stream);
  return rc == -8 ? -7 : rc;
}

int qr_factor_noalloc(double *A, int64_t M, int64_t N, int64_t lda, int NB, int IB, double *T,
                      void *stream) {
  if (M < 0) return -2;
  if (N < 0) return -3;
  if (!A && M * N > 0) return -1;
  if (lda < std::max<int64_t>(1, M)) return -4;
  if (NB != 0 && !nb_ok(NB)) return -5;
  if (IB < 0 || (NB != 0 && IB > NB)) return -6;
  if (M > INT32_MAX || N > INT32_MAX) return TILEQR_ERR_TOO_LARGE;
  int rc = resolve_tiling(M, N, 1, &NB, &IB);
  if (rc) return rc;
  if (!nb_ok(NB)) return -5;
  if (IB < 1 || IB > NB) return -6;
  if (!T && M * N > 0) return -7;
  if (!nb_enabled(NB)) return TILEQR_ERR_DISABLED;
  if (M == 0 || N == 0) return 0;
  MatDesc md;
  std::memset(&md, 0, sizeof(md));
  md_setup(md, M, N, NB, IB, 0);
  md.lda = lda;
  md.A = A;
  md.T = T;
  const int64_t nctr = ctr_count_factor(md);
  if (TQ_NOALLOC_CTR_OFFSET + nctr > TQ_NOALLOC_SCRATCH_INTS) return TILEQR_ERR_TOO_LARGE;
  // tasks of the program order (as the device decodes them)
  int64_t ntasks = 0;
  const int64_t slast = strips_of(md, md.NT - 1);
  for (int64_t k = 0; k < md.KT; ++k) {
    const int64_t r = md.MT - 1 - k, c = md.NT - 1 - k;
    const int64_t cs = c >= 1 ? (c - 1) * md.S + slast : 0;
    ntasks += 1 + r + cs + r * cs;
  }
  if (ntasks >= INT32_MAX) return TILEQR_ERR_TOO_LARGE;
  std::lock_guard<std::mutex> lk(g_mu);
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return TILEQR_ERR_NODEVICE;
  NoallocDev &nd = g_noalloc[dev];
  if (!nd.init) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return TILEQR_ERR_NODEVICE;
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) return TILEQR_ERR_NODEVICE;
    nd.ncu = prop.multiProcessorCount;
    int khz = 0;
    nd.wall_khz = (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) == hipSuccess &&
                   khz > 0) ? khz : 100000;
    nd.init = true;
  }
  int *sp = nullptr;
  if (tq_noalloc_scratch(dev, &sp) != 0) return TILEQR_ERR_HIP;
  const size_t lds = (size_t)lds_plan(NB, IB).doubles * 8;
  const int occ = tq_occupancy(lds);
  const int units = units_for(M, N, 1);
  const int cus = (units > 0 && units < nd.ncu) ? units : nd.ncu;
  const int grid = (int)std::min<int64_t>((int64_t)cus * occ, ntasks);
  DevState tmp;
  tmp.wall_khz = nd.wall_khz;
  if (tq_launch_noalloc(sp, md, ntasks, nctr, std::max(1, grid), lds, watchdog_ticks(tmp),
                        (hipStream_t)stream) != hipSuccess)
    return TILEQR_ERR_HIP;
  return 0;
}

static int apply_impl(const double *A, int64_t M, int64_t N, int64_t lda, int NB, int IB, int p,
                      const double *T, double *B, int64_t nrhs, int64_t ldb, void *stream,
                      bool notrans) {
  if (M < 0) return -2;
  if (N < 0) return -3;
  if (!A && M * N > 0) return -1;
  if (lda < std::max<int64_t>(1, M)) return -4;
  if (NB != 0 && !nb_ok(NB)) return -5;
  if (IB < 0 || (NB != 0 && IB > NB)) return -6;
  if (p < 0) return -7;
  int rc = resolve_tiling(M, N, 1, &NB, &IB);
  if (rc) return rc;
  if (!nb_ok(NB)) return -5;
  if (IB < 1 || IB > NB) return -6;
  if (!T && M * N > 0) return -8;
  if (nrhs < 0) return -10;
  if (!B && M * nrhs > 0) return -9;
  if (ldb < std::max<int64_t>(1, M)) return -11;
  if (M > INT32_MAX || N > INT32_MAX || nrhs > INT32_MAX) return TILEQR_ERR_TOO_LARGE;
  if (!nb_enabled(NB)) return TILEQR_ERR_DISABLED;
  if (M == 0 || N == 0 || nrhs == 0) return 0;
  std::lock_guard<std::mutex> lk(g_mu);
  if (p == 0) p = domains_for(M, N, NB);
  DevState *ds;
  if ((rc = dev_state(&ds))) return rc;
  MatDesc md;
  std::memset(&md, 0, sizeof(md));
  md_setup(md, M, N, NB, IB, nrhs, p);
  if ((int64_t)md.SB > 4095) return TILEQR_ERR_TOO_LARGE;
  md.lda = lda;
  md.ldb = ldb;
  md.notrans = notrans ? 1 : 0;
  PlanKey key{0, notrans ? 2 : 1, NB, IB, M, N, nrhs, 0};
  key.cus = units_for(M, N, 1);
  key.h = md.h;
  hipGetDevice(&key.dev);
  Plan *pl = nullptr;
  if ((rc = get_plan(key, {md}, true, *ds, &pl))) return rc;
  md.A = const_cast<double *>(A);
  md.T = const_cast<double *>(T);
  md.B = B;
  md.ctr = 0;
  TqLaunch a = make_launch(*pl, *ds, md);
  if (tq_launch_persistent(a, (hipStream_t)stream) != hipSuccess) return TILEQR_ERR_HIP;
  return 0;
}

int qr_apply_Qt_ca(const double *A, int64_t M, int64_t N, int64_t lda, int NB, int IB, int p,
                   const double *T, double *B, int64_t nrhs, int64_t ldb, void *stream) {
  return apply_impl(A, M, N, lda, NB, IB, p, T, B, nrhs, ldb, stream, false);
}

int qr_apply_Q_ca(const double *A, int64_t M, int64_t N, int64_t lda, int NB, int IB, int p,
                  const double *T, double *B, int64_t nrhs, int64_t ldb, void *stream) {
  return apply_impl(A, M, N, lda, NB, IB, p, T, B, nrhs, ldb, stream, true);
}

int qr_apply_Q(const double *A, int64_t M, int64_t N, int64_t lda, int NB, int IB,
               const double *T, double *B, int64_t nrhs, int64_t ldb, void *stream) {
  const int rc = qr_apply_Q_ca(A, M, N, lda, NB, IB, 1, T, B, nrhs, ldb, stream);
  return rc <= -8 ? rc + 1 : rc;
}

int qr_form_Q_ca(const double *A, int64_t M, int64_t N, int64_t lda, int NB, int IB, int p,
                 const double *T, double *Q, int64_t k, int64_t ldq, void *stream) {
  if (k < 0 || k > M) return -10;
  if (!Q && M * k > 0) return -9;
  if (ldq < std::max<int64_t>(1, M)) return -11;
  // the argument checks of the apply come first: nothing is written on error
  int rc = apply_impl(A, M, N, lda, NB, IB, p, T, nullptr, 0, std::max<int64_t>(1, M), stream,
                      true);
  if (rc) return rc;
  if (M == 0 || k == 0) return 0;
  if (tq_launch_eye(Q, M, k, ldq, (hipStream_t)stream) != hipSuccess) return TILEQR_ERR_HIP;
  if (N == 0) return 0;
  return apply_impl(A, M, N, lda, NB, IB, p, T, Q, k, ldq, stream, true);
}

int qr_solve_ls_ca(const double *A, int64_t M, int64_t N, int64_t lda, int NB, int IB, int p,
                   const double *T, double *B, int64_t nrhs, int64_t ldb, void *stream) {
  if (N > M) return -3;
  int rc = apply_impl(A, M, N, lda, NB, IB, p, T, B, nrhs, ldb, stream, false);
  if (rc) return rc;
  if (N == 0 || nrhs == 0) return 0;
  if (tq_launch_trsv_upper(A, lda, N, B, ldb, nrhs, (hipStream_t)stream) != hipSuccess)
    return TILEQR_ERR_HIP;
  return 0;
}

int qr_apply_Qt(const double *A, int64_t M, int64_t N, int64_t lda, int NB, int IB,
                const double *T, double *B, int64_t nrhs, int64_t ldb, void *stream) {
  const int rc = qr_apply_Qt_ca(A, M, N, lda, NB, IB, 1, T, B, nrhs, ldb, stream);
  return rc <= -8 ? rc + 1 : rc;  // the argument positions without p
}

static int batched_check(double *const *A, const int64_t *M, const int64_t *N, const int64_t *lda,
                         int64_t count, const int *NB, const int *IB, double *const *T,
                         std::vector<int> &nbs, std::vector<int> &ibs) {
  if (count < 0) return -5;
  if (count > 0 && (!A || !M || !N || !lda || !NB || !IB || !T)) {
    if (!A) return -1;
    if (!M) return -2;
    if (!N) return -3;
    if (!lda) return -4;
    if (!NB) return -6;
    if (!IB) return -7;
    return -8;
  }
  if (count > 65535) return TILEQR_ERR_TOO_LARGE;
  nbs.resize(count);
  ibs.resize(count);
  for (int64_t b = 0; b < count; ++b) {
    if (M[b] < 0) return -2;
    if (N[b] < 0) return -3;
    if (M[b] > INT32_MAX || N[b] > INT32_MAX) return TILEQR_ERR_TOO_LARGE;
    if (!A[b] && M[b] * N[b] > 0) return -1;
    if (lda[b] < std::max<int64_t>(1, M[b])) return -4;
    int nb = NB[b], ib = IB[b];
    if (nb != 0 && !nb_ok(nb)) return -6;
    if (ib < 0 || (nb != 0 && ib > nb)) return -7;
    int rc = resolve_tiling(M[b], N[b], count, &nb, &ib);
    if (rc) return rc;
    if (!nb_ok(nb)) return -6;
    if (ib < 1 || ib > nb) return -7;
    if (!T[b] && M[b] * N[b] > 0) return -8;
    if (!nb_enabled(nb)) return TILEQR_ERR_DISABLED;
    nbs[b] = nb;
    ibs[b] = ib;
  }
  return 0;
}

int qr_factor_batched(double *const *A, const int64_t *M, const int64_t *N, const int64_t *lda,
                      int64_t count, const int *NB, const int *IB, double *const *T, void *stream) {
  std::vector<int> nbs, ibs;
  int rc = batched_check(A, M, N, lda, count, NB, IB, T, nbs, ibs);
  if (rc) return rc;
  std::lock_guard<std::mutex> lk(g_mu);
  DevState *ds;
  if ((rc = dev_state(&ds))) return rc;
  std::vector<MatDesc> mats;
  uint64_t h = 1469598103934665603ull;
  for (int64_t b = 0; b < count; ++b) {
    if (M[b] == 0 || N[b] == 0) continue;
    MatDesc md;
    std::memset(&md, 0, sizeof(md));
    md_setup(md, M[b], N[b], nbs[b], ibs[b], 0);
    md.lda = lda[b];
    md.A = A[b];
    md.T = T[b];
    mats.push_back(md);
    h = mix(h, (uint64_t)(uintptr_t)A[b]);
    h = mix(h, (uint64_t)(uintptr_t)T[b]);
    h = mix(h, (uint64_t)M[b]);
    h = mix(h, (uint64_t)N[b]);
    h = mix(h, (uint64_t)lda[b]);
    h = mix(h, ((uint64_t)nbs[b] << 32) | (uint32_t)ibs[b]);
  }
  if (mats.empty()) return 0;
  PlanKey key{0, 2, 0, 0, (int64_t)mats.size(), 0, 0, h};
  hipGetDevice(&key.dev);
  Plan *p = nullptr;
  if ((rc = get_plan(key, mats, false, *ds, &p))) return rc;
  hipStream_t st = (hipStream_t)stream;
  if (!p->graph) {
    // Capture the counter reset + persistent launch once; replay after.
    hipStream_t cap;
    if (hipStreamCreateWithFlags(&cap, hipStreamNonBlocking) != hipSuccess) return TILEQR_ERR_HIP;
    MatDesc dummy;
    std::memset(&dummy, 0, sizeof(dummy));
    TqLaunch a = make_launch(*p, *ds, dummy);
    hipGraph_t g = nullptr;
    bool ok = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal) == hipSuccess;
    ok = ok && tq_launch_persistent(a, cap) == hipSuccess;
    ok = (hipStreamEndCapture(cap, &g) == hipSuccess) && ok;
    ok = ok && hipGraphInstantiate(&p->graph, g, nullptr, nullptr, 0) == hipSuccess;
    if (g) hipGraphDestroy(g);
    hipStreamDestroy(cap);
    if (!ok) {
      p->graph = nullptr;
      return TILEQR_ERR_HIP;
    }
  }
  if (hipGraphLaunch(p->graph, st) != hipSuccess) return TILEQR_ERR_HIP;
  return 0;
}

int qr_factor_loop(double *const *A, const int64_t *M, const int64_t *N, const int64_t *lda,
                   int64_t count, const int *NB, const int *IB, double *const *T, void *stream) {
  std::vector<int> nbs, ibs;
  int rc = batched_check(A, M, N, lda, count, NB, IB, T, nbs, ibs);
  if (rc) return rc;
  std::lock_guard<std::mutex> lk(g_mu);
  DevState *ds;
  if ((rc = dev_state(&ds))) return rc;
  for (int64_t b = 0; b < count; ++b) {
    rc = factor_one(A[b], M[b], N[b], lda[b], nbs[b], ibs[b], 1, T[b], (hipStream_t)stream, *ds);
    if (rc) return rc;
  }
  return 0;
}

int qr_set_compute_units(int cus) {
  if (cus < 0) return -1;
  std::lock_guard<std::mutex> lk(g_mu);
  DevState *ds;
  int rc = dev_state(&ds);
  if (rc) return rc;
  if (cus > ds->ncu) return -1;
  g_cu_limit = cus;
  return 0;
}

int qr_sync(void *stream) {
  std::lock_guard<std::mutex> lk(g_mu);
  DevState *ds;
  int rc = dev_state(&ds);
  if (rc) return rc;
  if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess) return TILEQR_ERR_HIP;
  int e = 0;
  if (hipMemcpy(&e, ds->err, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess)
    return TILEQR_ERR_HIP;
  int dev = 0;
  hipGetDevice(&dev);
  if (int *sp = tq_noalloc_scratch_if_set(dev)) {
    int e2 = 0;
    if (hipMemcpy(&e2, sp, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess)
      return TILEQR_ERR_HIP;
    if (e2 != 0) {
      hipMemset(sp, 0, sizeof(int));
      if (e == 0) e = e2;
    }
  }
  if (e != 0) {
    hipMemset(ds->err, 0, sizeof(int));
    hipDeviceSynchronize();
    return e == TQ_DEVERR_WATCHDOG ? TILEQR_ERR_WATCHDOG : TILEQR_ERR_HIP;
  }
  return 0;
}

int qr_tile_task(int kind, double *A, int64_t M, int64_t N, int64_t lda, int NB, int IB, double *T,
                 int i, int j, int k, void *stream) {
  if (kind < 0 || kind > 3) return -1;
  if (!A) return -2;
  if (M < 1) return -3;
  if (N < 1) return -4;
  if (lda < M) return -5;
  if (!nb_ok(NB)) return -6;
  if (IB < 1 || IB > NB) return -7;
  if (!T) return -8;
  if (!nb_enabled(NB)) return TILEQR_ERR_DISABLED;
  MatDesc md;
  std::memset(&md, 0, sizeof(md));
  md_setup(md, M, N, NB, IB, 0);
  md.lda = lda;
  md.A = A;
  md.T = T;
  if (k < 0 || k >= md.KT) return -11;
  std::vector<Task> tasks;
  switch (kind) {
    case 0:
      tasks.push_back(make_task(TK_GEQRT, 0, k, k, k, 0));
      break;
    case 1:
      if (i <= k || i >= md.MT) return -9;
      tasks.push_back(make_task(TK_TSQRT, 0, i, k, k, 0));
      break;
    case 2:
      if (j <= k || j >= md.NT) return -10;
      for (int s = 0; s < strips_of(md, j); ++s) tasks.push_back(make_task(TK_LARFB, 0, k, j, k, s));
      break;
    case 3:
      if (i <= k || i >= md.MT) return -9;
      if (j <= k || j >= md.NT) return -10;
      for (int s = 0; s < strips_of(md, j); ++s)
        tasks.push_back(make_task(TK_SSRFB, 0, i, j, k, s));
      break;
  }
  std::lock_guard<std::mutex> lk(g_mu);
  DevState *ds;
  int rc = dev_state(&ds);
  if (rc) return rc;
  hipStream_t st = (hipStream_t)stream;
  Task *d_tasks = nullptr;
  int *d_ctr = nullptr;
  if (hipMalloc(&d_tasks, sizeof(Task) * tasks.size()) != hipSuccess) return TILEQR_ERR_NOMEM;
  if (hipMalloc(&d_ctr, 256) != hipSuccess) {
    hipFree(d_tasks);
    return TILEQR_ERR_NOMEM;
  }
  rc = 0;
  if (hipMemcpyAsync(d_tasks, tasks.data(), sizeof(Task) * tasks.size(), hipMemcpyHostToDevice,
                     st) != hipSuccess)
    rc = TILEQR_ERR_HIP;
  size_t lds = (size_t)lds_plan(NB, IB).doubles * 8;
  TqLaunch a;
  a.tasks = d_tasks;
  a.ntasks = (int64_t)tasks.size();
  a.single = md;
  a.mats = nullptr;
  a.ctr = d_ctr;
  a.ctr_base = d_ctr;
  a.nctr_zero = 1;
  a.ticket = (unsigned int *)d_ctr;
  a.err = ds->err;
  a.use_waits = 0;
  a.timeout = watchdog_ticks(*ds);
  a.lds_bytes = lds;
  a.grid = (int)tasks.size();
  a.trace = nullptr;
  if (!rc && tq_launch_persistent(a, st) != hipSuccess) rc = TILEQR_ERR_HIP;
  if (hipStreamSynchronize(st) != hipSuccess) rc = TILEQR_ERR_HIP;
  hipFree(d_tasks);
  hipFree(d_ctr);
  return rc;
}

int qr_ssrfb_bench(int NB, int IB, int calls, int workers, double *seconds) {
  if (!nb_ok(NB)) return -1;
  if (IB < 1 || IB > NB) return -2;
  if (calls < 1) return -3;
  if (workers < 0) return -4;
  if (!seconds) return -5;
  if (!nb_enabled(NB)) return TILEQR_ERR_DISABLED;
  std::lock_guard<std::mutex> lk(g_mu);
  DevState *ds;
  int rc = dev_state(&ds);
  if (rc) return rc;
  int grid = workers > 0 ? workers : ds->ncu;
  int64_t per = 3 * (int64_t)NB * NB + (int64_t)IB * NB;
  static double *buf = nullptr;
  static int64_t cap = 0;
  static int bdev = -1;
  int dev = 0;
  hipGetDevice(&dev);
  if (per * grid > cap || dev != bdev) {
    if (buf) hipFree(buf);
    buf = nullptr;
    cap = per * grid;
    bdev = dev;
    if (hipMalloc(&buf, sizeof(double) * cap) != hipSuccess) {
      cap = 0;
      return TILEQR_ERR_NOMEM;
    }
  }
  // Small values keep repeated updates bounded (no overflow or denormals).
  if (tq_launch_fill(buf, per * grid, 12345, 0.02, 0) != hipSuccess) return TILEQR_ERR_HIP;
  hipEvent_t e0, e1;
  hipEventCreate(&e0);
  hipEventCreate(&e1);
  hipEventRecord(e0, 0);
  hipError_t he = tq_launch_ssrfb_bench(buf, NB, IB, calls, grid, 0);
  hipEventRecord(e1, 0);
  if (hipEventSynchronize(e1) != hipSuccess || he != hipSuccess) rc = TILEQR_ERR_HIP;
  float ms = 0;
  hipEventElapsedTime(&ms, e0, e1);
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  *seconds = ms * 1e-3;
  return rc;
}

// Step 1 with cold caches: every call in its own launch, each preceded by a
// write over `flush_bytes` of scratch memory (larger than the L2 caches and
// the MALL together) that evicts the tiles; only the DSSRFB launches are
// timed. The tiles are the same per workgroup as in qr_ssrfb_bench.
int qr_ssrfb_bench_flush(int NB, int IB, int calls, int workers, int64_t flush_bytes,
                         double *seconds) {
  if (!nb_ok(NB)) return -1;
  if (IB < 1 || IB > NB) return -2;
  if (calls < 1) return -3;
  if (workers < 0) return -4;
  if (flush_bytes < 0 || flush_bytes > ((int64_t)64 << 30)) return -5;
  if (!seconds) return -6;
  if (!nb_enabled(NB)) return TILEQR_ERR_DISABLED;
  std::lock_guard<std::mutex> lk(g_mu);
  DevState *ds;
  int rc = dev_state(&ds);
  if (rc) return rc;
  const int grid = workers > 0 ? workers : ds->ncu;
  const int64_t per = 3 * (int64_t)NB * NB + (int64_t)IB * NB;
  const int64_t nflush = flush_bytes / 8;
  double *buf = nullptr, *flush = nullptr;
  if (hipMalloc(&buf, sizeof(double) * per * grid) != hipSuccess) return TILEQR_ERR_NOMEM;
  if (nflush > 0 && hipMalloc(&flush, sizeof(double) * nflush) != hipSuccess) {
    hipFree(buf);
    return TILEQR_ERR_NOMEM;
  }
  hipEvent_t e0, e1;
  hipEventCreate(&e0);
  hipEventCreate(&e1);
  double total = 0.0;
  if (tq_launch_fill(buf, per * grid, 12345, 0.02, 0) != hipSuccess) rc = TILEQR_ERR_HIP;
  for (int c = 0; c < calls && !rc; ++c) {
    if (nflush > 0 && tq_launch_fill(flush, nflush, 777 + (uint64_t)c, 1.0, 0) != hipSuccess) {
      rc = TILEQR_ERR_HIP;
      break;
    }
    hipEventRecord(e0, 0);
    if (tq_launch_ssrfb_bench(buf, NB, IB, 1, grid, 0) != hipSuccess) rc = TILEQR_ERR_HIP;
    hipEventRecord(e1, 0);
    if (hipEventSynchronize(e1) != hipSuccess) rc = TILEQR_ERR_HIP;
    float ms = 0.f;
    hipEventElapsedTime(&ms, e0, e1);
    total += ms * 1e-3;
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  hipFree(buf);
  if (flush) hipFree(flush);
  *seconds = total;
  return rc;
}

// The FP64 MFMA ceiling: wg_per_cu workgroups of four waves per compute unit
// run the register-only probe; rate from the launch time, clock from the
// probe's own shader-clock and wall-clock spans.
int qr_mfma_probe(int wg_per_cu, int iters, double *tflops, double *ghz) {
  if (wg_per_cu < 1 || wg_per_cu > 8) return -1;
  if (iters < 1) return -2;
  if (!tflops) return -3;
  std::lock_guard<std::mutex> lk(g_mu);
  DevState *ds;
  int rc = dev_state(&ds);
  if (rc) return rc;
  const int grid = wg_per_cu * ds->ncu;
  double *out = nullptr;
  if (hipMalloc(&out, sizeof(double) * (2 + (int64_t)grid * 256)) != hipSuccess)
    return TILEQR_ERR_NOMEM;
  hipEvent_t e0, e1;
  hipEventCreate(&e0);
  hipEventCreate(&e1);
  // a short launch first, so the timed one starts at the running clock
  hipError_t he = tq_launch_mfma_probe(out, grid, iters / 8 + 1, 0);
  hipEventRecord(e0, 0);
  if (he == hipSuccess) he = tq_launch_mfma_probe(out, grid, iters, 0);
  hipEventRecord(e1, 0);
  if (hipEventSynchronize(e1) != hipSuccess || he != hipSuccess) rc = TILEQR_ERR_HIP;
  float ms = 0;
  hipEventElapsedTime(&ms, e0, e1);
  double span[2] = {0.0, 0.0};
  if (!rc && hipMemcpy(span, out, sizeof(span), hipMemcpyDeviceToHost) != hipSuccess)
    rc = TILEQR_ERR_HIP;
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  hipFree(out);
  if (rc) return rc;
  const double flops = 2048.0 * tq_mfma_probe_chains() * (double)iters * 4.0 * grid;
  *tflops = ms > 0 ? flops / (ms * 1e-3) / 1e12 : 0.0;
  if (ghz)
    *ghz = (span[1] > 0 && ds->wall_khz > 0) ? span[0] / (span[1] / (ds->wall_khz * 1e3)) / 1e9
                                             : 0.0;
  return 0;
}

// ------------------------------------------------------------------ tuning

int qr_tune_load(const char *path) {
  if (!path) return -1;
  FILE *f = std::fopen(path, "r");
  if (!f) return TILEQR_ERR_NOTABLE;
  std::vector<TableEntry> t;
  int dnb = 128, dib = 32, budget = 0;
  char line[512];
  bool bad = false;
  while (std::fgets(line, sizeof line, f)) {
    char *p = line;
    while (*p == ' ' || *p == '\t') ++p;
    if (*p == '#' || *p == '\n' || *p == 0) continue;
    TableEntry e;
    long long m, n, b;
    e.cus = 0;
    e.p = 1;
    e.budget = budget;
    const int got = std::sscanf(p, "entry %lld %lld %lld %d %d %lf %d %d", &m, &n, &b, &e.nb,
                                &e.ib, &e.gflops, &e.cus, &e.p);
    if (got >= 6 && got <= 8) {
      if (e.cus < 0 || e.p < 1) bad = true;
      e.M = m;
      e.N = n;
      e.batch = b;
      if (!nb_ok(e.nb) || e.ib < 1 || e.ib > e.nb || m < 1 || n < 1 || b < 1) bad = true;
      t.push_back(e);
    } else if (std::sscanf(p, "budget %d", &budget) == 1) {
      if (budget < 0) bad = true;
    } else if (std::sscanf(p, "default %d %d", &dnb, &dib) == 2) {
      if (!nb_ok(dnb) || dib < 1 || dib > dnb) bad = true;
    } else {
      bad = true;
    }
  }
  std::fclose(f);
  if (bad) return TILEQR_ERR_NOTABLE;
  std::lock_guard<std::mutex> lk(g_mu);
  g_table = t;
  g_default_nb = dnb;
  g_default_ib = dib;
  return 0;
}

int qr_tune_set_model(const float *params, int nmodels, const float *feat_mean,
                      const float *feat_std, float y_mean, float y_std, const int *cand,
                      int ncand) {
  if (nmodels < 0 || nmodels > 64) return -1;
  if (nmodels > 0) {
    if (!params) return -2;
    if (!feat_mean) return -3;
    if (!feat_std) return -4;
    for (int i = 0; i < 5; ++i)
      if (!(feat_std[i] > 0.f)) return -4;
    if (!cand || ncand < 1 || ncand > 4096) return -7;
    for (int c = 0; c < ncand; ++c)
      if (!nb_ok(cand[2 * c]) || cand[2 * c + 1] < 1 || cand[2 * c + 1] > cand[2 * c]) return -7;
  }
  std::lock_guard<std::mutex> lk(g_mu);
  g_model = ModelState();
  if (nmodels == 0) return 0;
  g_model.nmodels = nmodels;
  g_model.params.assign(params, params + (size_t)nmodels * TQ_MLP_NPARAM);
  std::memcpy(g_model.fmean, feat_mean, sizeof(float) * 5);
  std::memcpy(g_model.fstd, feat_std, sizeof(float) * 5);
  g_model.ymean = y_mean;
  g_model.ystd = y_std;
  g_model.cand.assign(cand, cand + 2 * ncand);
  return 0;
}

int qr_tune(int64_t M, int64_t N, int64_t batch, int *NB, int *IB, int *source) {
  if (M < 0) return -1;
  if (N < 0) return -2;
  if (batch < 1) return -3;
  if (!NB) return -4;
  if (!IB) return -5;
  int src = 0;
  const char *enb = std::getenv("TILEQR_NB");
  const char *eib = std::getenv("TILEQR_IB");
  if (enb && eib) {
    int a = std::atoi(enb), b = std::atoi(eib);
    if (nb_ok(a) && b >= 1 && b <= a) {
      *NB = a;
      *IB = b;
      if (source) *source = 3;
      return 0;
    }
  }
  std::lock_guard<std::mutex> lk(g_mu);
  int nb = g_default_nb, ib = g_default_ib;
  const TableEntry *e = nearest_entry(M, N, batch);
  if (e) {
    nb = e->nb;
    ib = e->ib;
    src = 1;
  }
  // The cost model ranks (NB, IB) pairs of the flat tree on the whole
  // device: it is consulted only where the table's decision is one of those.
  if (g_model.nmodels > 0 && !(e && (e->p > 1 || e->budget > 0))) {
    int mnb = 0, mib = 0;
    double spread = 1.0;
    int rc = tq_mlp_choose(g_model.params.data(), g_model.nmodels, g_model.fmean, g_model.fstd,
                           g_model.ymean, g_model.ystd, g_model.cand.data(),
                           (int)(g_model.cand.size() / 2), M, N, batch, &mnb, &mib, &spread);
    if (rc == 0) {
      if (spread <= 0.05) {
        nb = mnb;
        ib = mib;
        src = 2;
      } else {
        src |= 8;
      }
    }
  }
  *NB = nb;
  *IB = std::min(ib, nb);
  if (source) *source = src;
  return 0;
}

int qr_tune_domains(int64_t M, int64_t N, int64_t batch, int *p) {
  if (M < 0) return -1;
  if (N < 0) return -2;
  if (batch < 1) return -3;
  if (!p) return -4;
  std::lock_guard<std::mutex> lk(g_mu);
  const TableEntry *e = nearest_entry(M, N, batch);
  *p = e && e->p > 0 ? e->p : 1;
  return 0;
}

int qr_tune_units(int64_t M, int64_t N, int64_t batch, int *cus) {
  if (M < 0) return -1;
  if (N < 0) return -2;
  if (batch < 1) return -3;
  if (!cus) return -4;
  std::lock_guard<std::mutex> lk(g_mu);
  *cus = units_for(M, N, batch);
  return 0;
}

int qr_trace_fetch(int64_t *out, int64_t cap, int64_t *ntasks) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (ntasks) *ntasks = g_trace.n;
  if (!out || !g_trace.d || g_trace.n == 0) return 0;
  if (hipDeviceSynchronize() != hipSuccess) return TILEQR_ERR_HIP;
  std::vector<long long> h((size_t)4 * g_trace.n);
  if (hipMemcpy(h.data(), g_trace.d, sizeof(long long) * h.size(), hipMemcpyDeviceToHost) !=
      hipSuccess)
    return TILEQR_ERR_HIP;
  DevState *ds;
  int rc = dev_state(&ds);
  if (rc) return rc;
  for (int64_t t = 0; t < g_trace.n && t < cap; ++t) {
    const Task &tk = g_trace.order[t];
    int64_t *o = out + 9 * t;
    o[0] = task_type(tk);
    o[1] = tk.i;
    o[2] = tk.j;
    o[3] = tk.k;
    o[4] = task_strip(tk);
    // wall-clock ticks -> nanoseconds
    o[5] = (int64_t)(h[4 * t + 0] * (1e6 / (double)ds->wall_khz));
    o[6] = (int64_t)(h[4 * t + 1] * (1e6 / (double)ds->wall_khz));
    o[7] = (int64_t)(h[4 * t + 2] * (1e6 / (double)ds->wall_khz));
    o[8] = h[4 * t + 3];
  }
  return 0;
}

// --------------------------------------------------------- host inspection

int qr_dag_counts(int64_t M, int64_t N, int NB, int64_t *counts) {
  if (M < 0) return -1;
  if (N < 0) return -2;
  if (NB < 1) return -3;
  if (!counts) return -4;
  dag_tile_counts(M, N, NB, counts);
  return 0;
}

double qr_flops(int64_t M, int64_t N) {
  double m = (double)M, n = (double)N;
  if (M >= N) return 2.0 * m * n * n - 2.0 * n * n * n / 3.0;
  return 2.0 * n * m * m - 2.0 * m * m * m / 3.0;
}

double qr_flops_executed(int64_t M, int64_t N, int NB, int IB) {
  if (M <= 0 || N <= 0 || NB < 1 || IB < 1) return 0.0;
  // Task by task: Householder generation + updates inside GEQRT/TSQRT, and
  // the compact-WY applications (two products with V plus the T product per
  // inner block) in LARFB/SSRFB.
  int64_t MT = (M + NB - 1) / NB, NT = (N + NB - 1) / NB, KT = std::min(MT, NT);
  auto rows = [&](int64_t i) { return (double)std::min<int64_t>(NB, M - i * NB); };
  auto cols = [&](int64_t j) { return (double)std::min<int64_t>(NB, N - j * NB); };
  // Applying kref reflectors of height h (unit: trapezoidal) to c columns in
  // blocks of IB, T applied as a triangular product.
  auto apply = [&](double h, double kref, double c, bool unit, bool top) {
    double f = 0.0;
    for (double s = 0; s < kref; s += IB) {
      double w = std::min<double>(IB, kref - s);
      double hh = unit ? h - s : h;  // rows touched
      double vtc = 2.0 * hh * w * c - (unit ? w * w * c : 0.0);
      f += 2.0 * vtc + w * w * c + (top ? 2.0 * w * c : 0.0);
    }
    return f;
  };
  double f = 0.0;
  for (int64_t k = 0; k < KT; ++k) {
    double mb = rows(k), nb = cols(k), kk = std::min(mb, nb);
    // GEQRT: unblocked QR of the tile (LAPACK geqr2 count) plus T.
    f += 2.0 * mb * nb * kk - (mb + nb) * kk * kk + 2.0 * kk * kk * kk / 3.0;
    for (int64_t j = k + 1; j < NT; ++j) f += apply(mb, kk, cols(j), true, false);
    for (int64_t i = k + 1; i < MT; ++i) {
      double mi = rows(i);
      f += 2.0 * mi * nb * nb + 0.0;  // TSQRT: reflectors of height mi+1 on nb columns
      for (int64_t j = k + 1; j < NT; ++j) f += apply(mi, nb, cols(j), false, true);
    }
  }
  return f;
}

int qr_plan_check(int64_t M, int64_t N, int NB, int IB, int p, int64_t nrhs, int apply,
                  int workers, uint64_t seed, int64_t *ntasks, int64_t *seq, int64_t *stress) {
  if (M < 1 || N < 1 || !nb_ok(NB) || IB < 1 || IB > NB || workers < 1 || p < 1)
    return TILEQR_ERR_INTERNAL;
  MatDesc md;
  std::memset(&md, 0, sizeof(md));
  md_setup(md, M, N, NB, IB, apply ? nrhs : 0, p);
  md.notrans = apply == 2 ? 1 : 0;
  md.ctr = 0;
  std::vector<MatDesc> mats{md};
  std::vector<Task> order;
  int64_t nctr = 0;
  if (build_order(mats, apply != 0, workers, order, &nctr) != 0) return TILEQR_ERR_INTERNAL;
  if (ntasks) *ntasks = (int64_t)order.size();
  if (seq) *seq = check_order_sequential(mats, order);
  if (stress) *stress = stress_order(mats, apply != 0, order, workers, seed);
  return 0;
}

int qr_plan_tasks(int64_t M, int64_t N, int NB, int IB, int p, int64_t nrhs, int apply,
                  int workers, int32_t *out, int64_t cap, int64_t *ntasks) {
  if (M < 1 || N < 1 || !nb_ok(NB) || IB < 1 || IB > NB || workers < 1 || p < 1)
    return TILEQR_ERR_INTERNAL;
  MatDesc md;
  std::memset(&md, 0, sizeof(md));
  md_setup(md, M, N, NB, IB, apply ? nrhs : 0, p);
  md.notrans = apply == 2 ? 1 : 0;
  md.ctr = 0;
  std::vector<MatDesc> mats{md};
  std::vector<Task> order;
  if (build_order(mats, apply != 0, workers, order, nullptr) != 0) return TILEQR_ERR_INTERNAL;
  if (ntasks) *ntasks = (int64_t)order.size();
  if (out) {
    for (int64_t t = 0; t < (int64_t)order.size() && t < cap; ++t) {
      out[5 * t + 0] = task_type(order[t]);
      out[5 * t + 1] = order[t].i;
      out[5 * t + 2] = order[t].j;
      out[5 * t + 3] = order[t].k;
      out[5 * t + 4] = task_strip(order[t]);
    }
  }
  return 0;
}

}  // extern "C"
