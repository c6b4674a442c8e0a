// Host construction of the tile QR DAG and its ticket order.
#include "plan.h"

#include <algorithm>
#include <cstring>
#include <queue>
#include <random>
#include <unordered_map>

void md_init(MatDesc &md, int64_t M, int64_t N, int nb, int ib, int w, int64_t nrhs, int p) {
  md.M = (int32_t)M;
  md.N = (int32_t)N;
  md.nb = nb;
  md.ib = ib;
  md.w = w;
  md.MT = (int32_t)((M + nb - 1) / nb);
  md.NT = (int32_t)((N + nb - 1) / nb);
  md.KT = md.MT < md.NT ? md.MT : md.NT;
  md.S = (nb + w - 1) / w;
  md.nrhs = (int32_t)nrhs;
  md.SB = nrhs > 0 ? (int32_t)((nrhs + w - 1) / w) : 0;
  md.gmax = 1;
  const int pp = p < 1 ? 1 : (p > md.MT ? (md.MT > 0 ? md.MT : 1) : p);
  md.h = md.MT > 0 ? (md.MT + pp - 1) / pp : 1;
  md.D = md.MT > 0 ? (md.MT + md.h - 1) / md.h : 1;
  md.notrans = 0;
}

void tree_step(const MatDesc &md, int k, std::vector<int> &heads, std::vector<int> &rest,
               std::vector<int> &bottoms) {
  heads.clear();
  rest.clear();
  bottoms.clear();
  for (int i = k; i < md.MT; ++i) (tree_is_head(md, i, k) ? heads : rest).push_back(i);
  const int dk = k / md.h, E = md.D - dk;
  for (int l = 0; (1 << l) < E; ++l)
    for (int e1 = 0; e1 + (1 << l) < E; e1 += 2 << l) bottoms.push_back((dk + e1 + (1 << l)) * md.h);
}

void enum_factor_tasks(const MatDesc &md, int mat, std::vector<Task> &out) {
  std::vector<int> heads, rest, bottoms;
  for (int k = 0; k < md.KT; ++k) {
    tree_step(md, k, heads, rest, bottoms);
    for (int i : heads) out.push_back(make_task(TK_GEQRT, mat, i, k, k, 0));
    for (int i : rest) out.push_back(make_task(TK_TSQRT, mat, i, k, k, 0));
    for (int i : bottoms) out.push_back(make_task(TK_TTQRT, mat, i, k, k, 0));
    const int types[3] = {TK_LARFB, TK_SSRFB, TK_TTMQR};
    const std::vector<int> *rows[3] = {&heads, &rest, &bottoms};
    for (int q = 0; q < 3; ++q)
      for (int i : *rows[q])
        for (int j = k + 1; j < md.NT; ++j)
          for (int s = 0; s < strips_of(md, j); ++s) out.push_back(make_task(types[q], mat, i, j, k, s));
  }
}

void enum_apply_tasks(const MatDesc &md, int mat, std::vector<Task> &out) {
  std::vector<int> heads, rest, bottoms;
  const size_t first = out.size();
  for (int k = 0; k < md.KT; ++k) {
    tree_step(md, k, heads, rest, bottoms);
    const int types[3] = {TK_LARFB_B, TK_SSRFB_B, TK_TTMQR_B};
    const std::vector<int> *rows[3] = {&heads, &rest, &bottoms};
    for (int q = 0; q < 3; ++q)
      for (int i : *rows[q])
        for (int s = 0; s < md.SB; ++s) out.push_back(make_task(types[q], mat, i, 0, k, s));
  }
  // B <- Q B: the reflectors in the opposite order
  if (md.notrans) std::reverse(out.begin() + first, out.end());
}

void dag_tile_counts(int64_t M, int64_t N, int nb, int64_t counts[4]) {
  int64_t MT = (M + nb - 1) / nb, NT = (N + nb - 1) / nb, KT = MT < NT ? MT : NT;
  counts[0] = KT;
  counts[1] = counts[2] = counts[3] = 0;
  for (int64_t k = 0; k < KT; ++k) {
    counts[1] += MT - 1 - k;
    counts[2] += NT - 1 - k;
    counts[3] += (MT - 1 - k) * (NT - 1 - k);
  }
}

double task_cost(const Task &t, const MatDesc &m) {
  // Duration of one task on one workgroup (ns) with two workgroups per
  // compute unit, fitted to task traces of the persistent kernel at NB = 64
  // and NB = 128 under full load: a panel costs a latency per Householder
  // column that grows with the rows it touches; an update strip costs a
  // fixed latency (staging, barriers, dependency fences) plus its MFMA work.
  // Only relative sizes matter: they set the list schedule's priorities.
  const double g_col0 = 3280.0, g_row = 80.3;   // GEQRT: ns per column, + per row
  const double t_col0 = 3460.0, t_row = 97.5;   // TSQRT
  const double l_fix = 48000.0, l_rate = 0.066;  // LARFB: ns + ns per (rows*refl*cols)
  const double s_fix = 94000.0, s_rate = 0.103;  // SSRFB
  int s = task_strip(t);
  const int ty = task_type(t);
  const double mb = tile_rows(m, t.i), nbk = tile_cols(m, t.k);
  double c = task_on_B(ty) ? m.nrhs - s * m.w : (ty == TK_GEQRT || ty == TK_TSQRT || ty == TK_TTQRT)
                                                      ? 0.0 : tile_cols(m, t.j) - s * m.w;
  c = c < m.w ? c : m.w;
  switch (ty) {
    case TK_GEQRT: {
      double kk = mb < nbk ? mb : nbk;
      return kk * (g_col0 + g_row * mb);
    }
    case TK_TSQRT:
    case TK_TTQRT: return nbk * (t_col0 + t_row * mb);
    case TK_LARFB:
    case TK_LARFB_B: return l_fix + l_rate * mb * nbk * c;
    case TK_SSRFB:
    case TK_TTMQR:
    case TK_SSRFB_B:
    case TK_TTMQR_B: return s_fix + s_rate * mb * nbk * c;
  }
  return 1.0;
}

namespace {

struct Dag {
  std::vector<Task> tasks;          // program order
  std::vector<int32_t> succ_off;    // CSR successors
  std::vector<int32_t> succ;
  std::vector<int32_t> ndeps;
};

// Derives the DAG edges from the counter protocol itself: the task a wait
// (counter c, target v) depends on is the one that gives counter c its v-th
// increment in program order.
int derive_dag(const std::vector<MatDesc> &mats, bool apply, Dag &d) {
  d.tasks.clear();
  for (size_t m = 0; m < mats.size(); ++m) {
    if (apply) enum_apply_tasks(mats[m], (int)m, d.tasks);
    else enum_factor_tasks(mats[m], (int)m, d.tasks);
  }
  const int64_t T = (int64_t)d.tasks.size();
  int64_t nctr = 0;
  for (const MatDesc &m : mats) {
    int64_t e = m.ctr + (apply ? ctr_count_apply(m) : ctr_count_factor(m));
    nctr = e > nctr ? e : nctr;
  }
  std::vector<std::vector<int32_t>> signalers((size_t)nctr);
  std::vector<int32_t> pred_off(T + 1, 0);
  std::vector<int32_t> pred;
  pred.reserve((size_t)T * 3);
  for (int64_t t = 0; t < T; ++t) {
    const Task &tk = d.tasks[t];
    const MatDesc &m = mats[task_mat(tk)];
    int nw = task_nwaits(tk, m);
    for (int q = 0; q < nw; ++q) {
      int64_t idx;
      int target;
      task_wait(tk, m, q, &idx, &target);
      if (target <= 0) continue;
      if (idx < 0 || idx >= nctr) return -2;
      if ((int)signalers[idx].size() < target) return -3;  // would wait on a later task
      pred.push_back(signalers[idx][target - 1]);
    }
    pred_off[t + 1] = (int32_t)pred.size();
    int ns = task_nsignals(tk);
    for (int q = 0; q < ns; ++q) {
      int64_t idx = task_signal(tk, m, q);
      if (idx < 0 || idx >= nctr) return -2;
      signalers[idx].push_back((int32_t)t);
    }
  }
  d.ndeps.assign(T, 0);
  std::vector<int32_t> cnt(T + 1, 0);
  for (int64_t t = 0; t < T; ++t) {
    for (int32_t e = pred_off[t]; e < pred_off[t + 1]; ++e) cnt[pred[e] + 1]++;
    d.ndeps[t] = pred_off[t + 1] - pred_off[t];
  }
  for (int64_t t = 0; t < T; ++t) cnt[t + 1] += cnt[t];
  d.succ_off = cnt;
  d.succ.assign(pred.size(), 0);
  std::vector<int32_t> fill(cnt.begin(), cnt.end() - 1);
  for (int64_t t = 0; t < T; ++t)
    for (int32_t e = pred_off[t]; e < pred_off[t + 1]; ++e) d.succ[fill[pred[e]]++] = (int32_t)t;
  return 0;
}

}  // namespace

int build_order(const std::vector<MatDesc> &mats, bool apply, int workers,
                std::vector<Task> &order, int64_t *counter_total) {
  Dag d;
  int rc = derive_dag(mats, apply, d);
  if (rc != 0) return rc;
  const int64_t T = (int64_t)d.tasks.size();
  if (counter_total) {
    int64_t nctr = 0;
    for (const MatDesc &m : mats) {
      int64_t e = m.ctr + (apply ? ctr_count_apply(m) : ctr_count_factor(m));
      nctr = e > nctr ? e : nctr;
    }
    *counter_total = nctr;
  }
  std::vector<double> cost(T), bl(T);
  for (int64_t t = 0; t < T; ++t) cost[t] = task_cost(d.tasks[t], mats[task_mat(d.tasks[t])]);
  for (int64_t t = T - 1; t >= 0; --t) {
    double b = 0.0;
    for (int32_t e = d.succ_off[t]; e < d.succ_off[t + 1]; ++e) b = std::max(b, bl[d.succ[e]]);
    bl[t] = cost[t] + b;
  }
  typedef std::pair<double, int32_t> RP;  // (bottom level, -index)
  std::priority_queue<RP> ready;
  typedef std::pair<double, int32_t> EV;  // (-finish, task)
  std::priority_queue<EV> events;
  std::vector<int32_t> rem(d.ndeps);
  for (int64_t t = 0; t < T; ++t)
    if (rem[t] == 0) ready.push(RP(bl[t], (int32_t)-t));
  order.clear();
  order.reserve(T);
  double now = 0.0;
  int free_w = workers > 0 ? workers : 1;
  while ((int64_t)order.size() < T) {
    while (free_w > 0 && !ready.empty()) {
      int32_t t = -ready.top().second;
      ready.pop();
      order.push_back(d.tasks[t]);
      events.push(EV(-(now + cost[t]), t));
      --free_w;
    }
    if (events.empty()) return -4;  // cycle: cannot happen for a DAG
    now = -events.top().first;
    while (!events.empty() && -events.top().first <= now) {
      int32_t t = events.top().second;
      events.pop();
      ++free_w;
      for (int32_t e = d.succ_off[t]; e < d.succ_off[t + 1]; ++e) {
        int32_t s = d.succ[e];
        if (--rem[s] == 0) ready.push(RP(bl[s], -s));
      }
    }
  }
  return 0;
}

int64_t check_order_sequential(const std::vector<MatDesc> &mats, const std::vector<Task> &order) {
  int64_t nctr = 0;
  for (const MatDesc &m : mats) {
    int64_t e = m.ctr + std::max(ctr_count_apply(m), ctr_count_factor(m));
    nctr = e > nctr ? e : nctr;
  }
  std::vector<int32_t> ctr((size_t)nctr, 0);
  int64_t bad = 0;
  for (const Task &t : order) {
    const MatDesc &m = mats[task_mat(t)];
    int nw = task_nwaits(t, m);
    for (int q = 0; q < nw; ++q) {
      int64_t idx;
      int target;
      task_wait(t, m, q, &idx, &target);
      if (ctr[idx] < target) ++bad;
    }
    int ns = task_nsignals(t);
    for (int q = 0; q < ns; ++q) ctr[task_signal(t, m, q)]++;
  }
  return bad;
}

namespace {

// Data items a task touches, written from what each kernel reads and writes
// (independently of the counter protocol). A head tile is split into its R
// part (upper, rewritten by the TSQRTs and merges of the step) and its V part
// (lower, read by the LARFBs of the step).
struct Access {
  int64_t item;
  bool write;
};

int64_t item_strip(const MatDesc &m, int mat, int i, int j, int s) {
  return ((int64_t)mat << 40) | ((((int64_t)i * m.NT + j) * m.S + s) * 4 + 0);
}
int64_t item_rpart(const MatDesc &m, int mat, int i, int k) {
  return ((int64_t)mat << 40) | ((((int64_t)i * m.NT + k) * m.S) * 4 + 1);
}
int64_t item_vpart(const MatDesc &m, int mat, int i, int k) {
  return ((int64_t)mat << 40) | ((((int64_t)i * m.NT + k) * m.S) * 4 + 2);
}
int64_t item_T(const MatDesc &m, int mat, int i, int k) {
  return ((int64_t)mat << 40) | ((((int64_t)i * m.NT + k) * m.S) * 4 + 3);
}
// A merge's reflector block and T factor (domain d of the bottom head, step k).
int64_t item_tree(const MatDesc &m, int mat, int d, int k, int which) {
  return ((int64_t)mat << 40) | ((int64_t)1 << 38) | ((((int64_t)k * m.D + d) << 1) + which);
}
int64_t item_B(const MatDesc &m, int mat, int i, int s) {
  return ((int64_t)mat << 40) | ((int64_t)1 << 39) | ((int64_t)i * m.SB + s);
}

void accesses(const Task &t, const MatDesc &m, std::vector<Access> &a) {
  a.clear();
  int mat = task_mat(t), i = t.i, j = t.j, k = t.k, s = task_strip(t);
  switch (task_type(t)) {
    case TK_GEQRT:
      for (int q = 0; q < strips_of(m, k); ++q) a.push_back({item_strip(m, mat, i, k, q), true});
      a.push_back({item_rpart(m, mat, i, k), true});
      a.push_back({item_vpart(m, mat, i, k), true});
      a.push_back({item_T(m, mat, i, k), true});
      break;
    case TK_TSQRT:
      a.push_back({item_rpart(m, mat, tree_head(m, i, k), k), true});
      for (int q = 0; q < strips_of(m, k); ++q) a.push_back({item_strip(m, mat, i, k, q), true});
      a.push_back({item_T(m, mat, i, k), true});
      break;
    case TK_TTQRT:
      a.push_back({item_rpart(m, mat, tree_partner(m, i, k), k), true});
      a.push_back({item_rpart(m, mat, i, k), false});
      a.push_back({item_tree(m, mat, i / m.h, k, 0), true});
      a.push_back({item_tree(m, mat, i / m.h, k, 1), true});
      break;
    case TK_LARFB:
      a.push_back({item_vpart(m, mat, i, k), false});
      a.push_back({item_T(m, mat, i, k), false});
      a.push_back({item_strip(m, mat, i, j, s), true});
      break;
    case TK_SSRFB:
      for (int q = 0; q < strips_of(m, k); ++q) a.push_back({item_strip(m, mat, i, k, q), false});
      a.push_back({item_T(m, mat, i, k), false});
      a.push_back({item_strip(m, mat, tree_head(m, i, k), j, s), true});
      a.push_back({item_strip(m, mat, i, j, s), true});
      break;
    case TK_TTMQR:
      a.push_back({item_tree(m, mat, i / m.h, k, 0), false});
      a.push_back({item_tree(m, mat, i / m.h, k, 1), false});
      a.push_back({item_strip(m, mat, tree_partner(m, i, k), j, s), true});
      a.push_back({item_strip(m, mat, i, j, s), true});
      break;
    case TK_LARFB_B:
      a.push_back({item_B(m, mat, i, s), true});
      break;
    case TK_SSRFB_B:
      a.push_back({item_B(m, mat, tree_head(m, i, k), s), true});
      a.push_back({item_B(m, mat, i, s), true});
      break;
    case TK_TTMQR_B:
      a.push_back({item_B(m, mat, tree_partner(m, i, k), s), true});
      a.push_back({item_B(m, mat, i, s), true});
      break;
  }
}

}  // namespace

int64_t stress_order(const std::vector<MatDesc> &mats, bool apply,
                     const std::vector<Task> &order, int workers, uint64_t seed) {
  // Program order and task identity.
  std::vector<Task> prog;
  for (size_t m = 0; m < mats.size(); ++m) {
    if (apply) enum_apply_tasks(mats[m], (int)m, prog);
    else enum_factor_tasks(mats[m], (int)m, prog);
  }
  const int64_t T = (int64_t)prog.size();
  if ((int64_t)order.size() != T) return -2;
  auto key = [](const Task &t) {
    return ((uint64_t)(uint32_t)t.w0 << 32) ^ ((uint64_t)(uint32_t)t.i << 42) ^
           ((uint64_t)(uint32_t)t.j << 21) ^ (uint64_t)(uint32_t)t.k;
  };
  std::unordered_map<uint64_t, int64_t> pos;
  pos.reserve((size_t)T * 2);
  for (int64_t p = 0; p < T; ++p) pos[key(prog[p])] = p;
  int64_t nctr = 0;
  for (const MatDesc &m : mats) {
    int64_t e = m.ctr + (apply ? ctr_count_apply(m) : ctr_count_factor(m));
    nctr = e > nctr ? e : nctr;
  }
  std::vector<int32_t> ctr((size_t)nctr, 0);
  std::vector<double> start(T, -1.0), finish(T, -1.0);
  std::mt19937_64 rng(seed);
  std::uniform_real_distribution<double> dur(0.1, 10.0);

  enum { IDLE, WAITING, RUNNING };
  std::vector<int> state(workers, IDLE);
  std::vector<int64_t> cur(workers, -1);
  std::vector<double> end_t(workers, 0.0);
  int64_t next = 0, done = 0;
  double now = 0.0;
  while (done < T) {
    for (int w = 0; w < workers; ++w)
      if (state[w] == IDLE && next < T) {
        cur[w] = next++;
        state[w] = WAITING;
      }
    for (int w = 0; w < workers; ++w) {
      if (state[w] != WAITING) continue;
      const Task &t = order[cur[w]];
      const MatDesc &m = mats[task_mat(t)];
      bool ok = true;
      int nw = task_nwaits(t, m);
      for (int q = 0; q < nw && ok; ++q) {
        int64_t idx;
        int target;
        task_wait(t, m, q, &idx, &target);
        ok = ctr[idx] >= target;
      }
      if (ok) {
        state[w] = RUNNING;
        end_t[w] = now + dur(rng);
        start[pos[key(t)]] = now;
      }
    }
    double tmin = 1e300;
    for (int w = 0; w < workers; ++w)
      if (state[w] == RUNNING && end_t[w] < tmin) tmin = end_t[w];
    if (tmin == 1e300) return -1;  // everyone waits: deadlock
    now = tmin;
    for (int w = 0; w < workers; ++w) {
      if (state[w] == RUNNING && end_t[w] <= now) {
        const Task &t = order[cur[w]];
        const MatDesc &m = mats[task_mat(t)];
        int ns = task_nsignals(t);
        for (int q = 0; q < ns; ++q) ctr[task_signal(t, m, q)]++;
        finish[pos[key(t)]] = now;
        state[w] = IDLE;
        ++done;
      }
    }
  }
  // Hazard check in program order per data item.
  struct Last {
    int64_t last_write = -1;
    std::vector<int64_t> reads_since;
  };
  std::unordered_map<int64_t, Last> items;
  std::vector<Access> acc;
  int64_t bad = 0;
  for (int64_t p = 0; p < T; ++p) {
    const Task &t = prog[p];
    accesses(t, mats[task_mat(t)], acc);
    for (const Access &a : acc) {
      Last &L = items[a.item];
      if (L.last_write >= 0 && finish[L.last_write] > start[p]) ++bad;
      if (a.write) {
        for (int64_t r : L.reads_since)
          if (finish[r] > start[p]) ++bad;
        L.reads_since.clear();
        L.last_write = p;
      } else {
        L.reads_since.push_back(p);
      }
    }
  }
  return bad;
}
