// Task descriptors and the dependency protocol of the tile QR DAG, shared by
// the device scheduler and the host plan checker.
//
// The tile algorithm (Section 2.1, Figure 1) factorizes an M x N matrix cut
// into MT x NT tiles of order NB as a DAG of four kinds of tasks. Step k
// (k < KT = min(MT, NT)) runs
//   GEQRT(k)          QR of the diagonal tile A_kk,
//   TSQRT(i, k)       QR of [R_kk; A_ik] for i > k (a chain in i),
//   LARFB(k, j, s)    A_kj <- Q_kk^T A_kj for j > k,
//   SSRFB(i, j, k, s) [A_kj; A_ij] <- Q_ik^T [A_kj; A_ij] for i, j > k,
// where s is a column strip of the tile column j (the updates act on each
// column independently, so one tile update is split over several workgroups).
// Applying Q^T to a right-hand side B uses LARFB_B(k, s) and SSRFB_B(i, k, s)
// on B's tile rows with the stored (V, T).
//
// Synchronisation is by monotone counters in device memory:
//   pan[k]        number of panel tasks of step k done (GEQRT counts 1, each
//                 TSQRT(i, k) one more, so TSQRT(i, k) done <=> pan[k] > i-k),
//   ver[i][j][s]  number of writes applied to strip s of tile (i, j),
//   verB[i][s]    number of writes applied to strip s of B's tile row i.
// A task waits until every counter it reads has reached its target, runs, and
// then increments the counters of the data it wrote. The targets follow from
// the order in which the sequential algorithm writes each tile.
#pragma once
#include <stdint.h>

#if defined(__HIPCC__)
#define TQ_HD __host__ __device__
#else
#define TQ_HD
#endif

enum TaskType : int32_t {
  TK_GEQRT = 0,
  TK_TSQRT = 1,
  TK_LARFB = 2,
  TK_SSRFB = 3,
  TK_LARFB_B = 4,
  TK_SSRFB_B = 5,
};

// 16 bytes: w0 = type | strip << 4 | mat << 16.
struct Task {
  int32_t w0, i, j, k;
};

TQ_HD inline int task_type(const Task &t) { return t.w0 & 15; }
TQ_HD inline int task_strip(const Task &t) { return (t.w0 >> 4) & 4095; }
TQ_HD inline int task_mat(const Task &t) { return (int)((uint32_t)t.w0 >> 16); }
TQ_HD inline Task make_task(int type, int mat, int i, int j, int k, int s) {
  Task t;
  t.w0 = (int32_t)((uint32_t)type | ((uint32_t)s << 4) | ((uint32_t)mat << 16));
  t.i = i;
  t.j = j;
  t.k = k;
  return t;
}

// Per-matrix descriptor. A, T: the factorization; B: right-hand side of an
// apply. All column-major. ctr: offset of this matrix's counters.
struct MatDesc {
  double *A;
  double *T;
  double *B;
  int64_t lda, ldb, ctr;
  int32_t M, N, nb, ib, MT, NT, KT;
  int32_t S;     // strips per tile column of A (uniform, ceil(nb / w))
  int32_t w;     // strip width in columns (16 * active waves)
  int32_t nrhs;  // columns of B
  int32_t SB;    // strips of B (ceil(nrhs / w))
  int32_t gmax;  // V chunks staged in LDS at once
};

TQ_HD inline int tile_rows(const MatDesc &m, int i) {
  int r = m.M - i * m.nb;
  return r < m.nb ? r : m.nb;
}
TQ_HD inline int tile_cols(const MatDesc &m, int j) {
  int c = m.N - j * m.nb;
  return c < m.nb ? c : m.nb;
}
TQ_HD inline int strips_of(const MatDesc &m, int j) {
  return (tile_cols(m, j) + m.w - 1) / m.w;
}

TQ_HD inline int64_t ctr_pan(const MatDesc &m, int k) { return m.ctr + k; }
TQ_HD inline int64_t ctr_ver(const MatDesc &m, int i, int j, int s) {
  return m.ctr + m.KT + ((int64_t)i * m.NT + j) * m.S + s;
}
TQ_HD inline int64_t ctr_verB(const MatDesc &m, int i, int s) {
  return m.ctr + (int64_t)i * m.SB + s;
}
// Counters a matrix needs for a factorization / an apply.
TQ_HD inline int64_t ctr_count_factor(const MatDesc &m) {
  return (int64_t)m.KT + (int64_t)m.MT * m.NT * m.S;
}
TQ_HD inline int64_t ctr_count_apply(const MatDesc &m) {
  return (int64_t)m.MT * m.SB;
}

// Wait conditions: number, then the q-th (counter index, target).
TQ_HD inline int task_nwaits(const Task &t, const MatDesc &m) {
  int k = t.k;
  switch (task_type(t)) {
    case TK_GEQRT: return k > 0 ? strips_of(m, k) : 0;
    case TK_TSQRT: return 1 + (k > 0 ? strips_of(m, k) : 0);
    case TK_LARFB: return 1 + (k > 0 ? 1 : 0);
    case TK_SSRFB: return 2 + (k > 0 ? 1 : 0);
    case TK_LARFB_B: return k > 0 ? 1 : 0;
    case TK_SSRFB_B: return 1 + (k > 0 ? 1 : 0);
  }
  return 0;
}

TQ_HD inline void task_wait(const Task &t, const MatDesc &m, int q, int64_t *idx,
                            int *target) {
  int i = t.i, j = t.j, k = t.k, s = task_strip(t);
  switch (task_type(t)) {
    case TK_GEQRT:  // every strip of A_kk has received its k updates
      *idx = ctr_ver(m, k, k, q);
      *target = k;
      return;
    case TK_TSQRT:
      if (q == 0) {  // GEQRT(k) (i = k+1) or TSQRT(i-1, k) done
        *idx = ctr_pan(m, k);
        *target = i - k;
      } else {
        *idx = ctr_ver(m, i, k, q - 1);
        *target = k;
      }
      return;
    case TK_LARFB:
      if (q == 0) {  // V_kk, T_kk ready
        *idx = ctr_pan(m, k);
        *target = 1;
      } else {
        *idx = ctr_ver(m, k, j, s);
        *target = k;
      }
      return;
    case TK_SSRFB:
      if (q == 0) {  // TSQRT(i, k) done: V_ik, T_ik ready
        *idx = ctr_pan(m, k);
        *target = i - k + 1;
      } else if (q == 1) {  // LARFB(k,j,s) and SSRFB(k+1..i-1, j, k, s) applied to A_kj
        *idx = ctr_ver(m, k, j, s);
        *target = i;
      } else {  // A_ij has its k earlier updates
        *idx = ctr_ver(m, i, j, s);
        *target = k;
      }
      return;
    case TK_LARFB_B:
      *idx = ctr_verB(m, k, s);
      *target = k;
      return;
    case TK_SSRFB_B:
      if (q == 0) {
        *idx = ctr_verB(m, k, s);
        *target = i;
      } else {
        *idx = ctr_verB(m, i, s);
        *target = k;
      }
      return;
  }
}

// Signals: number, then the q-th counter index to increment.
TQ_HD inline int task_nsignals(const Task &t) {
  switch (task_type(t)) {
    case TK_SSRFB:
    case TK_SSRFB_B: return 2;
    default: return 1;
  }
}

TQ_HD inline int64_t task_signal(const Task &t, const MatDesc &m, int q) {
  int i = t.i, j = t.j, k = t.k, s = task_strip(t);
  switch (task_type(t)) {
    case TK_GEQRT:
    case TK_TSQRT: return ctr_pan(m, k);
    case TK_LARFB: return ctr_ver(m, k, j, s);
    case TK_SSRFB: return q == 0 ? ctr_ver(m, k, j, s) : ctr_ver(m, i, j, s);
    case TK_LARFB_B: return ctr_verB(m, k, s);
    case TK_SSRFB_B: return q == 0 ? ctr_verB(m, k, s) : ctr_verB(m, i, s);
  }
  return m.ctr;
}
