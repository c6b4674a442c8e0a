// Task descriptors and the dependency protocol of the tile QR DAG, shared by
// the device scheduler and the host plan checker.
//
// The tile algorithm (Section 2.1, Figure 1) factorizes an M x N matrix cut
// into MT x NT tiles of order NB as a DAG of tile tasks. The tile rows are
// grouped into domains of h consecutive rows (the communication-avoiding
// variant of Section 7: p = ceil(MT / h) domains; h >= MT is the flat tree of
// Section 2.1). At step k (k < KT = min(MT, NT)) the active rows are k..MT-1;
// the head of a domain is its first active row (row k for the domain holding
// k). Step k runs
//   GEQRT(i, k)        QR of the head tile A_ik of every domain,
//   TSQRT(i, k)        QR of [R_hk; A_ik] for every other row i, h its head
//                      (a chain in i within each domain, the domains in
//                      parallel),
//   TTQRT(i, k)        QR of [R_i1k; R_ik] merging the triangle of head i into
//                      the head i1 of a preceding domain, over a binary tree
//                      of the domains (level l joins domain index e + 2^l into
//                      e for e a multiple of 2^(l+1), counted from the domain
//                      of row k), whose root is row k,
//   LARFB(i, j, k, s)  A_ij <- Q_ik^T A_ij for heads i, j > k,
//   SSRFB(i, j, k, s)  [A_hj; A_ij] <- Q_ik^T [A_hj; A_ij] for the other rows,
//   TTMQR(i, j, k, s)  [A_i1j; A_ij] <- Q^T [A_i1j; A_ij] with a merge's Q,
// where s is a column strip of the tile column j (the updates act on each
// column independently, so one tile update is split over several workgroups).
// Applying Q^T to a right-hand side B runs the same updates (the _B kinds) on
// B's tile rows with the stored reflectors.
//
// A TTQRT copies the triangle of its bottom head into a separate nb x nb
// block (zeros below the diagonal) and factorizes [R_i1k; that block] with
// the TSQRT kernel, so the reflectors of the merge and their T live apart
// from the tile, whose lower part keeps the head's GEQRT reflectors.
//
// Synchronisation is by monotone counters in device memory:
//   pv[k][i]      panel writes to tile (i, k) at step k (its GEQRT, the
//                 TSQRTs of its domain while it is the head, its own TSQRT,
//                 the merges it takes part in),
//   ver[i][j][s]  number of writes applied to strip s of tile (i, j),
//   verB[i][s]    number of writes applied to strip s of B's tile row i.
// A task waits until every counter it reads has reached its target, runs, and
// then increments the counters of the data it wrote. The targets follow from
// the order in which the sequential algorithm writes each tile: within a
// step, a head row is written by its GEQRT's reflectors, then by the chain of
// its domain (rows ascending), then by the merges in level order.
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
  TK_TTQRT = 6,
  TK_TTMQR = 7,
  TK_TTMQR_B = 8,
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
TQ_HD inline bool task_on_B(int type) {
  return type == TK_LARFB_B || type == TK_SSRFB_B || type == TK_TTMQR_B;
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
  int32_t h;     // tile rows per domain (>= MT: flat tree)
  int32_t D;     // domains, ceil(MT / h)
  int32_t notrans;  // apply: B <- Q B (the Q^T program reversed) instead of Q^T B
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

// ------------------------------------------------------------ domain tree
TQ_HD inline int tq_min(int a, int b) { return a < b ? a : b; }
TQ_HD inline int tq_max(int a, int b) { return a > b ? a : b; }

// Head of row i's domain at step k (i >= k).
TQ_HD inline int tree_head(const MatDesc &m, int i, int k) {
  return tq_max(k, (i / m.h) * m.h);
}
TQ_HD inline bool tree_is_head(const MatDesc &m, int i, int k) {
  return i == k || i % m.h == 0;
}
// Active rows of domain d at step k.
TQ_HD inline int tree_rows(const MatDesc &m, int d, int k) {
  return tq_min((d + 1) * m.h, m.MT) - tq_max(k, d * m.h);
}
// Merges at levels below lmax in which element e of a binary tree over E
// elements is the top: levels l with e a multiple of 2^(l+1) and e + 2^l < E.
TQ_HD inline int tree_tops(int e, int E, int lmax) {
  int n = 0;
  for (int l = 0; l < lmax && l < 31; ++l) {
    if ((e & ((2 << l) - 1)) != 0 || e + (1 << l) >= E) break;
    ++n;
  }
  return n;
}
// Level at which element e > 0 is merged into e - 2^level.
TQ_HD inline int tree_level(int e) {
  int l = 0;
  while (((e >> l) & 1) == 0) ++l;
  return l;
}
// The head row that TTQRT(i2, k) merges into.
TQ_HD inline int tree_partner(const MatDesc &m, int i2, int k) {
  const int dk = k / m.h, e2 = i2 / m.h - dk;
  return tree_head(m, (dk + e2 - (1 << tree_level(e2))) * m.h, k);
}
// Updates applied to a tile (i, j), j >= k, by steps 0 .. k-1 (i >= k). A row
// that is not a domain's first row was a non-head at every earlier step (one
// write each); a domain's first row d*h was its head at every step before
// d*h: the GEQRT reflectors, the domain's chain and its merges.
TQ_HD inline int tree_writes_before(const MatDesc &m, int i, int k) {
  if (i % m.h != 0 || k == 0) return k;
  const int d = i / m.h, nd = tq_min(m.h, m.MT - d * m.h);
  int w = 0;
  for (int dd = 0; dd * m.h < k; ++dd) {
    const int cnt = tq_min((dd + 1) * m.h, k) - dd * m.h;
    w += cnt * (nd + tree_tops(d - dd, m.D - dd, 31) + 1);
  }
  return w;
}

// Writes to B's tile row i over the whole Q^T application: one per earlier
// step, and, for a row that becomes a diagonal row (i < KT), the root head's
// writes at step i (its LARFB, the SSRFBs of its domain, its merges).
TQ_HD inline int tree_writes_total(const MatDesc &m, int i) {
  const int kk = tq_min(i, m.KT);
  int w = tree_writes_before(m, i, kk);
  if (i < m.KT) w += tree_rows(m, i / m.h, i) + tree_tops(0, m.D - i / m.h, 31);
  return w;
}

// Storage of the merges' reflectors and T factors after the per-tile T:
// (k, d) -> nb x nb block and ib x nb block.
TQ_HD inline int64_t tile_T_doubles(const MatDesc &m) {
  return (int64_t)m.KT * m.MT * m.ib * m.nb;
}
TQ_HD inline int64_t tree_V_offset(const MatDesc &m, int d, int k) {
  return tile_T_doubles(m) + ((int64_t)k * m.D + d) * m.nb * m.nb;
}
TQ_HD inline int64_t tree_T_offset(const MatDesc &m, int d, int k) {
  return tile_T_doubles(m) + (int64_t)m.KT * m.D * m.nb * m.nb +
         ((int64_t)k * m.D + d) * m.ib * m.nb;
}
TQ_HD inline int64_t T_doubles(const MatDesc &m) {
  return tile_T_doubles(m) +
         (m.D > 1 ? (int64_t)m.KT * m.D * ((int64_t)m.nb * m.nb + (int64_t)m.ib * m.nb) : 0);
}

TQ_HD inline int64_t ctr_pan(const MatDesc &m, int i, int k) {
  return m.ctr + (int64_t)k * m.MT + i;
}
TQ_HD inline int64_t ctr_ver(const MatDesc &m, int i, int j, int s) {
  return m.ctr + (int64_t)m.KT * m.MT + ((int64_t)i * m.NT + j) * m.S + s;
}
TQ_HD inline int64_t ctr_verB(const MatDesc &m, int i, int s) {
  return m.ctr + (int64_t)i * m.SB + s;
}
// Counters a matrix needs for a factorization / an apply.
TQ_HD inline int64_t ctr_count_factor(const MatDesc &m) {
  return (int64_t)m.KT * m.MT + (int64_t)m.MT * m.NT * m.S;
}
TQ_HD inline int64_t ctr_count_apply(const MatDesc &m) {
  return (int64_t)m.MT * m.SB;
}

// Writes of step k to a head row i1 before the merge of level l into it, and
// to the bottom head i2 of a merge before that merge.
TQ_HD inline int tree_top_before(const MatDesc &m, int i1, int k, int l) {
  return tree_rows(m, i1 / m.h, k) + l;
}
TQ_HD inline int tree_bottom_before(const MatDesc &m, int i2, int k) {
  const int dk = k / m.h, d2 = i2 / m.h, e2 = d2 - dk;
  return tree_rows(m, d2, k) + tree_tops(e2, m.D - dk, tree_level(e2));
}

// Wait conditions: number, then the q-th (counter index, target).
TQ_HD inline int task_nwaits(const Task &t, const MatDesc &m) {
  int k = t.k;
  switch (task_type(t)) {
    case TK_GEQRT: return k > 0 ? strips_of(m, k) : 0;
    case TK_TSQRT: return 1 + (k > 0 ? strips_of(m, k) : 0);
    case TK_TTQRT: return 2;
    case TK_LARFB: return 2;
    case TK_SSRFB:
    case TK_TTMQR: return 3;
    case TK_LARFB_B: return 1;
    case TK_SSRFB_B:
    case TK_TTMQR_B: return 2;
  }
  return 0;
}

TQ_HD inline void task_wait_fwd(const Task &t, const MatDesc &m, int q, int64_t *idx,
                                int *target, int *row) {
  const int i = t.i, j = t.j, k = t.k, s = task_strip(t);
  *row = i;
  const int type = task_type(t);
  switch (type) {
    case TK_GEQRT:  // every strip of A_ik has received its earlier updates
      *idx = ctr_ver(m, i, k, q);
      *target = tree_writes_before(m, i, k);
      return;
    case TK_TSQRT: {
      const int hd = tree_head(m, i, k);
      if (q == 0) {  // the head's GEQRT and the chain's earlier TSQRTs done
        *idx = ctr_pan(m, hd, k);
        *target = i - hd;
      } else {
        *idx = ctr_ver(m, i, k, q - 1);
        *target = k;
      }
      return;
    }
    case TK_TTQRT: {
      const int i1 = tree_partner(m, i, k);
      if (q == 0) {
        *idx = ctr_pan(m, i1, k);
        *target = tree_top_before(m, i1, k, tree_level(i / m.h - k / m.h));
      } else {
        *idx = ctr_pan(m, i, k);
        *target = tree_bottom_before(m, i, k);
      }
      return;
    }
    case TK_LARFB:
      if (q == 0) {  // V_ik, T_ik ready
        *idx = ctr_pan(m, i, k);
        *target = 1;
      } else {
        *idx = ctr_ver(m, i, j, s);
        *target = tree_writes_before(m, i, k);
      }
      return;
    case TK_SSRFB: {
      const int hd = tree_head(m, i, k);
      if (q == 0) {  // TSQRT(i, k) done: V_ik, T_ik ready
        *idx = ctr_pan(m, i, k);
        *target = 1;
      } else if (q == 1) {  // the head's LARFB and the chain's earlier SSRFBs applied
        *idx = ctr_ver(m, hd, j, s);
        *target = tree_writes_before(m, hd, k) + i - hd;
      } else {  // A_ij has its earlier updates
        *idx = ctr_ver(m, i, j, s);
        *target = k;
      }
      return;
    }
    case TK_TTMQR: {
      const int i1 = tree_partner(m, i, k);
      const int l = tree_level(i / m.h - k / m.h);
      if (q == 0) {  // the merge done
        *idx = ctr_pan(m, i, k);
        *target = tree_bottom_before(m, i, k) + 1;
      } else if (q == 1) {
        *idx = ctr_ver(m, i1, j, s);
        *target = tree_writes_before(m, i1, k) + tree_top_before(m, i1, k, l);
      } else {
        *idx = ctr_ver(m, i, j, s);
        *target = tree_writes_before(m, i, k) + tree_bottom_before(m, i, k);
      }
      return;
    }
    case TK_LARFB_B:
      *idx = ctr_verB(m, i, s);
      *target = tree_writes_before(m, i, k);
      return;
    case TK_SSRFB_B: {
      const int hd = tree_head(m, i, k);
      if (q == 0) {
        *idx = ctr_verB(m, hd, s);
        *target = tree_writes_before(m, hd, k) + i - hd;
        *row = hd;
      } else {
        *idx = ctr_verB(m, i, s);
        *target = k;
      }
      return;
    }
    case TK_TTMQR_B: {
      const int i1 = tree_partner(m, i, k);
      const int l = tree_level(i / m.h - k / m.h);
      if (q == 0) {
        *idx = ctr_verB(m, i1, s);
        *target = tree_writes_before(m, i1, k) + tree_top_before(m, i1, k, l);
        *row = i1;
      } else {
        *idx = ctr_verB(m, i, s);
        *target = tree_writes_before(m, i, k) + tree_bottom_before(m, i, k);
      }
      return;
    }
  }
}

// The wait in the program actually run: for B <- Q B the Q^T program runs
// backwards, so a task waits for the writes that follow it in the forward
// order.
TQ_HD inline void task_wait(const Task &t, const MatDesc &m, int q, int64_t *idx, int *target) {
  int row;
  task_wait_fwd(t, m, q, idx, target, &row);
  if (m.notrans && task_on_B(task_type(t))) *target = tree_writes_total(m, row) - *target - 1;
}

// Signals: number, then the q-th counter index to increment.
TQ_HD inline int task_nsignals(const Task &t) {
  switch (task_type(t)) {
    case TK_GEQRT:
    case TK_LARFB:
    case TK_LARFB_B: return 1;
    default: return 2;
  }
}

TQ_HD inline int64_t task_signal(const Task &t, const MatDesc &m, int q) {
  const int i = t.i, j = t.j, k = t.k, s = task_strip(t);
  switch (task_type(t)) {
    case TK_GEQRT: return ctr_pan(m, i, k);
    case TK_TSQRT: return ctr_pan(m, q == 0 ? tree_head(m, i, k) : i, k);
    case TK_TTQRT: return ctr_pan(m, q == 0 ? tree_partner(m, i, k) : i, k);
    case TK_LARFB: return ctr_ver(m, i, j, s);
    case TK_SSRFB: return ctr_ver(m, q == 0 ? tree_head(m, i, k) : i, j, s);
    case TK_TTMQR: return ctr_ver(m, q == 0 ? tree_partner(m, i, k) : i, j, s);
    case TK_LARFB_B: return ctr_verB(m, i, s);
    case TK_SSRFB_B: return ctr_verB(m, q == 0 ? tree_head(m, i, k) : i, s);
    case TK_TTMQR_B: return ctr_verB(m, q == 0 ? tree_partner(m, i, k) : i, s);
  }
  return m.ctr;
}
