// Tile Householder QR kernels for gfx950 (MI355X), FP64.
//
// One persistent kernel runs every task of the tile DAG (Section 2.1): each
// workgroup (4 x wave64) repeatedly takes the next ticket of a host-built
// topological order, waits on the dependency counters of that task, runs it,
// and bumps the counters of the data it wrote.
//
// Task bodies:
//  * LARFB / SSRFB (and the updates inside the panels) apply a run of
//    compact-WY block reflectors H = I - V T V^T, IB columns at a time:
//        W = T^T (C1_s + V_s^T C2),  C1_s -= W,  C2 -= V_s W.
//    Each wave owns a 16-column strip of C2 for the whole task, held in
//    registers in the FP64 MFMA accumulator layout, so the contraction with
//    V_s^T uses the accumulators directly as the B operand of
//    v_mfma_f64_16x16x4 and the update accumulates into them. V is staged
//    through LDS 16 columns at a time (coalesced loads, conflict-free
//    transposed reads thanks to an odd leading dimension).
//  * GEQRT / TSQRT factor IB-wide column blocks: up to 16 columns at a time
//    are held in registers (rows spread over the 256 threads); each
//    Householder column needs one reduction for its norm and one batched
//    transpose-reduction for all its dot products, and builds the compact-WY
//    factor T column by column from the same dot products. The rest of the
//    tile is updated with the MFMA routine above.
//
// Storage: A column-major with leading dimension lda, tiles addressed in
// place (ragged last tile row/column allowed). T of tile (i, k) is an
// IB x nb_k array at T + (k*MT + i)*IB*NB, leading dimension IB; the block
// of columns [s, s+IB) holds the upper-triangular T_s of those reflectors.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device_api.h"
#include "layout.h"
#include "tq_sched.h"

typedef double d4 __attribute__((ext_vector_type(4)));

namespace {

constexpr int NTHR = TQ_NTHR;
enum { VK_UNIT = 0, VK_FULL = 1 };

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }
__device__ __forceinline__ int wave_id() { return threadIdx.x >> 6; }

__device__ __forceinline__ d4 mfma(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

struct Lds {
  double *vc;     // 16 x ldvc: one 16-column chunk of V
  double *y;      // nw regions of ibp x 16 (Y, then W in place)
  double *red1;   // 4
  double *red32;  // 4 x 32
  double *tot;    // 32
  double *scal;   // 8
  double *tmm;    // 32 x 33 micro-panel T, [a*33 + c]
  double *top;    // 32 x 33 TSQRT top block
  int ldvc, ibp;
};

__device__ inline Lds make_lds(double *base, int mbt, int ib, int nw) {
  Lds L;
  L.ldvc = lds_ldvc(mbt);
  L.ibp = ib_pad16(ib);
  double *p = base;
  L.vc = p;
  p += 16 * L.ldvc;
  L.y = p;
  p += nw * L.ibp * 16;
  L.red1 = p;
  p += 4;
  L.red32 = p;
  p += 128;
  L.tot = p;
  p += 32;
  L.scal = p;
  p += 8;
  L.tmm = p;
  p += 32 * 33;
  L.top = p;
  return L;
}

// ---------------------------------------------------------------------------
// Block reductions
// ---------------------------------------------------------------------------

__device__ inline double block_sum1(const Lds &L, double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
  __syncthreads();
  if (lane_id() == 0) L.red1[wave_id()] = v;
  __syncthreads();
  return L.red1[0] + L.red1[1] + L.red1[2] + L.red1[3];
}

// Width of the register-resident micro-panel in the panel kernels.
constexpr int PWM = 16;

// Sums v[0..15] over the workgroup into L.tot[0..15] (plus add[t] for
// 1 <= t <= nadd). Within a wave each exchange step hands half of the
// remaining values to the partner lane, so 16 values cost 15 shuffles
// instead of 16 separate butterflies.
__device__ inline void block_sum16(const Lds &L, const double (&v)[PWM], const double *add, int nadd) {
  const int ln = lane_id();
  double h8[8], h4[4], h2[2], h1;
  {
    const bool hi = ln & 32;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      double snd = hi ? v[i] : v[8 + i];
      double keep = hi ? v[8 + i] : v[i];
      h8[i] = keep + __shfl_xor(snd, 32);
    }
  }
  {
    const bool hi = ln & 16;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      double snd = hi ? h8[i] : h8[4 + i];
      double keep = hi ? h8[4 + i] : h8[i];
      h4[i] = keep + __shfl_xor(snd, 16);
    }
  }
  {
    const bool hi = ln & 8;
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      double snd = hi ? h4[i] : h4[2 + i];
      double keep = hi ? h4[2 + i] : h4[i];
      h2[i] = keep + __shfl_xor(snd, 8);
    }
  }
  {
    const bool hi = ln & 4;
    double snd = hi ? h2[0] : h2[1];
    double keep = hi ? h2[1] : h2[0];
    h1 = keep + __shfl_xor(snd, 4);
  }
  h1 += __shfl_xor(h1, 2);
  h1 += __shfl_xor(h1, 1);
  const int idx = ((ln >> 5) & 1) * 8 + ((ln >> 4) & 1) * 4 + ((ln >> 3) & 1) * 2 + ((ln >> 2) & 1);
  if (!(ln & 3)) L.red32[wave_id() * PWM + idx] = h1;
  __syncthreads();
  if (threadIdx.x < PWM) {
    const int t = threadIdx.x;
    double s = L.red32[t] + L.red32[PWM + t] + L.red32[2 * PWM + t] + L.red32[3 * PWM + t];
    if (add && t >= 1 && t <= nadd) s += add[t];
    L.tot[t] = s;
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// Block-reflector application (LARFB / SSRFB bodies)
// ---------------------------------------------------------------------------

// V[:, gc0 .. gc0+16) -> L.vc, rows 0..16*MBT-1, zero outside the reflector
// support. VK_UNIT: column gc has an implicit 1 at row gc and 0 above.
template <int MBT>
__device__ inline void load_vchunk(const Lds &L, const double *V, int64_t ldv, int vrows,
                                   int kind, int gc0, int kvalid) {
  constexpr int RP = MBT * 16;
  const int rlim = (vrows + 15) & ~15;
  for (int e = threadIdx.x; e < 16 * RP; e += NTHR) {
    const int c = e / RP, r = e % RP;
    if (r >= rlim) continue;
    const int gc = gc0 + c;
    double v = 0.0;
    if (gc < kvalid && r < vrows) {
      if (kind == VK_UNIT)
        v = r < gc ? 0.0 : (r == gc ? 1.0 : V[r + (int64_t)gc * ldv]);
      else
        v = V[r + (int64_t)gc * ldv];
    }
    L.vc[c * L.ldvc + r] = v;
  }
}

// C[0..crows) x column `col` into the accumulator layout of the FP64 MFMA:
// tile rt, register r holds row 16*rt + 4*r + lane/16 (column lane%16).
// VK_UNIT applies the unit-lower mask of a reflector whose head row is
// diag + col.
template <int MBT>
__device__ inline void load_c2(d4 (&c2)[MBT], const double *C, int64_t ldc, int crows, int col,
                               bool colok, int kind, int diag) {
  const int g = lane_id() >> 4;
#pragma unroll
  for (int rt = 0; rt < MBT; ++rt) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = rt * 16 + 4 * r + g;
      double v = 0.0;
      if (colok && row < crows) {
        if (kind == VK_UNIT) {
          const int h = diag + col;
          v = row < h ? 0.0 : (row == h ? 1.0 : C[row + (int64_t)col * ldc]);
        } else {
          v = C[row + (int64_t)col * ldc];
        }
      }
      c2[rt][r] = v;
    }
  }
}

template <int MBT>
__device__ inline void store_c2(const d4 (&c2)[MBT], double *C, int64_t ldc, int crows, int col,
                                bool colok) {
  if (!colok) return;
  const int g = lane_id() >> 4;
#pragma unroll
  for (int rt = 0; rt < MBT; ++rt) {
    if (rt * 16 >= crows) break;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = rt * 16 + 4 * r + g;
      if (row < crows) C[row + (int64_t)col * ldc] = c2[rt][r];
    }
  }
}

// Y[0..ibw) x 16 = V[:, s..s+ibw)^T C2 for this wave's strip -> wave region.
template <int MBT>
__device__ inline void y_phase(const Lds &L, const double *V, int64_t ldv, int vrows, int kind,
                               int s, int ibw, const d4 (&c2)[MBT], bool active) {
  const int ln = lane_id();
  double *yw = L.y + wave_id() * L.ibp * 16;
  const int nq = (ibw + 15) >> 4;
  for (int q = 0; q < nq; ++q) {
    __syncthreads();
    load_vchunk<MBT>(L, V, ldv, vrows, kind, s + q * 16, s + ibw);
    __syncthreads();
    if (active) {
      d4 y0 = {0.0, 0.0, 0.0, 0.0}, y1 = {0.0, 0.0, 0.0, 0.0};
      const int rt0 = (kind == VK_UNIT) ? ((s + q * 16) >> 4) : 0;
      // B operand = accumulator register r of C2 tile rt: k index lane/16
      // <-> row 16*rt + 4*r + lane/16; A operand = V^T at those rows.
      const double *vp = L.vc + (ln & 15) * L.ldvc + (ln >> 4);
#pragma unroll
      for (int rt = 0; rt < MBT; ++rt) {
        if (rt >= rt0 && rt * 16 < vrows) {
          y0 = mfma(vp[rt * 16 + 0], c2[rt][0], y0);
          y1 = mfma(vp[rt * 16 + 4], c2[rt][1], y1);
          y0 = mfma(vp[rt * 16 + 8], c2[rt][2], y0);
          y1 = mfma(vp[rt * 16 + 12], c2[rt][3], y1);
        }
      }
#pragma unroll
      for (int r = 0; r < 4; ++r)
        yw[(q * 16 + 4 * r + (ln >> 4)) * 16 + (ln & 15)] = y0[r] + y1[r];
    }
  }
}

// Applies the reflectors V[:, 0..kref) (blocks of ib, compact-WY factors in
// T: block s at T + s*ldt) to one strip of at most 16*nw columns:
//   C1 (optional): rows s..s+ib of the block's top part, C2: vrows rows.
template <int MBT>
__device__ __forceinline__ void apply_strip(const Lds &L, const double *V, int64_t ldv, int vrows, int kind,
                            int kref, int ib, const double *T, int64_t ldt, double *C1,
                            int64_t ldc1, double *C2, int64_t ldc2, int ncols, int nw) {
  const int ln = lane_id(), wv = wave_id();
  const bool active = (wv < nw) && (wv * 16 < ncols);
  const int col = wv * 16 + (ln & 15);
  const bool colok = active && col < ncols;
  d4 c2[MBT];
  load_c2<MBT>(c2, C2, ldc2, vrows, col, colok, VK_FULL, 0);
  double *yw = L.y + wv * L.ibp * 16;
  for (int s = 0; s < kref; s += ib) {
    const int ibw = min(ib, kref - s);
    const int nq = (ibw + 15) >> 4;
    y_phase<MBT>(L, V, ldv, vrows, kind, s, ibw, c2, active);
    __syncthreads();
    if (active && C1) {
      for (int e = ln; e < ibw * 16; e += 64) {
        const int a = e >> 4, c = wv * 16 + (e & 15);
        if (c < ncols) yw[e] += C1[(s + a) + (int64_t)c * ldc1];
      }
    }
    __syncthreads();
    if (active) {
      // W = T_s^T Y in place, bottom block first (W block q needs Y blocks <= q).
      const double *Ts = T + (int64_t)s * ldt;
      for (int q = nq - 1; q >= 0; --q) {
        d4 w = {0.0, 0.0, 0.0, 0.0};
        const int ccol = q * 16 + (ln & 15);
        for (int q2 = 0; q2 <= q; ++q2) {
#pragma unroll
          for (int kk = 0; kk < 4; ++kk) {
            const int arow = q2 * 16 + 4 * kk + (ln >> 4);
            const double a = (arow <= ccol && ccol < ibw) ? Ts[arow + (int64_t)ccol * ldt] : 0.0;
            w = mfma(a, yw[arow * 16 + (ln & 15)], w);
          }
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) yw[(q * 16 + 4 * r + (ln >> 4)) * 16 + (ln & 15)] = w[r];
      }
    }
    __syncthreads();
    if (active && C1) {
      for (int e = ln; e < ibw * 16; e += 64) {
        const int a = e >> 4, c = wv * 16 + (e & 15);
        if (c < ncols) C1[(s + a) + (int64_t)c * ldc1] -= yw[e];
      }
    }
    // C2 -= V_s W
    for (int q = 0; q < nq; ++q) {
      __syncthreads();
      load_vchunk<MBT>(L, V, ldv, vrows, kind, s + q * 16, s + ibw);
      __syncthreads();
      if (active) {
        const int rt0 = (kind == VK_UNIT) ? ((s + q * 16) >> 4) : 0;
        double b[4];
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) b[kk] = yw[(q * 16 + 4 * kk + (ln >> 4)) * 16 + (ln & 15)];
#pragma unroll
        for (int rt = 0; rt < MBT; ++rt) {
          if (rt >= rt0 && rt * 16 < vrows) {
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) {
              const double a = -L.vc[(4 * kk + (ln >> 4)) * L.ldvc + rt * 16 + (ln & 15)];
              c2[rt] = mfma(a, b[kk], c2[rt]);
            }
          }
        }
      }
    }
  }
  __syncthreads();
  store_c2<MBT>(c2, C2, ldc2, vrows, col, colok);
}

// All columns of C2 (and C1), in strips of 16*nw.
template <int MBT>
__device__ __forceinline__ void apply_cols(const Lds &L, const double *V, int64_t ldv, int vrows, int kind,
                           int kref, int ib, const double *T, int64_t ldt, double *C1,
                           int64_t ldc1, double *C2, int64_t ldc2, int ncols, int nw) {
  const int w = 16 * nw;
  for (int c0 = 0; c0 < ncols; c0 += w) {
    apply_strip<MBT>(L, V, ldv, vrows, kind, kref, ib, T, ldt,
                     C1 ? C1 + (int64_t)c0 * ldc1 : nullptr, ldc1, C2 + (int64_t)c0 * ldc2, ldc2,
                     min(w, ncols - c0), nw);
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// Panel factorization (GEQRT / TSQRT bodies)
// ---------------------------------------------------------------------------

// Householder scalars from alpha and the squared norm of the tail.
__device__ inline void householder(double alpha, double ss, double &beta, double &tau,
                                   double &scale) {
  if (ss == 0.0) {
    beta = alpha;
    tau = 0.0;
    scale = 1.0;
  } else {
    const double nrm = sqrt(alpha * alpha + ss);
    beta = alpha >= 0.0 ? -nrm : nrm;
    tau = (beta - alpha) / beta;
    scale = 1.0 / (alpha - beta);
  }
}

// Register slots rotate left once per column, so the current column is
// always slot 0, the remaining ones slots 1..pw-1-c and the finished ones
// slots PWM-c..PWM-1 (column p at slot PWM-c+p).
template <int HR>
__device__ inline void rotate_slots(double (&x)[HR][PWM]) {
#pragma unroll
  for (int h = 0; h < HR; ++h) {
    const double t0 = x[h][0];
#pragma unroll
    for (int i = 0; i < PWM - 1; ++i) x[h][i] = x[h][i + 1];
    x[h][PWM - 1] = t0;
  }
}

// T column c of the micro-panel from the Gram entries tot[PWM-c+p] (p < c).
__device__ inline void micro_T_column(const Lds &L, int c, double tau) {
  const int t = threadIdx.x;
  if (t < c) {
    double acc = 0.0;
    for (int p = t; p < c; ++p) acc += L.tmm[t * 33 + p] * L.tot[PWM - c + p];
    L.tmm[t * 33 + c] = -tau * acc;
  }
  if (t == 0) L.tmm[c * 33 + c] = tau;
}

__device__ inline void store_micro_T(const Lds &L, double *Tmm, int64_t ldt, int pw) {
  __syncthreads();
  for (int e = threadIdx.x; e < pw * pw; e += NTHR) {
    const int a = e % pw, c = e / pw;
    Tmm[a + (int64_t)c * ldt] = a <= c ? L.tmm[a * 33 + c] : 0.0;
  }
  __syncthreads();
}

// Unblocked Householder QR of one micro-panel of pw <= 16 columns, held in
// registers (thread t owns rows t, t+256, ...).
//  GEQRT (ts == false): X = P[0..mrows) x [m0, m0+pw) in the block frame;
//    reflector c has its unit at row m0+c, zeros above.
//  TSQRT (ts == true): X = U[0..mrows) x [0, pw) under the pw x pw upper
//    block of R kept in L.top; reflector c is [e_c; u_c].
// Each column costs one reduction for the norm and one batched reduction for
// all its dot products (remaining columns: the update; finished columns: the
// Gram entries that build column c of the micro-panel's T).
template <int HR>
__device__ __forceinline__ void level2_panel(const Lds &L, bool ts, double *X, int64_t ldx, int mrows, int m0,
                             int pw, double *Tmm, int64_t ldt) {
  const int tid = threadIdx.x;
  double x[HR][PWM];
#pragma unroll
  for (int h = 0; h < HR; ++h) {
    const int row = tid + NTHR * h;
#pragma unroll
    for (int i = 0; i < PWM; ++i)
      x[h][i] = (i < pw && row < mrows) ? X[row + (int64_t)(m0 + i) * ldx] : 0.0;
  }
  for (int c = 0; c < pw; ++c) {
    const int jr = ts ? -1 : m0 + c;  // rows > jr form the reflector tail
    double ss = 0.0;
#pragma unroll
    for (int h = 0; h < HR; ++h) {
      const int row = tid + NTHR * h;
      if (row > jr) ss += x[h][0] * x[h][0];
      if (row == jr) L.scal[0] = x[h][0];
    }
    ss = block_sum1(L, ss);
    const double alpha = ts ? L.top[c * 33 + c] : L.scal[0];
    double beta, tau, scale;
    householder(alpha, ss, beta, tau, scale);
    double v[HR];
#pragma unroll
    for (int h = 0; h < HR; ++h) {
      const int row = tid + NTHR * h;
      if (row > jr) {
        x[h][0] *= scale;
        v[h] = x[h][0];
      } else if (row == jr) {
        v[h] = 1.0;
        x[h][0] = beta;
      } else {
        v[h] = 0.0;
      }
    }
    double d[PWM];
    d[0] = 0.0;
#pragma unroll
    for (int i = 1; i < PWM; ++i) {
      double a = 0.0;
#pragma unroll
      for (int h = 0; h < HR; ++h) a += v[h] * x[h][i];
      d[i] = a;
    }
    const int nrem = pw - 1 - c;
    // TSQRT: the remaining columns' dot products include row c of R.
    block_sum16(L, d, ts ? L.top + c * 33 + c : nullptr, nrem);
#pragma unroll
    for (int i = 1; i < PWM; ++i) {
      if (i <= nrem) {
        const double f = tau * L.tot[i];
#pragma unroll
        for (int h = 0; h < HR; ++h) x[h][i] -= f * v[h];
      }
    }
    if (ts) {
      if (tid >= 1 && tid <= nrem) L.top[c * 33 + c + tid] -= tau * L.tot[tid];
      if (tid == 0) L.top[c * 33 + c] = beta;
    }
    micro_T_column(L, c, tau);
    rotate_slots<HR>(x);
  }
#pragma unroll
  for (int h = 0; h < HR; ++h) {
    const int row = tid + NTHR * h;
#pragma unroll
    for (int i = 0; i < PWM; ++i) {
      const int p = (i + pw) & (PWM - 1);
      if (p < pw && row < mrows) X[row + (int64_t)(m0 + p) * ldx] = x[h][i];
    }
  }
  store_micro_T(L, Tmm, ldt, pw);
}

// After micro-panel [m0, m0+pw) (pw <= 16) of an IB block: fills
// T[0:m0, m0:m0+pw] = -T[0:m0, 0:m0] (V[:,0:m0]^T V[:,m0:m0+pw]) T[m0:,m0:].
template <int MBT>
__device__ __forceinline__ void assemble_T(const Lds &L, const double *V, int64_t ldv, int vrows, int kind, int m0,
                           int pw, double *Tb, int64_t ldt) {
  const bool act = wave_id() == 0;
  const int col = lane_id() & 15;
  d4 c2[MBT];
  load_c2<MBT>(c2, V + (int64_t)m0 * ldv, ldv, vrows, col, act && col < pw, kind, m0);
  y_phase<MBT>(L, V, ldv, vrows, kind, 0, m0, c2, act);
  __syncthreads();
  double *G = L.y;  // wave 0 region: G[a*16 + c]
  for (int a = threadIdx.x; a < m0; a += NTHR) {
    for (int c = pw - 1; c >= 0; --c) {
      double acc = 0.0;
      for (int p = 0; p <= c; ++p) acc += G[a * 16 + p] * Tb[(m0 + p) + (int64_t)(m0 + c) * ldt];
      G[a * 16 + c] = acc;
    }
  }
  __syncthreads();
  for (int e = threadIdx.x; e < m0 * pw; e += NTHR) {
    const int a = e % m0, c = e / m0;
    double acc = 0.0;
    for (int b = a; b < m0; ++b) acc += Tb[a + (int64_t)b * ldt] * G[b * 16 + c];
    Tb[a + (int64_t)(m0 + c) * ldt] = -acc;
  }
  for (int e = threadIdx.x; e < m0 * pw; e += NTHR) {
    const int a = e % pw, c = e / pw;
    Tb[(m0 + a) + (int64_t)c * ldt] = 0.0;
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// Task dispatch and the persistent scheduler
// ---------------------------------------------------------------------------

struct ApplyArgs {
  const double *V;
  const double *T;
  double *C1;
  double *C2;
  int64_t ldv, ldt, ldc1, ldc2;
  int vrows, kind, kref, ib, ncols;
};

// Runs one task. Every task is a sequence of steps that end with one
// block-reflector application; panels precede it with the factorization of
// a micro-panel. Keeping a single call site of the MFMA routine (and of the
// panel routine) keeps the register allocation of the fused kernel tight.
template <int MBT>
__device__ __forceinline__ void run_task(const Task &t, const MatDesc &m, const Lds &L) {
  constexpr int HR = (MBT * 16 + NTHR - 1) / NTHR;
  const int nb = m.nb, ib = m.ib, nw = m.w >> 4;
  const int i = t.i, j = t.j, k = t.k, strip = task_strip(t);
  const int type = task_type(t);
  auto At = [&](int r, int c) { return m.A + (int64_t)c * nb * m.lda + (int64_t)r * nb; };
  auto Tt = [&](int r, int c) { return m.T + ((int64_t)c * m.MT + r) * (int64_t)ib * nb; };
  const int64_t lda = m.lda;

  if (type == TK_GEQRT || type == TK_TSQRT) {
    const bool ts = type == TK_TSQRT;
    double *R = At(k, k);                 // diagonal tile (TSQRT: R on top)
    double *U = ts ? At(i, k) : R;        // tile being factored
    double *T = ts ? Tt(i, k) : Tt(k, k);
    const int mb = ts ? tile_rows(m, i) : tile_rows(m, k);
    const int ncol = tile_cols(m, k);
    const int K = ts ? ncol : min(mb, ncol);
    int s = 0, m0 = 0;
    while (s < K) {
      const int ibw = min(ib, K - s);
      const int pw = min(PWM, ibw - m0);
      // Block frame: GEQRT rows/cols start at s; TSQRT rows of U start at 0.
      double *Xb = ts ? U + (int64_t)s * lda : U + s + (int64_t)s * lda;
      double *Rb = R + s + (int64_t)s * lda;
      double *Tb = T + (int64_t)s * ib;
      const int mrows = ts ? mb : mb - s;
      if (ts) {
        for (int e = threadIdx.x; e < 32 * 32; e += NTHR) {
          const int a = e >> 5, c = e & 31;
          L.top[a * 33 + c] = (a <= c && c < pw) ? Rb[(m0 + a) + (int64_t)(m0 + c) * lda] : 0.0;
        }
        __syncthreads();
      }
      level2_panel<HR>(L, ts, Xb, lda, mrows, m0, pw, Tb + m0 + (int64_t)m0 * ib, ib);
      if (ts) {
        for (int e = threadIdx.x; e < 32 * 32; e += NTHR) {
          const int a = e >> 5, c = e & 31;
          if (a <= c && c < pw) Rb[(m0 + a) + (int64_t)(m0 + c) * lda] = L.top[a * 33 + c];
        }
        __syncthreads();
      }
      const int kind = ts ? VK_FULL : VK_UNIT;
      if (m0 > 0) assemble_T<MBT>(L, Xb, lda, mrows, kind, m0, pw, Tb, ib);
      ApplyArgs a;
      bool go = true;
      if (m0 + pw < ibw) {
        // this micro-panel's reflectors onto the rest of the IB block
        a.V = ts ? Xb + (int64_t)m0 * lda : Xb + m0 + (int64_t)m0 * lda;
        a.vrows = ts ? mrows : mrows - m0;
        a.kref = pw;
        a.ib = pw;
        a.T = Tb + m0 + (int64_t)m0 * ib;
        a.C1 = ts ? Rb + m0 + (int64_t)(m0 + pw) * lda : nullptr;
        a.C2 = ts ? Xb + (int64_t)(m0 + pw) * lda : Xb + m0 + (int64_t)(m0 + pw) * lda;
        a.ncols = ibw - m0 - pw;
        m0 += pw;
      } else {
        // the whole IB block onto the trailing columns of the tile
        a.V = Xb;
        a.vrows = mrows;
        a.kref = ibw;
        a.ib = ibw;
        a.T = Tb;
        a.C1 = ts ? Rb + (int64_t)ibw * lda : nullptr;
        a.C2 = Xb + (int64_t)ibw * lda;
        a.ncols = ncol - s - ibw;
        go = a.ncols > 0;
        s += ibw;
        m0 = 0;
      }
      a.kind = kind;
      a.ldv = lda;
      a.ldt = ib;
      a.ldc1 = lda;
      a.ldc2 = lda;
      if (go)
        apply_cols<MBT>(L, a.V, a.ldv, a.vrows, a.kind, a.kref, a.ib, a.T, a.ldt, a.C1, a.ldc1,
                        a.C2, a.ldc2, a.ncols, nw);
    }
    return;
  }

  ApplyArgs a;
  a.ib = ib;
  a.ldv = lda;
  a.ldt = ib;
  a.C1 = nullptr;
  a.ldc1 = lda;
  a.ldc2 = lda;
  const int c0 = strip * m.w;
  const bool onB = type == TK_LARFB_B || type == TK_SSRFB_B;
  const bool larfb = type == TK_LARFB || type == TK_LARFB_B;
  if (larfb) {
    const int mb = tile_rows(m, k);
    a.V = At(k, k);
    a.vrows = mb;
    a.kind = VK_UNIT;
    a.kref = min(mb, tile_cols(m, k));
    a.T = Tt(k, k);
  } else {
    a.V = At(i, k);
    a.vrows = tile_rows(m, i);
    a.kind = VK_FULL;
    a.kref = tile_cols(m, k);
    a.T = Tt(i, k);
  }
  if (onB) {
    a.ncols = min(m.w, m.nrhs - c0);
    a.ldc1 = a.ldc2 = m.ldb;
    double *Bk = m.B + (int64_t)k * nb + (int64_t)c0 * m.ldb;
    if (larfb) {
      a.C2 = Bk;
    } else {
      a.C1 = Bk;
      a.C2 = m.B + (int64_t)i * nb + (int64_t)c0 * m.ldb;
    }
  } else {
    a.ncols = min(m.w, tile_cols(m, j) - c0);
    if (larfb) {
      a.C2 = At(k, j) + (int64_t)c0 * lda;
    } else {
      a.C1 = At(k, j) + (int64_t)c0 * lda;
      a.C2 = At(i, j) + (int64_t)c0 * lda;
    }
  }
  apply_strip<MBT>(L, a.V, a.ldv, a.vrows, a.kind, a.kref, a.ib, a.T, a.ldt, a.C1, a.ldc1, a.C2,
                   a.ldc2, a.ncols, nw);
}

__device__ inline int ld_acquire(const int *p) {
  return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}

// Thread 0 polls the task's counters; gives up (and flags `err`) after
// `timeout` wall-clock ticks or when another workgroup flagged an error.
__device__ __forceinline__ bool wait_deps(const Task &t, const MatDesc &m, const int *ctr, int *err,
                          long long timeout) {
  __shared__ int s_ok;
  if (threadIdx.x == 0) {
    int ok = 1;
    const long long t0 = wall_clock64();
    const int nw = task_nwaits(t, m);
    for (int q = 0; q < nw && ok; ++q) {
      int64_t idx;
      int target;
      task_wait(t, m, q, &idx, &target);
      unsigned spins = 0;
      while (ld_acquire(ctr + idx) < target) {
        __builtin_amdgcn_s_sleep(2);
        if ((++spins & 63u) == 0) {
          if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
            ok = 0;
            break;
          }
          if (wall_clock64() - t0 > timeout) {
            __hip_atomic_store(err, TQ_DEVERR_WATCHDOG, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            ok = 0;
            break;
          }
        }
      }
    }
    s_ok = ok;
  }
  __syncthreads();
  const int ok = __builtin_amdgcn_readfirstlane(s_ok);
  __syncthreads();
  return ok != 0;
}

template <int MBT>
__global__ __launch_bounds__(NTHR) __attribute__((amdgpu_waves_per_eu(MBT <= 8 ? 2 : 1, MBT <= 8 ? 2 : 1))) void tq_persistent(const Task *__restrict__ tasks,
                                                      int64_t ntasks, MatDesc single,
                                                      const MatDesc *__restrict__ mats, int *ctr,
                                                      unsigned int *ticket, int *err,
                                                      int use_waits, long long timeout) {
  extern __shared__ double lds_dyn[];
  __shared__ int s_t;
  for (;;) {
    if (threadIdx.x == 0) {
      const int e = __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      s_t = e ? -1 : (int)atomicAdd(ticket, 1u);
    }
    __syncthreads();
    // Uniform across the workgroup: read into a scalar register so that the
    // task's parameters (and every loop bound derived from them) are scalar.
    const int64_t t = __builtin_amdgcn_readfirstlane(s_t);
    __syncthreads();
    if (t < 0 || t >= ntasks) break;
    const Task tk = tasks[t];
    const MatDesc m = mats ? mats[task_mat(tk)] : single;
    if (use_waits && !wait_deps(tk, m, ctr, err, timeout)) break;
    const Lds L = make_lds(lds_dyn, MBT, m.ib, m.w >> 4);
    run_task<MBT>(tk, m, L);
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0 && use_waits) {
      const int ns = task_nsignals(tk);
      for (int q = 0; q < ns; ++q)
        __hip_atomic_fetch_add(ctr + task_signal(tk, m, q), 1, __ATOMIC_RELEASE,
                               __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

__global__ void tq_zero_ints(int *p, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0;
}

// Step-1 kernel benchmark: every workgroup applies `calls` full-tile SSRFBs
// (all strips) to its own tiles, one after the other.
template <int MBT>
__global__ __launch_bounds__(NTHR) void tq_ssrfb_bench(double *buf, int nb, int ib, int calls,
                                                       int nw) {
  extern __shared__ double lds_dyn[];
  const Lds L = make_lds(lds_dyn, MBT, ib, nw);
  const int64_t per = 3 * (int64_t)nb * nb + (int64_t)ib * nb;
  double *V = buf + per * blockIdx.x;
  double *C1 = V + (int64_t)nb * nb, *C2 = C1 + (int64_t)nb * nb, *T = C2 + (int64_t)nb * nb;
  for (int call = 0; call < calls; ++call)
    apply_cols<MBT>(L, V, nb, nb, VK_FULL, nb, ib, T, ib, C1, nb, C2, nb, nb, nw);
}

// Deterministic fill with values in [-scale, scale] (splitmix64 hash).
__global__ void tq_fill_hash(double *p, int64_t n, uint64_t seed, double scale) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    uint64_t z = seed + 0x9E3779B97F4A7C15ull * (uint64_t)(i + 1);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    p[i] = scale * (2.0 * ((double)(z >> 11) * (1.0 / 9007199254740992.0)) - 1.0);
  }
}

template <int MBT>
hipError_t launch_persistent_t(const TqLaunch &a, hipStream_t st) {
  auto kern = tq_persistent<MBT>;
  if (a.lds_bytes > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)a.lds_bytes);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(kern, dim3(a.grid), dim3(NTHR), a.lds_bytes, st, a.tasks, a.ntasks, a.single,
                     a.mats, a.ctr, a.ticket, a.err, a.use_waits, a.timeout);
  return hipGetLastError();
}

template <int MBT>
int occupancy_t(size_t lds) {
  auto kern = tq_persistent<MBT>;
  if (lds > 64 * 1024)
    hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  int nblk = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nblk, kern, NTHR, lds) != hipSuccess) return 1;
  return nblk > 0 ? nblk : 1;
}

template <int MBT>
hipError_t launch_bench_t(double *buf, int nb, int ib, int calls, int nw, int grid, hipStream_t st) {
  auto kern = tq_ssrfb_bench<MBT>;
  size_t lds = (size_t)lds_doubles(MBT, ib, nw) * 8;
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(kern, dim3(grid), dim3(NTHR), lds, st, buf, nb, ib, calls, nw);
  return hipGetLastError();
}

}  // namespace

hipError_t tq_launch_persistent(const TqLaunch &a, hipStream_t st) {
  if (a.nctr_zero > 0) {
    int64_t n = a.nctr_zero;
    int g = (int)((n + 255) / 256);
    g = g > 1024 ? 1024 : (g < 1 ? 1 : g);
    hipLaunchKernelGGL(tq_zero_ints, dim3(g), dim3(256), 0, st, a.ctr_base, n);
  }
  switch (a.mbt) {
    case 4: return launch_persistent_t<4>(a, st);
    case 8: return launch_persistent_t<8>(a, st);
    case 16: return launch_persistent_t<16>(a, st);
    case 32: return launch_persistent_t<32>(a, st);
  }
  return hipErrorInvalidValue;
}

int tq_occupancy(int mbt, size_t lds) {
  switch (mbt) {
    case 4: return occupancy_t<4>(lds);
    case 8: return occupancy_t<8>(lds);
    case 16: return occupancy_t<16>(lds);
    case 32: return occupancy_t<32>(lds);
  }
  return 1;
}

hipError_t tq_launch_ssrfb_bench(double *buf, int nb, int ib, int calls, int grid, hipStream_t st) {
  const int nw = nwaves_for(nb, ib);
  switch (mbt_for_nb(nb)) {
    case 4: return launch_bench_t<4>(buf, nb, ib, calls, nw, grid, st);
    case 8: return launch_bench_t<8>(buf, nb, ib, calls, nw, grid, st);
    case 16: return launch_bench_t<16>(buf, nb, ib, calls, nw, grid, st);
    case 32: return launch_bench_t<32>(buf, nb, ib, calls, nw, grid, st);
  }
  return hipErrorInvalidValue;
}

hipError_t tq_launch_fill(double *p, int64_t n, uint64_t seed, double scale, hipStream_t st) {
  int g = (int)((n + 255) / 256);
  g = g > 4096 ? 4096 : (g < 1 ? 1 : g);
  hipLaunchKernelGGL(tq_fill_hash, dim3(g), dim3(256), 0, st, p, n, seed, scale);
  return hipGetLastError();
}
