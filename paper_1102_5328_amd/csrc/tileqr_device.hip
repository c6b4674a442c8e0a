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

// Address-space-qualified views of global (1) and LDS (3) memory, so that
// accesses compile to global_* / ds_* instructions with 32-bit LDS
// addresses rather than to generic flat ones.
typedef __attribute__((address_space(1))) double gdbl;
typedef __attribute__((address_space(3))) double ldbl;
__device__ inline gdbl *gp(double *p) { return (gdbl *)p; }
__device__ inline const gdbl *gp(const double *p) { return (const gdbl *)p; }

namespace {

constexpr int NTHR = TQ_NTHR;

// Register classes up to this one are compiled for two waves per SIMD
// (256 registers per lane); larger ones get the full register file.
#ifndef TQ_WPE2_MAX_MBT
#define TQ_WPE2_MAX_MBT 8
#endif
enum { VK_UNIT = 0, VK_FULL = 1 };

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }
__device__ __forceinline__ int wave_id() { return threadIdx.x >> 6; }

__device__ __forceinline__ d4 mfma(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

struct Lds {
  ldbl *vc;     // gmax chunks of 16 columns of V, column c at c * ldvc
  ldbl *y;      // nw regions of ibp x 16 (Y, then W in place)
  ldbl *ts;     // T_s of the current block, [a * ldts + c] (aliases the panel scratch)
  ldbl *red1;   // 4
  ldbl *red32;  // 4 x 16
  ldbl *tot;    // 16 (+16)
  ldbl *scal;   // 8
  ldbl *tmm;    // 32 x 33 micro-panel T, [a*33 + c]
  ldbl *top;    // 32 x 33 TSQRT top block
  int ldvc, ibp, gmax;
};

__device__ inline Lds make_lds(double *lds_base, int mbt, int ib, int nw, int gmax) {
  Lds L;
  L.ldvc = lds_ldvc(mbt);
  L.ibp = ib_pad16(ib);
  L.gmax = gmax;
  ldbl *p = (ldbl *)lds_base;
  L.vc = p;
  p += (int64_t)gmax * 16 * L.ldvc;
  L.y = p;
  p += nw * L.ibp * 16;
  L.ts = p;
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

// Width of the register-resident micro-panel in the panel kernels.
constexpr int PWM = 16;

// ---------------------------------------------------------------------------
// Block-reflector application (LARFB / SSRFB bodies)
// ---------------------------------------------------------------------------

// Stages chunks of V into LDS: columns gc0 .. gc0 + 16*ng of V (column c of
// the group at L.vc + c*ldvc), rows 0..vrows rounded up to 16, zero outside
// the reflector support. VK_UNIT: column gc has an implicit 1 at row gc and
// 0 above. Four independent loads per thread are issued before their LDS
// stores so that one memory latency covers them.
template <int MBT>
__device__ inline void load_vgroup(const Lds &L, const double *V, int64_t ldv, int vrows,
                                   int kind, int gc0, int kvalid, int ng) {
  constexpr int RP = MBT * 16;
  const int rlim = (vrows + 15) & ~15;
  const int total = ng * 16 * RP;
  const gdbl *Vg = gp(V);
  for (int base = 0; base < total; base += NTHR * 4) {
    double v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = base + u * NTHR + threadIdx.x;
      const int c = e / RP, r = e % RP;
      const int gc = gc0 + c;
      double x = 0.0;
      if (e < total && r < vrows && gc < kvalid) {
        if (kind == VK_UNIT)
          x = r < gc ? 0.0 : (r == gc ? 1.0 : Vg[r + (int64_t)gc * ldv]);
        else
          x = Vg[r + (int64_t)gc * ldv];
      }
      v[u] = x;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = base + u * NTHR + threadIdx.x;
      const int c = e / RP, r = e % RP;
      if (e < total && r < rlim) L.vc[c * L.ldvc + r] = v[u];
    }
  }
}

// T_s (ibw x ibw upper triangle of the block at Tb, leading dimension ldt)
// into L.ts as [a * (ibp + 1) + c], zero elsewhere up to ibp x ibp, where ibp
// is the padded inner block of the application in progress (not the task's).
__device__ inline void load_tblock(const Lds &L, const double *Tb, int64_t ldt, int ibw, int ibp) {
  const int total = ibp * ibp, ldts = lds_ldts(ibp);
  const gdbl *Tg = gp(Tb);
  for (int base = 0; base < total; base += NTHR * 4) {
    double v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = base + u * NTHR + threadIdx.x;
      const int a = e / ibp, c = e % ibp;
      v[u] = (e < total && a <= c && c < ibw) ? Tg[a + (int64_t)c * ldt] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = base + u * NTHR + threadIdx.x;
      if (e < total) L.ts[(e / ibp) * ldts + (e % ibp)] = v[u];
    }
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
  const gdbl *Cg = gp(C);
#pragma unroll
  for (int rt = 0; rt < MBT; ++rt) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = rt * 16 + 4 * r + g;
      double v = 0.0;
      if (colok && row < crows) {
        if (kind == VK_UNIT) {
          const int h = diag + col;
          v = row < h ? 0.0 : (row == h ? 1.0 : Cg[row + (int64_t)col * ldc]);
        } else {
          v = Cg[row + (int64_t)col * ldc];
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
  gdbl *Cg = gp(C);
#pragma unroll
  for (int rt = 0; rt < MBT; ++rt) {
    if (rt * 16 >= crows) break;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = rt * 16 + 4 * r + g;
      if (row < crows) Cg[row + (int64_t)col * ldc] = c2[rt][r];
    }
  }
}

// Y rows of the staged chunks (group starting at chunk g0 of the block whose
// first reflector is s): Y[q] = V[:, s+16q..]^T C2 -> wave region yw. The B
// operand is accumulator register r of C2 tile rt (k index lane/16 <-> row
// 16*rt + 4*r + lane/16); the A operand is V^T at those rows.
template <int MBT>
__device__ inline void y_group(const Lds &L, int kind, int s, int g0, int ng, int vrows,
                               const d4 (&c2)[MBT], ldbl *yw) {
  const int ln = lane_id();
  for (int g = 0; g < ng; ++g) {
    const int q = g0 + g;
    d4 y0 = {0.0, 0.0, 0.0, 0.0}, y1 = {0.0, 0.0, 0.0, 0.0};
    const int rt0 = (kind == VK_UNIT) ? ((s + q * 16) >> 4) : 0;
    const ldbl *vp = L.vc + (g * 16 + (ln & 15)) * L.ldvc + (ln >> 4);
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

// C2 -= V_s W for the staged chunks: A = -V[row 16*rt + lane%16][col 4kk +
// lane/16 of chunk q], B = W[16q + 4kk + lane/16][lane%16].
template <int MBT>
__device__ inline void update_group(const Lds &L, int kind, int s, int g0, int ng, int vrows,
                                    const ldbl *yw, d4 (&c2)[MBT]) {
  const int ln = lane_id();
  for (int g = 0; g < ng; ++g) {
    const int q = g0 + g;
    const int rt0 = (kind == VK_UNIT) ? ((s + q * 16) >> 4) : 0;
    double b[4];
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) b[kk] = yw[(q * 16 + 4 * kk + (ln >> 4)) * 16 + (ln & 15)];
    const ldbl *vp = L.vc + (g * 16 + (ln >> 4)) * L.ldvc + (ln & 15);
#pragma unroll
    for (int rt = 0; rt < MBT; ++rt) {
      if (rt >= rt0 && rt * 16 < vrows) {
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) c2[rt] = mfma(-vp[4 * kk * L.ldvc + rt * 16], b[kk], c2[rt]);
      }
    }
  }
}

// W = T_s^T Ytot in place in the wave region, bottom block first (W block q
// needs Y blocks <= q). T_s from the LDS stage or from global memory.
template <bool TLDS>
__device__ inline void w_phase(const Lds &L, const double *Ts, int64_t ldt, int ibw, int ldts,
                               ldbl *yw) {
  const gdbl *Tg = gp(Ts);
  const int ln = lane_id();
  const int nq = (ibw + 15) >> 4;
  for (int q = nq - 1; q >= 0; --q) {
    d4 w = {0.0, 0.0, 0.0, 0.0};
    const int ccol = q * 16 + (ln & 15);
    for (int q2 = 0; q2 <= q; ++q2) {
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) {
        const int arow = q2 * 16 + 4 * kk + (ln >> 4);
        double a;
        if (TLDS)
          a = L.ts[arow * ldts + ccol];
        else
          a = (arow <= ccol && ccol < ibw) ? Tg[arow + (int64_t)ccol * ldt] : 0.0;
        w = mfma(a, yw[arow * 16 + (ln & 15)], w);
      }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) yw[(q * 16 + 4 * r + (ln >> 4)) * 16 + (ln & 15)] = w[r];
  }
}

// yw[a][c] += C1[s + a][col c] (add = true) or C1 -= yw (add = false) for the
// wave's columns; loads batched four per lane.
__device__ inline void c1_pass(ldbl *yw, double *C1, int64_t ldc1, int s, int ibw, int ncols,
                               bool add) {
  const int ln = lane_id(), wv = wave_id();
  gdbl *Cg = gp(C1);
  const int total = ibw * 16;
  for (int base = 0; base < total; base += 64 * 4) {
    double v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = base + u * 64 + ln;
      const int a = e >> 4, c = wv * 16 + (e & 15);
      v[u] = (e < total && c < ncols) ? Cg[(s + a) + (int64_t)c * ldc1] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = base + u * 64 + ln;
      const int a = e >> 4, c = wv * 16 + (e & 15);
      if (e < total) {
        if (add)
          yw[e] += v[u];
        else if (c < ncols)
          Cg[(s + a) + (int64_t)c * ldc1] = v[u] - yw[e];
      }
    }
  }
}

// Applies the reflectors V[:, 0..kref) (blocks of ib, compact-WY factors in
// T: block s at T + s*ldt) to one strip of at most 16*nw columns:
//   C1 (optional): rows s..s+ib of the block's top part, C2: vrows rows.
// Per block: stage V_s (and T_s) in LDS once, Y = V_s^T C2 + C1_s,
// W = T_s^T Y, C1_s -= W, C2 -= V_s W.
//
// yonly: stop after Y of the first block (Y left in the wave region), with C2
// read as reflectors (unit-lower with head row c2diag + col if c2diag >= 0,
// full otherwise): the Gram product of the T assembly; nothing is written.
template <int MBT>
__device__ __forceinline__ void apply_strip(const Lds &L, const double *V, int64_t ldv, int vrows,
                                            int kind, int kref, int ib, const double *T,
                                            int64_t ldt, double *C1, int64_t ldc1, double *C2,
                                            int64_t ldc2, int ncols, int nw, bool yonly,
                                            int c2diag) {
  const int ln = lane_id(), wv = wave_id();
  const bool active = (wv < nw) && (wv * 16 < ncols);
  const int col = wv * 16 + (ln & 15);
  const bool colok = active && col < ncols;
  d4 c2[MBT];
  load_c2<MBT>(c2, C2, ldc2, vrows, col, colok, (yonly && c2diag >= 0) ? VK_UNIT : VK_FULL,
               c2diag);
  ldbl *yw = L.y + wv * L.ibp * 16;
  // T_s staged in LDS when the block is narrow enough; the stage region is
  // sized for the task's inner block and for the panel scratch, so any
  // application with ib_pad16(ib) <= 64 fits.
  const bool tl = t_in_lds(ib);
  const int ibp_a = ib_pad16(ib), ldts_a = lds_ldts(ibp_a);
  for (int s = 0; s < kref; s += ib) {
    const int ibw = min(ib, kref - s);
    const int nq = (ibw + 15) >> 4;
    const bool resident = nq <= L.gmax;
    for (int g0 = 0; g0 < nq; g0 += L.gmax) {
      const int ng = min(L.gmax, nq - g0);
      __syncthreads();
      load_vgroup<MBT>(L, V, ldv, vrows, kind, s + g0 * 16, s + ibw, ng);
      if (g0 == 0 && tl && !yonly) load_tblock(L, T + (int64_t)s * ldt, ldt, ibw, ibp_a);
      __syncthreads();
      if (active) y_group<MBT>(L, kind, s, g0, ng, vrows, c2, yw);
    }
    __syncthreads();
    if (yonly) return;
    if (active && C1) c1_pass(yw, C1, ldc1, s, ibw, ncols, true);
    __syncthreads();
    if (active) {
      if (tl)
        w_phase<true>(L, nullptr, 0, ibw, ldts_a, yw);
      else
        w_phase<false>(L, T + (int64_t)s * ldt, ldt, ibw, ldts_a, yw);
    }
    __syncthreads();
    if (active && C1) c1_pass(yw, C1, ldc1, s, ibw, ncols, false);
    for (int g0 = 0; g0 < nq; g0 += L.gmax) {
      const int ng = min(L.gmax, nq - g0);
      if (!resident) {
        __syncthreads();
        load_vgroup<MBT>(L, V, ldv, vrows, kind, s + g0 * 16, s + ibw, ng);
        __syncthreads();
      }
      if (active) update_group<MBT>(L, kind, s, g0, ng, vrows, yw, c2);
    }
  }
  __syncthreads();
  store_c2<MBT>(c2, C2, ldc2, vrows, col, colok);
}

// All columns of C2 (and C1), in strips of 16*nw.
template <int MBT>
__device__ __forceinline__ void apply_cols(const Lds &L, const double *V, int64_t ldv, int vrows, int kind,
                           int kref, int ib, const double *T, int64_t ldt, double *C1,
                           int64_t ldc1, double *C2, int64_t ldc2, int ncols, int nw, bool yonly,
                           int c2diag) {
  const int w = 16 * nw;
  for (int c0 = 0; c0 < ncols; c0 += w) {
    apply_strip<MBT>(L, V, ldv, vrows, kind, kref, ib, T, ldt,
                     C1 ? C1 + (int64_t)c0 * ldc1 : nullptr, ldc1, C2 + (int64_t)c0 * ldc2, ldc2,
                     min(w, ncols - c0), nw, yonly, c2diag);
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
// slots PW-c..PW-1 (column p at slot PW-c+p).
template <int HR, int PW>
__device__ inline void rotate_slots(double (&x)[HR][PW]) {
#pragma unroll
  for (int h = 0; h < HR; ++h) {
    const double t0 = x[h][0];
#pragma unroll
    for (int i = 0; i < PW - 1; ++i) x[h][i] = x[h][i + 1];
    x[h][PW - 1] = t0;
  }
}

__device__ inline void store_micro_T(const Lds &L, double *Tmm, int64_t ldt, int pw) {
  __syncthreads();
  gdbl *Tg = gp(Tmm);
  for (int e = threadIdx.x; e < pw * pw; e += NTHR) {
    const int a = e % pw, c = e / pw;
    Tg[a + (int64_t)c * ldt] = a <= c ? L.tmm[a * 33 + c] : 0.0;
  }
  __syncthreads();
}

// Orders the wave's LDS accesses before this point against those after it
// (the lanes of a wave run in lockstep; this pins the compiler's ordering).
__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Wave-level sum of one double (xor butterfly; every lane gets the total).
__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// Wave-level sums of v[0..NV) (NV = 8 or 16) into slot[0..NV), an LDS slot
// private to the calling wave; every lane then reads the totals it needs.
// Each exchange step hands half of the remaining values to the partner lane,
// so NV values cost NV - 1 shuffles instead of NV butterflies.
template <int NV>
__device__ inline void wave_sumN(ldbl *slot, const double (&v)[NV]) {
  const int ln = lane_id();
  double h[NV];
#pragma unroll
  for (int i = 0; i < NV; ++i) h[i] = v[i];
  int n = NV;
  int idx = 0;
#pragma unroll
  for (int bit = 5; bit >= 0; --bit) {
    const int half = n >> 1;
    if (half == 0) {
      h[0] += __shfl_xor(h[0], 1 << bit);
    } else {
      const bool hi = (ln >> bit) & 1;
#pragma unroll
      for (int i = 0; i < NV / 2; ++i) {
        if (i < half) {
          const double snd = hi ? h[i] : h[half + i];
          const double keep = hi ? h[half + i] : h[i];
          h[i] = keep + __shfl_xor(snd, 1 << bit);
        }
      }
      idx = idx * 2 + (hi ? 1 : 0);
      n = half;
    }
  }
  // Lanes sharing the low (6 - log2 NV) bits hold the same total, index idx.
  constexpr int LOW = (NV == 16) ? 2 : 3;
  if (!(ln & ((1 << LOW) - 1))) slot[idx] = h[0];
  wave_sync();
}

// Unblocked Householder QR of one micro-panel of pw <= PW columns on ONE
// wave (wave 0): lane l holds rows l, l+64, ... in registers, so every
// reduction is wave-local and the column loop has no workgroup barrier.
//  GEQRT (ts == false): X = P[0..mrows) x [m0, m0+pw) in the block frame;
//    reflector c has its unit at row m0+c, zeros above.
//  TSQRT (ts == true): X = U[0..mrows) x [0, pw) under the pw x pw upper
//    block of R kept in L.top; reflector c is [e_c; u_c].
// Each column costs one reduction for the norm and one batched reduction for
// all its dot products (remaining columns: the update; finished columns: the
// Gram entries that build column c of the micro-panel's T). Waves 1..3 wait
// at the closing barrier.
template <int HRW, int PW>
__device__ __forceinline__ void level2_panel(const Lds &L, bool ts, double *X, int64_t ldx,
                                             int mrows, int m0, int pw, double *Tmm, int64_t ldt) {
  if (wave_id() == 0) {
    const int ln = lane_id();
    gdbl *Xg = gp(X);
    double x[HRW][PW];
#pragma unroll
    for (int h = 0; h < HRW; ++h) {
      const int row = ln + 64 * h;
#pragma unroll
      for (int i = 0; i < PW; ++i)
        x[h][i] = (i < pw && row < mrows) ? Xg[row + (int64_t)(m0 + i) * ldx] : 0.0;
    }
    for (int c = 0; c < pw; ++c) {
      const int jr = ts ? -1 : m0 + c;  // rows > jr form the reflector tail
      double ss = 0.0, own = x[0][0];
#pragma unroll
      for (int h = 0; h < HRW; ++h) {
        const int row = ln + 64 * h;
        if (row > jr) ss += x[h][0] * x[h][0];
        if (h > 0 && (jr >> 6) == h) own = x[h][0];
      }
      ss = wave_sum(ss);
      const double alpha = ts ? L.top[c * 33 + c] : __shfl(own, jr & 63);
      double beta, tau, scale;
      householder(alpha, ss, beta, tau, scale);
      double v[HRW];
#pragma unroll
      for (int h = 0; h < HRW; ++h) {
        const int row = ln + 64 * h;
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
      double d[PW];
      d[0] = 0.0;
#pragma unroll
      for (int i = 1; i < PW; ++i) {
        double a = 0.0;
#pragma unroll
        for (int h = 0; h < HRW; ++h) a += v[h] * x[h][i];
        d[i] = a;
      }
      ldbl *tot = L.tot;
      wave_sumN<PW>(tot, d);
      const int nrem = pw - 1 - c;
      if (ts) {
        // Remaining columns' dot products include row c of R; then row c of
        // R is updated.
        if (ln >= 1 && ln <= nrem) tot[ln] += L.top[c * 33 + c + ln];
        wave_sync();
        if (ln >= 1 && ln <= nrem) L.top[c * 33 + c + ln] -= tau * tot[ln];
        if (ln == 0) L.top[c * 33 + c] = beta;
      }
#pragma unroll
      for (int i = 1; i < PW; ++i) {
        if (i <= nrem) {
          const double f = tau * tot[i];
#pragma unroll
          for (int h = 0; h < HRW; ++h) x[h][i] -= f * v[h];
        }
      }
      // T column c from the Gram entries of the finished columns (slot
      // PW-c+p holds column p < c).
      if (ln < c) {
        double tval = 0.0;
        for (int p = ln; p < c; ++p) tval += L.tmm[ln * 33 + p] * tot[PW - c + p];
        L.tmm[ln * 33 + c] = -tau * tval;
      }
      if (ln == 0) L.tmm[c * 33 + c] = tau;
      wave_sync();
      rotate_slots<HRW, PW>(x);
    }
#pragma unroll
    for (int h = 0; h < HRW; ++h) {
      const int row = ln + 64 * h;
#pragma unroll
      for (int i = 0; i < PW; ++i) {
        const int p = (i + pw) & (PW - 1);
        if (p < pw && row < mrows) Xg[row + (int64_t)(m0 + p) * ldx] = x[h][i];
      }
    }
  }
  store_micro_T(L, Tmm, ldt, pw);
}

// After micro-panel [m0, m0+pw) of an IB block, with the Gram block
// G = V[:, 0:m0]^T V[:, m0:m0+pw] already in the wave-0 region of L.y:
// T[0:m0, m0:m0+pw] = -T[0:m0, 0:m0] G T[m0:, m0:], lower block zeroed.
__device__ inline void assemble_T_post(const Lds &L, int m0, int pw, double *Tb, int64_t ldt) {
  ldbl *G = L.y;  // wave 0 region: G[a*16 + c]
  gdbl *Tg = gp(Tb);
  for (int a = threadIdx.x; a < m0; a += NTHR) {
    for (int c = pw - 1; c >= 0; --c) {
      double acc = 0.0;
      for (int p = 0; p <= c; ++p) acc += G[a * 16 + p] * Tg[(m0 + p) + (int64_t)(m0 + c) * ldt];
      G[a * 16 + c] = acc;
    }
  }
  __syncthreads();
  for (int e = threadIdx.x; e < m0 * pw; e += NTHR) {
    const int a = e % m0, c = e / m0;
    double acc = 0.0;
    for (int b = a; b < m0; ++b) acc += Tg[a + (int64_t)b * ldt] * G[b * 16 + c];
    Tg[a + (int64_t)(m0 + c) * ldt] = -acc;
  }
  for (int e = threadIdx.x; e < m0 * pw; e += NTHR) {
    const int a = e % pw, c = e / pw;
    Tg[(m0 + a) + (int64_t)c * ldt] = 0.0;
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// Task dispatch and the persistent scheduler
// ---------------------------------------------------------------------------


// Runs one task. Every task is a sequence of steps that end with one
// block-reflector application; panels precede it with the factorization of
// a micro-panel. A single call site of the MFMA routine (and of the panel
// routine) keeps the register allocation of the fused kernel tight.
template <int MBT>
__device__ __forceinline__ void run_task(const Task &t, const MatDesc &m, const Lds &L) {
  constexpr int HRW = (MBT * 16 + 63) / 64;  // panel rows per lane of the panel wave
  constexpr int PWV = HRW >= 2 ? 8 : 16;     // micro-panel width held in registers
  const int nb = m.nb, ib = m.ib, nw = m.w >> 4;
  const int i = t.i, j = t.j, k = t.k, strip = task_strip(t);
  const int type = task_type(t);
  auto At = [&](int r, int c) { return m.A + (int64_t)c * nb * m.lda + (int64_t)r * nb; };
  auto Tt = [&](int r, int c) { return m.T + ((int64_t)c * m.MT + r) * (int64_t)ib * nb; };
  const int64_t lda = m.lda;
  const bool panel = type == TK_GEQRT || type == TK_TSQRT;
  const bool ts = type == TK_TSQRT;

  // Panel state (GEQRT: factor A_kk; TSQRT: factor [R_kk; A_ik]).
  double *R = At(k, k);
  double *U = ts ? At(i, k) : R;
  double *Tp = ts ? Tt(i, k) : Tt(k, k);
  const int pmb = ts ? tile_rows(m, i) : tile_rows(m, k);
  const int pcol = tile_cols(m, k);
  const int K = ts ? pcol : min(pmb, pcol);
  int s = 0, m0 = 0;
  if (panel) {
    // Panels are the critical path: their waves win instruction issue over
    // co-resident update waves.
    __builtin_amdgcn_s_setprio(2);
  }

  // Panel steps: factor a micro-panel, then (if it is not the first of its
  // IB block) the Gram product of the T assembly, then the update of the
  // rest of the block or, after the block's last micro-panel, of the
  // trailing columns. Each loop iteration makes exactly one application.
  int phase = 0;  // 0: factor next micro-panel, 1: T assembly done -> update
  int pw = 0;
  for (;;) {
    const double *aV, *aT;
    double *aC1, *aC2;
    int64_t ldc1 = lda, ldc2 = lda;
    int vrows, kind, kref, aib, ncols, c2diag = 0;
    bool go = true, yonly = false, post_asm = false;
    if (panel) {
      if (s >= K) break;
      const int ibw = min(ib, K - s);
      // Block frame: GEQRT rows/cols start at s; TSQRT rows of U start at 0.
      double *Xb = ts ? U + (int64_t)s * lda : U + s + (int64_t)s * lda;
      double *Rb = R + s + (int64_t)s * lda;
      double *Tb = Tp + (int64_t)s * ib;
      const int mrows = ts ? pmb : pmb - s;
      kind = ts ? VK_FULL : VK_UNIT;
      if (phase == 0) {
        pw = min(PWV, ibw - m0);
        if (ts) {
          const gdbl *Rg = gp(Rb);
          for (int e = threadIdx.x; e < 32 * 32; e += NTHR) {
            const int a = e >> 5, c = e & 31;
            L.top[a * 33 + c] = (a <= c && c < pw) ? Rg[(m0 + a) + (int64_t)(m0 + c) * lda] : 0.0;
          }
          __syncthreads();
        }
        level2_panel<HRW, PWV>(L, ts, Xb, lda, mrows, m0, pw, Tb + m0 + (int64_t)m0 * ib, ib);
        if (ts) {
          gdbl *Rg = gp(Rb);
          for (int e = threadIdx.x; e < 32 * 32; e += NTHR) {
            const int a = e >> 5, c = e & 31;
            if (a <= c && c < pw) Rg[(m0 + a) + (int64_t)(m0 + c) * lda] = L.top[a * 33 + c];
          }
          __syncthreads();
        }
      }
      if (phase == 0 && m0 > 0) {
        // Gram block V[:, 0:m0]^T V[:, m0:m0+pw] (Y of a one-block application)
        aV = Xb;
        vrows = mrows;
        kref = m0;
        aib = m0;
        aT = Tb;
        aC1 = nullptr;
        aC2 = Xb + (int64_t)m0 * lda;
        ncols = pw;
        yonly = true;
        post_asm = true;
        c2diag = ts ? -1 : m0;  // GEQRT vectors: unit at row m0 + col
        phase = 1;
      } else if (m0 + pw < ibw) {
        // this micro-panel's reflectors onto the rest of the IB block
        aV = ts ? Xb + (int64_t)m0 * lda : Xb + m0 + (int64_t)m0 * lda;
        vrows = ts ? mrows : mrows - m0;
        kref = pw;
        aib = pw;
        aT = Tb + m0 + (int64_t)m0 * ib;
        aC1 = ts ? Rb + m0 + (int64_t)(m0 + pw) * lda : nullptr;
        aC2 = ts ? Xb + (int64_t)(m0 + pw) * lda : Xb + m0 + (int64_t)(m0 + pw) * lda;
        ncols = ibw - m0 - pw;
        m0 += pw;
        phase = 0;
      } else {
        // the whole IB block onto the trailing columns of the tile
        aV = Xb;
        vrows = mrows;
        kref = ibw;
        aib = ibw;
        aT = Tb;
        aC1 = ts ? Rb + (int64_t)ibw * lda : nullptr;
        aC2 = Xb + (int64_t)ibw * lda;
        ncols = pcol - s - ibw;
        go = ncols > 0;
        s += ibw;
        m0 = 0;
        phase = 0;
      }
    } else {
      aib = ib;
      aC1 = nullptr;
      const int c0 = strip * m.w;
      const bool onB = type == TK_LARFB_B || type == TK_SSRFB_B;
      const bool larfb = type == TK_LARFB || type == TK_LARFB_B;
      if (larfb) {
        const int mb = tile_rows(m, k);
        aV = At(k, k);
        vrows = mb;
        kind = VK_UNIT;
        kref = min(mb, tile_cols(m, k));
        aT = Tt(k, k);
      } else {
        aV = At(i, k);
        vrows = tile_rows(m, i);
        kind = VK_FULL;
        kref = tile_cols(m, k);
        aT = Tt(i, k);
      }
      if (onB) {
        ncols = min(m.w, m.nrhs - c0);
        ldc1 = ldc2 = m.ldb;
        double *Bk = m.B + (int64_t)k * nb + (int64_t)c0 * m.ldb;
        if (larfb) {
          aC2 = Bk;
        } else {
          aC1 = Bk;
          aC2 = m.B + (int64_t)i * nb + (int64_t)c0 * m.ldb;
        }
      } else {
        ncols = min(m.w, tile_cols(m, j) - c0);
        if (larfb) {
          aC2 = At(k, j) + (int64_t)c0 * lda;
        } else {
          aC1 = At(k, j) + (int64_t)c0 * lda;
          aC2 = At(i, j) + (int64_t)c0 * lda;
        }
      }
    }
    if (go)
      apply_cols<MBT>(L, aV, lda, vrows, kind, kref, aib, aT, ib, aC1, ldc1, aC2, ldc2, ncols, nw,
                      yonly, c2diag);
    if (post_asm) assemble_T_post(L, m0, pw, Tp + (int64_t)s * ib, ib);
    if (!panel) break;
  }
  if (panel) __builtin_amdgcn_s_setprio(0);
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
__global__ __launch_bounds__(NTHR) __attribute__((amdgpu_waves_per_eu(MBT <= TQ_WPE2_MAX_MBT ? 2 : 1, MBT <= TQ_WPE2_MAX_MBT ? 2 : 1))) void tq_persistent(const Task *__restrict__ tasks,
                                                      int64_t ntasks, MatDesc single,
                                                      const MatDesc *__restrict__ mats, int *ctr,
                                                      unsigned int *ticket, int *err,
                                                      int use_waits, long long timeout,
                                                      long long *trace) {
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
    const long long t_take = trace ? wall_clock64() : 0;
    if (use_waits && !wait_deps(tk, m, ctr, err, timeout)) break;
    const long long t_run = trace ? wall_clock64() : 0;
    const Lds L = make_lds(lds_dyn, MBT, m.ib, m.w >> 4, m.gmax);
    run_task<MBT>(tk, m, L);
    __threadfence();
    __syncthreads();
    if (trace && threadIdx.x == 0) {
      trace[4 * t + 0] = t_take;
      trace[4 * t + 1] = t_run;
      trace[4 * t + 2] = wall_clock64();
      trace[4 * t + 3] = blockIdx.x;
    }
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
  const Lds L = make_lds(lds_dyn, MBT, ib, nw, lds_plan(MBT, ib).gmax);
  const int64_t per = 3 * (int64_t)nb * nb + (int64_t)ib * nb;
  double *V = buf + per * blockIdx.x;
  double *C1 = V + (int64_t)nb * nb, *C2 = C1 + (int64_t)nb * nb, *T = C2 + (int64_t)nb * nb;
  for (int call = 0; call < calls; ++call)
    apply_cols<MBT>(L, V, nb, nb, VK_FULL, nb, ib, T, ib, C1, nb, C2, nb, nb, nw, false, 0);
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
                     a.mats, a.ctr, a.ticket, a.err, a.use_waits, a.timeout, a.trace);
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
  size_t lds = (size_t)lds_plan(MBT, ib).doubles * 8;
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
