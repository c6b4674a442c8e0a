// Tile Householder QR kernels for gfx950 (MI355X), FP64.
//
// One persistent kernel runs every task of the tile DAG (Section 2.1): each
// workgroup (4 x wave64) repeatedly takes the next ticket of a host-built
// topological order, waits on the dependency counters of that task, runs it,
// and bumps the counters of the data it wrote.
//
// Register layout: a wave holds a block of 128 rows x 16 columns in the
// accumulator layout of v_mfma_f64_16x16x4f64 (lane l, item (t, r) holds row
// 16t + 4r + l/16 of column l%16). Tiles taller than 128 rows are covered by
// several waves ("row waves") that hold consecutive 128-row slabs of the
// same 16 columns; see layout.h.
//
// Task bodies:
//  * LARFB / SSRFB (and the updates inside the panels) apply a run of
//    compact-WY block reflectors H = I - V T V^T, IB columns at a time:
//        W = T^T (C1_s + V_s^T C2),  C1_s -= W,  C2 -= V_s W.
//    C2 stays in the wave registers for the whole task; its products with
//    V_s^T and V_s run on the FP64 MFMA with the accumulators as operands.
//    V_s and T_s are staged in LDS; when a block is small enough, the next
//    block's V, T and C1 rows are loaded into registers while the current
//    one computes, so each block costs two barriers and no exposed memory
//    latency.
//  * GEQRT / TSQRT factor a register panel of up to 64 columns held in
//    registers by all four waves: per Householder column, one wave-level
//    reduction for the norm, one LDS broadcast of the reflector, and one
//    reduction for all the dot products (one barrier per column when the
//    tile has at most 128 rows). The lanes of finished columns compute the
//    Gram entries of the compact-WY factor T at no extra cost, and wave 0
//    runs the T recurrence one column behind. The rest of the tile is then
//    updated with the MFMA routine above.
//
// Storage: A column-major with leading dimension lda, tiles addressed in
// place (ragged last tile row/column allowed). T of tile (i, k) is an
// IB x nb_k array at T + (k*MT + i)*IB*NB, leading dimension IB; the block
// of columns [s, s+IB) holds the upper-triangular T_s (zero below).
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
constexpr int RT = TQ_ROWS_PER_WAVE / 16;  // 16-row tiles per wave block
constexpr int PF = 16;                     // doubles per lane of a register-staged V block
enum { VK_UNIT = 0, VK_FULL = 1 };

// The thread index, opaque to the optimizer at every use: in a persistent
// kernel every value derived from it (addresses, predicates of unrolled
// loops) is loop-invariant, and hoisting all of them out of the task loop
// would keep hundreds of them live for the whole kernel. The empty asm makes
// the compiler recompute them where they are used instead.
__device__ __forceinline__ int tid_x() {
  int t = threadIdx.x;
  asm volatile("" : "+v"(t));
  return t;
}
__device__ __forceinline__ int lane_id() { return tid_x() & 63; }
// Wave index in a scalar register (uniform across the wave).
__device__ __forceinline__ int wave_id() { return __builtin_amdgcn_readfirstlane(tid_x() >> 6); }

__device__ __forceinline__ d4 mfma(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Orders the wave's LDS accesses before this point against those after it
// (the lanes of a wave run in lockstep; this pins the compiler's ordering).
__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// A double from lane l ^ 1 (CTRL = 0xB1, quad_perm [1,0,3,2]) or l ^ 2
// (CTRL = 0x4E, quad_perm [2,3,0,1]) by DPP: a register move, no LDS trip.
template <int CTRL>
__device__ __forceinline__ double dpp_quad(double v) {
  const uint64_t b = __builtin_bit_cast(uint64_t, v);
  const int lo = __builtin_amdgcn_mov_dpp((int)(uint32_t)b, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(uint32_t)(b >> 32), CTRL, 0xF, 0xF, false);
  return __builtin_bit_cast(double, ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

// Sum over the four adjacent lanes of a quad (the lanes holding the rows of
// one column in the panel layout); every one of them gets the total.
__device__ inline double quad_sum(double v) {
  v += dpp_quad<0xB1>(v);
  v += dpp_quad<0x4E>(v);
  return v;
}

// Geometry of a tile class with RW row waves per column group.
template <int RW>
struct Geo {
  static constexpr int ROWS = TQ_ROWS_PER_WAVE * RW;  // rows of a staged V column
  static constexpr int LDVC = ROWS + 1;               // odd: conflict-free transposed reads
  static constexpr int CGN = 4 / RW;                  // column groups of 16
  static constexpr int P = 16 * CGN;                  // strip / register panel width
};

struct Lds {
  // update phase
  ldbl *vc;  // gmax chunks of 16 columns of V, column c at c * ldvc
  ldbl *y;   // one ibp x 16 region per column group (Y, then W in place)
  ldbl *ts;  // T_s of the current block, [a * (ibp + 1) + c]
  // panel phase (aliases the update phase)
  ldbl *vb;    // 2 x rows: reflector broadcast, double-buffered
  ldbl *taus;  // 64
  ldbl *red;   // 4 x 2: norm and alpha partials of the row waves
  ldbl *dred;  // 4 x 64: dot-product partials of the row waves
  ldbl *tg;    // P x (P+1): T (upper, with diagonal) and G^T (strictly lower)
  ldbl *top;   // P x (P+1): TSQRT block of R
  ldbl *z;     // wide-T assembly product (aliases the panel phase)
  int ibp, gmax;
};

template <int RW>
__device__ inline Lds make_lds(double *lds_base, const MatDesc &m) {
  using Gm = Geo<RW>;
  Lds L;
  L.ibp = ib_pad16(m.ib);
  L.gmax = m.gmax;
  ldbl *base = (ldbl *)lds_base;
  L.vc = base;
  L.y = base + L.gmax * 16 * Gm::LDVC;
  L.ts = L.y + Gm::CGN * L.ibp * 16;
  ldbl *p = base;
  L.vb = p;
  p += 2 * Gm::ROWS;
  L.taus = p;
  p += 64;
  L.red = p;
  p += 128;
  L.dred = p;
  p += 256;
  L.tg = p;
  p += Gm::P * (Gm::P + 1);
  L.top = p;
  L.z = base;
  return L;
}

// ---------------------------------------------------------------------------
// Block-reflector application (LARFB / SSRFB bodies, panel trailing updates)
// ---------------------------------------------------------------------------

// V chunks [gc0, gc0 + 16*ng) (columns of V, rows 0 .. 128*RW) into per-lane
// registers: element e = ebase + u*256 + tid sits at column e / ROWS, row
// e % ROWS, so a lane walks one row (or two, ROWS = 512) and steps over
// columns with a fixed stride. The registers hold the values as loaded (every
// read inside the block, at clamped indices); vstage_store applies the
// reflector support and the unit diagonal. Selecting here would make each
// load wait at once, and with it every load issued before it.
template <int RW>
__device__ inline void vstage_load(double (&v)[PF], const double *V, int64_t ldv, int vrows,
                                   int gc0, int kvalid, int ebase, int total) {
  constexpr int ROWS = Geo<RW>::ROWS;
  constexpr int CPU = ROWS <= NTHR ? NTHR / ROWS : 1;  // columns per step of u (ROWS <= 256)
  const int tid = tid_x();
  const int e0 = ebase + tid;
  const int r0 = e0 % ROWS, c0 = gc0 + e0 / ROWS;
  const gdbl *Vg = gp(V);
  // uniform: every element below `total` lies inside the block (total is a
  // multiple of 256, so e < total is the uniform test ebase + 256u < total)
  const int eend = min(total, ebase + PF * NTHR);
  if (vrows == ROWS && gc0 + eend / ROWS <= kvalid) {
    const gdbl *Vb = Vg + (int64_t)c0 * ldv + r0;
#pragma unroll
    for (int u = 0; u < PF; ++u) {
      if (ebase + u * NTHR >= total) break;
      const int du = ROWS <= NTHR ? u * CPU : u >> 1;
      const int dr = ROWS <= NTHR ? 0 : (u & 1) * NTHR;
      v[u] = Vb[(int64_t)du * ldv + dr];
    }
    return;
  }
#pragma unroll
  for (int u = 0; u < PF; ++u) {
    // ROWS = 512: u even -> rows r0, u odd -> rows r0 + 256 of the same column
    const int du = ROWS <= NTHR ? u * CPU : u >> 1;
    const int dr = ROWS <= NTHR ? 0 : (u & 1) * NTHR;
    const int r = r0 + dr, gc = c0 + du;
    // always read an element of the block (clamped indices): no branch per element
    v[u] = Vg[min(r, vrows - 1) + (int64_t)min(gc, kvalid - 1) * ldv];
  }
}

// Registers of vstage_load (same block: vrows, gc0, kvalid, ebase, total)
// into the LDS chunks (chunk-relative column c at c * ldvc), rows up to vrows
// rounded to 16 (the zero padding of the last row tile): zero outside the
// reflector support; VK_UNIT: column gc has an implicit 1 at row gc and 0
// above.
template <int RW>
__device__ inline void vstage_store(const Lds &L, const double (&v)[PF], int vrows, int kind,
                                    int gc0, int kvalid, int ebase, int total) {
  constexpr int ROWS = Geo<RW>::ROWS, LDVC = Geo<RW>::LDVC;
  constexpr int CPU = ROWS <= NTHR ? NTHR / ROWS : 1;
  const int rlim = (vrows + 15) & ~15;
  const int e0 = ebase + tid_x();
  const int r0 = e0 % ROWS, c0 = e0 / ROWS;
  ldbl *lb = L.vc + c0 * LDVC + r0;
  auto value = [&](int u, int du, int dr) {
    const int r = r0 + dr, gc = gc0 + c0 + du;
    const bool ok = e0 + u * NTHR < total && r < vrows && gc < kvalid;
    const double y = (kind == VK_UNIT) ? (r < gc ? 0.0 : (r == gc ? 1.0 : v[u])) : v[u];
    return ok ? y : 0.0;
  };
  if (rlim == ROWS) {  // uniform: every row stored; e < total is uniform per u
#pragma unroll
    for (int u = 0; u < PF; ++u) {
      if (ebase + u * NTHR >= total) break;
      const int du = ROWS <= NTHR ? u * CPU : u >> 1;
      const int dr = ROWS <= NTHR ? 0 : (u & 1) * NTHR;
      lb[du * LDVC + dr] = value(u, du, dr);
    }
    return;
  }
#pragma unroll
  for (int u = 0; u < PF; ++u) {
    const int du = ROWS <= NTHR ? u * CPU : u >> 1;
    const int dr = ROWS <= NTHR ? 0 : (u & 1) * NTHR;
    if (e0 + u * NTHR < total && r0 + dr < rlim) lb[du * LDVC + dr] = value(u, du, dr);
  }
}

// Chunks [gc0, gc0 + 16*ng) of V straight into LDS.
template <int RW>
__device__ inline void stage_v(const Lds &L, const double *V, int64_t ldv, int vrows, int kind,
                               int gc0, int kvalid, int ng) {
  const int total = ng * 16 * Geo<RW>::ROWS;
  for (int base = 0; base < total; base += PF * NTHR) {
    double v[PF];
    vstage_load<RW>(v, V, ldv, vrows, gc0, kvalid, base, total);
    vstage_store<RW>(L, v, vrows, kind, gc0, kvalid, base, total);
  }
}

// T_s (ibw x ibw upper triangle of the block at Tb, leading dimension ldt)
// as ibp x ibp with zeros elsewhere (ibp <= TQ_TS_MAX); element
// e = u*256 + tid at (a = e / TQ_TS_MAX, c = e % TQ_TS_MAX). Loaded as is
// (clamped indices); tstage_store keeps the triangle.
constexpr int TPF = TQ_TS_MAX * TQ_TS_MAX / NTHR;
__device__ inline void tstage_load(double (&v)[TPF], const double *Tb, int64_t ldt, int ibw) {
  const gdbl *Tg = gp(Tb);
#pragma unroll
  for (int u = 0; u < TPF; ++u) {
    const int e = u * NTHR + tid_x();
    const int a = e / TQ_TS_MAX, c = e % TQ_TS_MAX;
    v[u] = Tg[min(a, ibw - 1) + (int64_t)min(c, ibw - 1) * ldt];
  }
}
__device__ inline void tstage_store(const Lds &L, const double (&v)[TPF], int ibp, int ibw) {
  const int ldts = ibp + 1;
#pragma unroll
  for (int u = 0; u < TPF; ++u) {
    const int e = u * NTHR + tid_x();
    const int a = e / TQ_TS_MAX, c = e % TQ_TS_MAX;
    if (a < ibp && c < ibp) L.ts[a * ldts + c] = (a <= c && c < ibw) ? v[u] : 0.0;
  }
}

// C1 rows [s, s + ibw) of the wave's 16 columns (column group cg), element
// e = u*64 + lane at (a = e / 16, c = e % 16); ibw <= 32. Loaded as is
// (clamped indices): rows a >= ibw and columns c >= ncols hold copies of
// valid elements, which the users mask.
constexpr int CPF = TQ_TS_MAX * 16 / 64;
__device__ inline void c1_load(double (&v)[CPF], const double *C1, int64_t ldc1, int s, int ibw,
                               int ncols, int cg) {
  const int ln = lane_id();
  const int c = cg * 16 + (ln & 15);
  const gdbl *Cb = gp(C1) + (int64_t)min(c, ncols - 1) * ldc1 + s;
#pragma unroll
  for (int u = 0; u < CPF; ++u) {
    const int a = 4 * u + (ln >> 4);
    v[u] = Cb[min(a, ibw - 1)];
  }
}

// C[rbase + 0 .. 128) x column `col` into registers: item (rt, r) of the
// lane holds row 16*rt + 4*r + g, where g = lane/16 in the accumulator layout
// of the MFMA (QUAD = false) and g = lane%4 in the panel layout (QUAD = true,
// whose four lanes of a column are adjacent).
template <bool QUAD = false>
__device__ inline void load_c2(d4 (&c2)[RT], const double *C, int64_t ldc, int crows, int col,
                               bool colok, int rbase) {
  // (crows >= 1, and col is clamped to a valid column when !colok)
  const int g = QUAD ? (lane_id() & 3) : (lane_id() >> 4);
  const gdbl *Cc = gp(C) + (int64_t)col * ldc;
#pragma unroll
  for (int rt = 0; rt < RT; ++rt) {
    const int lo = rbase + rt * 16;  // uniform
    if (lo + 16 <= crows) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const double val = Cc[lo + 4 * r + g];
        c2[rt][r] = colok ? val : 0.0;
      }
    } else if (lo < crows) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = lo + 4 * r + g;
        const double val = Cc[min(row, crows - 1)];
        c2[rt][r] = (colok && row < crows) ? val : 0.0;
      }
    } else {
      c2[rt] = d4{0.0, 0.0, 0.0, 0.0};
    }
  }
}

template <bool QUAD = false>
__device__ inline void store_c2(const d4 (&c2)[RT], double *C, int64_t ldc, int crows, int col,
                                bool colok, int rbase) {
  if (!colok) return;
  const int g = QUAD ? (lane_id() & 3) : (lane_id() >> 4);
  gdbl *Cc = gp(C) + (int64_t)col * ldc;
#pragma unroll
  for (int rt = 0; rt < RT; ++rt) {
    const int lo = rbase + rt * 16;  // uniform
    if (lo >= crows) break;
    if (lo + 16 <= crows) {
#pragma unroll
      for (int r = 0; r < 4; ++r) Cc[lo + 4 * r + g] = c2[rt][r];
    } else {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = lo + 4 * r + g;
        if (row < crows) Cc[row] = c2[rt][r];
      }
    }
  }
}

// First row tile of the wave block that can hold a nonzero of the staged
// chunk q of the block starting at reflector s (unit-lower V: rows above
// s + 16q are zero).
__device__ inline int first_rt(int kind, int s, int q, int rbase) {
  if (kind != VK_UNIT) return 0;
  const int d = s + q * 16 - rbase;
  return d > 0 ? (d >> 4) : 0;
}

// Y rows of the staged chunks [g0, g0+ng) (chunk g0 + g is block chunk q):
// Y[q] (+)= V[:, s+16q ..]^T C2 over the wave's rows, into the group region
// yw. The B operand is accumulator register r of C2 tile rt (k index
// lane/16 <-> row 16*rt + 4*r + lane/16); the A operand is V^T at those rows.
// Four independent accumulator chains (one per register r), summed at the end.
template <int RW>
__device__ inline void y_group(const Lds &L, int kind, int s, int q0, int ng, int vrows,
                               const d4 (&c2)[RT], ldbl *yw, int rbase, bool acc) {
  constexpr int LDVC = Geo<RW>::LDVC;
  const int ln = lane_id();
  for (int g = 0; g < ng; ++g) {
    const int q = q0 + g;
    d4 y[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) y[r] = d4{0.0, 0.0, 0.0, 0.0};
    const int rt0 = first_rt(kind, s, q, rbase);
    const ldbl *vp = L.vc + (g * 16 + (ln & 15)) * LDVC + rbase + (ln >> 4);
    // A operands one row tile ahead of their MFMAs (every read stays inside
    // the staged column), so the LDS latency hides behind the MFMAs
    double a[4], an[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) a[r] = vp[4 * r];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
      if (rt + 1 < RT) {
#pragma unroll
        for (int r = 0; r < 4; ++r) an[r] = vp[(rt + 1) * 16 + 4 * r];
      }
      __builtin_amdgcn_sched_barrier(0);  // keep the loads ahead of the MFMAs
      if (rt >= rt0 && rbase + rt * 16 < vrows) {
#pragma unroll
        for (int r = 0; r < 4; ++r) y[r] = mfma(a[r], c2[rt][r], y[r]);
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) a[r] = an[r];
    }
    const d4 ys = (y[0] + y[1]) + (y[2] + y[3]);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      ldbl *d = yw + (q * 16 + 4 * r + (ln >> 4)) * 16 + (ln & 15);
      if (acc)
        *d += ys[r];
      else
        *d = ys[r];
    }
  }
}

// C2 -= V_s W over the wave's rows for the staged chunks: A = V[row 16*rt +
// lane%16][col 4kk + lane/16 of chunk q], B = -W[16q + 4kk + lane/16][lane%16].
// The row tiles are the independent accumulator chains (kk outermost).
template <int RW>
__device__ inline void update_group(const Lds &L, int kind, int s, int q0, int ng, int vrows,
                                    const ldbl *yw, d4 (&c2)[RT], int rbase) {
  constexpr int LDVC = Geo<RW>::LDVC;
  const int ln = lane_id();
  for (int g = 0; g < ng; ++g) {
    const int q = q0 + g;
    const int rt0 = first_rt(kind, s, q, rbase);
    double b[4];
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) b[kk] = -yw[(q * 16 + 4 * kk + (ln >> 4)) * 16 + (ln & 15)];
    const ldbl *vp = L.vc + (g * 16 + (ln >> 4)) * LDVC + rbase + (ln & 15);
    // A operands two MFMAs ahead (a ring of two), for the same reason
    double a0 = vp[0], a1 = vp[16];
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
#pragma unroll
      for (int rt = 0; rt < RT; ++rt) {
        const int nx = kk * RT + rt + 2;  // the operand two steps ahead
        const double an = nx < 4 * RT ? (double)vp[4 * (nx / RT) * LDVC + (nx % RT) * 16] : 0.0;
        __builtin_amdgcn_sched_barrier(0);  // keep the load ahead of the MFMA
        if (rt >= rt0 && rbase + rt * 16 < vrows) c2[rt] = mfma(a0, b[kk], c2[rt]);
        a0 = a1;
        a1 = an;
      }
    }
  }
}

// W = T_s^T Ytot (or T_s Ytot when notrans) in place in the group region:
// W block q needs the Y blocks <= q (>= q), so the blocks go bottom (top)
// first. T_s from the LDS stage or from global memory.
template <bool TLDS>
__device__ inline void w_phase(const Lds &L, const double *Ts, int64_t ldt, int ibw, int ldts,
                               ldbl *yw, bool notrans = false) {
  const gdbl *Tg = gp(Ts);
  const int ln = lane_id();
  const int nq = (ibw + 15) >> 4;
  for (int qi = 0; qi < nq; ++qi) {
    const int q = notrans ? qi : nq - 1 - qi;
    d4 w = {0.0, 0.0, 0.0, 0.0};
    const int orow = q * 16 + (ln & 15);  // output row of W
    const int q2lo = notrans ? q : 0, q2hi = notrans ? nq - 1 : q;
    for (int q2 = q2lo; q2 <= q2hi; ++q2) {
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) {
        const int kr = q2 * 16 + 4 * kk + (ln >> 4);  // contraction index
        // transposed: T[kr][orow]; not transposed: T[orow][kr] (upper)
        const int tr = notrans ? orow : kr, tc = notrans ? kr : orow;
        double a;
        if (TLDS)
          a = L.ts[tr * ldts + tc];
        else
          a = (tr <= tc && tc < ibw) ? Tg[tr + (int64_t)tc * ldt] : 0.0;
        w = mfma(a, yw[kr * 16 + (ln & 15)], w);
      }
    }
    wave_sync();
#pragma unroll
    for (int r = 0; r < 4; ++r) yw[(q * 16 + 4 * r + (ln >> 4)) * 16 + (ln & 15)] = w[r];
    wave_sync();
  }
}

// yw[a][c] += C1[s + a][col c] (add) or C1 = C1 - yw (sub) for the wave's
// column group, straight from global memory.
__device__ inline void c1_pass(ldbl *yw, double *C1, int64_t ldc1, int s, int ibw, int ncols,
                               int cg, bool add) {
  const int ln = lane_id();
  gdbl *Cg = gp(C1);
  const int total = ibw * 16;
  for (int base = 0; base < total; base += 64 * 4) {
    double v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = base + u * 64 + ln;
      const int a = e >> 4, c = cg * 16 + (e & 15);
      v[u] = (e < total && c < ncols) ? Cg[(s + a) + (int64_t)c * ldc1] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = base + u * 64 + ln;
      const int a = e >> 4, c = cg * 16 + (e & 15);
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
// T: block s at T + s*ldt) to one strip of at most 16 * (4 / RW) columns:
//   C1 (optional): rows s .. s+ib of the block's top part, C2: vrows rows.
// Per block: stage V_s (and T_s) in LDS, Y = V_s^T C2 + C1_s (row waves add
// their slabs one after the other), W = T_s^T Y, C1_s -= W, C2 -= V_s W.
template <int RW>
__device__ __forceinline__ void apply_strip(const Lds &L, const double *V, int64_t ldv, int vrows,
                                            int kind, int kref, int ib, const double *T,
                                            int64_t ldt, double *C1, int64_t ldc1, double *C2,
                                            int64_t ldc2, int ncols, bool notrans) {
  constexpr int ROWS = Geo<RW>::ROWS;
  const int ln = lane_id(), wv = wave_id();
  const int cg = wv / RW, rb = wv % RW, rbase = rb * TQ_ROWS_PER_WAVE;
  const bool gact = cg * 16 < ncols;  // wave-uniform
  const int col = cg * 16 + (ln & 15);
  const bool colok = col < ncols;
  const int ibp = ib_pad16(ib), ldts = ibp + 1;
  const bool tl = t_in_lds(ib);
  const int nqb = ibp >> 4;
  // Register pipeline: the whole block fits the staged chunks and the
  // prefetch registers, and T_s the LDS stage.
  const bool pf = tl && nqb <= L.gmax && nqb * 16 * ROWS <= PF * NTHR && !notrans;
  ldbl *yw = L.y + cg * L.ibp * 16;
  const bool c1w = C1 != nullptr && rb == 0 && gact;
  // C2 as loaded (clamped rows of a valid column), then the first block's
  // prefetch, then the masks: the masks wait for the C2 loads only
  d4 c2[RT];
  {
    const int g = ln >> 4;
    const gdbl *Cc = gp(C2) + (int64_t)min(col, ncols - 1) * ldc2;
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
      const int lo = rbase + rt * 16;  // uniform
      if (lo < vrows) {
#pragma unroll
        for (int r = 0; r < 4; ++r) c2[rt][r] = Cc[min(lo + 4 * r + g, vrows - 1)];
      } else {
        c2[rt] = d4{0.0, 0.0, 0.0, 0.0};
      }
    }
  }
  double pv[PF], pt[TPF], pc[CPF];
  if (pf) {
    const int ibw0 = min(ib, kref);
    vstage_load<RW>(pv, V, ldv, vrows, 0, ibw0, 0, ((ibw0 + 15) >> 4) * 16 * ROWS);
    tstage_load(pt, T, ldt, ibw0);
    if (c1w) c1_load(pc, C1, ldc1, 0, ibw0, ncols, cg);
  }
  {
    const int g = ln >> 4;
    const bool cok = colok && gact;
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = rbase + rt * 16 + 4 * r + g;
        c2[rt][r] = (cok && row < vrows) ? c2[rt][r] : 0.0;
      }
  }
  const int nblk = (kref + ib - 1) / ib;
  for (int bi = 0; bi < nblk; ++bi) {
    // Q^T: blocks in order; Q: the last block first
    const int s = (notrans ? nblk - 1 - bi : bi) * ib;
    const int ibw = min(ib, kref - s);
    const int nq = (ibw + 15) >> 4;
    const bool resident = nq <= L.gmax;
    const int sn = s + ib;
    // --- Y = V_s^T C2 ---
    for (int g0 = 0; g0 < nq; g0 += L.gmax) {
      const int ng = min(L.gmax, nq - g0);
      __syncthreads();
      if (pf) {
        vstage_store<RW>(L, pv, vrows, kind, s, s + ibw, 0, nq * 16 * ROWS);
        tstage_store(L, pt, ibp, ibw);
        if (sn < kref) {
          const int ibwn = min(ib, kref - sn);
          vstage_load<RW>(pv, V, ldv, vrows, sn, sn + ibwn, 0, ((ibwn + 15) >> 4) * 16 * ROWS);
          tstage_load(pt, T + (int64_t)sn * ldt, ldt, ibwn);
        }
      } else {
        stage_v<RW>(L, V, ldv, vrows, kind, s + g0 * 16, s + ibw, ng);
        if (g0 == 0 && tl) {
          double t[TPF];
          tstage_load(t, T + (int64_t)s * ldt, ldt, ibw);
          tstage_store(L, t, ibp, ibw);
        }
      }
      __syncthreads();
      for (int rr = 0; rr < RW; ++rr) {
        if (rr > 0) __syncthreads();
        if (rb == rr && gact) y_group<RW>(L, kind, s, g0, ng, vrows, c2, yw, rbase, rr > 0);
      }
    }
    if (RW > 1) __syncthreads();
    // --- Y += C1_s; W = T_s^T Y; C1_s -= W (first row wave of each group) ---
    if (c1w) {
      if (pf) {
        // element e = 64u + lane is row 4u + lane/16: rows < ibw in all lanes
        // for 4u + 4 <= ibw (uniform), per lane only in a ragged last group
#pragma unroll
        for (int u = 0; u < CPF; ++u) {
          const int e = u * 64 + ln;
          const double cv = colok ? pc[u] : 0.0;  // columns past ncols hold copies
          if (4 * u + 4 <= ibw)
            yw[e] += cv;
          else if (4 * u < ibw && e < ibw * 16)
            yw[e] += cv;
        }
      } else {
        c1_pass(yw, C1, ldc1, s, ibw, ncols, cg, true);
      }
    }
    if (rb == 0 && gact) {
      wave_sync();
      if (tl)
        w_phase<true>(L, nullptr, 0, ibw, ldts, yw, notrans);
      else
        w_phase<false>(L, T + (int64_t)s * ldt, ldt, ibw, ldts, yw, notrans);
    }
    if (c1w) {
      if (pf) {
        gdbl *Cb = gp(C1) + (int64_t)col * ldc1 + s + (ln >> 4);
        double w[CPF];
#pragma unroll
        for (int u = 0; u < CPF; ++u) w[u] = pc[u] - yw[u * 64 + ln];
        if (colok) {
#pragma unroll
          for (int u = 0; u < CPF; ++u) {
            if (4 * u + 4 <= ibw)
              Cb[4 * u] = w[u];
            else if (4 * u + (ln >> 4) < ibw)
              Cb[4 * u] = w[u];
          }
        }
        if (sn < kref) c1_load(pc, C1, ldc1, sn, min(ib, kref - sn), ncols, cg);
      } else {
        c1_pass(yw, C1, ldc1, s, ibw, ncols, cg, false);
      }
    }
    if (RW > 1)
      __syncthreads();
    else
      wave_sync();
    // --- C2 -= V_s W ---
    for (int g0 = 0; g0 < nq; g0 += L.gmax) {
      const int ng = min(L.gmax, nq - g0);
      if (!resident) {
        __syncthreads();
        stage_v<RW>(L, V, ldv, vrows, kind, s + g0 * 16, s + ibw, ng);
        __syncthreads();
      }
      if (gact) update_group<RW>(L, kind, s, g0, ng, vrows, yw, c2, rbase);
    }
  }
  __syncthreads();
  store_c2(c2, C2, ldc2, vrows, col, colok && gact, rbase);
}

// Straight-line form of apply_strip for the common case: one row wave per
// column group (tiles of at most 128 rows), a full 128-row V, a full 64-column
// strip and whole IB blocks of 16 or 32 columns. No per-element predicates and
// one block structure, so the compiler's wait counts stay exact across the
// loop: the next block's V, T (issued when the current block is staged) and
// C1 rows (issued after the current C1 write-back) are in flight while the
// current block computes.
template <int IB>
__device__ __forceinline__ void apply_strip_fast(const Lds &L, const double *V, int64_t ldv,
                                                 int kind, int kref, const double *T, int64_t ldt,
                                                 double *C1, int64_t ldc1, double *C2,
                                                 int64_t ldc2) {
  constexpr int RW = 1, ROWS = Geo<RW>::ROWS, LDVC = Geo<RW>::LDVC;
  constexpr int NQ = IB / 16;            // chunks per block
  constexpr int VPL = NQ * 16 * ROWS / NTHR;  // V doubles per lane per block (8 or 16)
  constexpr int LDTS = IB + 1;
  static_assert(VPL <= PF, "V block exceeds the prefetch registers");
  const int ln = lane_id(), wv = wave_id();
  const int col = wv * 16 + (ln & 15);
  ldbl *yw = L.y + wv * L.ibp * 16;
  const bool c1 = C1 != nullptr;  // uniform
  // per-lane staging positions: V element e = u*256 + tid -> column e / 128,
  // row e % 128; T element e -> (e / IB, e % IB)
  const int tid = tid_x();
  const int vr = tid & (ROWS - 1), vc = tid >> 7;
  d4 c2[RT];
  {
    const gdbl *Cc = gp(C2) + (int64_t)col * ldc2 + (ln >> 4);
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
      for (int r = 0; r < 4; ++r) c2[rt][r] = Cc[rt * 16 + 4 * r];
  }
  double pv[VPL], pt[IB * IB / NTHR > 0 ? IB * IB / NTHR : 1], pc[IB / 4];
  constexpr int TPL = IB * IB / NTHR > 0 ? IB * IB / NTHR : 1;
  // The prefetch registers hold the values as loaded: the unit-lower and
  // triangle selections are applied when the block is staged, so that no
  // instruction right after the loads waits for them (a select there would
  // make the prefetch synchronous).
  auto load_v = [&](int s) {
    const gdbl *Vb = gp(V) + (int64_t)(s + vc) * ldv + vr;
#pragma unroll
    for (int u = 0; u < VPL; ++u) pv[u] = Vb[(int64_t)(2 * u) * ldv];
  };
  auto load_t = [&](int s) {
    const gdbl *Tb = gp(T) + (int64_t)s * ldt;
#pragma unroll
    for (int u = 0; u < TPL; ++u) {
      const int e = u * NTHR + tid;
      const int a = e / IB, c = e % IB;
      pt[u] = Tb[min(a, IB - 1) + (int64_t)c * ldt];
    }
  };
  auto load_c1 = [&](int s) {
    const gdbl *Cb = gp(C1) + (int64_t)col * ldc1 + s + (ln >> 4);
#pragma unroll
    for (int u = 0; u < IB / 4; ++u) pc[u] = Cb[4 * u];
  };
  load_v(0);
  load_t(0);
  if (c1) load_c1(0);
  for (int s = 0; s < kref; s += IB) {
    __syncthreads();
    {
      ldbl *lb = L.vc + vc * LDVC + vr;
#pragma unroll
      for (int u = 0; u < VPL; ++u) {
        const int gc = s + vc + 2 * u;
        const double v = pv[u];
        lb[2 * u * LDVC] = (kind == VK_UNIT) ? (vr < gc ? 0.0 : (vr == gc ? 1.0 : v)) : v;
      }
#pragma unroll
      for (int u = 0; u < TPL; ++u) {
        const int e = u * NTHR + tid;
        const int a = e / IB, c = e % IB;
        if (e < IB * IB) L.ts[a * LDTS + c] = a <= c ? pt[u] : 0.0;
      }
    }
    const int sn = s + IB;
    if (sn < kref) {
      load_v(sn);
      load_t(sn);
    }
    __syncthreads();
    y_group<RW>(L, kind, s, 0, NQ, ROWS, c2, yw, 0, false);
    if (c1) {
#pragma unroll
      for (int u = 0; u < IB / 4; ++u) yw[u * 64 + ln] += pc[u];
    }
    wave_sync();
    // W = T_s^T Y: every operand read before the block's result overwrites Y
    d4 w[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) w[q] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int q = 0; q < NQ; ++q)
#pragma unroll
      for (int q2 = 0; q2 <= q; ++q2)
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) {
          const int arow = q2 * 16 + 4 * kk + (ln >> 4);
          w[q] = mfma(L.ts[arow * LDTS + q * 16 + (ln & 15)], yw[arow * 16 + (ln & 15)], w[q]);
        }
    wave_sync();
#pragma unroll
    for (int q = 0; q < NQ; ++q)
#pragma unroll
      for (int r = 0; r < 4; ++r) yw[(q * 16 + 4 * r + (ln >> 4)) * 16 + (ln & 15)] = w[q][r];
    wave_sync();
    if (c1) {
      gdbl *Cb = gp(C1) + (int64_t)col * ldc1 + s + (ln >> 4);
#pragma unroll
      for (int u = 0; u < IB / 4; ++u) Cb[4 * u] = pc[u] - yw[u * 64 + ln];
      if (sn < kref) load_c1(sn);
    }
    update_group<RW>(L, kind, s, 0, NQ, ROWS, yw, c2, 0);
  }
  __syncthreads();
  {
    gdbl *Cc = gp(C2) + (int64_t)col * ldc2 + (ln >> 4);
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
      for (int r = 0; r < 4; ++r) Cc[rt * 16 + 4 * r] = c2[rt][r];
  }
}

// All columns of C2 (and C1), in strips of 16 * (4 / RW).
template <int RW>
__device__ __forceinline__ void apply_cols(const Lds &L, const double *V, int64_t ldv, int vrows,
                                           int kind, int kref, int ib, const double *T,
                                           int64_t ldt, double *C1, int64_t ldc1, double *C2,
                                           int64_t ldc2, int ncols, bool notrans = false) {
  constexpr int w = Geo<RW>::P;
  for (int c0 = 0; c0 < ncols; c0 += w) {
    double *c1 = C1 ? C1 + (int64_t)c0 * ldc1 : nullptr;
    double *c2 = C2 + (int64_t)c0 * ldc2;
    const int nc = min(w, ncols - c0);
    // uniform choice of the straight-line form
    const bool fast = RW == 1 && vrows == TQ_ROWS_PER_WAVE && nc == w && kref % ib == 0 &&
                      L.gmax * 16 >= ib && !notrans;
    if (fast && ib == 32)
      apply_strip_fast<32>(L, V, ldv, kind, kref, T, ldt, c1, ldc1, c2, ldc2);
    else if (fast && ib == 16)
      apply_strip_fast<16>(L, V, ldv, kind, kref, T, ldt, c1, ldc1, c2, ldc2);
    else
      apply_strip<RW>(L, V, ldv, vrows, kind, kref, ib, T, ldt, c1, ldc1, c2, ldc2, nc, notrans);
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

// C (m x n) = sum_k A(i, k) B(k, j) on the FP64 MFMA, 16 x 16 output tiles
// spread over the waves; the operands come from functors that return 0
// outside their ranges (four k-steps of loads are issued before their
// MFMAs), the result goes to a functor per element.
template <class FA, class FB, class FS>
__device__ inline void small_gemm(int m, int n, int kd, FA fa, FB fb, FS fs) {
  const int ln = lane_id(), wv = wave_id();
  const int tm = (m + 15) >> 4, tn = (n + 15) >> 4;
  for (int t = wv; t < tm * tn; t += 4) {
    const int i0 = (t % tm) * 16, j0 = (t / tm) * 16;
    d4 acc = {0.0, 0.0, 0.0, 0.0};
    for (int k0 = 0; k0 < kd; k0 += 16) {
      double av[4], bv[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int kk = k0 + 4 * u + (ln >> 4);
        av[u] = fa(i0 + (ln & 15), kk);
        bv[u] = fb(kk, j0 + (ln & 15));
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) acc = mfma(av[u], bv[u], acc);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) fs(i0 + 4 * r + (ln >> 4), j0 + (ln & 15), acc[r]);
  }
}

// G = V[:, 0:a]^T V[:, a:a+pw] (pw <= one strip) into Tb[i + (a + j) * ldt]:
// the Y phase of the block application with C2 = the reflectors [a, a+pw).
template <int RW>
__device__ __forceinline__ void gram_cross(const Lds &L, const double *V, int64_t ldv, int vrows, int kind, int a,
                           int pw, double *Tb, int64_t ldt) {
  const int ln = lane_id(), wv = wave_id();
  const int cg = wv / RW, rb = wv % RW, rbase = rb * TQ_ROWS_PER_WAVE;
  const int col = cg * 16 + (ln & 15);
  const bool gact = cg * 16 < pw;
  const gdbl *Vc = gp(V) + (int64_t)(a + min(col, pw - 1)) * ldv;
  const int gc = a + col;
  d4 c2[RT];
#pragma unroll
  for (int rt = 0; rt < RT; ++rt)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = rbase + rt * 16 + 4 * r + (ln >> 4);
      const double val = Vc[min(row, vrows - 1)];
      const double y = kind == VK_UNIT ? (row < gc ? 0.0 : (row == gc ? 1.0 : val)) : val;
      c2[rt][r] = (col < pw && row < vrows) ? y : 0.0;
    }
  ldbl *yw = L.y + cg * L.ibp * 16;
  const int nq = (a + 15) >> 4;
  for (int g0 = 0; g0 < nq; g0 += L.gmax) {
    const int ng = min(L.gmax, nq - g0);
    __syncthreads();
    stage_v<RW>(L, V, ldv, vrows, kind, g0 * 16, a, ng);
    __syncthreads();
    for (int rr = 0; rr < RW; ++rr) {
      if (rr > 0) __syncthreads();
      if (rb == rr && gact) y_group<RW>(L, kind, 0, g0, ng, vrows, c2, yw, rbase, rr > 0);
    }
  }
  __syncthreads();
  if (rb == 0 && gact) {
    gdbl *Tg = gp(Tb);
    for (int e = ln; e < a * 16; e += 64) {
      const int i = e >> 4, c = cg * 16 + (e & 15);
      if (c < pw) Tg[i + (int64_t)(a + c) * ldt] = yw[e];
    }
  }
  __threadfence_block();
  __syncthreads();
}

// Off-diagonal parts of the T factor of an IB block wider than a register
// panel: the diagonal blocks of width P (one per register panel) are there;
// for each later panel [a, a + pw) of the block,
//   T[0:a, a:a+pw] = -T[0:a, 0:a] (V[:, 0:a]^T V[:, a:a+pw]) T[a:a+pw, a:a+pw].
// V: the block's reflectors (unit lower from row 0 of the block frame for
// GEQRT, full for TSQRT), Tb: the block's T (leading dimension ldt).
template <int RW>
__device__ __forceinline__ void assemble_wide_T(const Lds &L, const double *V, int64_t ldv, int vrows, int kind,
                                int ibw, double *Tb, int64_t ldt) {
  constexpr int P = Geo<RW>::P;
  gdbl *Tg = gp(Tb);
  for (int a = P; a < ibw; a += P) {
    const int pw = min(P, ibw - a);
    gram_cross<RW>(L, V, ldv, vrows, kind, a, pw, Tb, ldt);
    // Z = G T[a:a+pw, a:a+pw] into LDS (a x pw, [i * pw + j])
    ldbl *Z = L.z;
    small_gemm(
        a, pw, pw,
        [=](int i, int k) { return (i < a && k < pw) ? (double)Tg[i + (int64_t)(a + k) * ldt] : 0.0; },
        [=](int k, int j) {
          return (k < pw && j < pw && k <= j) ? (double)Tg[(a + k) + (int64_t)(a + j) * ldt] : 0.0;
        },
        [=](int i, int j, double v) {
          if (i < a && j < pw) Z[i * pw + j] = v;
        });
    __syncthreads();
    // T[0:a, a:a+pw] = -T[0:a, 0:a] Z
    small_gemm(
        a, pw, a,
        [=](int i, int k) {
          return (i < a && k < a && i <= k) ? (double)Tg[i + (int64_t)k * ldt] : 0.0;
        },
        [=](int k, int j) { return (k < a && j < pw) ? (double)Z[k * pw + j] : 0.0; },
        [=](int i, int j, double v) {
          if (i < a && j < pw) Tg[i + (int64_t)(a + j) * ldt] = -v;
        });
    __threadfence_block();
    __syncthreads();
  }
}

// Column cc of the T block that starts at local column tb: lanes a in
// [tb, cc) of the calling wave compute T[a][cc] = -tau_cc * sum_{p=a}^{cc-1}
// T[a][p] G[p][cc]; lane cc sets T[cc][cc] = tau_cc. T is the upper part of
// L.tg, G^T its strictly lower part.
template <int RW>
__device__ inline void t_column(const Lds &L, int cc, int tb) {
  constexpr int ld = Geo<RW>::P + 1;
  const int a = lane_id();
  const double tau = L.taus[cc];
  if (a >= tb && a < cc) {
    const ldbl *tr = L.tg + a * ld, *gr = L.tg + cc * ld;
    double t[4] = {0.0, 0.0, 0.0, 0.0};
    int p = a;
    for (; p + 3 < cc; p += 4) {
#pragma unroll
      for (int u = 0; u < 4; ++u) t[u] += tr[p + u] * gr[p + u];
    }
    for (; p < cc; ++p) t[0] += tr[p] * gr[p];
    L.tg[a * ld + cc] = -tau * ((t[0] + t[1]) + (t[2] + t[3]));
  }
  if (a == cc) L.tg[cc * ld + cc] = tau;
  wave_sync();
}

// The T blocks of a register panel of pw columns, from the Gram entries and
// tau in LDS (T blocks of ib columns when IB <= P, else the panel's own
// diagonal block). First the recurrence runs on sub-blocks of at most 16
// columns, one wave per sub-block; then each T block is assembled from its
// sub-blocks by one wave, 16 columns at a time, on the MFMA:
//   T[0:a, a:a+w] = -T[0:a, 0:a] (G[0:a, a:a+w] T[a:a+w, a:a+w]),
// with the product in the lower bracket kept in registers in the
// accumulator layout, which is the B-operand layout of the next product.
template <int RW>
__device__ inline void panel_T(const Lds &L, int pw, int ib) {
  constexpr int P = Geo<RW>::P, ld = P + 1;
  constexpr int NZ = P / 16;  // row tiles of a T block (at most)
  const int wv = wave_id(), ln = lane_id();
  const int bw = ib <= P ? ib : pw;  // T block width
  const int nblk = (pw + bw - 1) / bw;
  // sub-block recurrences
  const int nsub_b = (bw + 15) / 16;  // sub-blocks per T block
  for (int sb = wv; sb < nblk * nsub_b; sb += 4) {
    const int b = sb / nsub_b, q = sb % nsub_b;
    const int tb = b * bw + q * 16;
    const int te = min(min(tb + 16, b * bw + bw), pw);
    for (int cc = tb; cc < te; ++cc) t_column<RW>(L, cc, tb);
  }
  if (nsub_b == 1) return;
  __syncthreads();
  // assembly of each T block from its sub-blocks (one wave per block)
  for (int b = wv; b < nblk; b += 4) {
    const int t0 = b * bw, tw = min(bw, pw - t0);
    for (int a = 16; a < tw; a += 16) {
      const int w = min(16, tw - a);
      const int na = a / 16;  // row tiles above
      d4 z[NZ];
      // Z = G[0:a, a:a+w] T[a:a+w, a:a+w]: A = G[i][a+k] = tg[(t0+a+k)][t0+i],
      // B = T[a+k][a+j] (upper, k <= j, j < w)
#pragma unroll
      for (int it = 0; it < NZ; ++it) {
        z[it] = d4{0.0, 0.0, 0.0, 0.0};
        if (it < na) {
#pragma unroll
          for (int kk = 0; kk < 4; ++kk) {
            const int k = 4 * kk + (ln >> 4), i = it * 16 + (ln & 15), j = ln & 15;
            const int kc = min(k, w - 1), jc = min(j, w - 1);  // in-range addresses
            const double ga = k < w ? (double)L.tg[(t0 + a + kc) * ld + t0 + i] : 0.0;
            const double tb_ = (k <= j && j < w) ? (double)L.tg[(t0 + a + kc) * ld + t0 + a + jc] : 0.0;
            z[it] = mfma(ga, tb_, z[it]);
          }
        }
      }
      // X = T[0:a, 0:a] Z: output row tile it, k over row tiles it2 >= it of Z
#pragma unroll
      for (int it = 0; it < NZ; ++it) {
        if (it < na) {
          d4 xacc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
          for (int it2 = 0; it2 < NZ; ++it2) {
            if (it2 >= it && it2 < na) {
#pragma unroll
              for (int kk = 0; kk < 4; ++kk) {
                const int i = it * 16 + (ln & 15), k = it2 * 16 + 4 * kk + (ln >> 4);
                const double ta = i <= k ? (double)L.tg[(t0 + i) * ld + t0 + k] : 0.0;
                xacc = mfma(ta, z[it2][kk], xacc);
              }
            }
          }
          // T[it*16 + row][a + j] = -X (rows < a, columns a.. a+w: not read above)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int i = it * 16 + 4 * r + (ln >> 4), j = ln & 15;
            if (j < w) L.tg[(t0 + i) * ld + t0 + a + j] = -xacc[r];
          }
        }
      }
      wave_sync();
    }
  }
}

// ts = false (GEQRT): QR in place of the mrows x ncol block X (= R).
// ts = true (TSQRT, and the merges): QR of [R; X] with R the upper triangle
// of an ncol x ncol block of A (updated in place) and X an mrows x ncol block
// (leading dimension ldx) overwritten by the lower parts of the reflectors
// [e_j; u_j]. The block factors T go to Tp (ib x ncol).
// Columns are taken in register panels of at most P = 16 * (4 / RW) columns
// that never straddle an IB block unless IB > P.
template <int RW>
__device__ __forceinline__ void panel_task(const MatDesc &m, const Lds &L, bool ts, double *R,
                                           double *X, int64_t ldx, double *Tp, int mrows,
                                           int ncol) {
  constexpr int ROWS = Geo<RW>::ROWS, P = Geo<RW>::P, ld = P + 1;
  const int ib = m.ib;
  const int64_t lda = m.lda;
  const int K = ts ? ncol : min(mrows, ncol);
  const int ln = lane_id(), wv = wave_id();
  const int cg = wv / RW, rb = wv % RW, rbase = rb * TQ_ROWS_PER_WAVE;
  // panel layout: the four lanes of a column are adjacent (lane/4 = column
  // within the wave's 16, lane%4 = row group), so column sums are DPP moves
  const int mc = cg * 16 + (ln >> 2);  // my column within the register panel
  const int g4 = ln & 3;
  gdbl *Rg = gp(R);
  gdbl *Tg = gp(Tp);

  int pw = 0;
  for (int c0 = 0; c0 < K; c0 += pw) {
    const int sg = (c0 / ib) * ib;
    pw = ib <= P ? min(K - c0, (P / ib) * ib) : min(P, min(sg + ib, K) - c0);
    const bool colok = mc < pw;
    d4 x[RT];
    load_c2<true>(x, X + (int64_t)c0 * ldx, ldx, mrows, min(mc, pw - 1), colok, rbase);
    if (ts) {
      for (int e = tid_x(); e < P * P; e += NTHR) {
        const int a = e / P, c = e % P;
        L.top[a * ld + c] = (a <= c && c < pw) ? Rg[(c0 + a) + (int64_t)(c0 + c) * lda] : 0.0;
      }
    }
    __syncthreads();
    for (int c = 0; c < pw; ++c) {
      // lane-derived values recomputed per column (kept out of the loop's
      // live registers; see tid_x)
      const int g4 = lane_id() & 3;
      const int mc = cg * 16 + (lane_id() >> 2);
      const int j = c0 + c;
      const int h = ts ? -1 : j;  // rows > h form the reflector tail
      const int par = c & 1;
      const bool owner = cg == (c >> 4);
      const bool mine = (lane_id() >> 2) == (c & 15);
      // --- norm of the tail and alpha (owner column group) ---
      double ss = 0.0, al = 0.0, alpha = 0.0;
      if (owner) {
        // tiles wholly below the head row, wholly above it, or holding it
        // (uniform tests; only the last needs per-row compares)
        double s4[4] = {0.0, 0.0, 0.0, 0.0};  // independent chains
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) {
          const int lo = rbase + rt * 16;
          if (lo > h) {
#pragma unroll
            for (int r = 0; r < 4; ++r) s4[r] += x[rt][r] * x[rt][r];
          } else if (lo + 15 >= h) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int row = lo + 4 * r + g4;
              const double v = x[rt][r];
              s4[r] += row > h ? v * v : 0.0;
              al += row == h ? v : 0.0;
            }
          }
        }
        ss = quad_sum((s4[0] + s4[1]) + (s4[2] + s4[3]));
        al = quad_sum(al);
        if (ts) alpha = L.top[c * ld + c];
        if (RW > 1 && mine && g4 == 0) {
          L.red[2 * rb] = ss;
          L.red[2 * rb + 1] = al;
        }
      }
      if (RW > 1) {
        __syncthreads();
        if (owner) {
          ss = 0.0;
          al = 0.0;
          for (int q = 0; q < RW; ++q) {
            ss += L.red[2 * q];
            al += L.red[2 * q + 1];
          }
        }
      }
      // --- reflector: v in registers and in the broadcast buffer ---
      if (owner) {
        double beta, tau, scale;
        householder(ts ? alpha : al, ss, beta, tau, scale);
        wave_sync();  // every lane has read alpha before R_jj is overwritten
        if (mine) {
          ldbl *vb = L.vb + par * ROWS + 4 * g4;  // [tile][g4][r]
#pragma unroll
          for (int rt = 0; rt < RT; ++rt) {
            const int lo = rbase + rt * 16;
            if (lo > h) {
#pragma unroll
              for (int r = 0; r < 4; ++r) {
                x[rt][r] *= scale;
                vb[lo + r] = x[rt][r];
              }
            } else if (lo + 15 < h) {
#pragma unroll
              for (int r = 0; r < 4; ++r) vb[lo + r] = 0.0;
            } else {
#pragma unroll
              for (int r = 0; r < 4; ++r) {
                const int row = lo + 4 * r + g4;
                const double xv = x[rt][r];
                const double v = row > h ? xv * scale : (row == h ? 1.0 : 0.0);
                x[rt][r] = row > h ? v : (row == h ? beta : xv);
                vb[lo + r] = v;
              }
            }
          }
          if (g4 == 0 && rb == 0) {
            L.taus[c] = tau;
            if (ts) L.top[c * ld + c] = beta;
          }
        }
      }
      __syncthreads();
      // --- dot products of every column with v ---
      const double tau = L.taus[c];
      const ldbl *vb = L.vb + par * ROWS + rbase + 4 * g4;  // [tile][g4][r]
      double dd[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int r = 0; r < 4; ++r) dd[r] += x[rt][r] * vb[rt * 16 + r];
      double d = quad_sum((dd[0] + dd[1]) + (dd[2] + dd[3]));
      const bool active = mc > c && mc < pw;
      const double rtop = (ts && active) ? L.top[c * ld + mc] : 0.0;
      wave_sync();  // R_j row read by every lane of the column before it is written
      if (RW > 1) {
        if (g4 == 0) L.dred[rb * 64 + mc] = d;
        __syncthreads();
        d = 0.0;
        for (int q = 0; q < RW; ++q) d += L.dred[q * 64 + mc];
      }
      if (active) {
        d += rtop;
        const double f = tau * d;
#pragma unroll
        for (int rt = 0; rt < RT; ++rt)
#pragma unroll
          for (int r = 0; r < 4; ++r) x[rt][r] -= f * vb[rt * 16 + r];
        if (ts && g4 == 0 && rb == 0) L.top[c * ld + mc] = rtop - f;
      }
      // Gram entry G[mc][c] of two reflectors of the same T block
      const int tbc = ib <= P ? (j / ib) * ib - c0 : 0;
      if (mc < c && mc >= tbc && g4 == 0 && rb == 0) L.tg[c * ld + mc] = d;
    }
    __syncthreads();
    panel_T<RW>(L, pw, ib);
    // --- write back the panel: R above, reflectors below ---
    store_c2<true>(x, X + (int64_t)c0 * ldx, ldx, mrows, mc, colok, rbase);
    __syncthreads();
    if (ts) {
      for (int e = tid_x(); e < pw * pw; e += NTHR) {
        const int a = e / pw, c = e % pw;
        if (a <= c) Rg[(c0 + a) + (int64_t)(c0 + c) * lda] = L.top[a * ld + c];
      }
    }
    // T of the panel's columns: whole blocks (IB <= P) or the diagonal block
    // of this panel and the zeros below it (IB > P).
    {
      const int rlo = ib <= P ? 0 : c0 - sg;
      const int bw = min(ib, K - sg);  // rows of the (last) block
      const int span = ib <= P ? ib : bw - rlo;
      for (int e = tid_x(); e < span * pw; e += NTHR) {
        const int rr = e % span, c = e / span;
        const int cc = c0 + c;
        const int sb = ib <= P ? (cc / ib) * ib : sg;  // block start of column cc
        const int ra = rlo + rr;                       // row within T_s
        const int rc = cc - sb;                        // column within T_s
        if (ra < min(ib, K - sb)) {
          const int la = ra - rlo + (ib <= P ? sb - c0 : 0);  // local row in tg
          Tg[ra + (int64_t)cc * ib] = ra <= rc ? (double)L.tg[la * ld + c] : 0.0;
        }
      }
    }
    __syncthreads();
    // --- the rest of the tile: trailing columns [c0 + pw, ncol) ---
    const int rest = ncol - c0 - pw;
    if (rest > 0) {
      const double *Vp = ts ? X + (int64_t)c0 * ldx : X + c0 + (int64_t)c0 * ldx;
      const int vrows = ts ? mrows : mrows - c0;
      double *C1 = ts ? R + c0 + (int64_t)(c0 + pw) * lda : nullptr;
      double *C2 = ts ? X + (int64_t)(c0 + pw) * ldx : X + c0 + (int64_t)(c0 + pw) * ldx;
      const double *Ta = ib <= P ? Tp + (int64_t)c0 * ib : Tp + (c0 - sg) + (int64_t)c0 * ib;
      apply_cols<RW>(L, Vp, ldx, vrows, ts ? VK_FULL : VK_UNIT, pw, ib <= P ? ib : pw, Ta, ib, C1, lda,
                 C2, ldx, rest);
    }
  }
  if (ib > P) {
    for (int sg = 0; sg < K; sg += ib) {
      const int bw = min(ib, K - sg);
      if (bw <= P) continue;
      const double *Vb = ts ? X + (int64_t)sg * ldx : X + sg + (int64_t)sg * ldx;
      assemble_wide_T<RW>(L, Vb, ldx, ts ? mrows : mrows - sg, ts ? VK_FULL : VK_UNIT, bw,
                      Tp + (int64_t)sg * ib, ib);
    }
  }
}

// ---------------------------------------------------------------------------
// Task dispatch and the persistent scheduler
// ---------------------------------------------------------------------------

template <int RW>
__device__ __forceinline__ void run_task(const Task &t, const MatDesc &m, const Lds &L) {
  const int nb = m.nb, ib = m.ib;
  const int i = t.i, j = t.j, k = t.k, strip = task_strip(t);
  const int type = task_type(t);
  const int64_t lda = m.lda;
  auto At = [&](int r, int c) { return m.A + (int64_t)c * nb * lda + (int64_t)r * nb; };
  auto Tt = [&](int r, int c) { return m.T + ((int64_t)c * m.MT + r) * (int64_t)ib * nb; };
  if (type == TK_GEQRT || type == TK_TSQRT || type == TK_TTQRT) {
    // Panels are the critical path: their waves win instruction issue over
    // co-resident update waves.
    __builtin_amdgcn_s_setprio(2);
    const int mrows = tile_rows(m, i), ncol = tile_cols(m, k);
    if (type == TK_GEQRT) {
      panel_task<RW>(m, L, false, At(i, k), At(i, k), lda, Tt(i, k), mrows, ncol);
    } else if (type == TK_TSQRT) {
      panel_task<RW>(m, L, true, At(tree_head(m, i, k), k), At(i, k), lda, Tt(i, k), mrows, ncol);
    } else {
      // merge: the bottom head's triangle (zeros below it) into its own
      // block, then the TSQRT of [R_top; block]
      double *Vt = m.T + tree_V_offset(m, i / m.h, k);
      const gdbl *Ab = gp(At(i, k));
      gdbl *Vg = gp(Vt);
      for (int c = 0; c < ncol; ++c)
        for (int r = tid_x(); r < mrows; r += NTHR)
          Vg[r + (int64_t)c * nb] = r <= c ? Ab[r + (int64_t)c * lda] : 0.0;
      __syncthreads();
      panel_task<RW>(m, L, true, At(tree_partner(m, i, k), k), Vt, nb,
                     m.T + tree_T_offset(m, i / m.h, k), mrows, ncol);
    }
    __builtin_amdgcn_s_setprio(0);
    return;
  }
  const int c0 = strip * m.w;
  const bool onB = task_on_B(type);
  const bool larfb = type == TK_LARFB || type == TK_LARFB_B;
  const bool merge = type == TK_TTMQR || type == TK_TTMQR_B;
  const double *aV, *aT;
  int64_t ldv = lda;
  int vrows = tile_rows(m, i), kind = VK_FULL, kref = tile_cols(m, k), top = i;
  if (larfb) {  // the head's GEQRT reflectors (unit lower part of A_ik)
    aV = At(i, k);
    kind = VK_UNIT;
    kref = min(vrows, kref);
    aT = Tt(i, k);
  } else if (merge) {  // a merge's reflector block
    aV = m.T + tree_V_offset(m, i / m.h, k);
    ldv = nb;
    aT = m.T + tree_T_offset(m, i / m.h, k);
    top = tree_partner(m, i, k);
  } else {
    aV = At(i, k);
    aT = Tt(i, k);
    top = tree_head(m, i, k);
  }
  double *aC1 = nullptr, *aC2;
  int64_t ldc = lda;
  int ncols;
  if (onB) {
    ncols = min(m.w, m.nrhs - c0);
    ldc = m.ldb;
    aC2 = m.B + (int64_t)i * nb + (int64_t)c0 * m.ldb;
    if (!larfb) aC1 = m.B + (int64_t)top * nb + (int64_t)c0 * m.ldb;
  } else {
    ncols = min(m.w, tile_cols(m, j) - c0);
    aC2 = At(i, j) + (int64_t)c0 * lda;
    if (!larfb) aC1 = At(top, j) + (int64_t)c0 * lda;
  }
  apply_cols<RW>(L, aV, ldv, vrows, kind, kref, ib, aT, ib, aC1, ldc, aC2, ldc, ncols,
                 onB && m.notrans);
}

// The task's matrix descriptor, field by field from the batch array or the
// kernel argument (a whole-struct select between the two would give the
// descriptor an address and a private-memory copy).
__device__ __forceinline__ MatDesc load_desc(const MatDesc *__restrict__ mats, int idx,
                                             const MatDesc &single) {
  if (!mats) return single;
  const MatDesc *g = mats + idx;
  MatDesc m;
  m.A = g->A;
  m.T = g->T;
  m.B = g->B;
  m.lda = g->lda;
  m.ldb = g->ldb;
  m.ctr = g->ctr;
  m.M = g->M;
  m.N = g->N;
  m.nb = g->nb;
  m.ib = g->ib;
  m.MT = g->MT;
  m.NT = g->NT;
  m.KT = g->KT;
  m.S = g->S;
  m.w = g->w;
  m.nrhs = g->nrhs;
  m.SB = g->SB;
  m.gmax = g->gmax;
  m.h = g->h;
  m.D = g->D;
  m.notrans = g->notrans;
  return m;
}

// Counter poll: a relaxed agent-scope load reads the coherent value without
// the cache invalidation an acquire load implies. On this multi-XCD chip an
// agent-scope acquire invalidates the whole L2 of the XCD and a release
// writes all of its dirty lines back, so the protocol does each once per
// task (after the last wait, and after the task's stores), never per poll.
__device__ inline int ld_relaxed(const int *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// s_waitcnt vmcnt(0): this wave's global loads and stores have completed.
__device__ __forceinline__ void wait_vm() { __builtin_amdgcn_s_waitcnt(0x0F70); }

// Thread 0 polls the task's counters; gives up (and flags `err`) after
// `timeout` wall-clock ticks or when another workgroup flagged an error.
// Returns after an agent-scope acquire (one L2 invalidation) and a barrier.
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
      while (ld_relaxed(ctr + idx) < target) {
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
    if (ok) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    s_ok = ok;
  }
  __syncthreads();
  const int ok = __builtin_amdgcn_readfirstlane(s_ok);
  __syncthreads();
  return ok != 0;
}

// Task t of the factorization DAG of one matrix in the sequential program
// order of the tile algorithm (step k: GEQRT, the TSQRT chain, the LARFBs,
// then the SSRFBs with i ascending), which is a topological order. (k, pk)
// carry the step of the previous decode and the number of tasks before it;
// tickets of one workgroup only grow, so the scan over k is amortized O(1).
__device__ inline Task decode_program_order(const MatDesc &m, int64_t t, int &k, int64_t &pk) {
  const int S = m.S, slast = strips_of(m, m.NT - 1);
  for (;;) {
    const int64_t r = m.MT - 1 - k, c = m.NT - 1 - k;
    const int64_t cs = c >= 1 ? (c - 1) * S + slast : 0;
    const int64_t cnt = 1 + r + cs + r * cs;
    if (t < pk + cnt) {
      const int64_t o = t - pk;
      if (o == 0) return make_task(TK_GEQRT, 0, k, k, k, 0);
      if (o <= r) return make_task(TK_TSQRT, 0, (int)(k + o), k, k, 0);
      if (o <= r + cs) {
        const int64_t idx = o - 1 - r;
        return make_task(TK_LARFB, 0, k, (int)(k + 1 + idx / S), k, (int)(idx % S));
      }
      const int64_t idx = o - 1 - r - cs, rem = idx % cs;
      return make_task(TK_SSRFB, 0, (int)(k + 1 + idx / cs), (int)(k + 1 + rem / S), k,
                       (int)(rem % S));
    }
    pk += cnt;
    ++k;
  }
}

__global__ __launch_bounds__(NTHR) __attribute__((amdgpu_waves_per_eu(2, 2))) void tq_persistent(
    const Task *__restrict__ tasks, int64_t ntasks, MatDesc single,
    const MatDesc *__restrict__ mats, int *ctr, unsigned int *ticket, int *err, int use_waits,
    long long timeout, long long *trace) {
  extern __shared__ double lds_dyn[];
  __shared__ int s_t;
  __shared__ Task s_task;
  int dk = 0;       // program-order decode state (thread 0, tasks == nullptr)
  int64_t dpk = 0;
  for (;;) {
    if (threadIdx.x == 0) {
      const int e = __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      const int tt = e ? -1 : (int)atomicAdd(ticket, 1u);
      s_t = tt;
      if (!tasks && tt >= 0 && tt < ntasks) s_task = decode_program_order(single, tt, dk, dpk);
    }
    __syncthreads();
    // Uniform across the workgroup: read into a scalar register so that the
    // task's parameters (and every loop bound derived from them) are scalar.
    const int64_t t = __builtin_amdgcn_readfirstlane(s_t);
    Task tk;
    if (tasks && t >= 0 && t < ntasks) {
      tk = tasks[t];
    } else {
      tk.w0 = __builtin_amdgcn_readfirstlane(s_task.w0);
      tk.i = __builtin_amdgcn_readfirstlane(s_task.i);
      tk.j = __builtin_amdgcn_readfirstlane(s_task.j);
      tk.k = __builtin_amdgcn_readfirstlane(s_task.k);
    }
    __syncthreads();
    if (t < 0 || t >= ntasks) break;
    const MatDesc m = load_desc(mats, task_mat(tk), single);
    const long long t_take = trace ? wall_clock64() : 0;
    if (use_waits && !wait_deps(tk, m, ctr, err, timeout)) break;
    const long long t_run = trace ? wall_clock64() : 0;
    switch (m.w) {
      case 64: run_task<1>(tk, m, make_lds<1>(lds_dyn, m)); break;
      case 32: run_task<2>(tk, m, make_lds<2>(lds_dyn, m)); break;
      default: run_task<4>(tk, m, make_lds<4>(lds_dyn, m)); break;
    }
    // Every wave's stores have reached the L2; then one agent-scope release
    // (the L2 write-back) for the whole workgroup before the counters move.
    wait_vm();
    __syncthreads();
    if (trace && threadIdx.x == 0) {
      trace[4 * t + 0] = t_take;
      trace[4 * t + 1] = t_run;
      trace[4 * t + 2] = wall_clock64();
      trace[4 * t + 3] = blockIdx.x;
    }
    if (threadIdx.x == 0 && use_waits) {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      const int ns = task_nsignals(tk);
      for (int q = 0; q < ns; ++q)
        __hip_atomic_fetch_add(ctr + task_signal(tk, m, q), 1, __ATOMIC_RELAXED,
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
__global__ __launch_bounds__(NTHR) __attribute__((amdgpu_waves_per_eu(2, 2))) void tq_ssrfb_bench(
    double *buf, MatDesc m, int calls) {
  extern __shared__ double lds_dyn[];
  const int nb = m.nb, ib = m.ib;
  const int64_t per = 3 * (int64_t)nb * nb + (int64_t)ib * nb;
  double *V = buf + per * blockIdx.x;
  double *C1 = V + (int64_t)nb * nb, *C2 = C1 + (int64_t)nb * nb, *T = C2 + (int64_t)nb * nb;
  for (int call = 0; call < calls; ++call) {
    switch (m.w) {
      case 64:
        apply_cols<1>(make_lds<1>(lds_dyn, m), V, nb, nb, VK_FULL, nb, ib, T, ib, C1, nb, C2, nb, nb);
        break;
      case 32:
        apply_cols<2>(make_lds<2>(lds_dyn, m), V, nb, nb, VK_FULL, nb, ib, T, ib, C1, nb, C2, nb, nb);
        break;
      default:
        apply_cols<4>(make_lds<4>(lds_dyn, m), V, nb, nb, VK_FULL, nb, ib, T, ib, C1, nb, C2, nb, nb);
        break;
    }
  }
}

// Deterministic fill with values in [-scale, scale] (splitmix64 hash).
// Q <- [I_k; 0] (M x k).
__global__ void tq_eye(double *Q, int64_t M, int64_t k, int64_t ldq) {
  const int64_t total = M * k;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = e % M, c = e / M;
    Q[r + c * ldq] = r == c ? 1.0 : 0.0;
  }
}

// Back substitution R x = b for one right-hand side per workgroup (column
// blockIdx.x of B), a column of R at a time: x_j = b_j / R_jj, then
// b[0:j] -= x_j R[0:j, j] by all threads.
__global__ __launch_bounds__(NTHR) void tq_trsv_upper(const double *R, int64_t ldr, int64_t N,
                                                      double *B, int64_t ldb) {
  gdbl *b = gp(B) + (int64_t)blockIdx.x * ldb;
  const gdbl *Rg = gp(R);
  const int tid = threadIdx.x;
  __shared__ double s_x;
  for (int64_t j = N - 1; j >= 0; --j) {
    if (tid == 0) {
      const double x = b[j] / Rg[j + j * ldr];
      b[j] = x;
      s_x = x;
    }
    __syncthreads();
    const double x = s_x;
    const gdbl *rc = Rg + j * ldr;
    for (int64_t i = tid; i < j; i += NTHR) b[i] -= x * rc[i];
    __syncthreads();
  }
}

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

hipError_t set_lds(const void *kern, size_t lds) {
  if (lds > 64 * 1024)
    return hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  return hipSuccess;
}

}  // namespace

hipError_t tq_launch_persistent(const TqLaunch &a, hipStream_t st) {
  if (a.nctr_zero > 0) {
    int64_t n = a.nctr_zero;
    int g = (int)((n + 255) / 256);
    g = g > 1024 ? 1024 : (g < 1 ? 1 : g);
    hipLaunchKernelGGL(tq_zero_ints, dim3(g), dim3(256), 0, st, a.ctr_base, n);
  }
  hipError_t e = set_lds((const void *)tq_persistent, a.lds_bytes);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(tq_persistent, dim3(a.grid), dim3(NTHR), a.lds_bytes, st, a.tasks, a.ntasks,
                     a.single, a.mats, a.ctr, a.ticket, a.err, a.use_waits, a.timeout, a.trace);
  return hipGetLastError();
}

int tq_occupancy(size_t lds) {
  if (set_lds((const void *)tq_persistent, lds) != hipSuccess) return 1;
  int nblk = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nblk, tq_persistent, NTHR, lds) != hipSuccess)
    return 1;
  return nblk > 0 ? nblk : 1;
}

hipError_t tq_launch_ssrfb_bench(double *buf, int nb, int ib, int calls, int grid, hipStream_t st) {
  const LdsPlan lp = lds_plan(nb, ib);
  if (lp.gmax < 1) return hipErrorInvalidValue;
  MatDesc m;
  __builtin_memset(&m, 0, sizeof(m));
  m.nb = nb;
  m.ib = ib;
  m.w = strip_width(nb);
  m.gmax = lp.gmax;
  m.h = 1;
  m.D = 1;
  const size_t lds = (size_t)lp.doubles * 8;
  hipError_t e = set_lds((const void *)tq_ssrfb_bench, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(tq_ssrfb_bench, dim3(grid), dim3(NTHR), lds, st, buf, m, calls);
  return hipGetLastError();
}

hipError_t tq_launch_eye(double *Q, int64_t M, int64_t k, int64_t ldq, hipStream_t st) {
  if (M <= 0 || k <= 0) return hipSuccess;
  int64_t g = (M * k + 255) / 256;
  g = g > 4096 ? 4096 : g;
  hipLaunchKernelGGL(tq_eye, dim3((unsigned)g), dim3(256), 0, st, Q, M, k, ldq);
  return hipGetLastError();
}

hipError_t tq_launch_trsv_upper(const double *R, int64_t ldr, int64_t N, double *B, int64_t ldb,
                                int64_t nrhs, hipStream_t st) {
  if (N <= 0 || nrhs <= 0) return hipSuccess;
  hipLaunchKernelGGL(tq_trsv_upper, dim3((unsigned)nrhs), dim3(NTHR), 0, st, R, ldr, N, B, ldb);
  return hipGetLastError();
}

hipError_t tq_launch_fill(double *p, int64_t n, uint64_t seed, double scale, hipStream_t st) {
  int g = (int)((n + 255) / 256);
  g = g > 4096 ? 4096 : (g < 1 ? 1 : g);
  hipLaunchKernelGGL(tq_fill_hash, dim3(g), dim3(256), 0, st, p, n, seed, scale);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Allocation-free factorization: a static device array holds everything the
// persistent launch needs besides A and T (error word, ticket, dependency
// counters); the tasks are decoded from the ticket in program order, so no
// task list is stored either.
// ---------------------------------------------------------------------------

static __device__ __align__(256) int scratch[TQ_NOALLOC_SCRATCH_INTS];

namespace {
int *g_scratch_ptr[64];  // device address of `scratch`, per device (null: not looked up)
}

int tq_noalloc_scratch(int dev, int **ptr) {
  if (dev < 0 || dev >= 64) return -1;
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return -2;
    g_scratch_ptr[dev] = (int *)p;
  }
  *ptr = g_scratch_ptr[dev];
  return 0;
}

int *tq_noalloc_scratch_if_set(int dev) {
  return (dev >= 0 && dev < 64) ? g_scratch_ptr[dev] : nullptr;
}

hipError_t tq_launch_noalloc(int *sp, const MatDesc &md, int64_t ntasks, int64_t nctr, int grid,
                             size_t lds, long long timeout, hipStream_t st) {
  // ticket and counters start at zero; the error word is left to qr_sync
  const int64_t nz = TQ_NOALLOC_CTR_OFFSET - 1 + nctr;
  int g = (int)((nz + 255) / 256);
  g = g > 1024 ? 1024 : (g < 1 ? 1 : g);
  hipLaunchKernelGGL(tq_zero_ints, dim3(g), dim3(256), 0, st, sp + 1, nz);
  hipError_t e = set_lds((const void *)tq_persistent, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(tq_persistent, dim3(grid), dim3(NTHR), lds, st, (const Task *)nullptr, ntasks,
                     md, (const MatDesc *)nullptr, sp + TQ_NOALLOC_CTR_OFFSET,
                     (unsigned int *)(sp + 1), sp, 1, timeout, (long long *)nullptr);
  return hipGetLastError();
}
