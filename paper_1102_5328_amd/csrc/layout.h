// Work distribution and LDS layout of the tile kernels, shared by the device
// code and the host (which sizes the dynamic LDS and the strips of a launch).
//
// Every task runs on one workgroup of four wave64s. A wave always holds a
// block of 128 rows x 16 columns in registers, in the accumulator layout of
// v_mfma_f64_16x16x4f64 (32 doubles per lane), whatever the tile order:
//   NB <= 128: RW = 1 row wave per column group, 4 groups -> 64-column strips,
//   NB <= 256: RW = 2, 2 groups -> 32-column strips,
//   NB <= 512: RW = 4, 1 group  -> 16-column strips.
// Larger tiles are thus walked in 128-row slabs by more waves instead of
// needing more registers per lane, so every tile order runs the same code
// within 256 VGPRs and without accumulation registers or scratch.
#pragma once
#include <stdint.h>

#include "tq_sched.h"

#define TQ_NTHR 256                // threads per workgroup: 4 wave64
#define TQ_LDS_LIMIT (158 * 1024)  // bytes of dynamic LDS we allow (gfx950: 160 KiB per CU)
#define TQ_LDS_TWO (78 * 1024)     // per-workgroup budget for two workgroups per CU
#define TQ_ROWS_PER_WAVE 128
#define TQ_TS_MAX 32               // T_s of an application is staged in LDS up to this width

// Largest tile order the library accepts (TILEQR_ERR_DISABLED above it).
#ifndef TQ_MAX_ENABLED_NB
#define TQ_MAX_ENABLED_NB 512
#endif

TQ_HD inline int rw_for_nb(int nb) { return nb <= 128 ? 1 : nb <= 256 ? 2 : 4; }
// Strip width of the update tasks (columns of one workgroup).
TQ_HD inline int strip_width(int nb) { return 64 / rw_for_nb(nb); }
// Width of a register panel in the panel tasks (columns held at once).
TQ_HD inline int panel_width(int nb) { return 64 / rw_for_nb(nb); }
TQ_HD inline int ib_pad16(int ib) { return (ib + 15) & ~15; }
// V staging: rows 0 .. 128*RW, odd leading dimension for conflict-free
// transposed reads.
TQ_HD inline int lds_ldvc(int rw) { return TQ_ROWS_PER_WAVE * rw + 1; }
TQ_HD inline bool t_in_lds(int ib) { return ib_pad16(ib) <= TQ_TS_MAX; }

// Panel phase: reflector broadcast (2 x rows), tau (64), norm and dot
// partials (128 + 256), the T/Gram block and the TSQRT top block (P x (P+1)
// each); the assembly of a T block wider than a register panel reuses the
// region for an (IB - P) x P product.
TQ_HD inline int64_t lds_panel_doubles(int nb, int ib) {
  const int rw = rw_for_nb(nb), p = panel_width(nb);
  int64_t d = 2 * TQ_ROWS_PER_WAVE * rw + 64 + 128 + 256 + 2 * (int64_t)p * (p + 1);
  const int ibc = ib < nb ? ib : nb;
  if (ibc > p) {
    const int64_t z = (int64_t)(ibc - p) * p;
    if (z > d) d = z;
  }
  return d;
}
// Update phase: g staged 16-column chunks of V, one ibp x 16 Y/W region per
// column group, the T_s stage.
TQ_HD inline int64_t lds_update_doubles(int nb, int ib, int g) {
  const int rw = rw_for_nb(nb), cgn = 4 / rw, ibp = ib_pad16(ib);
  return (int64_t)g * 16 * lds_ldvc(rw) + (int64_t)cgn * ibp * 16 + TQ_TS_MAX * (TQ_TS_MAX + 1);
}

// Resident V chunks and dynamic LDS of one (NB, IB): the whole V block
// resident if possible, within a budget that keeps two workgroups per
// compute unit, else within the whole LDS.
struct LdsPlan {
  int gmax;
  int64_t doubles;
};
TQ_HD inline LdsPlan lds_plan(int nb, int ib) {
  const int nq = ib_pad16(ib) / 16;
  const int64_t pan = lds_panel_doubles(nb, ib);
  const int64_t budgets[2] = {TQ_LDS_TWO / 8, TQ_LDS_LIMIT / 8};
  for (int b = 0; b < 2; ++b)
    for (int g = nq; g >= 1; --g) {
      int64_t d = lds_update_doubles(nb, ib, g);
      if (pan > d) d = pan;
      if (d <= budgets[b]) return LdsPlan{g, d};
    }
  return LdsPlan{0, 0};
}
