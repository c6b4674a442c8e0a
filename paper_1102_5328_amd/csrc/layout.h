// LDS layout of the tile kernels, shared by the device code and the host
// (which sizes the dynamic LDS of each launch).
#pragma once
#include <stdint.h>

#include "tq_sched.h"

#define TQ_NTHR 256            // threads per workgroup: 4 wave64
#define TQ_LDS_LIMIT (158 * 1024)  // bytes of dynamic LDS we allow (gfx950: 160 KiB per CU)

// Largest tile order the library accepts at present. The register classes
// for NB in (128, 512] exist, but an earlier build of the NB <= 256 class
// made a memory fault on the device whose cause is not established; until it
// is, those classes are switched off (TILEQR_ERR_DISABLED).
#define TQ_MAX_ENABLED_NB 128

// Row tiles of 16 held in registers for a tile order of at most 16*mbt.
TQ_HD inline int mbt_for_nb(int nb) {
  return nb <= 64 ? 4 : nb <= 128 ? 8 : nb <= 256 ? 16 : 32;
}
TQ_HD inline int ib_pad16(int ib) { return (ib + 15) & ~15; }
TQ_HD inline int lds_ldvc(int mbt) { return mbt * 16 + 1; }  // odd: conflict-free transposed reads
TQ_HD inline int lds_ldts(int ibp) { return ibp + 1; }
// T_s of a block is staged in LDS when the block is at most 64 wide.
TQ_HD inline bool t_in_lds(int ib) { return ib_pad16(ib) <= 64; }
// Panel scratch: reductions, scalars, the micro-panel T and the TSQRT top
// block (aliases the T_s stage: they are never live at the same time).
TQ_HD inline int64_t lds_panel_doubles() { return 4 + 128 + 32 + 8 + 2 * 32 * 33; }

// Doubles of dynamic LDS: gmax staged 16-column chunks of V, one ibp x 16
// W/Y region per active wave, and the T_s stage / panel scratch.
TQ_HD inline int64_t lds_doubles(int mbt, int ib, int nw, int gmax) {
  const int ibp = ib_pad16(ib);
  const int64_t ts = t_in_lds(ib) ? (int64_t)ibp * lds_ldts(ibp) : 0;
  const int64_t pan = lds_panel_doubles();
  return (int64_t)gmax * 16 * lds_ldvc(mbt) + (int64_t)nw * ibp * 16 + (ts > pan ? ts : pan);
}

// Active waves (16 columns each) and resident V chunks for a tile class and
// inner block: the whole V block resident if possible, within a budget that
// keeps two workgroups per compute unit for the smaller classes.
struct LdsPlan {
  int nw, gmax;
  int64_t doubles;
};
TQ_HD inline LdsPlan lds_plan(int mbt, int ib) {
  const int64_t budget = (int64_t)(mbt <= 8 ? 78 : 158) * 1024 / 8;
  const int nq = ib_pad16(ib) / 16;
  for (int nw = 4; nw >= 1; nw >>= 1)
    for (int g = nq; g >= 1; --g) {
      const int64_t d = lds_doubles(mbt, ib, nw, g);
      if (d <= budget) return LdsPlan{nw, g, d};
    }
  for (int g = nq; g >= 1; --g) {
    const int64_t d = lds_doubles(mbt, ib, 1, g);
    if (d * 8 <= TQ_LDS_LIMIT) return LdsPlan{1, g, d};
  }
  return LdsPlan{0, 0, 0};
}
TQ_HD inline int nwaves_for(int nb, int ib) { return lds_plan(mbt_for_nb(nb), ib).nw; }
