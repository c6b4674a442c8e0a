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

// Doubles of dynamic LDS: V chunk (16 columns), one ibp x 16 W/Y region per
// active wave, reduction scratch, the micro-panel T and the TSQRT top block.
TQ_HD inline int64_t lds_doubles(int mbt, int ib, int nw) {
  return (int64_t)16 * lds_ldvc(mbt) + (int64_t)nw * ib_pad16(ib) * 16 + 4 + 128 + 32 + 8 +
         2 * 32 * 33;
}

// Active waves (16 columns each) per workgroup for a (NB, IB) pair: as many
// as the LDS budget allows (4, 2 or 1).
TQ_HD inline int nwaves_for(int nb, int ib) {
  int mbt = mbt_for_nb(nb);
  for (int nw = 4; nw >= 1; nw >>= 1)
    if (lds_doubles(mbt, ib, nw) * 8 <= TQ_LDS_LIMIT) return nw;
  return 0;
}
