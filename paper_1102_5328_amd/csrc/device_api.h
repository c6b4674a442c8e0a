// Host-side launchers of the device kernels (C++ linkage, internal to the
// library).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "tq_sched.h"

#define TQ_DEVERR_WATCHDOG 2

struct TqLaunch {
  const Task *tasks;
  int64_t ntasks;
  MatDesc single;       // used when mats == nullptr
  const MatDesc *mats;  // device array of descriptors (batched) or nullptr
  int *ctr;             // dependency counters (already offset by matrix ctr fields)
  int *ctr_base;        // region zeroed before the launch
  int64_t nctr_zero;    // ints to zero at ctr_base (counters + ticket), 0 = none
  unsigned int *ticket;
  int *err;
  int use_waits;
  long long timeout;    // wall-clock ticks
  size_t lds_bytes;
  int grid;
  long long *trace;     // optional: 4 wall-clock stamps per task, or nullptr
};

hipError_t tq_launch_persistent(const TqLaunch &a, hipStream_t st);
int tq_occupancy(size_t lds_bytes);
hipError_t tq_launch_ssrfb_bench(double *buf, int nb, int ib, int calls, int grid, hipStream_t st);
hipError_t tq_launch_fill(double *p, int64_t n, uint64_t seed, double scale, hipStream_t st);
// Q (M x k, leading dimension ldq) <- the first k columns of the identity.
hipError_t tq_launch_eye(double *Q, int64_t M, int64_t k, int64_t ldq, hipStream_t st);
// B[0:N, 0:nrhs] <- R^-1 B[0:N, 0:nrhs] with R the upper triangle of the
// N x N block at R (leading dimension ldr): back substitution, one workgroup
// per right-hand side.
hipError_t tq_launch_trsv_upper(const double *R, int64_t ldr, int64_t N, double *B, int64_t ldb,
                                int64_t nrhs, hipStream_t st);

// Allocation-free factorization (qr_factor_noalloc): a static device array
// of TQ_NOALLOC_SCRATCH_INTS ints per device; int 0 is the error word, int 1
// the ticket, the dependency counters start at TQ_NOALLOC_CTR_OFFSET.
#define TQ_NOALLOC_SCRATCH_INTS (4 << 20)
#define TQ_NOALLOC_CTR_OFFSET 64
// Device address of the array on device `dev` (looked up once with
// hipGetSymbolAddress while `dev` is current); 0 or a negative code.
int tq_noalloc_scratch(int dev, int **ptr);
// The address if it was looked up on `dev` already, else nullptr.
int *tq_noalloc_scratch_if_set(int dev);
// Zeroes the ticket and counters, then runs the persistent kernel over the
// program-order DAG of one matrix (tasks decoded from the ticket).
hipError_t tq_launch_noalloc(int *scratch_ptr, const MatDesc &md, int64_t ntasks, int64_t nctr,
                             int grid, size_t lds, long long timeout, hipStream_t st);
// FP64 MFMA rate probe: `grid` workgroups of four waves, each wave `iters`
// rounds of tq_mfma_probe_chains() independent v_mfma_f64_16x16x4f64 chains.
// out holds 2 + 256 * grid doubles: [0] shader-clock ticks and [1] wall-clock
// ticks of workgroup 0, then one checksum per lane.
int tq_mfma_probe_chains();
hipError_t tq_launch_mfma_probe(double *out, int grid, int iters, hipStream_t st);
