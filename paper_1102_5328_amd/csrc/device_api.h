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
