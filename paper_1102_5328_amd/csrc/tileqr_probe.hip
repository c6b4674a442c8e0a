// Measurement support: the sustained rate of the FP64 matrix instruction the
// update kernels are built on (v_mfma_f64_16x16x4f64), with nothing else in
// the way. It gives the ceiling against which their rates are read next to
// the chip's published FP64 peak.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device_api.h"

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int PROBE_CHAINS = 8;  // independent accumulator chains per wave

// Every wave runs `iters` rounds of PROBE_CHAINS independent MFMA chains with
// register operands: no memory traffic, no barriers, no dependence stalls
// (each chain's next product is issued PROBE_CHAINS products later). The
// chains are summed and stored so that none of them is dead. Workgroup 0's
// first lane records its shader-clock and wall-clock spans, so the host can
// tell the clock the launch ran at.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4, 4))) void tq_mfma_probe(
    double *out, int iters) {
  const int ln = threadIdx.x & 63;
  const long long c0 = clock64(), w0 = wall_clock64();
  d4 acc[PROBE_CHAINS];
#pragma unroll
  for (int c = 0; c < PROBE_CHAINS; ++c) acc[c] = d4{0.0, 0.0, 0.0, 0.0};
  const double a = 1.0 + 0x1p-30 * ln, b = 1.0 - 0x1p-30 * ln;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int c = 0; c < PROBE_CHAINS; ++c)
      acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[c], 0, 0, 0);
  }
  const long long c1 = clock64(), w1 = wall_clock64();
  double s = 0.0;
#pragma unroll
  for (int c = 0; c < PROBE_CHAINS; ++c) s += (acc[c][0] + acc[c][1]) + (acc[c][2] + acc[c][3]);
  out[2 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    out[0] = (double)(c1 - c0);
    out[1] = (double)(w1 - w0);
  }
}

}  // namespace

int tq_mfma_probe_chains() { return PROBE_CHAINS; }

hipError_t tq_launch_mfma_probe(double *out, int grid, int iters, hipStream_t st) {
  hipLaunchKernelGGL(tq_mfma_probe, dim3(grid), dim3(256), 0, st, out, iters);
  return hipGetLastError();
}
