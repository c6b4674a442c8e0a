// Learned (NB, IB) cost model: a 5 -> 64 -> 64 -> 64 -> 1 ReLU MLP in FP32,
// with hand-written forward, backward and Adam kernels. It is trained on the
// timings the empirical tuner measures and predicts log GFLOP/s of a tile QR
// for (log M, log N, log NB, IB/NB, log batch), so that the pruned search
// can be skipped for unseen shapes when the ensemble agrees.
//
// Parameter layout (8769 floats), weight matrices row-major [out][in]:
//   W1[64][5] @0, b1 @320, W2[64][64] @384, b2 @4480, W3[64][64] @4544,
//   b3 @8640, W4[1][64] @8704, b4 @8768.
// Loss over n rows: L = 1/(2n) sum (yhat - y)^2.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cmath>
#include <vector>

#include "../../include/tileqr.h"
#include "mlp_api.h"

namespace {

constexpr int NP = TQ_MLP_NPARAM;
constexpr int H = TQ_MLP_H;
constexpr int IN = TQ_MLP_IN;
constexpr int OW1 = 0, OB1 = 320, OW2 = 384, OB2 = 4480, OW3 = 4544, OB3 = 8640, OW4 = 8704,
              OB4 = 8768;
constexpr int CH = 64;  // rows per chunk in the backward pass
constexpr int NT = 256;

__device__ inline float relu(float z) { return z > 0.f ? z : 0.f; }

// One thread per row; weights staged in LDS (broadcast reads).
__global__ __launch_bounds__(NT) void mlp_forward_kernel(const float *__restrict__ params,
                                                         const float *__restrict__ X, int64_t n,
                                                         float *__restrict__ y) {
  __shared__ float w[NP];
  const float *p = params + (int64_t)blockIdx.y * NP;
  for (int e = threadIdx.x; e < NP; e += NT) w[e] = p[e];
  __syncthreads();
  const int64_t r = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (r >= n) return;
  float x[IN];
#pragma unroll
  for (int i = 0; i < IN; ++i) x[i] = X[r * IN + i];
  float h1[H], h2[H];
#pragma unroll
  for (int o = 0; o < H; ++o) {
    float s = w[OB1 + o];
#pragma unroll
    for (int i = 0; i < IN; ++i) s += w[OW1 + o * IN + i] * x[i];
    h1[o] = relu(s);
  }
#pragma unroll
  for (int o = 0; o < H; ++o) {
    float s = w[OB2 + o];
#pragma unroll
    for (int i = 0; i < H; ++i) s += w[OW2 + o * H + i] * h1[i];
    h2[o] = relu(s);
  }
  float out = w[OB4];
  for (int o = 0; o < H; ++o) {
    float s = w[OB3 + o];
#pragma unroll
    for (int i = 0; i < H; ++i) s += w[OW3 + o * H + i] * h2[i];
    out += w[OW4 + o] * relu(s);
  }
  y[(int64_t)blockIdx.y * n + r] = out;
}

struct Scratch {
  float *w, *g;           // NP each
  float *z1, *z2, *z3;    // CH x H pre-activations
  float *d;               // CH x H deltas
  float *xs;              // CH x IN
  float *ys, *dy;         // CH
  float *red;             // NT
};

__device__ inline Scratch carve(float *base) {
  Scratch s;
  float *p = base;
  s.w = p; p += NP;
  s.g = p; p += NP;
  s.z1 = p; p += CH * H;
  s.z2 = p; p += CH * H;
  s.z3 = p; p += CH * H;
  s.d = p; p += CH * H;
  s.xs = p; p += CH * IN;
  s.ys = p; p += CH;
  s.dy = p; p += CH;
  s.red = p;
  return s;
}
constexpr int SCRATCH_FLOATS = 2 * NP + 4 * CH * H + CH * IN + 2 * CH + NT;

// Adds the gradient of sum_b 0.5 (yhat_b - y_b)^2 * inv_n over the rows
// rows[0..bc) into S.g; returns this chunk's sum of 0.5 e^2 (thread 0).
__device__ float chunk_grad(const Scratch &S, const float *X, const float *Y, const int64_t *rows,
                            int bc, float inv_n) {
  const int t = threadIdx.x;
  for (int e = t; e < bc * IN; e += NT) S.xs[e] = X[rows[e / IN] * IN + e % IN];
  for (int b = t; b < bc; b += NT) S.ys[b] = Y[rows[b]];
  __syncthreads();
  for (int e = t; e < bc * H; e += NT) {
    const int b = e / H, o = e % H;
    float s = S.w[OB1 + o];
#pragma unroll
    for (int i = 0; i < IN; ++i) s += S.w[OW1 + o * IN + i] * S.xs[b * IN + i];
    S.z1[e] = s;
  }
  __syncthreads();
  for (int e = t; e < bc * H; e += NT) {
    const int b = e / H, o = e % H;
    float s = S.w[OB2 + o];
    for (int i = 0; i < H; ++i) s += S.w[OW2 + o * H + i] * relu(S.z1[b * H + i]);
    S.z2[e] = s;
  }
  __syncthreads();
  for (int e = t; e < bc * H; e += NT) {
    const int b = e / H, o = e % H;
    float s = S.w[OB3 + o];
    for (int i = 0; i < H; ++i) s += S.w[OW3 + o * H + i] * relu(S.z2[b * H + i]);
    S.z3[e] = s;
  }
  __syncthreads();
  float lpart = 0.f;
  for (int b = t; b < bc; b += NT) {
    float s = S.w[OB4];
    for (int i = 0; i < H; ++i) s += S.w[OW4 + i] * relu(S.z3[b * H + i]);
    const float e = s - S.ys[b];
    lpart += 0.5f * e * e;
    S.dy[b] = e * inv_n;
  }
  S.red[t] = lpart;
  __syncthreads();
  // Output layer.
  if (t < H) {
    float s = 0.f;
    for (int b = 0; b < bc; ++b) s += S.dy[b] * relu(S.z3[b * H + t]);
    S.g[OW4 + t] += s;
  }
  if (t == H) {
    float s = 0.f;
    for (int b = 0; b < bc; ++b) s += S.dy[b];
    S.g[OB4] += s;
  }
  for (int e = t; e < bc * H; e += NT) {
    const int b = e / H, o = e % H;
    S.d[e] = S.z3[e] > 0.f ? S.dy[b] * S.w[OW4 + o] : 0.f;
  }
  __syncthreads();
  // Layer 3: gW3[o][i] += sum_b d3[b][o] h2[b][i]; then d2 -> z3 buffer.
  for (int e = t; e < H * H; e += NT) {
    const int o = e / H, i = e % H;
    float s = 0.f;
    for (int b = 0; b < bc; ++b) s += S.d[b * H + o] * relu(S.z2[b * H + i]);
    S.g[OW3 + e] += s;
  }
  if (t < H) {
    float s = 0.f;
    for (int b = 0; b < bc; ++b) s += S.d[b * H + t];
    S.g[OB3 + t] += s;
  }
  for (int e = t; e < bc * H; e += NT) {
    const int b = e / H, i = e % H;
    float s = 0.f;
    for (int o = 0; o < H; ++o) s += S.w[OW3 + o * H + i] * S.d[b * H + o];
    S.z3[e] = S.z2[e] > 0.f ? s : 0.f;
  }
  __syncthreads();
  // Layer 2 with d2 in z3; d1 -> d.
  for (int e = t; e < H * H; e += NT) {
    const int o = e / H, i = e % H;
    float s = 0.f;
    for (int b = 0; b < bc; ++b) s += S.z3[b * H + o] * relu(S.z1[b * H + i]);
    S.g[OW2 + e] += s;
  }
  if (t < H) {
    float s = 0.f;
    for (int b = 0; b < bc; ++b) s += S.z3[b * H + t];
    S.g[OB2 + t] += s;
  }
  for (int e = t; e < bc * H; e += NT) {
    const int b = e / H, i = e % H;
    float s = 0.f;
    for (int o = 0; o < H; ++o) s += S.w[OW2 + o * H + i] * S.z3[b * H + o];
    S.d[e] = S.z1[e] > 0.f ? s : 0.f;
  }
  __syncthreads();
  // Layer 1.
  for (int e = t; e < H * IN; e += NT) {
    const int o = e / IN, i = e % IN;
    float s = 0.f;
    for (int b = 0; b < bc; ++b) s += S.d[b * H + o] * S.xs[b * IN + i];
    S.g[OW1 + e] += s;
  }
  if (t < H) {
    float s = 0.f;
    for (int b = 0; b < bc; ++b) s += S.d[b * H + t];
    S.g[OB1 + t] += s;
  }
  // Loss of the chunk.
  for (int o = NT / 2; o > 0; o >>= 1) {
    if (t < o) S.red[t] += S.red[t + o];
    __syncthreads();
  }
  const float l = S.red[0];
  __syncthreads();
  return l;
}

__global__ __launch_bounds__(NT) void mlp_grad_kernel(const float *params, const float *X,
                                                      const float *Y, int64_t n, float *grad,
                                                      float *loss) {
  extern __shared__ float smem[];
  Scratch S = carve(smem);
  __shared__ int64_t rows[CH];
  for (int e = threadIdx.x; e < NP; e += NT) {
    S.w[e] = params[e];
    S.g[e] = 0.f;
  }
  __syncthreads();
  float lsum = 0.f;
  const float inv_n = 1.f / (float)n;
  for (int64_t r0 = 0; r0 < n; r0 += CH) {
    const int bc = (int)((n - r0) < CH ? (n - r0) : CH);
    if (threadIdx.x < bc) rows[threadIdx.x] = r0 + threadIdx.x;
    __syncthreads();
    lsum += chunk_grad(S, X, Y, rows, bc, inv_n);
  }
  __syncthreads();
  for (int e = threadIdx.x; e < NP; e += NT) grad[e] = S.g[e];
  if (threadIdx.x == 0) *loss = lsum * inv_n;
}

__device__ inline uint64_t splitmix(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// One workgroup per model: minibatch Adam on its own parameters.
__global__ __launch_bounds__(NT) void mlp_train_kernel(float *params, float *adam, const float *X,
                                                       const float *Y, int64_t n, int epochs,
                                                       int batch, float lr, uint64_t seed,
                                                       int64_t step0, float *loss_out,
                                                       int nmodels) {
  extern __shared__ float smem[];
  Scratch S = carve(smem);
  __shared__ int64_t rows[CH];
  const int m = blockIdx.x;
  float *p = params + (int64_t)m * NP;
  float *am = adam + (int64_t)m * NP;
  float *av = adam + (int64_t)nmodels * NP + (int64_t)m * NP;
  for (int e = threadIdx.x; e < NP; e += NT) S.w[e] = p[e];
  __syncthreads();
  const int64_t steps = (n + batch - 1) / batch;
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  float last_epoch_loss = 0.f;
  int64_t step = step0;
  for (int ep = 0; ep < epochs; ++ep) {
    float eloss = 0.f;
    for (int64_t st = 0; st < steps; ++st) {
      for (int e = threadIdx.x; e < NP; e += NT) S.g[e] = 0.f;
      __syncthreads();
      const float inv_b = 1.f / (float)batch;
      float bl = 0.f;
      for (int c0 = 0; c0 < batch; c0 += CH) {
        const int bc = batch - c0 < CH ? batch - c0 : CH;
        if (threadIdx.x < bc) {
          const uint64_t h = splitmix((seed + (uint64_t)m) * 0x100000001B3ull +
                                      (uint64_t)step * (uint64_t)batch + (uint64_t)(c0 + threadIdx.x));
          rows[threadIdx.x] = (int64_t)(h % (uint64_t)n);
        }
        __syncthreads();
        bl += chunk_grad(S, X, Y, rows, bc, inv_b);
      }
      ++step;
      const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
      const float lr_t = lr * sqrtf(c2) / c1;
      for (int e = threadIdx.x; e < NP; e += NT) {
        const float g = S.g[e];
        const float mm = b1 * am[e] + (1.f - b1) * g;
        const float vv = b2 * av[e] + (1.f - b2) * g * g;
        am[e] = mm;
        av[e] = vv;
        S.w[e] -= lr_t * mm / (sqrtf(vv) + eps);
      }
      __syncthreads();
      eloss += bl * inv_b;
    }
    last_epoch_loss = eloss / (float)steps;
  }
  for (int e = threadIdx.x; e < NP; e += NT) p[e] = S.w[e];
  if (threadIdx.x == 0) loss_out[m] = last_epoch_loss;
}

size_t scratch_bytes() { return sizeof(float) * SCRATCH_FLOATS; }

bool set_smem(const void *k) {
  return hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)scratch_bytes()) ==
         hipSuccess;
}

}  // namespace

extern "C" {

int qr_mlp_forward(const float *params, int nmodels, const float *X, int64_t n, float *y,
                   void *stream) {
  if (!params) return -1;
  if (nmodels < 1 || nmodels > 65535) return -2;
  if (!X && n > 0) return -3;
  if (n < 0) return -4;
  if (!y && n > 0) return -5;
  if (n == 0) return 0;
  dim3 grid((unsigned)((n + NT - 1) / NT), (unsigned)nmodels);
  hipLaunchKernelGGL(mlp_forward_kernel, grid, dim3(NT), 0, (hipStream_t)stream, params, X, n, y);
  return hipGetLastError() == hipSuccess ? 0 : TILEQR_ERR_HIP;
}

int qr_mlp_grad(const float *params, const float *X, const float *y, int64_t n, float *grad,
                float *loss, void *stream) {
  if (!params) return -1;
  if (!X) return -2;
  if (!y) return -3;
  if (n < 1) return -4;
  if (!grad) return -5;
  if (!loss) return -6;
  if (!set_smem((const void *)mlp_grad_kernel)) return TILEQR_ERR_HIP;
  hipLaunchKernelGGL(mlp_grad_kernel, dim3(1), dim3(NT), scratch_bytes(), (hipStream_t)stream,
                     params, X, y, n, grad, loss);
  return hipGetLastError() == hipSuccess ? 0 : TILEQR_ERR_HIP;
}

int qr_mlp_train(float *params, int nmodels, float *adam, const float *X, const float *y,
                 int64_t n, int epochs, int batch, float lr, uint64_t seed, int64_t step0,
                 float *loss_out, void *stream) {
  if (!params) return -1;
  if (nmodels < 1 || nmodels > 65535) return -2;
  if (!adam) return -3;
  if (!X) return -4;
  if (!y) return -5;
  if (n < 1) return -6;
  if (epochs < 0) return -7;
  if (batch < 1 || batch > 4096) return -8;
  if (!(lr > 0.f)) return -9;
  if (!loss_out) return -11;
  if (!set_smem((const void *)mlp_train_kernel)) return TILEQR_ERR_HIP;
  hipLaunchKernelGGL(mlp_train_kernel, dim3(nmodels), dim3(NT), scratch_bytes(),
                     (hipStream_t)stream, params, adam, X, y, n, epochs, batch, lr, seed, step0,
                     loss_out, nmodels);
  return hipGetLastError() == hipSuccess ? 0 : TILEQR_ERR_HIP;
}

}  // extern "C"

int tq_mlp_choose(const float *params_host, int nmodels, const float *fmean, const float *fstd,
                  float ymean, float ystd, const int *cand, int ncand, int64_t M, int64_t N,
                  int64_t batch, int *nb, int *ib, double *spread) {
  static float *d_p = nullptr, *d_x = nullptr, *d_y = nullptr;
  static int cap_m = 0, cap_c = 0, dev = -1;
  int cur = 0;
  if (hipGetDevice(&cur) != hipSuccess) return TILEQR_ERR_NODEVICE;
  if (cur != dev || nmodels > cap_m || ncand > cap_c) {
    if (d_p) hipFree(d_p);
    if (d_x) hipFree(d_x);
    if (d_y) hipFree(d_y);
    d_p = d_x = d_y = nullptr;
    cap_m = nmodels;
    cap_c = ncand;
    dev = cur;
    if (hipMalloc(&d_p, sizeof(float) * NP * cap_m) != hipSuccess ||
        hipMalloc(&d_x, sizeof(float) * IN * cap_c) != hipSuccess ||
        hipMalloc(&d_y, sizeof(float) * cap_c * cap_m) != hipSuccess) {
      cap_m = cap_c = 0;
      return TILEQR_ERR_NOMEM;
    }
  }
  std::vector<float> x((size_t)IN * ncand);
  for (int c = 0; c < ncand; ++c) {
    const double f[IN] = {std::log((double)std::max<int64_t>(M, 1)),
                          std::log((double)std::max<int64_t>(N, 1)), std::log((double)cand[2 * c]),
                          (double)cand[2 * c + 1] / (double)cand[2 * c],
                          std::log((double)std::max<int64_t>(batch, 1))};
    for (int i = 0; i < IN; ++i) x[(size_t)c * IN + i] = (float)((f[i] - fmean[i]) / fstd[i]);
  }
  if (hipMemcpy(d_p, params_host, sizeof(float) * NP * nmodels, hipMemcpyHostToDevice) != hipSuccess)
    return TILEQR_ERR_HIP;
  if (hipMemcpy(d_x, x.data(), sizeof(float) * x.size(), hipMemcpyHostToDevice) != hipSuccess)
    return TILEQR_ERR_HIP;
  int rc = qr_mlp_forward(d_p, nmodels, d_x, ncand, d_y, nullptr);
  if (rc) return rc;
  std::vector<float> y((size_t)ncand * nmodels);
  if (hipMemcpy(y.data(), d_y, sizeof(float) * y.size(), hipMemcpyDeviceToHost) != hipSuccess)
    return TILEQR_ERR_HIP;
  // Choice: the candidate with the best ensemble-mean prediction. Spread:
  // the largest loss any member predicts for that choice against its own
  // best candidate, max_m (1 - g_m(choice) / max_c g_m(c)); members that
  // agree on the ranking give 0 even when their absolute rates differ.
  std::vector<double> g((size_t)ncand * nmodels), mean(ncand, 0.0);
  for (int m = 0; m < nmodels; ++m)
    for (int c = 0; c < ncand; ++c) {
      g[(size_t)m * ncand + c] = std::exp((double)y[(size_t)m * ncand + c] * ystd + ymean);
      mean[c] += g[(size_t)m * ncand + c] / nmodels;
    }
  int best = 0;
  for (int c = 1; c < ncand; ++c)
    if (mean[c] > mean[best]) best = c;
  double bestspread = 0.0;
  for (int m = 0; m < nmodels; ++m) {
    double top = 0.0;
    for (int c = 0; c < ncand; ++c) top = std::max(top, g[(size_t)m * ncand + c]);
    const double loss = top > 0.0 ? 1.0 - g[(size_t)m * ncand + best] / top : 1.0;
    bestspread = std::max(bestspread, loss);
  }
  *nb = cand[2 * best];
  *ib = cand[2 * best + 1];
  *spread = bestspread;
  return 0;
}
