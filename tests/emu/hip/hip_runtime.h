// CPU emulation of the subset of HIP the library's kernels use, so that the
// device source can be compiled for the host and run under AddressSanitizer:
// every lane is a host thread, workgroups run one after the other, barriers
// are std::barrier, LDS is a host array laid out as on the device (an 8-byte
// static segment, then the dynamic part), and v_mfma_f64_16x16x4f64 follows
// the lane layout measured on gfx950. Lanes do not run in lockstep, so the
// emulation also checks that lanes exchanging data through LDS synchronise.
#pragma once
#include <atomic>
#include <barrier>
#include <cassert>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <thread>
#include <vector>
#include <algorithm>

struct dim3 { unsigned x, y, z; dim3(unsigned a = 1, unsigned b = 1, unsigned c = 1) : x(a), y(b), z(c) {} };
extern thread_local dim3 threadIdx;
extern thread_local dim3 blockIdx;
extern dim3 blockDim, gridDim;

#define __global__
#define __device__
#define __host__
#define __forceinline__ inline
#define __launch_bounds__(...)
#define __restrict__
#define __shared__ static
#define __align__(x) __attribute__((aligned(x)))
#define HIP_SYMBOL(x) ((const void *)&(x))

typedef int hipError_t;
#define hipSuccess 0
#define hipErrorInvalidValue 1
typedef void *hipStream_t;
enum { hipFuncAttributeMaxDynamicSharedMemorySize = 8 };
inline hipError_t hipFuncSetAttribute(const void *, int, int) { return 0; }
inline hipError_t hipOccupancyMaxActiveBlocksPerMultiprocessor(int *n, ...) { *n = 1; return 0; }
inline hipError_t hipGetLastError() { return 0; }
enum { hipMemcpyHostToDevice = 1, hipMemcpyDeviceToHost = 2, hipMemcpyDeviceToDevice = 3 };
inline hipError_t hipGetDevice(int *d) { *d = 0; return 0; }
template <class T> inline hipError_t hipMalloc(T **p, size_t n) { *p = (T *)malloc(n); return *p ? 0 : 1; }
inline hipError_t hipFree(void *p) { free(p); return 0; }
inline hipError_t hipMemcpy(void *d, const void *s, size_t n, int) { memcpy(d, s, n); return 0; }
inline hipError_t hipGetSymbolAddress(void **p, const void *sym) { *p = (void *)sym; return 0; }

extern std::barrier<> *g_block_bar;
extern std::barrier<> *g_wave_bar[4];
extern double g_wave_a[4][64], g_wave_b[4][64];
extern double g_wave_c[4][64][4];
extern double *g_dyn_lds;
extern char *g_lds_origin;
extern size_t g_dyn_lds_bytes;

inline void __syncthreads() { std::atomic_thread_fence(std::memory_order_seq_cst); g_block_bar->arrive_and_wait(); }
inline void __threadfence() { std::atomic_thread_fence(std::memory_order_seq_cst); }
inline void __threadfence_block() { std::atomic_thread_fence(std::memory_order_seq_cst); }
inline long long wall_clock64() { return 0; }
inline void __builtin_amdgcn_s_sleep(int) { std::this_thread::yield(); }

#define __builtin_amdgcn_fence(...) std::atomic_thread_fence(std::memory_order_seq_cst)
#define __builtin_amdgcn_s_waitcnt(x) std::atomic_thread_fence(std::memory_order_seq_cst)
#define __builtin_amdgcn_s_setprio(x) ((void)0)
#define __builtin_amdgcn_sched_barrier(x) ((void)0)
inline void __builtin_amdgcn_wave_barrier() { g_wave_bar[threadIdx.x >> 6]->arrive_and_wait(); }
inline double __shfl(double v, int src, int width = 64) {
  int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  g_wave_a[w][l] = v;
  g_wave_bar[w]->arrive_and_wait();
  double r = g_wave_a[w][src & 63];
  g_wave_bar[w]->arrive_and_wait();
  return r;
}
inline double __shfl_xor(double v, int mask, int width = 64) {
  int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  g_wave_a[w][l] = v;
  g_wave_bar[w]->arrive_and_wait();
  double r = g_wave_a[w][l ^ mask];
  g_wave_bar[w]->arrive_and_wait();
  return r;
}

// DPP move within a row of 16 lanes, quad_perm patterns only (ctrl < 0x100):
// lane l takes src from lane (l & ~3) | sel(l & 3).
inline int __builtin_amdgcn_mov_dpp(int v, int ctrl, int, int, bool) {
  int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  assert(ctrl < 0x100);
  static thread_local int dummy;
  (void)dummy;
  double *slot = &g_wave_a[w][0];
  int *islot = (int *)slot;  // reuse the exchange buffer as ints
  islot[l] = v;
  g_wave_bar[w]->arrive_and_wait();
  int src = (l & ~3) | ((ctrl >> (2 * (l & 3))) & 3);
  int r = islot[src];
  g_wave_bar[w]->arrive_and_wait();
  return r;
}

// v_readlane_b32: lane `src`'s value to the whole wave (every lane calls it).
inline int __builtin_amdgcn_readlane(int v, int src) {
  int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  assert(src >= 0 && src < 64);
  int *islot = (int *)&g_wave_a[w][0];
  islot[l] = v;
  g_wave_bar[w]->arrive_and_wait();
  int r = islot[src];
  g_wave_bar[w]->arrive_and_wait();
  return r;
}

typedef double emu_d4 __attribute__((ext_vector_type(4)));
// v_mfma_f64_16x16x4f64 with the assumed lane layout:
//   A[i][k] in lane i + 16k, B[k][j] in lane j + 16k, D[i][j] in lane j + 16*(i%4), item i/4
//   (measured on gfx950).
inline emu_d4 __builtin_amdgcn_mfma_f64_16x16x4f64(double a, double b, emu_d4 c, int, int, int) {
  int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  g_wave_a[w][l] = a;
  g_wave_b[w][l] = b;
  g_wave_bar[w]->arrive_and_wait();
  emu_d4 d;
  for (int r = 0; r < 4; ++r) {
    int i = 4 * r + l / 16, j = l % 16;
    double s = c[r];
    for (int k = 0; k < 4; ++k) s += g_wave_a[w][i + 16 * k] * g_wave_b[w][j + 16 * k];
    d[r] = s;
  }
  g_wave_bar[w]->arrive_and_wait();
  return d;
}

#define __ATOMIC_AGENT_DUMMY 0
#define __HIP_MEMORY_SCOPE_AGENT 0
#define __hip_atomic_load(p, o, s) __atomic_load_n((p), __ATOMIC_SEQ_CST)
#define __hip_atomic_store(p, v, o, s) __atomic_store_n((p), (v), __ATOMIC_SEQ_CST)
#define __hip_atomic_fetch_add(p, v, o, s) __atomic_fetch_add((p), (v), __ATOMIC_SEQ_CST)
inline unsigned atomicAdd(unsigned *p, unsigned v) { return __atomic_fetch_add(p, v, __ATOMIC_SEQ_CST); }
#define __builtin_amdgcn_readfirstlane(x) (x)

using std::min;
using std::max;

// Runs the grid one block at a time; each block on 256 host threads.
template <class F, class... Args>
void emu_launch(dim3 grid, dim3 block, size_t lds, F kern, Args... args) {
  gridDim = grid;
  blockDim = block;
  // As on the device: an 8-byte static segment (the ticket broadcast) at LDS
  // offset 0, dynamic LDS right after it at offset 8.
  std::vector<double> dyn((lds + 7) / 8 + 1, std::nan(""));
  g_lds_origin = (char *)dyn.data();
  g_dyn_lds = dyn.data() + 1;
  g_dyn_lds_bytes = lds;
  for (unsigned bx = 0; bx < grid.x; ++bx)
    for (unsigned by = 0; by < grid.y; ++by) {
      std::barrier<> bb(block.x);
      std::barrier<> wb0(64), wb1(64), wb2(64), wb3(64);
      g_block_bar = &bb;
      g_wave_bar[0] = &wb0; g_wave_bar[1] = &wb1; g_wave_bar[2] = &wb2; g_wave_bar[3] = &wb3;
      std::vector<std::thread> th;
      for (unsigned t = 0; t < block.x; ++t)
        th.emplace_back([=]() { threadIdx = dim3(t); blockIdx = dim3(bx, by); kern(args...); });
      for (auto &x : th) x.join();
    }
}
#define hipLaunchKernelGGL(kern, grid, block, lds, stream, ...) emu_launch(grid, block, lds, kern, __VA_ARGS__)
