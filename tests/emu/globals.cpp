// Definitions of the emulator's globals.
#include <hip/hip_runtime.h>
thread_local dim3 threadIdx;
thread_local dim3 blockIdx;
dim3 blockDim, gridDim;
std::barrier<> *g_block_bar;
std::barrier<> *g_wave_bar[4];
double g_wave_a[4][64], g_wave_b[4][64];
double g_wave_c[4][64][4];
double *g_dyn_lds;
char *g_lds_origin;
size_t g_dyn_lds_bytes;
