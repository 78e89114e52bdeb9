// Standalone microbenchmark of the instruction rates the roofline uses:
// v_exp_f32 (alone and with an add), v_fma_f64, v_fma_f32 (non-packed) and an
// exp + 4 x fma64 mix, each over 8 independent chains per lane.
// Build: python -m paper_2507_23602_amd.build --probes ; run ./_build/probe_rates
#include <hip/hip_runtime.h>
#include <cstdio>
#define ITERS 4096
__global__ __launch_bounds__(256) void k_exp(float* out, float seed) {
  float a[8]; for (int i = 0; i < 8; ++i) a[i] = seed * (threadIdx.x + i) * 1e-6f - 1.0f;
  for (int it = 0; it < ITERS; ++it) {
#pragma unroll
    for (int i = 0; i < 8; ++i) a[i] = __builtin_amdgcn_exp2f(a[i]) - 1.5f;  // exp + add
  }
  float s = 0; for (int i = 0; i < 8; ++i) s += a[i];
  out[blockIdx.x * 256 + threadIdx.x] = s;
}
__global__ __launch_bounds__(256) void k_exp_only(float* out, float seed) {
  float a[8]; for (int i = 0; i < 8; ++i) a[i] = seed * (threadIdx.x + i) * 1e-6f;
  for (int it = 0; it < ITERS; ++it) {
#pragma unroll
    for (int i = 0; i < 8; ++i) a[i] = __builtin_amdgcn_exp2f(-a[i]);
  }
  float s = 0; for (int i = 0; i < 8; ++i) s += a[i];
  out[blockIdx.x * 256 + threadIdx.x] = s;
}
__global__ __launch_bounds__(256) void k_fma64(double* out, double seed) {
  double a[8]; for (int i = 0; i < 8; ++i) a[i] = seed * (threadIdx.x + i);
  for (int it = 0; it < ITERS; ++it) {
#pragma unroll
    for (int i = 0; i < 8; ++i) a[i] = fma(a[i], 0.999999, 1e-7);
  }
  double s = 0; for (int i = 0; i < 8; ++i) s += a[i];
  out[blockIdx.x * 256 + threadIdx.x] = s;
}
__global__ __launch_bounds__(256) void k_fma32(float* out, float seed) {
  float a[8]; for (int i = 0; i < 8; ++i) a[i] = seed * (threadIdx.x + i);
  for (int it = 0; it < ITERS; ++it) {
#pragma unroll
    for (int i = 0; i < 8; ++i) a[i] = fmaf(a[i], 0.999999f, 1e-7f);
  }
  float s = 0; for (int i = 0; i < 8; ++i) s += a[i];
  out[blockIdx.x * 256 + threadIdx.x] = s;
}
// per element: 1 exp + 4 fma64 (interleaved, independent chains)
__global__ __launch_bounds__(256) void k_mix(float* out, double seed) {
  float a[8]; double b[8];
  for (int i = 0; i < 8; ++i) { a[i] = seed * (threadIdx.x + i) * 1e-6 - 1.0; b[i] = seed * i; }
  for (int it = 0; it < ITERS; ++it) {
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      a[i] = __builtin_amdgcn_exp2f(a[i]) - 1.5f;
      b[i] = fma(b[i], 0.999999, 1e-7); b[i] = fma(b[i], 0.999999, 1e-7);
      b[i] = fma(b[i], 0.999999, 1e-7); b[i] = fma(b[i], 0.999999, 1e-7);
    }
  }
  float s = 0; for (int i = 0; i < 8; ++i) s += a[i] + (float)b[i];
  out[blockIdx.x * 256 + threadIdx.x] = s;
}
template <typename F> double timeit(F f) {
  hipEvent_t a, b; hipEventCreate(&a); hipEventCreate(&b);
  f(); hipDeviceSynchronize();
  hipEventRecord(a); f(); hipEventRecord(b); hipEventSynchronize(b);
  float ms; hipEventElapsedTime(&ms, a, b); return ms * 1e-3;
}
int main() {
  const int blocks = 256 * 8 * 4;   // 8192 workgroups of 256
  const double lanes = (double)blocks * 256;
  float* o32; double* o64;
  hipMalloc(&o32, sizeof(float) * blocks * 256); hipMalloc(&o64, sizeof(double) * blocks * 256);
  double t;
  t = timeit([&] { hipLaunchKernelGGL(k_exp, dim3(blocks), dim3(256), 0, 0, o32, 1.0f); });
  printf("exp2f+add: %.3e exp/s (%.3e instr/s incl. add)\n", lanes * ITERS * 8 / t, lanes * ITERS * 16 / t);
  t = timeit([&] { hipLaunchKernelGGL(k_exp_only, dim3(blocks), dim3(256), 0, 0, o32, 1.0f); });
  printf("exp2f only: %.3e exp/s\n", lanes * ITERS * 8 / t);
  t = timeit([&] { hipLaunchKernelGGL(k_fma64, dim3(blocks), dim3(256), 0, 0, o64, 1.0); });
  printf("fma64: %.3e lane-fma/s\n", lanes * ITERS * 8 / t);
  t = timeit([&] { hipLaunchKernelGGL(k_fma32, dim3(blocks), dim3(256), 0, 0, o32, 1.0f); });
  printf("fma32: %.3e lane-fma/s\n", lanes * ITERS * 8 / t);
  t = timeit([&] { hipLaunchKernelGGL(k_mix, dim3(blocks), dim3(256), 0, 0, o32, 1.0); });
  printf("mix (1 exp+1 add+4 fma64): %.3e elem/s -> %.3e exp/s\n", lanes * ITERS * 8 / t, lanes * ITERS * 8 / t);
  return 0;
}
