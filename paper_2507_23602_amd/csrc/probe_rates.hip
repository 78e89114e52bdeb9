// Standalone microbenchmark of the instruction rates the roofline uses:
// v_exp_f32 (alone and with an add), v_fma_f64, v_fma_f32 (non-packed) and an
// exp + 4 x fma64 mix, each over 8 independent chains per lane; and
// v_mfma_f64_16x16x4_f64 alone and with the conversion, exponential and sum
// of its 256 outputs, to see whether the matrix core runs beside the vector ALU.
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
typedef double d4 __attribute__((ext_vector_type(4)));
// four chained accumulators per wave: matrix-core rate alone
__global__ __launch_bounds__(256) void k_mfma64(double* out, double seed) {
  const int l = threadIdx.x & 63;
  const double a = seed * l, b = seed * (l + 1);
  d4 acc[4];
  for (int u = 0; u < 4; ++u) acc[u] = (d4){0.0, 0.0, 0.0, 0.0};
  for (int it = 0; it < ITERS / 2; ++it) {
#pragma unroll
    for (int u = 0; u < 4; ++u) acc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[u], 0, 0, 0);
  }
  double s = 0;
  for (int u = 0; u < 4; ++u) s += acc[u][0] + acc[u][1] + acc[u][2] + acc[u][3];
  out[blockIdx.x * 256 + threadIdx.x] = s;
}
// the same products consumed one iteration later by 16 x (cvt, exp, add)
__global__ __launch_bounds__(256) void k_mfma64_exp(double* out, double seed) {
  const int l = threadIdx.x & 63;
  const double a = 1e-3 * (l % 16);
  double b = seed * 1e-6 * (l / 16);
  const d4 c0 = {-0.5, -0.25, -0.125, -0.0625};
  d4 cur[4], nxt[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) cur[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b + u, c0, 0, 0, 0);
  float s[4] = {0.f, 0.f, 0.f, 0.f};
  for (int it = 0; it < ITERS / 2; ++it) {
    b += 1e-9;
#pragma unroll
    for (int u = 0; u < 4; ++u) nxt[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b + 1e-12 * u, c0, 0, 0, 0);
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int r = 0; r < 4; ++r) s[r] += __builtin_amdgcn_exp2f((float)cur[u][r]);
#pragma unroll
    for (int u = 0; u < 4; ++u) cur[u] = nxt[u];
  }
  out[blockIdx.x * 256 + threadIdx.x] = (double)(s[0] + s[1] + s[2] + s[3]);
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
  // matrix core: 1024 FMA per instruction; cycles per instruction per SIMD
  const double mf = (double)blocks * 4 * (ITERS / 2) * 4;
  t = timeit([&] { hipLaunchKernelGGL(k_mfma64, dim3(blocks), dim3(256), 0, 0, o64, 1.0); });
  printf("mfma f64 16x16x4: %.3e flop/s, %.1f cycles per instruction per SIMD\n", mf * 2048 / t,
         1024 * 2.4e9 * t / mf);
  t = timeit([&] { hipLaunchKernelGGL(k_mfma64_exp, dim3(blocks), dim3(256), 0, 0, o64, 1.0); });
  printf("mfma f64 + 256 x (cvt, exp, add): %.1f cycles per instruction per SIMD\n",
         1024 * 2.4e9 * t / mf);
  return 0;
}
