// Device helpers shared by the library's kernels (wavefront reductions and
// box distances). Wavefront = 64 lanes on CDNA.
#pragma once
#include <hip/hip_runtime.h>

__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ inline double wave_max(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ inline double wave_min(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ inline int wave_sum_int(int v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Workgroups are dispatched to the 8 XCDs round-robin (workgroup i to XCD
// i % 8). xcd_group maps workgroup i to a group index so that each XCD runs
// one contiguous range of groups: neighbouring work items, which read the
// same point or target records, then share that XCD's L2. Launch
// xcd_grid(n_groups) workgroups; a result >= n_groups means no work.
__device__ __forceinline__ int64_t xcd_group(int64_t n_groups) {
    const int64_t per = (n_groups + 7) / 8;
    return (int64_t)(blockIdx.x & 7) * per + (int64_t)(blockIdx.x >> 3);
}
static inline unsigned xcd_grid(int64_t n_groups) {
    return (unsigned)(((n_groups + 7) / 8) * 8);
}

// Work items taken in a sorted order (neighbours read the same records) are
// dealt to the XCDs in runs of RSOT_XCD_RUN consecutive items, run r to XCD
// r % 8, and each XCD takes its runs in order. A run keeps sorted neighbours
// on one XCD's L2, and the runs spread the heavy and light parts of the order
// evenly over the XCDs, which one contiguous range per XCD does not when item
// costs drift along the order. xcd_run_item gives the sorted position of
// this wave's item (wave = wave index in a 4-wave workgroup); launch
// xcd_run_grid(n) workgroups; a result >= n means no work. Every position
// below n is produced exactly once.
#define RSOT_XCD_RUN 64
__device__ __forceinline__ int64_t xcd_run_item(int wave) {
    const int64_t s = (int64_t)(blockIdx.x >> 3) * 4 + wave;   // slot within this XCD
    const int64_t run = (s / RSOT_XCD_RUN) * 8 + (int64_t)(blockIdx.x & 7);
    return run * RSOT_XCD_RUN + s % RSOT_XCD_RUN;
}
static inline unsigned xcd_run_grid(int64_t n) {
    const int64_t runs = (n + RSOT_XCD_RUN - 1) / RSOT_XCD_RUN;
    const int64_t runs_per_xcd = (runs + 7) / 8;
    return (unsigned)(runs_per_xcd * (RSOT_XCD_RUN / 4) * 8);
}

// A 64-bit value from its two 32-bit halves in the signed-int form a 32-bit
// register move returns them: each half is widened through uint32_t, because
// a plain (uint64_t) cast of a low half with bit 31 set would sign-extend
// into the high one. Host-callable so the widening is tested on the CPU.
__host__ __device__ constexpr uint64_t join_halves(int lo, int hi) {
    return ((uint64_t)(uint32_t)hi << 32) | (uint64_t)(uint32_t)lo;
}

// Lane 0's value of a 64-bit quantity, in scalar registers.
__device__ __forceinline__ uint64_t uniform_u64(uint64_t v) {
    return join_halves(__builtin_amdgcn_readfirstlane((int)(uint32_t)v),
                       __builtin_amdgcn_readfirstlane((int)(uint32_t)(v >> 32)));
}

// least distance between the intervals [a0,a1] and [b0,b1] along one axis
__device__ inline double box_gap(double a0, double a1, double b0, double b1) {
    if (b0 > a1) return b0 - a1;
    if (a0 > b1) return a0 - b1;
    return 0.0;
}
// greatest distance between a point of [a0,a1] and a point of [b0,b1]
__device__ inline double box_far(double a0, double a1, double b0, double b1) {
    return fmax(fabs(b1 - a0), fabs(a1 - b0));
}
// greatest distance between a point of [a0,a1] and the value y
__device__ inline double box_far_pt(double a0, double a1, double y) {
    return fmax(fabs(y - a0), fabs(a1 - y));
}
