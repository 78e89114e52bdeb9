// Device helpers of the pair loops shared by the evaluation passes and the
// plan-moment kernels: exponent constants, pair-loop modes, record access
// through the scalar cache, the reference offsets and the canonical FP64
// exponent of a (point, target) pair.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

#define RSOT_LN2 0.69314718055994530942
#define RSOT_LOG2E 1.44269504088896340736
#define CH 8   // pairs per chunk between FP64 flushes

enum { MODE_DENSE = 0, MODE_LIST = 1, MODE_MASK = 2 };

// Fractional offset in [0, 1) of the reference grid of element i (a point of
// the objective pass, a tile of the gradient pass): successive elements step
// by the golden ratio, so the offsets are spread evenly over any run of
// elements. References are ceil(value - offset) + offset; rescaling a sum
// between two references of one element is an exact power of two.
__device__ __forceinline__ double ref_offset(int64_t i) {
    const double v = (double)(i + 1) * 0.6180339887498949;
    return v - floor(v);
}

// constant (read-only) address space: loads at uniform addresses through it
// may use the scalar cache
#define RSOT_CAS __attribute__((address_space(4)))

__device__ __forceinline__ double4 ld4(const double4 *p) { return *p; }
__device__ __forceinline__ double4 ld4(const RSOT_CAS double4 *p) {
    const RSOT_CAS double *q = (const RSOT_CAS double *)p;
    double4 r;
    r.x = q[0];
    r.y = q[1];
    r.z = q[2];
    r.w = q[3];
    return r;
}

// Target record k of a block for the objective pass. 3D: the 32-byte
// records {Y0, Y1, Y2, B}. 2D: the packed 24-byte copies {Y0, Y1, B}, so the
// eight records of a chunk are 192 contiguous bytes that load as three
// 64-byte scalar loads (the 32-byte records with their unused third
// component would load as sixteen 8- and 16-byte pieces).
template <int D, typename P>
__device__ __forceinline__ double4 trec_at(P T, int k) {
    if constexpr (D == 3) {
        return ld4(T + k);
    } else {
        double4 r;
        r.x = T[3 * k + 0];
        r.y = T[3 * k + 1];
        r.z = 0.0;
        r.w = T[3 * k + 2];
        return r;
    }
}

// The FP64 exponent t = B_j + x.Y_j of a (point, target) pair, always formed
// in this order, so that the objective pass and the gradient pass take the
// per-pair cutoff test t > G_j - A_q (c < C) on bitwise equal operands.
template <int D>
__device__ __forceinline__ double pair_exp(double x0, double x1, double x2, const double4 &r) {
    double v = fma(x0, r.x, r.w);
    v = fma(x1, r.y, v);
    if (D == 3) v = fma(x2, r.z, v);
    return v;
}

