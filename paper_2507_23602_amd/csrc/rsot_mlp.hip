// Learned warm start: the 6-256x4-1 GELU network, its training kernels and
// the solve from its prediction.
//
// Layout (rows padded to RP, a multiple of 1024; padded rows carry zero
// features and zero loss gradient, so they change no parameter gradient):
//   H_l   bf16 [RP][256]  activation of hidden layer l (row-major)
//   HT_l  bf16 [256][RP]  the same, transposed (l = 0..2): operand of dW_{l+1}
//   Z_l   fp32 [RP][256]  pre-activation (training only)
//   dZ    bf16 [RP][256]  pre-activation gradient, ping-pong; dZT its transpose
// The 256x256 layers are one MFMA kernel (v_mfma_f32_32x32x16_bf16) with the
// whole bf16 weight matrix in LDS; a workgroup tile is 128 rows x 256
// columns, four waves of 64 x 128. Weight gradients split the rows into
// chunks of 1024, each writing its own partial; every other sum over rows
// uses slots of 256 rows. One kernel then adds the partials in a fixed order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

#include "rsot_internal.h"
#include "rsot_mlp.h"

namespace {

constexpr int WID = RSOT_MLP_WIDTH;
constexpr int NIN = RSOT_MLP_IN;
constexpr int KPAD = WID + 8;       // LDS row stride (bf16): 528 B, rows 4 banks apart
constexpr int64_t ROW_ALIGN = 1024; // RP multiple; = CHUNK_DW
constexpr int CHUNK_DW = 1024;      // rows per weight-gradient partial
constexpr int SLOT = 256;           // rows per small-parameter partial

// flat parameter offsets
constexpr int64_t OFF_W0 = 0, OFF_B0 = 1536;
constexpr int64_t OFF_W[4] = {0, 1792, 67584, 133376};
constexpr int64_t OFF_B[4] = {1536, 67328, 133120, 198912};
constexpr int64_t OFF_W4 = 199168, OFF_B4 = 199424;
constexpr int64_t NPAR = RSOT_MLP_NPARAMS;
static_assert(OFF_B4 + 1 == NPAR, "parameter layout");
// small-parameter partial layout: W0 (1536) b0 (256) b1 b2 b3 (256 each) W4 (256) b4 (1)
constexpr int S_W0 = 0, S_B0 = 1536, S_B1 = 1792, S_W4 = 2560, S_B4 = 2816, S_N = 2817;

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ uint16_t f2bf(float x) {
    // round to nearest, ties to even (finite values)
    uint32_t b = __float_as_uint(x);
    b += 0x7FFFu + ((b >> 16) & 1u);
    return (uint16_t)(b >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ float gelu(float z) {
    return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f));
}
__device__ __forceinline__ float gelu_prime(float z) {
    return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) +
           z * expf(-0.5f * z * z) * 0.39894228040143268f;
}

__device__ __forceinline__ bf16x8 ld8(const uint16_t *p) {
    return __builtin_bit_cast(bf16x8, *(const uint4 *)p);
}

__device__ __forceinline__ float wsum(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// ---------------------------------------------------------------------------
// input layer: standardise, 6 -> 256 affine (FP32), GELU
// ---------------------------------------------------------------------------
// One workgroup = 16 rows, thread = output column. Training also keeps the
// standardised features (for dW0), Z0 and the transposed activation.
template <bool TRAIN>
__global__ __launch_bounds__(256) void k_mlp_in(const float *__restrict__ feats,
                                                const int64_t *__restrict__ idx, int64_t R,
                                                int64_t RP, const float *__restrict__ norm,
                                                const uint16_t *__restrict__ W0b,
                                                const float *__restrict__ b0,
                                                float *__restrict__ Fout, float *__restrict__ Z0,
                                                uint16_t *__restrict__ H0,
                                                uint16_t *__restrict__ HT0) {
    const int n = threadIdx.x;
    float w[NIN];
#pragma unroll
    for (int f = 0; f < NIN; ++f) w[f] = bf2f(W0b[f * WID + n]);
    const float bb = b0[n];
    const int64_t r0 = (int64_t)blockIdx.x * 16;
    uint16_t hv[16];
#pragma unroll
    for (int rr = 0; rr < 16; ++rr) {
        const int64_t r = r0 + rr;
        float F[NIN];
        if (r < R) {
            const int64_t src = idx ? idx[r] : r;
#pragma unroll
            for (int f = 0; f < NIN; ++f) F[f] = (feats[src * NIN + f] - norm[f]) / norm[NIN + f];
        } else {
#pragma unroll
            for (int f = 0; f < NIN; ++f) F[f] = 0.0f;
        }
        float z = bb;
#pragma unroll
        for (int f = 0; f < NIN; ++f) z = fmaf(F[f], w[f], z);
        const uint16_t h = f2bf(gelu(z));
        H0[r * WID + n] = h;
        hv[rr] = h;
        if (TRAIN) {
            Z0[r * WID + n] = z;
            if (n < 8) Fout[r * 8 + n] = n < NIN ? F[n] : 0.0f;
        }
    }
    if (TRAIN) {
        uint4 a, b;
        a.x = hv[0] | ((uint32_t)hv[1] << 16);
        a.y = hv[2] | ((uint32_t)hv[3] << 16);
        a.z = hv[4] | ((uint32_t)hv[5] << 16);
        a.w = hv[6] | ((uint32_t)hv[7] << 16);
        b.x = hv[8] | ((uint32_t)hv[9] << 16);
        b.y = hv[10] | ((uint32_t)hv[11] << 16);
        b.z = hv[12] | ((uint32_t)hv[13] << 16);
        b.w = hv[14] | ((uint32_t)hv[15] << 16);
        uint4 *dst = (uint4 *)(HT0 + (int64_t)n * RP + r0);
        dst[0] = a;
        dst[1] = b;
    }
}

// ---------------------------------------------------------------------------
// 256x256 layer on MFMA: C[RP][256] = A[RP][256] . B, B given as Bt[n][k]
// ---------------------------------------------------------------------------
// EPI_FWD:   z = C + bias; H = bf16(GELU(z)); training also stores Z and,
//            if HT is given, the transposed H.
// EPI_BWD:   C is dH of the layer below; dZ = bf16(C * GELU'(Zin)), stored
//            row-major and, if DT is given, transposed.
enum { EPI_FWD = 0, EPI_BWD = 1 };

template <int EPI, bool TRAIN>
__global__ __launch_bounds__(256) void k_mlp_gemm(const uint16_t *__restrict__ A,
                                                  const uint16_t *__restrict__ Bt,
                                                  const float *__restrict__ bias,
                                                  const float *__restrict__ Zin, int64_t RP,
                                                  float *__restrict__ Zout,
                                                  uint16_t *__restrict__ Hout,
                                                  uint16_t *__restrict__ HTout) {
    __shared__ uint16_t sB[WID * KPAD];
    for (int i = threadIdx.x; i < WID * (WID / 8); i += 256) {
        const int n = i >> 5, c = i & 31;
        *(uint4 *)&sB[n * KPAD + c * 8] = ((const uint4 *)Bt)[i];
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wr = wave >> 1, wc = wave & 1;
    const int li = lane & 31, lh = lane >> 5;
    const int64_t n_tiles = RP / 128;
    for (int64_t tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
        const int64_t row0 = tile * 128 + wr * 64;
        f32x16 acc[2][4];
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b)
#pragma unroll
                for (int r = 0; r < 16; ++r) acc[a][b][r] = 0.0f;
        const uint16_t *a0 = A + (row0 + li) * WID + lh * 8;
        const uint16_t *a1 = a0 + 32 * WID;
        const uint16_t *bl = sB + (wc * 128 + li) * KPAD + lh * 8;
#pragma unroll 4
        for (int k0 = 0; k0 < WID; k0 += 16) {
            const bf16x8 fa0 = ld8(a0 + k0), fa1 = ld8(a1 + k0);
#pragma unroll
            for (int cb = 0; cb < 4; ++cb) {
                const bf16x8 fb = ld8(bl + cb * 32 * KPAD + k0);
                acc[0][cb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa0, fb, acc[0][cb], 0, 0, 0);
                acc[1][cb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa1, fb, acc[1][cb], 0, 0, 0);
            }
        }
        // C[i][j] of a 32x32 block: j = lane % 32, i = 8 (r / 4) + 4 (lane / 32) + r % 4
#pragma unroll
        for (int rb = 0; rb < 2; ++rb) {
#pragma unroll
            for (int cb = 0; cb < 4; ++cb) {
                const int col = wc * 128 + cb * 32 + li;
                const float bc = EPI == EPI_FWD ? bias[col] : 0.0f;
#pragma unroll
                for (int g = 0; g < 4; ++g) {
                    const int64_t rbase = row0 + rb * 32 + 8 * g + 4 * lh;
                    uint16_t hq[4];
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const int64_t row = rbase + q;
                        const float c = acc[rb][cb][4 * g + q];
                        uint16_t h;
                        if (EPI == EPI_FWD) {
                            const float z = c + bc;
                            h = f2bf(gelu(z));
                            if (TRAIN) Zout[row * WID + col] = z;
                        } else {
                            h = f2bf(c * gelu_prime(Zin[row * WID + col]));
                        }
                        Hout[row * WID + col] = h;
                        hq[q] = h;
                    }
                    if (TRAIN && HTout) {
                        uint2 v;
                        v.x = hq[0] | ((uint32_t)hq[1] << 16);
                        v.y = hq[2] | ((uint32_t)hq[3] << 16);
                        *(uint2 *)(HTout + (int64_t)col * RP + rbase) = v;
                    }
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// weight gradient of a 256x256 layer: dW[k][n] = sum_r H[r][k] dZ[r][n]
// ---------------------------------------------------------------------------
// Grid = chunks x 4 quadrants of 128x128; wave = 64x64 of its quadrant over
// the chunk's 1024 rows. Operands come from the transposed copies, whose rows
// are contiguous in r. Chunk c of layer l is written at
// part_base + c * 3 * 65536, part_base = partW + (l - 1) * 65536.
__global__ __launch_bounds__(256) void k_mlp_gemm_dw(const uint16_t *__restrict__ HT,
                                                     const uint16_t *__restrict__ DT, int64_t RP,
                                                     float *__restrict__ part) {
    const int64_t chunk = blockIdx.x >> 2;
    const int quad = blockIdx.x & 3;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int li = lane & 31, lh = lane >> 5;
    const int k0r = (quad >> 1) * 128 + (wave >> 1) * 64;
    const int n0c = (quad & 1) * 128 + (wave & 1) * 64;
    f32x16 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[a][b][r] = 0.0f;
    const int64_t rs = chunk * CHUNK_DW + lh * 8;
    const uint16_t *pa0 = HT + (int64_t)(k0r + li) * RP + rs;
    const uint16_t *pa1 = pa0 + 32 * RP;
    const uint16_t *pb0 = DT + (int64_t)(n0c + li) * RP + rs;
    const uint16_t *pb1 = pb0 + 32 * RP;
#pragma unroll 4
    for (int r = 0; r < CHUNK_DW; r += 16) {
        const bf16x8 a0 = ld8(pa0 + r), a1 = ld8(pa1 + r);
        const bf16x8 b0 = ld8(pb0 + r), b1 = ld8(pb1 + r);
        acc[0][0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0, b0, acc[0][0], 0, 0, 0);
        acc[0][1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0, b1, acc[0][1], 0, 0, 0);
        acc[1][0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1, b0, acc[1][0], 0, 0, 0);
        acc[1][1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1, b1, acc[1][1], 0, 0, 0);
    }
    float *dst = part + chunk * (int64_t)(3 * WID * WID);
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int k = k0r + a * 32 + 8 * (r >> 2) + 4 * lh + (r & 3);
                const int n = n0c + b * 32 + li;
                dst[k * WID + n] = acc[a][b][r];
            }
}

// ---------------------------------------------------------------------------
// output layer and loss gradient
// ---------------------------------------------------------------------------
// MODE 0: prediction only (out = o * std + mean for rows < R).
// MODE 1: MSE against target: d_r = 2 (o_r - t_r) / R in standardised units.
// MODE 2: given dL/dout: d_r = dout_r * std.
// Training modes also write dZ3 = bf16(d_r W4 GELU'(Z3)) (row-major and
// transposed) and the slot's partials of W4, b4 and the loss.
template <int MODE>
__global__ __launch_bounds__(256) void k_mlp_out(
    const uint16_t *__restrict__ H3, const float *__restrict__ Z3, const uint16_t *__restrict__ w4b,
    const float *__restrict__ b4, const float *__restrict__ norm, const float *__restrict__ target,
    const float *__restrict__ dgiven, const int64_t *__restrict__ idx, int64_t R, int64_t RP,
    float *__restrict__ out, uint16_t *__restrict__ dZ, uint16_t *__restrict__ dZT,
    float *__restrict__ partS, double *__restrict__ lossp) {
    __shared__ float sd[SLOT];
    __shared__ double sl[4];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t base = (int64_t)blockIdx.x * SLOT;
    const float om = norm[2 * NIN], osd = norm[2 * NIN + 1];
    float wl[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) wl[q] = bf2f(w4b[lane * 4 + q]);
    double lacc = 0.0;
    for (int rr = wave; rr < SLOT; rr += 4) {
        const int64_t r = base + rr;
        const uint2 hv = *(const uint2 *)(H3 + r * WID + lane * 4);
        float p = bf2f((uint16_t)(hv.x & 0xFFFF)) * wl[0];
        p = fmaf(bf2f((uint16_t)(hv.x >> 16)), wl[1], p);
        p = fmaf(bf2f((uint16_t)(hv.y & 0xFFFF)), wl[2], p);
        p = fmaf(bf2f((uint16_t)(hv.y >> 16)), wl[3], p);
        const float o = wsum(p) + b4[0];
        if (MODE == 0) {
            if (lane == 0 && r < R) out[r] = fmaf(o, osd, om);
            continue;
        }
        float d = 0.0f;
        if (r < R) {
            if (MODE == 1) {
                const int64_t src = idx ? idx[r] : r;
                const float t = (target[src] - om) / osd;
                const float diff = o - t;
                d = 2.0f * diff / (float)R;
                lacc += (double)diff * (double)diff;
            } else {
                d = dgiven[r] * osd;
            }
        }
        if (lane == 0) sd[rr] = d;
    }
    if (MODE == 0) return;
    if (lane == 0) sl[wave] = lacc;
    __syncthreads();
    const int k = threadIdx.x;
    const float wk = bf2f(w4b[k]);
    float gw = 0.0f;
    for (int r8 = 0; r8 < SLOT; r8 += 8) {
        uint16_t dq[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int64_t r = base + r8 + q;
            const float d = sd[r8 + q];
            gw = fmaf(d, bf2f(H3[r * WID + k]), gw);
            const uint16_t dz = f2bf(d * wk * gelu_prime(Z3[r * WID + k]));
            dZ[r * WID + k] = dz;
            dq[q] = dz;
        }
        uint4 v;
        v.x = dq[0] | ((uint32_t)dq[1] << 16);
        v.y = dq[2] | ((uint32_t)dq[3] << 16);
        v.z = dq[4] | ((uint32_t)dq[5] << 16);
        v.w = dq[6] | ((uint32_t)dq[7] << 16);
        *(uint4 *)(dZT + (int64_t)k * RP + base + r8) = v;
    }
    float *ps = partS + (int64_t)blockIdx.x * S_N;
    ps[S_W4 + k] = gw;
    if (k == 0) {
        float sb = 0.0f;
        for (int r = 0; r < SLOT; ++r) sb += sd[r];
        ps[S_B4] = sb;
        lossp[blockIdx.x] = sl[0] + sl[1] + sl[2] + sl[3];
    }
}

// bias gradient of hidden layer l: slot partial of sum_r dZ[r][n]
__global__ __launch_bounds__(256) void k_mlp_colsum(const uint16_t *__restrict__ dZ,
                                                    float *__restrict__ partS, int soff) {
    const int n = threadIdx.x;
    const int64_t base = (int64_t)blockIdx.x * SLOT;
    float s = 0.0f;
    for (int r = 0; r < SLOT; ++r) s += bf2f(dZ[(base + r) * WID + n]);
    partS[(int64_t)blockIdx.x * S_N + soff + n] = s;
}

// input layer gradients: slot partials of dW0[f][n] = sum_r F[r][f] dZ0[r][n], db0
__global__ __launch_bounds__(256) void k_mlp_dw0(const float *__restrict__ F,
                                                 const uint16_t *__restrict__ dZ0,
                                                 float *__restrict__ partS) {
    const int n = threadIdx.x;
    const int64_t base = (int64_t)blockIdx.x * SLOT;
    float g[NIN] = {0, 0, 0, 0, 0, 0}, gb = 0.0f;
    for (int r = 0; r < SLOT; ++r) {
        const float dz = bf2f(dZ0[(base + r) * WID + n]);
        const float *fr = F + (base + r) * 8;
#pragma unroll
        for (int f = 0; f < NIN; ++f) g[f] = fmaf(fr[f], dz, g[f]);
        gb += dz;
    }
    float *ps = partS + (int64_t)blockIdx.x * S_N;
#pragma unroll
    for (int f = 0; f < NIN; ++f) ps[S_W0 + f * WID + n] = g[f];
    ps[S_B0 + n] = gb;
}

// fixed-order sum of the partials into the flat gradient; thread 0 of block 0
// also sums the loss partials
__global__ __launch_bounds__(256) void k_mlp_reduce(const float *__restrict__ partW,
                                                    int64_t n_chunks,
                                                    const float *__restrict__ partS,
                                                    int64_t n_slots,
                                                    const double *__restrict__ lossp, int64_t R,
                                                    float *__restrict__ grad,
                                                    double *__restrict__ loss) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i == 0 && loss) {
        double s = 0.0;
        for (int64_t c = 0; c < n_slots; ++c) s += lossp[c];
        *loss = s / (double)R;
    }
    if (i >= NPAR) return;
    int layer = 0;
    for (int l = 1; l < 4; ++l)
        if (i >= OFF_W[l] && i < OFF_W[l] + WID * WID) layer = l;
    double s = 0.0;
    if (layer > 0) {
        const int64_t off = (int64_t)(layer - 1) * WID * WID + (i - OFF_W[layer]);
        for (int64_t c = 0; c < n_chunks; ++c) s += partW[c * 3 * WID * WID + off];
    } else {
        int j;
        if (i < OFF_B0 + WID) j = (int)i;                                   // W0, b0
        else if (i >= OFF_W4) j = S_W4 + (int)(i - OFF_W4);                 // W4, b4
        else {
            int l = 1;
            while (!(i >= OFF_B[l] && i < OFF_B[l] + WID)) ++l;
            j = S_B1 + (l - 1) * WID + (int)(i - OFF_B[l]);
        }
        for (int64_t c = 0; c < n_slots; ++c) s += partS[c * S_N + j];
    }
    grad[i] = (float)s;
}

// Adam step (FP32) with bias corrections c1 = 1/(1-b1^t), c2 = 1/(1-b2^t);
// remakes the bf16 copies of the updated weights
__global__ __launch_bounds__(256) void k_mlp_adam(float *__restrict__ P, float *__restrict__ Mm,
                                                  float *__restrict__ Vv,
                                                  const float *__restrict__ grad, float lr,
                                                  float b1, float b2, float eps, float c1,
                                                  float c2, uint16_t *__restrict__ W0b,
                                                  uint16_t *__restrict__ Wb,
                                                  uint16_t *__restrict__ WTb,
                                                  uint16_t *__restrict__ w4b) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= NPAR) return;
    const float g = grad[i];
    const float m = b1 * Mm[i] + (1.0f - b1) * g;
    const float v = b2 * Vv[i] + (1.0f - b2) * g * g;
    Mm[i] = m;
    Vv[i] = v;
    const float p = P[i] - lr * (m * c1) / (sqrtf(v * c2) + eps);
    P[i] = p;
    const uint16_t h = f2bf(p);
    if (i < OFF_B0) W0b[i] = h;
    else if (i >= OFF_W4 && i < OFF_B4) w4b[i - OFF_W4] = h;
    for (int l = 1; l < 4; ++l) {
        if (i >= OFF_W[l] && i < OFF_W[l] + WID * WID) {
            const int64_t loc = i - OFF_W[l];
            const int64_t k = loc / WID, n = loc % WID;
            Wb[(int64_t)(l - 1) * WID * WID + loc] = h;
            WTb[(int64_t)(l - 1) * WID * WID + n * WID + k] = h;
        }
    }
}

// bf16 copies of the masters (after set_params)
__global__ __launch_bounds__(256) void k_mlp_copies(const float *__restrict__ P,
                                                    uint16_t *__restrict__ W0b,
                                                    uint16_t *__restrict__ Wb,
                                                    uint16_t *__restrict__ WTb,
                                                    uint16_t *__restrict__ w4b) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= NPAR) return;
    const uint16_t h = f2bf(P[i]);
    if (i < OFF_B0) W0b[i] = h;
    else if (i >= OFF_W4 && i < OFF_B4) w4b[i - OFF_W4] = h;
    for (int l = 1; l < 4; ++l) {
        if (i >= OFF_W[l] && i < OFF_W[l] + WID * WID) {
            const int64_t loc = i - OFF_W[l];
            const int64_t k = loc / WID, n = loc % WID;
            Wb[(int64_t)(l - 1) * WID * WID + loc] = h;
            WTb[(int64_t)(l - 1) * WID * WID + n * WID + k] = h;
        }
    }
}

// values the kernels use, as float: bf16 weights, FP32 biases
__global__ __launch_bounds__(256) void k_mlp_used(const float *__restrict__ P,
                                                  const uint16_t *__restrict__ W0b,
                                                  const uint16_t *__restrict__ Wb,
                                                  const uint16_t *__restrict__ w4b,
                                                  float *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= NPAR) return;
    float v = P[i];
    if (i < OFF_B0) v = bf2f(W0b[i]);
    else if (i >= OFF_W4 && i < OFF_B4) v = bf2f(w4b[i - OFF_W4]);
    for (int l = 1; l < 4; ++l)
        if (i >= OFF_W[l] && i < OFF_W[l] + WID * WID)
            v = bf2f(Wb[(int64_t)(l - 1) * WID * WID + (i - OFF_W[l])]);
    out[i] = v;
}

// mean and spread of features and targets (FP64), one workgroup
__global__ __launch_bounds__(1024) void k_mlp_moments(const float *__restrict__ feats,
                                                      const float *__restrict__ target,
                                                      int64_t rows, double *__restrict__ out) {
    __shared__ double sh[14][16];
    double s[14];
    for (int q = 0; q < 14; ++q) s[q] = 0.0;
    for (int64_t r = threadIdx.x; r < rows; r += blockDim.x) {
        for (int f = 0; f < NIN; ++f) {
            const double v = feats[r * NIN + f];
            s[f] += v;
            s[NIN + f] += v * v;
        }
        const double t = target[r];
        s[12] += t;
        s[13] += t * t;
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int q = 0; q < 14; ++q) {
        double v = s[q];
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
        if (lane == 0) sh[q][wave] = v;
    }
    __syncthreads();
    if (threadIdx.x < 14) {
        double v = 0.0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) v += sh[threadIdx.x][w];
        out[threadIdx.x] = v;
    }
}

__global__ __launch_bounds__(256) void k_mlp_features(int64_t n, const double *__restrict__ y,
                                                      double c0, double c1, double s, double leps,
                                                      float *__restrict__ feats) {
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j >= n) return;
    float *f = feats + j * NIN;
    f[0] = (float)y[2 * j];
    f[1] = (float)y[2 * j + 1];
    f[2] = (float)c0;
    f[3] = (float)c1;
    f[4] = (float)s;
    f[5] = (float)leps;
}

// features of a problem's targets in its sorted order (coordinates un-shifted)
__global__ __launch_bounds__(256) void k_mlp_features_sorted(int64_t n_pad,
                                                             const double *__restrict__ ty,
                                                             double sx, double sy, double c0,
                                                             double c1, double s, double leps,
                                                             float *__restrict__ feats) {
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j >= n_pad) return;
    float *f = feats + j * NIN;
    f[0] = (float)(ty[3 * j] + sx);
    f[1] = (float)(ty[3 * j + 1] + sy);
    f[2] = (float)c0;
    f[3] = (float)c1;
    f[4] = (float)s;
    f[5] = (float)leps;
}

// psi = pred - (sum nu pred) / (sum nu), FP64; pred and nu indexed alike,
// written to dst[perm[j]] (or dst[j] without perm) for entries with perm >= 0
__global__ __launch_bounds__(1024) void k_mlp_centre(int64_t n, const float *__restrict__ pred,
                                                     const double *__restrict__ nu,
                                                     const int32_t *__restrict__ perm,
                                                     double *__restrict__ dst) {
    __shared__ double sa[16], sb[16];
    double a = 0.0, b = 0.0;
    for (int64_t j = threadIdx.x; j < n; j += blockDim.x) {
        if (perm && perm[j] < 0) continue;
        a += nu[j] * (double)pred[j];
        b += nu[j];
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int o = 32; o > 0; o >>= 1) {
        a += __shfl_xor(a, o, 64);
        b += __shfl_xor(b, o, 64);
    }
    if (lane == 0) {
        sa[wave] = a;
        sb[wave] = b;
    }
    __syncthreads();
    double A = 0.0, B = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
        A += sa[w];
        B += sb[w];
    }
    const double mean = B > 0.0 ? A / B : 0.0;
    for (int64_t j = threadIdx.x; j < n; j += blockDim.x) {
        if (perm) {
            if (perm[j] >= 0) dst[perm[j]] = (double)pred[j] - mean;
        } else {
            dst[j] = (double)pred[j] - mean;
        }
    }
}

__global__ void k_mlp_nonfinite(int64_t n, const double *__restrict__ v, int *__restrict__ flag) {
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j < n && !isfinite(v[j])) *flag = 1;
}

__global__ void k_zero_int(int *p) { *p = 0; }

}  // namespace

struct rsot_mlp {
    hipStream_t stream = nullptr;
    float *P = nullptr, *Mm = nullptr, *Vv = nullptr;   // masters, Adam moments
    uint16_t *W0b = nullptr, *Wb = nullptr, *WTb = nullptr, *w4b = nullptr;
    float *norm = nullptr;                              // device [14]
    float hnorm[14];
    float *grad = nullptr;                              // device NPAR
    double *dloss = nullptr, *dmom = nullptr;
    int *dflag = nullptr;
    int64_t step = 0;
    // training workspace, sized for cap_tr rows
    int64_t cap_tr = 0;
    float *Z[4] = {nullptr, nullptr, nullptr, nullptr};
    uint16_t *H[4] = {nullptr, nullptr, nullptr, nullptr};
    uint16_t *HT[3] = {nullptr, nullptr, nullptr};
    uint16_t *dZ[2] = {nullptr, nullptr};
    uint16_t *dZT = nullptr;
    float *F = nullptr, *partW = nullptr, *partS = nullptr;
    double *lossp = nullptr;
    std::vector<void *> ws_tr;
    // inference workspace, sized for cap_inf rows
    int64_t cap_inf = 0;
    uint16_t *Hi[2] = {nullptr, nullptr};
    float *outb = nullptr;
    std::vector<void *> ws_inf;
    float *featb = nullptr;                             // feature rows of predictions
    int64_t featb_cap = 0;
    hipEvent_t e0 = nullptr, e1 = nullptr;

    static void free_list(std::vector<void *> &v) {
        for (void *p : v) (void)hipFree(p);
        v.clear();
    }
    ~rsot_mlp() {
        free_list(ws_tr);
        free_list(ws_inf);
        for (void *p : {(void *)P, (void *)Mm, (void *)Vv, (void *)W0b, (void *)Wb, (void *)WTb,
                        (void *)w4b, (void *)norm, (void *)grad, (void *)dloss, (void *)dmom,
                        (void *)dflag, (void *)featb})
            if (p) (void)hipFree(p);
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
    }
};

static int64_t padded_rows(int64_t R) { return (R + ROW_ALIGN - 1) / ROW_ALIGN * ROW_ALIGN; }

template <typename T>
static rsot_status ws_alloc(std::vector<void *> &list, T **p, size_t count) {
    void *q = nullptr;
    if (hipMalloc(&q, std::max<size_t>(count, 1) * sizeof(T)) != hipSuccess) {
        (void)hipGetLastError();
        return RSOT_ERR_OOM;
    }
    list.push_back(q);
    *p = (T *)q;
    return RSOT_OK;
}

// Training and inference keep separate workspaces, each grown to the largest
// padded row count it has seen, so that alternating the two (a held-out
// forward between training steps) reallocates nothing.
static rsot_status ensure_train_ws(rsot_mlp *m, int64_t RP) {
    if (RP <= m->cap_tr) return RSOT_OK;
    RSOT_HIP(hipStreamSynchronize(m->stream));
    rsot_mlp::free_list(m->ws_tr);
    m->cap_tr = 0;
    auto &L = m->ws_tr;
    const size_t rw = (size_t)RP * WID;
    for (int l = 0; l < 4; ++l) RSOT_TRY(ws_alloc(L, &m->Z[l], rw));
    for (int l = 0; l < 4; ++l) RSOT_TRY(ws_alloc(L, &m->H[l], rw));
    for (int l = 0; l < 3; ++l) RSOT_TRY(ws_alloc(L, &m->HT[l], rw));
    for (int l = 0; l < 2; ++l) RSOT_TRY(ws_alloc(L, &m->dZ[l], rw));
    RSOT_TRY(ws_alloc(L, &m->dZT, rw));
    RSOT_TRY(ws_alloc(L, &m->F, (size_t)RP * 8));
    RSOT_TRY(ws_alloc(L, &m->partW, (size_t)(RP / CHUNK_DW) * 3 * WID * WID));
    RSOT_TRY(ws_alloc(L, &m->partS, (size_t)(RP / SLOT) * S_N));
    RSOT_TRY(ws_alloc(L, &m->lossp, (size_t)(RP / SLOT)));
    m->cap_tr = RP;
    return RSOT_OK;
}

static rsot_status ensure_inf_ws(rsot_mlp *m, int64_t RP) {
    if (RP <= m->cap_inf) return RSOT_OK;
    RSOT_HIP(hipStreamSynchronize(m->stream));
    rsot_mlp::free_list(m->ws_inf);
    m->cap_inf = 0;
    auto &L = m->ws_inf;
    const size_t rw = (size_t)RP * WID;
    RSOT_TRY(ws_alloc(L, &m->Hi[0], rw));
    RSOT_TRY(ws_alloc(L, &m->Hi[1], rw));
    RSOT_TRY(ws_alloc(L, &m->outb, (size_t)RP));
    m->cap_inf = RP;
    return RSOT_OK;
}

static unsigned gemm_grid(int64_t RP) { return (unsigned)std::min<int64_t>(RP / 128, 256); }

// forward pass; training keeps Z, H, HT and the standardised inputs
static rsot_status run_forward(rsot_mlp *m, const float *feats, const int64_t *idx, int64_t R,
                               int64_t RP, bool train) {
    const hipStream_t st = m->stream;
    const float *bias[4] = {m->P + OFF_B[0], m->P + OFF_B[1], m->P + OFF_B[2], m->P + OFF_B[3]};
    if (train) {
        hipLaunchKernelGGL(k_mlp_in<true>, dim3((unsigned)(RP / 16)), dim3(256), 0, st, feats, idx,
                           R, RP, m->norm, m->W0b, bias[0], m->F, m->Z[0], m->H[0], m->HT[0]);
        for (int l = 1; l < 4; ++l)
            hipLaunchKernelGGL((k_mlp_gemm<EPI_FWD, true>), dim3(gemm_grid(RP)), dim3(256), 0, st,
                               m->H[l - 1], m->WTb + (size_t)(l - 1) * WID * WID, bias[l],
                               (const float *)nullptr, RP, m->Z[l], m->H[l],
                               l < 3 ? m->HT[l] : (uint16_t *)nullptr);
    } else {
        hipLaunchKernelGGL(k_mlp_in<false>, dim3((unsigned)(RP / 16)), dim3(256), 0, st, feats, idx,
                           R, RP, m->norm, m->W0b, bias[0], (float *)nullptr, (float *)nullptr,
                           m->Hi[0], (uint16_t *)nullptr);
        for (int l = 1; l < 4; ++l)
            hipLaunchKernelGGL((k_mlp_gemm<EPI_FWD, false>), dim3(gemm_grid(RP)), dim3(256), 0,
                               st, m->Hi[(l - 1) & 1], m->WTb + (size_t)(l - 1) * WID * WID,
                               bias[l], (const float *)nullptr, RP, (float *)nullptr, m->Hi[l & 1],
                               (uint16_t *)nullptr);
    }
    return hipGetLastError() == hipSuccess ? RSOT_OK : RSOT_ERR_DEVICE;
}

// backward from dZ3 (in dZ[0], dZT) to the flat gradient `grad` (device)
static rsot_status run_backward(rsot_mlp *m, int64_t R, int64_t RP, float *grad,
                                double *loss_dev) {
    const hipStream_t st = m->stream;
    const int64_t n_chunks = RP / CHUNK_DW, n_slots = RP / SLOT;
    int cur = 0;
    for (int l = 3; l >= 1; --l) {
        // dW_l from H_{l-1} and dZ_l (transposed copies)
        hipLaunchKernelGGL(k_mlp_gemm_dw, dim3((unsigned)(n_chunks * 4)), dim3(256), 0, st,
                           m->HT[l - 1], m->dZT, RP, m->partW + (size_t)(l - 1) * WID * WID);
        hipLaunchKernelGGL(k_mlp_colsum, dim3((unsigned)n_slots), dim3(256), 0, st, m->dZ[cur],
                           m->partS, S_B1 + (l - 1) * WID);
        // dZ_{l-1} = bf16((dZ_l W_l^T) * GELU'(Z_{l-1})); W_l as [k][n] is Bt of this product
        hipLaunchKernelGGL((k_mlp_gemm<EPI_BWD, true>), dim3(gemm_grid(RP)), dim3(256), 0, st,
                           m->dZ[cur], m->Wb + (size_t)(l - 1) * WID * WID, (const float *)nullptr,
                           m->Z[l - 1], RP, (float *)nullptr, m->dZ[cur ^ 1],
                           l - 1 >= 1 ? m->dZT : (uint16_t *)nullptr);
        cur ^= 1;
    }
    hipLaunchKernelGGL(k_mlp_dw0, dim3((unsigned)n_slots), dim3(256), 0, st, m->F, m->dZ[cur],
                       m->partS);
    hipLaunchKernelGGL(k_mlp_reduce, dim3((unsigned)((NPAR + 255) / 256)), dim3(256), 0, st,
                       m->partW, n_chunks, m->partS, n_slots, m->lossp, R, grad, loss_dev);
    return hipGetLastError() == hipSuccess ? RSOT_OK : RSOT_ERR_DEVICE;
}

static rsot_status upload_params(rsot_mlp *m, const float *params) {
    RSOT_HIP(hipMemcpyAsync(m->P, params, sizeof(float) * NPAR, hipMemcpyHostToDevice, m->stream));
    RSOT_HIP(hipMemsetAsync(m->Mm, 0, sizeof(float) * NPAR, m->stream));
    RSOT_HIP(hipMemsetAsync(m->Vv, 0, sizeof(float) * NPAR, m->stream));
    hipLaunchKernelGGL(k_mlp_copies, dim3((unsigned)((NPAR + 255) / 256)), dim3(256), 0, m->stream,
                       m->P, m->W0b, m->Wb, m->WTb, m->w4b);
    RSOT_HIP(hipGetLastError());
    RSOT_HIP(hipStreamSynchronize(m->stream));
    m->step = 0;
    return RSOT_OK;
}

static rsot_status upload_norm(rsot_mlp *m) {
    RSOT_HIP(hipMemcpyAsync(m->norm, m->hnorm, sizeof(m->hnorm), hipMemcpyHostToDevice, m->stream));
    RSOT_HIP(hipStreamSynchronize(m->stream));
    return RSOT_OK;
}

extern "C" rsot_status rsot_mlp_create(const float *params, void *hip_stream, rsot_mlp **out) {
    if (!out) return RSOT_ERR_INVALID_ARG;
    *out = nullptr;
    if (!params) return RSOT_ERR_INVALID_ARG;
    for (int64_t i = 0; i < NPAR; ++i)
        if (!std::isfinite(params[i])) return RSOT_ERR_NONFINITE;
    auto *m = new (std::nothrow) rsot_mlp();
    if (!m) return RSOT_ERR_OOM;
    m->stream = (hipStream_t)hip_stream;
    bool ok = hipMalloc((void **)&m->P, sizeof(float) * NPAR) == hipSuccess &&
              hipMalloc((void **)&m->Mm, sizeof(float) * NPAR) == hipSuccess &&
              hipMalloc((void **)&m->Vv, sizeof(float) * NPAR) == hipSuccess &&
              hipMalloc((void **)&m->grad, sizeof(float) * NPAR) == hipSuccess &&
              hipMalloc((void **)&m->W0b, sizeof(uint16_t) * NIN * WID) == hipSuccess &&
              hipMalloc((void **)&m->Wb, sizeof(uint16_t) * 3 * WID * WID) == hipSuccess &&
              hipMalloc((void **)&m->WTb, sizeof(uint16_t) * 3 * WID * WID) == hipSuccess &&
              hipMalloc((void **)&m->w4b, sizeof(uint16_t) * WID) == hipSuccess &&
              hipMalloc((void **)&m->norm, sizeof(float) * 14) == hipSuccess &&
              hipMalloc((void **)&m->dloss, sizeof(double) * 2) == hipSuccess &&
              hipMalloc((void **)&m->dmom, sizeof(double) * 14) == hipSuccess &&
              hipMalloc((void **)&m->dflag, sizeof(int)) == hipSuccess &&
              hipEventCreate(&m->e0) == hipSuccess && hipEventCreate(&m->e1) == hipSuccess;
    if (!ok) {
        (void)hipGetLastError();
        delete m;
        return RSOT_ERR_OOM;
    }
    for (int f = 0; f < NIN; ++f) {
        m->hnorm[f] = 0.0f;
        m->hnorm[NIN + f] = 1.0f;
    }
    m->hnorm[12] = 0.0f;
    m->hnorm[13] = 1.0f;
    rsot_status s = upload_params(m, params);
    if (s == RSOT_OK) s = upload_norm(m);
    if (s != RSOT_OK) {
        delete m;
        return s;
    }
    *out = m;
    return RSOT_OK;
}

extern "C" void rsot_mlp_destroy(rsot_mlp *m) {
    if (!m) return;
    (void)hipStreamSynchronize(m->stream);
    delete m;
}

extern "C" rsot_status rsot_mlp_get_params(rsot_mlp *m, int which, float *params_out) {
    if (!m || !params_out || (which != 0 && which != 1)) return RSOT_ERR_INVALID_ARG;
    if (which == 0) {
        RSOT_HIP(hipMemcpyAsync(params_out, m->P, sizeof(float) * NPAR, hipMemcpyDeviceToHost,
                                m->stream));
    } else {
        hipLaunchKernelGGL(k_mlp_used, dim3((unsigned)((NPAR + 255) / 256)), dim3(256), 0,
                           m->stream, m->P, m->W0b, m->Wb, m->w4b, m->grad);
        RSOT_HIP(hipGetLastError());
        RSOT_HIP(hipMemcpyAsync(params_out, m->grad, sizeof(float) * NPAR, hipMemcpyDeviceToHost,
                                m->stream));
    }
    RSOT_HIP(hipStreamSynchronize(m->stream));
    return RSOT_OK;
}

extern "C" rsot_status rsot_mlp_set_params(rsot_mlp *m, const float *params) {
    if (!m || !params) return RSOT_ERR_INVALID_ARG;
    for (int64_t i = 0; i < NPAR; ++i)
        if (!std::isfinite(params[i])) return RSOT_ERR_NONFINITE;
    return upload_params(m, params);
}

extern "C" rsot_status rsot_mlp_set_normalization(rsot_mlp *m, const float *feat_mean,
                                                  const float *feat_std, float out_mean,
                                                  float out_std) {
    if (!m || !feat_mean || !feat_std) return RSOT_ERR_INVALID_ARG;
    for (int f = 0; f < NIN; ++f)
        if (!std::isfinite(feat_mean[f]) || !(feat_std[f] > 0.0f) || !std::isfinite(feat_std[f]))
            return RSOT_ERR_INVALID_ARG;
    if (!std::isfinite(out_mean) || !(out_std > 0.0f) || !std::isfinite(out_std))
        return RSOT_ERR_INVALID_ARG;
    for (int f = 0; f < NIN; ++f) {
        m->hnorm[f] = feat_mean[f];
        m->hnorm[NIN + f] = feat_std[f];
    }
    m->hnorm[12] = out_mean;
    m->hnorm[13] = out_std;
    return upload_norm(m);
}

extern "C" rsot_status rsot_mlp_get_normalization(rsot_mlp *m, float *feat_mean, float *feat_std,
                                                  float *out_mean, float *out_std) {
    if (!m) return RSOT_ERR_INVALID_ARG;
    for (int f = 0; f < NIN; ++f) {
        if (feat_mean) feat_mean[f] = m->hnorm[f];
        if (feat_std) feat_std[f] = m->hnorm[NIN + f];
    }
    if (out_mean) *out_mean = m->hnorm[12];
    if (out_std) *out_std = m->hnorm[13];
    return RSOT_OK;
}

extern "C" rsot_status rsot_mlp_fit_normalization(rsot_mlp *m, const float *feats,
                                                  const float *target, int64_t rows) {
    if (!m || !feats || !target || rows < 1) return RSOT_ERR_INVALID_ARG;
    hipLaunchKernelGGL(k_mlp_moments, dim3(1), dim3(1024), 0, m->stream, feats, target, rows,
                       m->dmom);
    RSOT_HIP(hipGetLastError());
    double h[14];
    RSOT_HIP(hipMemcpyAsync(h, m->dmom, sizeof(h), hipMemcpyDeviceToHost, m->stream));
    RSOT_HIP(hipStreamSynchronize(m->stream));
    auto spread = [&](double s1, double s2) {
        const double mean = s1 / rows;
        const double var = std::max(0.0, s2 / rows - mean * mean);
        const double sd = std::sqrt(var);
        return sd > 1e-12 * std::max(1.0, std::fabs(mean)) ? sd : 1.0;
    };
    for (int f = 0; f < NIN; ++f) {
        m->hnorm[f] = (float)(h[f] / rows);
        m->hnorm[NIN + f] = (float)spread(h[f], h[NIN + f]);
    }
    m->hnorm[12] = (float)(h[12] / rows);
    m->hnorm[13] = (float)spread(h[12], h[13]);
    for (int q = 0; q < 14; ++q)
        if (!std::isfinite(m->hnorm[q])) return RSOT_ERR_NONFINITE;
    return upload_norm(m);
}

extern "C" rsot_status rsot_mlp_features(int64_t n, const double *y, const double *cond,
                                         float *feats, void *hip_stream) {
    if (n < 0 || (n > 0 && (!y || !feats)) || !cond) return RSOT_ERR_INVALID_ARG;
    if (!(cond[3] > 0.0) || !std::isfinite(cond[3])) return RSOT_ERR_INVALID_ARG;
    if (n == 0) return RSOT_OK;
    hipLaunchKernelGGL(k_mlp_features, dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                       (hipStream_t)hip_stream, n, y, cond[0], cond[1], cond[2], std::log(cond[3]),
                       feats);
    RSOT_HIP(hipGetLastError());
    return RSOT_OK;
}

extern "C" rsot_status rsot_mlp_forward(rsot_mlp *m, const float *feats, int64_t rows, float *out) {
    if (!m || rows < 0 || (rows > 0 && (!feats || !out))) return RSOT_ERR_INVALID_ARG;
    if (rows == 0) return RSOT_OK;
    const int64_t RP = padded_rows(rows);
    RSOT_TRY(ensure_inf_ws(m, RP));
    RSOT_TRY(run_forward(m, feats, nullptr, rows, RP, false));
    hipLaunchKernelGGL(k_mlp_out<0>, dim3((unsigned)(RP / SLOT)), dim3(256), 0, m->stream,
                       m->Hi[1], (const float *)nullptr, m->w4b,
                       m->P + OFF_B4, m->norm, (const float *)nullptr, (const float *)nullptr,
                       (const int64_t *)nullptr, rows, RP, out, (uint16_t *)nullptr,
                       (uint16_t *)nullptr, (float *)nullptr, (double *)nullptr);
    RSOT_HIP(hipGetLastError());
    RSOT_HIP(hipStreamSynchronize(m->stream));
    return RSOT_OK;
}

// prediction of `rows` feature rows into m->outb (no synchronisation)
static rsot_status predict_rows(rsot_mlp *m, const float *feats, int64_t rows) {
    const int64_t RP = padded_rows(rows);
    RSOT_TRY(ensure_inf_ws(m, RP));
    RSOT_TRY(run_forward(m, feats, nullptr, rows, RP, false));
    hipLaunchKernelGGL(k_mlp_out<0>, dim3((unsigned)(RP / SLOT)), dim3(256), 0, m->stream,
                       m->Hi[1], (const float *)nullptr, m->w4b, m->P + OFF_B4, m->norm,
                       (const float *)nullptr, (const float *)nullptr, (const int64_t *)nullptr,
                       rows, RP, m->outb, (uint16_t *)nullptr, (uint16_t *)nullptr,
                       (float *)nullptr, (double *)nullptr);
    RSOT_HIP(hipGetLastError());
    return RSOT_OK;
}

static rsot_status ensure_featb(rsot_mlp *m, int64_t rows) {
    if (rows <= m->featb_cap) return RSOT_OK;
    RSOT_HIP(hipStreamSynchronize(m->stream));
    if (m->featb) (void)hipFree(m->featb);
    m->featb = nullptr;
    m->featb_cap = 0;
    if (hipMalloc((void **)&m->featb, sizeof(float) * NIN * (size_t)rows) != hipSuccess) {
        (void)hipGetLastError();
        return RSOT_ERR_OOM;
    }
    m->featb_cap = rows;
    return RSOT_OK;
}

extern "C" rsot_status rsot_mlp_backward(rsot_mlp *m, const float *feats, int64_t rows,
                                         const float *dout, float *grad) {
    if (!m || rows < 1 || !feats || !dout || !grad) return RSOT_ERR_INVALID_ARG;
    const int64_t RP = padded_rows(rows);
    RSOT_TRY(ensure_train_ws(m, RP));
    RSOT_TRY(run_forward(m, feats, nullptr, rows, RP, true));
    hipLaunchKernelGGL(k_mlp_out<2>, dim3((unsigned)(RP / SLOT)), dim3(256), 0, m->stream,
                       m->H[3], m->Z[3], m->w4b, m->P + OFF_B4, m->norm, (const float *)nullptr,
                       dout, (const int64_t *)nullptr, rows, RP, (float *)nullptr, m->dZ[0], m->dZT,
                       m->partS, m->lossp);
    RSOT_HIP(hipGetLastError());
    RSOT_TRY(run_backward(m, rows, RP, grad, nullptr));
    RSOT_HIP(hipStreamSynchronize(m->stream));
    return RSOT_OK;
}

static bool adam_args_ok(float lr, float b1, float b2, float eps) {
    return lr > 0.0f && std::isfinite(lr) && b1 >= 0.0f && b1 < 1.0f && b2 >= 0.0f && b2 < 1.0f &&
           eps >= 0.0f && std::isfinite(eps);
}

static rsot_status launch_adam(rsot_mlp *m, const float *grad, float lr, float b1, float b2,
                               float eps) {
    ++m->step;
    const double c1 = 1.0 / (1.0 - std::pow((double)b1, (double)m->step));
    const double c2 = 1.0 / (1.0 - std::pow((double)b2, (double)m->step));
    hipLaunchKernelGGL(k_mlp_adam, dim3((unsigned)((NPAR + 255) / 256)), dim3(256), 0, m->stream,
                       m->P, m->Mm, m->Vv, grad, lr, b1, b2, eps, (float)c1, (float)c2, m->W0b,
                       m->Wb, m->WTb, m->w4b);
    RSOT_HIP(hipGetLastError());
    return RSOT_OK;
}

extern "C" rsot_status rsot_mlp_adam_step(rsot_mlp *m, const float *grad, float lr, float b1,
                                          float b2, float eps) {
    if (!m || !grad || !adam_args_ok(lr, b1, b2, eps)) return RSOT_ERR_INVALID_ARG;
    RSOT_TRY(launch_adam(m, grad, lr, b1, b2, eps));
    RSOT_HIP(hipStreamSynchronize(m->stream));
    return RSOT_OK;
}

extern "C" rsot_status rsot_mlp_train_step(rsot_mlp *m, const float *feats, const float *target,
                                           const int64_t *idx, int64_t rows, float lr, float b1,
                                           float b2, float eps, double *loss) {
    if (!m || rows < 1 || !feats || !target || !adam_args_ok(lr, b1, b2, eps))
        return RSOT_ERR_INVALID_ARG;
    const int64_t RP = padded_rows(rows);
    RSOT_TRY(ensure_train_ws(m, RP));
    RSOT_TRY(run_forward(m, feats, idx, rows, RP, true));
    hipLaunchKernelGGL(k_mlp_out<1>, dim3((unsigned)(RP / SLOT)), dim3(256), 0, m->stream,
                       m->H[3], m->Z[3], m->w4b, m->P + OFF_B4, m->norm, target,
                       (const float *)nullptr, idx, rows, RP, (float *)nullptr, m->dZ[0], m->dZT, m->partS,
                       m->lossp);
    RSOT_HIP(hipGetLastError());
    RSOT_TRY(run_backward(m, rows, RP, m->grad, m->dloss));
    RSOT_TRY(launch_adam(m, m->grad, lr, b1, b2, eps));
    if (loss) {
        RSOT_HIP(hipMemcpyAsync(loss, m->dloss, sizeof(double), hipMemcpyDeviceToHost, m->stream));
        RSOT_HIP(hipStreamSynchronize(m->stream));
    }
    return RSOT_OK;
}

extern "C" rsot_status rsot_mlp_predict_psi(rsot_mlp *m, int64_t n, const double *y,
                                            const double *nu, const double *cond, double *psi) {
    if (!m || n < 1 || !y || !nu || !cond || !psi) return RSOT_ERR_INVALID_ARG;
    RSOT_TRY(ensure_featb(m, n));
    RSOT_TRY(rsot_mlp_features(n, y, cond, m->featb, m->stream));
    RSOT_TRY(predict_rows(m, m->featb, n));
    hipLaunchKernelGGL(k_mlp_centre, dim3(1), dim3(1024), 0, m->stream, n, m->outb, nu,
                       (const int32_t *)nullptr, psi);
    RSOT_HIP(hipGetLastError());
    RSOT_HIP(hipStreamSynchronize(m->stream));
    return RSOT_OK;
}

extern "C" rsot_status rsot_solve_learned(rsot_problem *p, rsot_mlp *m, const double *cond,
                                          const rsot_solve_params *sp, double *psi_out,
                                          rsot_solve_info *info, rsot_learned_info *linfo) {
    if (!p || !m || !cond || !sp || !psi_out || !sp->eps_schedule || sp->n_eps < 1)
        return RSOT_ERR_INVALID_ARG;
    if (p->dim != 2 || !(cond[3] > 0.0) || !std::isfinite(cond[3])) return RSOT_ERR_INVALID_ARG;
    const double eps_f = sp->eps_schedule[sp->n_eps - 1];
    if (!(eps_f > 0.0) || !std::isfinite(eps_f)) return RSOT_ERR_INVALID_ARG;
    rsot_learned_info li{};
    const int64_t n = p->n, n_pad = p->n_pad;
    RSOT_HIP(hipStreamSynchronize(p->stream));
    // prediction on the problem's sorted targets, centred and scattered to
    // the caller's order in p->dpsi
    RSOT_TRY(ensure_featb(m, n_pad));
    RSOT_HIP(hipEventRecord(m->e0, m->stream));
    hipLaunchKernelGGL(k_mlp_features_sorted, dim3((unsigned)((n_pad + 255) / 256)), dim3(256), 0,
                       m->stream, n_pad, p->ty, p->shift[0], p->shift[1], cond[0], cond[1],
                       cond[2], std::log(cond[3]), m->featb);
    RSOT_HIP(hipGetLastError());
    RSOT_TRY(predict_rows(m, m->featb, n_pad));
    hipLaunchKernelGGL(k_mlp_centre, dim3(1), dim3(1024), 0, m->stream, n_pad, m->outb, p->tnu,
                       p->tperm, p->dpsi);
    hipLaunchKernelGGL(k_zero_int, dim3(1), dim3(1), 0, m->stream, m->dflag);
    hipLaunchKernelGGL(k_mlp_nonfinite, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, m->stream,
                       n, p->dpsi, m->dflag);
    RSOT_HIP(hipGetLastError());
    RSOT_HIP(hipEventRecord(m->e1, m->stream));
    int flag = 0;
    RSOT_HIP(hipMemcpyAsync(&flag, m->dflag, sizeof(int), hipMemcpyDeviceToHost, m->stream));
    RSOT_HIP(hipStreamSynchronize(m->stream));
    float ms = 0.0f;
    (void)hipEventElapsedTime(&ms, m->e0, m->e1);
    li.predict_ms = ms;
    std::vector<double> psi((size_t)n, 0.0);
    li.J_pred = NAN;
    rsot_eval_info ei{};
    if (!flag) {
        RSOT_HIP(hipMemcpy(psi.data(), p->dpsi, sizeof(double) * n, hipMemcpyDeviceToHost));
        double J = 0.0;
        RSOT_TRY(rsot_eval_impl(p, eps_f, p->dpsi, &J, p->dgrad, &ei));
        li.J_pred = J;
    }
    {
        RSOT_HIP(hipMemsetAsync(p->dpsi, 0, sizeof(double) * n, p->stream));
        double J = 0.0;
        RSOT_TRY(rsot_eval_impl(p, eps_f, p->dpsi, &J, p->dgrad, &ei));
        li.J_zero = J;
    }
    rsot_status s;
    if (!flag && std::isfinite(li.J_pred) && li.J_pred < li.J_zero) {
        li.used_learned = 1;
        rsot_solve_params one = *sp;
        one.eps_schedule = &eps_f;
        one.n_eps = 1;
        s = rsot_solve(p, &one, psi.data(), info);
    } else {
        li.used_learned = 0;
        std::fill(psi.begin(), psi.end(), 0.0);
        s = rsot_solve(p, sp, psi.data(), info);
    }
    std::memcpy(psi_out, psi.data(), sizeof(double) * n);
    if (linfo) *linfo = li;
    return s;
}
