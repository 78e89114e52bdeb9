// Learned warm start: the 6-256x4-1 GELU network, its training kernels and
// the solve from its prediction.
//
// Layouts (rows padded to RP, a multiple of 1024; padded rows carry zero
// features and zero loss gradient, so they change no parameter gradient):
//   k-blocked bf16   X[c/16][r][c%16]       operand of the layer products
//                                          (each MFMA operand load is 1 KB
//                                          contiguous)
//   row-blocked bf16 X[r/16][c][r%16]       operand of the weight gradients
//   fragment FP32    per 32x32 block (r/32, c/32) in row-major block order,
//                    inside it the MFMA accumulator order [g][lane][q]
//                    (r%32 = 8g + 4(lane/32) + q, c%32 = lane%32): the
//                    pre-activations, written and read as float4 by the
//                    layer epilogues
// The 256x256 layers run on v_mfma_f32_32x32x16_bf16 with the whole bf16
// weight matrix in LDS; a workgroup of 8 waves owns 128 rows x 256 columns,
// a wave 32 x 128. The output layer and the loss are fused into the last
// layer's epilogue, the bias gradients into the epilogues that produce the
// pre-activation gradients. Sums over rows go to per-workgroup (or per
// 256-row slot) partials that one kernel adds in a fixed order, so repeated
// calls give the same bits.
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
constexpr int SLOT = 256;           // rows per input-layer partial
constexpr int GW = 8;               // waves per layer workgroup (two per SIMD)
constexpr int GROWS = GW / 2 * 32;  // rows per layer workgroup tile (128)
constexpr int MAX_GRID = 256;       // layer workgroups (one per CU)

// flat parameter offsets
constexpr int64_t OFF_B0 = 1536;
constexpr int64_t OFF_W[4] = {0, 1792, 67584, 133376};
constexpr int64_t OFF_B[4] = {1536, 67328, 133120, 198912};
constexpr int64_t OFF_W4 = 199168, OFF_B4 = 199424;
constexpr int64_t NPAR = RSOT_MLP_NPARAMS;
static_assert(OFF_B4 + 1 == NPAR, "parameter layout");
// partial layout per slot: W0 (1536) b0 (256) b1 b2 b3 (256 each) W4 (256) b4 (1).
// W0, b0 come from the input-layer kernel (one slot per 256 rows); the rest
// from the layer epilogues (one slot per workgroup).
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

// GELU and its derivative from one erf and one exp (same roundings as above)
__device__ __forceinline__ void gelu_and_prime(float z, float &g, float &gp) {
    const float phi = 0.5f * (1.0f + erff(z * 0.70710678118654752f));
    g = z * phi;
    gp = phi + z * expf(-0.5f * z * z) * 0.39894228040143268f;
}

__device__ __forceinline__ bf16x8 ld8(const uint16_t *p) {
    return __builtin_bit_cast(bf16x8, *(const uint4 *)p);
}

__host__ __device__ __forceinline__ int64_t kb_idx(int64_t r, int c, int64_t RP) {
    return ((int64_t)(c >> 4) * RP + r) * 16 + (c & 15);
}
__host__ __device__ __forceinline__ int64_t rb_idx(int64_t r, int c) {
    return ((r >> 4) * WID + c) * 16 + (r & 15);
}
// first element (q = 0) of the float4 holding rows r..r+3 (r % 4 = 0) of column c
__host__ __device__ __forceinline__ int64_t fr_idx(int64_t r, int c) {
    const int i = (int)(r & 31);
    return (((r >> 5) * 8 + (c >> 5)) * 4 + (i >> 3)) * 256 + (((i >> 2) & 1) * 32 + (c & 31)) * 4;
}

__device__ __forceinline__ float wsum(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ uint2 pack4(const uint16_t h[4]) {
    uint2 v;
    v.x = h[0] | ((uint32_t)h[1] << 16);
    v.y = h[2] | ((uint32_t)h[3] << 16);
    return v;
}

// ---------------------------------------------------------------------------
// input layer: standardise, 6 -> 256 affine (FP32), GELU
// ---------------------------------------------------------------------------
// One workgroup = 32 rows; thread (column block cbk, lane) owns column
// cbk*32 + lane%32 and the 16 rows 8g + 4(lane/32) + q of the accumulator
// layout, so every store matches the layer kernels' layouts. Training also
// keeps the standardised features (for dW0), Z0 and the row-blocked copy.
template <bool TRAIN>
__global__ __launch_bounds__(512) void k_mlp_in(const float *__restrict__ feats,
                                                const int64_t *__restrict__ idx, int64_t R,
                                                int64_t RP, const float *__restrict__ norm,
                                                const uint16_t *__restrict__ W0b,
                                                const float *__restrict__ b0,
                                                float *__restrict__ Fout, float *__restrict__ Z0,
                                                uint16_t *__restrict__ Hkb,
                                                uint16_t *__restrict__ Hrb) {
    __shared__ float sF[32][8];
    __shared__ uint16_t sH[32][WID + 8];   // the tile's bf16 activations (528-byte rows)
    const int lane = threadIdx.x & 63, cbk = threadIdx.x >> 6;
    const int li = lane & 31, lh = lane >> 5;
    const int col = cbk * 32 + li;
    const int64_t r0 = (int64_t)blockIdx.x * 32;
    // standardised features of the workgroup's 32 rows, once per row
    if (threadIdx.x < 32 * 8) {
        const int rr = threadIdx.x >> 3, f = threadIdx.x & 7;
        const int64_t r = r0 + rr;
        float v = 0.0f;
        if (r < R && f < NIN) {
            const int64_t src = idx ? idx[r] : r;
            v = (feats[src * NIN + f] - norm[f]) / norm[NIN + f];
        }
        sF[rr][f] = v;
        if (TRAIN) Fout[r * 8 + f] = v;
    }
    __syncthreads();
    float w[NIN];
#pragma unroll
    for (int f = 0; f < NIN; ++f) w[f] = bf2f(W0b[f * WID + col]);
    const float bb = b0[col];
#pragma unroll
    for (int g = 0; g < 4; ++g) {
        const int64_t rb = r0 + 8 * g + 4 * lh;
        float z4[4];
        uint16_t h4[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int rl = 8 * g + 4 * lh + q;
            float z = bb;
#pragma unroll
            for (int f = 0; f < NIN; ++f) z = fmaf(sF[rl][f], w[f], z);
            z4[q] = z;
            h4[q] = f2bf(gelu(z));
            sH[rl][col] = h4[q];
        }
        if (TRAIN) {
            *(float4 *)(Z0 + fr_idx(rb, col)) = make_float4(z4[0], z4[1], z4[2], z4[3]);
            *(uint2 *)(Hrb + rb_idx(rb, col)) = pack4(h4);
        }
    }
    __syncthreads();
    // k-blocked copy from LDS in 16-byte pieces (8 columns of one row): each
    // 64 consecutive pieces are 1 KB of contiguous output
    for (int i = threadIdx.x; i < 32 * (WID / 8); i += 512) {
        const int c16 = i >> 6, rl = (i >> 1) & 31, hf = i & 1;
        const int c = c16 * 16 + hf * 8;
        *(uint4 *)(Hkb + kb_idx(r0 + rl, c, RP)) = *(const uint4 *)&sH[rl][c];
    }
}

// ---------------------------------------------------------------------------
// 256x256 layer on MFMA: C[RP][256] = A[RP][256] . B, B given as Bt[n][k]
// ---------------------------------------------------------------------------
// EPI_FWD  hidden layer: z = C + bias, H = bf16(GELU(z)) k-blocked; training
//          also stores z (fragment order) and H row-blocked.
// EPI_OUT  last hidden layer fused with the output layer: o_r = H_r . W4 + b4
//          (rows reduced across lanes and the two column waves through LDS);
//          prediction writes o * std + mean; training forms the loss
//          gradient d_r, dZ3 = bf16(d_r W4 GELU'(z)) in both bf16 layouts and
//          the slot partials of b3 (column sums of dZ3), W4, b4 and the loss.
// EPI_BWD  C is dH of the layer below: dZ = bf16(C GELU'(Zin)) k-blocked, and
//          row-blocked if asked; with `colsum` the slot partial of its bias.
enum { EPI_FWD = 0, EPI_OUT = 1, EPI_BWD = 2 };
enum { OUT_PREDICT = 0, OUT_MSE = 1, OUT_GIVEN = 2 };

struct LayerArgs {
    const uint16_t *A;    // k-blocked operand [RP][256]
    const uint16_t *Bt;   // [256 n][256 k] bf16
    const float *bias;    // FWD / OUT
    const float *Zin;     // BWD: pre-activation of the output layer, fragment order
    float *Zout;          // FWD, training
    uint16_t *Hkb, *Hrb;  // outputs (Hrb may be null)
    float *partS;         // slot partials [slot][S_N]
    int soff;             // column-sum offset in a slot (-1: none)
    // output layer
    const uint16_t *w4b;
    const float *b4, *norm, *target, *dgiven;
    const int64_t *idx;
    float *out;
    double *lossp;
    int out_mode;
    int64_t R, RP;
};

template <int EPI, bool TRAIN>
__global__ __launch_bounds__(GW * 64) void k_mlp_layer(LayerArgs a) {
    __shared__ uint16_t sB[WID * KPAD];
    __shared__ float sPart[2][GROWS];   // EPI_OUT: row dots of each column wave
    __shared__ float sD[GROWS];         // EPI_OUT: loss gradient d_r of each row
    __shared__ float sRed[GW / 2][WID];
    __shared__ double sLoss[GW];
    for (int i = threadIdx.x; i < WID * (WID / 8); i += GW * 64) {
        const int n = i >> 5, c = i & 31;
        *(uint4 *)&sB[n * KPAD + c * 8] = ((const uint4 *)a.Bt)[i];
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wr = wave >> 1, wc = wave & 1;
    const int li = lane & 31, lh = lane >> 5;
    const int64_t RP = a.RP;
    const int64_t n_tiles = RP / GROWS;
    constexpr bool OUT_TRAIN = EPI == EPI_OUT && TRAIN;
    float csum[4] = {0.0f, 0.0f, 0.0f, 0.0f};   // column sums of the bf16 output
    float gw4[4] = {0.0f, 0.0f, 0.0f, 0.0f};    // sum_r d_r h[r][col]
    float gb4 = 0.0f;
    double lacc = 0.0;
    float w4c[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    if (EPI == EPI_OUT) {
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) w4c[cb] = bf2f(a.w4b[wc * 128 + cb * 32 + li]);
    }
    const float om = EPI == EPI_OUT ? a.norm[2 * NIN] : 0.0f;
    const float osd = EPI == EPI_OUT ? a.norm[2 * NIN + 1] : 1.0f;
    for (int64_t tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
        const int64_t row0 = tile * GROWS + wr * 32;
        f32x16 acc[4];
#pragma unroll
        for (int cb = 0; cb < 4; ++cb)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[cb][r] = 0.0f;
        const uint16_t *ap = a.A + (row0 + li) * 16 + lh * 8;
        const uint16_t *bl = sB + (wc * 128 + li) * KPAD + lh * 8;
        // operand fragments are requested eight k steps at a time, so the
        // wave waits for memory twice per tile instead of once per k step
#pragma unroll 1
        for (int k0 = 0; k0 < WID / 16; k0 += 8) {
            bf16x8 fa[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) fa[k] = ld8(ap + (int64_t)(k0 + k) * RP * 16);
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int k = 0; k < 8; ++k) {
#pragma unroll
                for (int cb = 0; cb < 4; ++cb) {
                    const bf16x8 fb = ld8(bl + cb * 32 * KPAD + (k0 + k) * 16);
                    acc[cb] =
                        __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[k], fb, acc[cb], 0, 0, 0);
                }
            }
        }
        // accumulator element (cb, 4g+q): row row0 + 8g + 4lh + q, column
        // wc*128 + cb*32 + li
        if (EPI == EPI_FWD) {
#pragma unroll
            for (int cb = 0; cb < 4; ++cb) {
                const int col = wc * 128 + cb * 32 + li;
                const float bc = a.bias[col];
#pragma unroll
                for (int g = 0; g < 4; ++g) {
                    const int64_t rb = row0 + 8 * g + 4 * lh;
                    float z4[4];
                    uint16_t h4[4];
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        z4[q] = acc[cb][4 * g + q] + bc;
                        h4[q] = f2bf(gelu(z4[q]));
                        a.Hkb[kb_idx(rb + q, col, RP)] = h4[q];
                    }
                    if (TRAIN) {
                        *(float4 *)(a.Zout + fr_idx(rb, col)) =
                            make_float4(z4[0], z4[1], z4[2], z4[3]);
                        if (a.Hrb) *(uint2 *)(a.Hrb + rb_idx(rb, col)) = pack4(h4);
                    }
                }
            }
        } else if (EPI == EPI_BWD) {
#pragma unroll
            for (int cb = 0; cb < 4; ++cb) {
                const int col = wc * 128 + cb * 32 + li;
#pragma unroll
                for (int g = 0; g < 4; ++g) {
                    const int64_t rb = row0 + 8 * g + 4 * lh;
                    const float4 z = *(const float4 *)(a.Zin + fr_idx(rb, col));
                    const float zq[4] = {z.x, z.y, z.z, z.w};
                    uint16_t h4[4];
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        h4[q] = f2bf(acc[cb][4 * g + q] * gelu_prime(zq[q]));
                        a.Hkb[kb_idx(rb + q, col, RP)] = h4[q];
                        csum[cb] += bf2f(h4[q]);
                    }
                    if (a.Hrb) *(uint2 *)(a.Hrb + rb_idx(rb, col)) = pack4(h4);
                }
            }
        } else {
            // this lane's partial dots for its 16 rows; training keeps the
            // bf16 activations packed and overwrites acc with GELU'(z)
            float pd[16];
            uint32_t hb[4][8];
#pragma unroll
            for (int r = 0; r < 16; ++r) pd[r] = 0.0f;
#pragma unroll
            for (int cb = 0; cb < 4; ++cb) {
                const float bc = a.bias[wc * 128 + cb * 32 + li];
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const float z = acc[cb][r] + bc;
                    uint16_t h;
                    if (OUT_TRAIN) {
                        float g, gp;
                        gelu_and_prime(z, g, gp);
                        h = f2bf(g);
                        acc[cb][r] = gp;
                        if (r & 1) hb[cb][r >> 1] |= (uint32_t)h << 16;
                        else hb[cb][r >> 1] = h;
                    } else {
                        h = f2bf(gelu(z));
                    }
                    pd[r] = fmaf(bf2f(h), w4c[cb], pd[r]);
                    // four rows at a time: bounds the live temporaries
                    if ((r & 3) == 3) __builtin_amdgcn_sched_barrier(0);
                }
            }
            // sum over the 32 columns of each half-wave; lanes li == 0 publish
            // their 16 rows, then one thread per row adds the two column
            // waves and forms the prediction or the loss gradient
#pragma unroll
            for (int r = 0; r < 16; ++r) {
#pragma unroll
                for (int o = 1; o < 32; o <<= 1) pd[r] += __shfl_xor(pd[r], o, 64);
            }
            if (li == 0) {
#pragma unroll
                for (int r = 0; r < 16; ++r)
                    sPart[wc][wr * 32 + 8 * (r >> 2) + 4 * lh + (r & 3)] = pd[r];
            }
            __syncthreads();
            if (threadIdx.x < GROWS) {
                const int rl = threadIdx.x;
                const int64_t row = tile * GROWS + rl;
                const float o = sPart[0][rl] + sPart[1][rl] + a.b4[0];
                float d = 0.0f;
                if (row < a.R) {
                    if (a.out_mode == OUT_PREDICT) {
                        a.out[row] = fmaf(o, osd, om);
                    } else if (a.out_mode == OUT_MSE) {
                        const int64_t src = a.idx ? a.idx[row] : row;
                        const float t = (a.target[src] - om) / osd;
                        const float diff = o - t;
                        d = 2.0f * diff / (float)a.R;
                        lacc += (double)diff * (double)diff;
                    } else {
                        d = a.dgiven[row] * osd;
                    }
                }
                sD[rl] = d;
                gb4 += d;
            }
            // second barrier: the next tile's writes of sPart must not
            // overtake these reads, and training reads sD below
            __syncthreads();
            if (OUT_TRAIN) {
#pragma unroll
                for (int cb = 0; cb < 4; ++cb) {
                    const int col = wc * 128 + cb * 32 + li;
#pragma unroll
                    for (int g = 0; g < 4; ++g) {
                        const int64_t rb = row0 + 8 * g + 4 * lh;
                        uint16_t h4[4];
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            const float d = sD[wr * 32 + 8 * g + 4 * lh + q];
                            const int r = 4 * g + q;
                            const uint16_t h = (uint16_t)(hb[cb][r >> 1] >> (16 * (r & 1)));
                            gw4[cb] = fmaf(d, bf2f(h), gw4[cb]);
                            h4[q] = f2bf(d * w4c[cb] * acc[cb][r]);
                            a.Hkb[kb_idx(rb + q, col, RP)] = h4[q];
                            csum[cb] += bf2f(h4[q]);
                        }
                        *(uint2 *)(a.Hrb + rb_idx(rb, col)) = pack4(h4);
                    }
                    __builtin_amdgcn_sched_barrier(0);
                }
            }
        }
    }
    // slot partials of this workgroup: per column, fixed order (lane halves,
    // then the eight row waves)
    const bool want_cols = (EPI == EPI_BWD && a.soff >= 0) || OUT_TRAIN;
    if (!want_cols) return;
    float *ps = a.partS + (int64_t)blockIdx.x * S_N;
    for (int pass = 0; pass < (OUT_TRAIN ? 2 : 1); ++pass) {
        float v[4];
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) {
            v[cb] = pass == 0 ? csum[cb] : gw4[cb];
            v[cb] += __shfl_xor(v[cb], 32, 64);
        }
        __syncthreads();
        if (lh == 0) {
#pragma unroll
            for (int cb = 0; cb < 4; ++cb) sRed[wr][wc * 128 + cb * 32 + li] = v[cb];
        }
        __syncthreads();
        if (threadIdx.x < WID) {
            float s = 0.0f;
            for (int w = 0; w < GW / 2; ++w) s += sRed[w][threadIdx.x];
            ps[(pass == 0 ? (EPI == EPI_OUT ? S_B1 + 2 * WID : a.soff) : S_W4) + threadIdx.x] = s;
        }
    }
    if (OUT_TRAIN) {
        // b4 and loss: threads 0..GROWS-1 hold them (one row each per tile)
        const float b = wsum(gb4);
        double l = lacc;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) l += __shfl_xor(l, o, 64);
        __syncthreads();
        if (lane == 0) {
            sPart[0][wave] = b;
            sLoss[wave] = l;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            float sb = 0.0f;
            double sl = 0.0;
            for (int w = 0; w < GW; ++w) {
                sb += sPart[0][w];
                sl += sLoss[w];
            }
            ps[S_B4] = sb;
            a.lossp[blockIdx.x] = sl;
        }
    }
}

// ---------------------------------------------------------------------------
// weight gradient of a 256x256 layer: dW[k][n] = sum_r H[r][k] dZ[r][n]
// ---------------------------------------------------------------------------
// Grid = chunks x 4 quadrants of 128x128; wave = 64x64 of its quadrant over
// the chunk's 1024 rows. Both operands are row-blocked, so each fragment
// load is 1 KB contiguous. Chunk c of layer l is written at
// part_base + c * 3 * 65536, part_base = partW + (l - 1) * 65536.
__global__ __launch_bounds__(256) void k_mlp_gemm_dw(const uint16_t *__restrict__ Hrb,
                                                     const uint16_t *__restrict__ Drb,
                                                     float *__restrict__ part) {
    const int64_t chunk = blockIdx.x >> 2;
    const int quad = blockIdx.x & 3;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int li = lane & 31, lh = lane >> 5;
    const int k0r = (quad >> 1) * 128 + (wave >> 1) * 64;
    const int n0c = (quad & 1) * 128 + (wave & 1) * 64;
    f32x16 acc[2][2];
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[x][y][r] = 0.0f;
    // rows r0..r0+15 of row block r0/16 start at (r0/16) * 256 * 16
    const uint16_t *pa = Hrb + (chunk * (CHUNK_DW / 16) * WID + k0r + li) * 16 + lh * 8;
    const uint16_t *pb = Drb + (chunk * (CHUNK_DW / 16) * WID + n0c + li) * 16 + lh * 8;
    // one wave per SIMD: the fragments of eight row blocks are requested
    // together, so the wave waits for memory eight times per chunk, not 64
#pragma unroll 1
    for (int rb0 = 0; rb0 < CHUNK_DW / 16; rb0 += 8) {
        bf16x8 fa[8][2], fb[8][2];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int64_t o = (int64_t)(rb0 + u) * WID * 16;
            fa[u][0] = ld8(pa + o);
            fa[u][1] = ld8(pa + o + 32 * 16);
            fb[u][0] = ld8(pb + o);
            fb[u][1] = ld8(pb + o + 32 * 16);
        }
        // keep the scheduler from interleaving the loads with the products
        // (it would trade the batching back for fewer live registers)
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int u = 0; u < 8; ++u)
#pragma unroll
            for (int x = 0; x < 2; ++x)
#pragma unroll
                for (int y = 0; y < 2; ++y)
                    acc[x][y] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[u][x], fb[u][y],
                                                                        acc[x][y], 0, 0, 0);
    }
    float *dst = part + chunk * (int64_t)(3 * WID * WID);
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int k = k0r + x * 32 + 8 * (r >> 2) + 4 * lh + (r & 3);
                const int n = n0c + y * 32 + li;
                dst[k * WID + n] = acc[x][y][r];
            }
}

// input layer gradients: slot partials of dW0[f][n] = sum_r F[r][f] dZ0[r][n]
// and db0, dZ0 k-blocked
__global__ __launch_bounds__(256) void k_mlp_dw0(const float *__restrict__ F,
                                                 const uint16_t *__restrict__ dZ0, int64_t RP,
                                                 float *__restrict__ partS) {
    const int n = threadIdx.x;
    const int64_t base = (int64_t)blockIdx.x * SLOT;
    float g[NIN] = {0, 0, 0, 0, 0, 0}, gb = 0.0f;
    for (int r = 0; r < SLOT; ++r) {
        const float dz = bf2f(dZ0[kb_idx(base + r, n, RP)]);
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

// fixed-order sum of the partials into the flat gradient: hidden weights
// over the row chunks, W0 and b0 over the 256-row slots, the other entries
// over the layer workgroups; thread 0 of block 0 also sums the loss partials
__global__ __launch_bounds__(256) void k_mlp_reduce(const float *__restrict__ partW,
                                                    int64_t n_chunks,
                                                    const float *__restrict__ partS,
                                                    int64_t n_slots, int64_t n_groups,
                                                    const double *__restrict__ lossp, int64_t R,
                                                    float *__restrict__ grad,
                                                    double *__restrict__ loss) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i == 0 && loss) {
        double s = 0.0;
        for (int64_t c = 0; c < n_groups; ++c) s += lossp[c];
        *loss = s / (double)R;
    }
    if (i >= NPAR) return;
    int layer = 0;
    for (int l = 1; l < 4; ++l)
        if (i >= OFF_W[l] && i < OFF_W[l] + WID * WID) layer = l;
    const float *src;
    int64_t stride, count;
    if (layer > 0) {
        src = partW + (int64_t)(layer - 1) * WID * WID + (i - OFF_W[layer]);
        stride = 3 * WID * WID;
        count = n_chunks;
    } else {
        int j;
        if (i < OFF_B0 + WID) j = (int)i;                                   // W0, b0
        else if (i >= OFF_W4) j = S_W4 + (int)(i - OFF_W4);                 // W4, b4
        else {
            int l = 1;
            while (!(i >= OFF_B[l] && i < OFF_B[l] + WID)) ++l;
            j = S_B1 + (l - 1) * WID + (int)(i - OFF_B[l]);
        }
        src = partS + j;
        stride = S_N;
        count = j < S_B1 ? n_slots : n_groups;
    }
    // eight independent sums (c = 8m + u), added in a fixed order
    double s8[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    int64_t c = 0;
    for (; c + 16 <= count; c += 16) {
        // sixteen partials requested together; partial c still goes to
        // sum c % 8, in increasing c
        float v[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) v[u] = src[(c + u) * stride];
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int u = 0; u < 16; ++u) s8[u & 7] += v[u];
    }
    for (; c + 8 <= count; c += 8) {
#pragma unroll
        for (int u = 0; u < 8; ++u) s8[u] += src[(c + u) * stride];
    }
    for (int u = 0; c < count; ++c, ++u) s8[u] += src[c * stride];
    grad[i] = (float)(((s8[0] + s8[1]) + (s8[2] + s8[3])) + ((s8[4] + s8[5]) + (s8[6] + s8[7])));
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
    float *Zf[3] = {nullptr, nullptr, nullptr};         // Z0..Z2, fragment order
    uint16_t *Hkb[3] = {nullptr, nullptr, nullptr};     // H0..H2, k-blocked
    uint16_t *Hrb[3] = {nullptr, nullptr, nullptr};     // H0..H2, row-blocked
    uint16_t *dZkb[2] = {nullptr, nullptr};             // ping-pong, k-blocked
    uint16_t *dZrb = nullptr;                           // row-blocked
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
static unsigned layer_grid(int64_t RP) { return (unsigned)std::min<int64_t>(RP / GROWS, MAX_GRID); }

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
    for (int l = 0; l < 3; ++l) RSOT_TRY(ws_alloc(L, &m->Zf[l], rw));
    for (int l = 0; l < 3; ++l) RSOT_TRY(ws_alloc(L, &m->Hkb[l], rw));
    for (int l = 0; l < 3; ++l) RSOT_TRY(ws_alloc(L, &m->Hrb[l], rw));
    for (int l = 0; l < 2; ++l) RSOT_TRY(ws_alloc(L, &m->dZkb[l], rw));
    RSOT_TRY(ws_alloc(L, &m->dZrb, rw));
    RSOT_TRY(ws_alloc(L, &m->F, (size_t)RP * 8));
    RSOT_TRY(ws_alloc(L, &m->partW, (size_t)(RP / CHUNK_DW) * 3 * WID * WID));
    RSOT_TRY(ws_alloc(L, &m->partS, (size_t)std::max<int64_t>(RP / SLOT, MAX_GRID) * S_N));
    RSOT_TRY(ws_alloc(L, &m->lossp, (size_t)MAX_GRID));
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

static LayerArgs layer_args(rsot_mlp *m, int64_t R, int64_t RP) {
    LayerArgs a{};
    a.R = R;
    a.RP = RP;
    a.soff = -1;
    a.partS = m->partS;
    a.w4b = m->w4b;
    a.b4 = m->P + OFF_B4;
    a.norm = m->norm;
    a.lossp = m->lossp;
    return a;
}

// Forward pass. Prediction writes o * std + mean into `out`; training keeps
// what the backward pass needs and ends with dZ3 in dZkb[0] / dZrb and the
// output-layer partials (out_mode OUT_MSE with target/idx, or OUT_GIVEN with
// dout).
static rsot_status run_forward(rsot_mlp *m, const float *feats, const int64_t *idx, int64_t R,
                               int64_t RP, bool train, int out_mode, const float *target,
                               const float *dout, float *out) {
    const hipStream_t st = m->stream;
    const unsigned gl = layer_grid(RP);
    if (train) {
        hipLaunchKernelGGL(k_mlp_in<true>, dim3((unsigned)(RP / 32)), dim3(512), 0, st, feats,
                           idx, R, RP, m->norm, m->W0b, m->P + OFF_B[0], m->F, m->Zf[0],
                           m->Hkb[0], m->Hrb[0]);
        for (int l = 1; l < 3; ++l) {
            LayerArgs a = layer_args(m, R, RP);
            a.A = m->Hkb[l - 1];
            a.Bt = m->WTb + (size_t)(l - 1) * WID * WID;
            a.bias = m->P + OFF_B[l];
            a.Zout = m->Zf[l];
            a.Hkb = m->Hkb[l];
            a.Hrb = m->Hrb[l];
            hipLaunchKernelGGL((k_mlp_layer<EPI_FWD, true>), dim3(gl), dim3(GW * 64), 0, st, a);
        }
        LayerArgs a = layer_args(m, R, RP);
        a.A = m->Hkb[2];
        a.Bt = m->WTb + (size_t)2 * WID * WID;
        a.bias = m->P + OFF_B[3];
        a.Hkb = m->dZkb[0];
        a.Hrb = m->dZrb;
        a.target = target;
        a.dgiven = dout;
        a.idx = idx;
        a.out_mode = out_mode;
        hipLaunchKernelGGL((k_mlp_layer<EPI_OUT, true>), dim3(gl), dim3(GW * 64), 0, st, a);
    } else {
        hipLaunchKernelGGL(k_mlp_in<false>, dim3((unsigned)(RP / 32)), dim3(512), 0, st, feats,
                           idx, R, RP, m->norm, m->W0b, m->P + OFF_B[0], (float *)nullptr,
                           (float *)nullptr, m->Hi[0], (uint16_t *)nullptr);
        for (int l = 1; l < 3; ++l) {
            LayerArgs a = layer_args(m, R, RP);
            a.A = m->Hi[(l - 1) & 1];
            a.Bt = m->WTb + (size_t)(l - 1) * WID * WID;
            a.bias = m->P + OFF_B[l];
            a.Hkb = m->Hi[l & 1];
            hipLaunchKernelGGL((k_mlp_layer<EPI_FWD, false>), dim3(gl), dim3(GW * 64), 0, st, a);
        }
        LayerArgs a = layer_args(m, R, RP);
        a.A = m->Hi[0];
        a.Bt = m->WTb + (size_t)2 * WID * WID;
        a.bias = m->P + OFF_B[3];
        a.out_mode = OUT_PREDICT;
        a.out = out;
        hipLaunchKernelGGL((k_mlp_layer<EPI_OUT, false>), dim3(gl), dim3(GW * 64), 0, st, a);
    }
    return hipGetLastError() == hipSuccess ? RSOT_OK : RSOT_ERR_DEVICE;
}

// backward from dZ3 (dZkb[0], dZrb) to the flat gradient `grad` (device)
static rsot_status run_backward(rsot_mlp *m, int64_t R, int64_t RP, float *grad,
                                double *loss_dev) {
    const hipStream_t st = m->stream;
    const int64_t n_chunks = RP / CHUNK_DW, n_slots = RP / SLOT;
    const unsigned gl = layer_grid(RP);
    int cur = 0;
    for (int l = 3; l >= 1; --l) {
        // dW_l from H_{l-1} and dZ_l (row-blocked)
        hipLaunchKernelGGL(k_mlp_gemm_dw, dim3((unsigned)(n_chunks * 4)), dim3(256), 0, st,
                           m->Hrb[l - 1], m->dZrb, m->partW + (size_t)(l - 1) * WID * WID);
        // dZ_{l-1} = bf16((dZ_l W_l^T) * GELU'(Z_{l-1})); W_l as [k][n] is Bt here
        LayerArgs a = layer_args(m, R, RP);
        a.A = m->dZkb[cur];
        a.Bt = m->Wb + (size_t)(l - 1) * WID * WID;
        a.Zin = m->Zf[l - 1];
        a.Hkb = m->dZkb[cur ^ 1];
        a.Hrb = l - 1 >= 1 ? m->dZrb : nullptr;
        a.soff = l - 1 >= 1 ? S_B1 + (l - 2) * WID : -1;
        hipLaunchKernelGGL((k_mlp_layer<EPI_BWD, true>), dim3(gl), dim3(GW * 64), 0, st, a);
        cur ^= 1;
    }
    hipLaunchKernelGGL(k_mlp_dw0, dim3((unsigned)n_slots), dim3(256), 0, st, m->F, m->dZkb[cur],
                       RP, m->partS);
    hipLaunchKernelGGL(k_mlp_reduce, dim3((unsigned)((NPAR + 255) / 256)), dim3(256), 0, st,
                       m->partW, n_chunks, m->partS, n_slots, (int64_t)gl, m->lossp, R, grad,
                       loss_dev);
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
    RSOT_TRY(run_forward(m, feats, nullptr, rows, RP, false, OUT_PREDICT, nullptr, nullptr, out));
    RSOT_HIP(hipStreamSynchronize(m->stream));
    return RSOT_OK;
}

// prediction of `rows` feature rows into m->outb (no synchronisation)
static rsot_status predict_rows(rsot_mlp *m, const float *feats, int64_t rows) {
    const int64_t RP = padded_rows(rows);
    RSOT_TRY(ensure_inf_ws(m, RP));
    return run_forward(m, feats, nullptr, rows, RP, false, OUT_PREDICT, nullptr, nullptr,
                       m->outb);
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
    RSOT_TRY(run_forward(m, feats, nullptr, rows, RP, true, OUT_GIVEN, nullptr, dout, nullptr));
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
    RSOT_TRY(run_forward(m, feats, idx, rows, RP, true, OUT_MSE, target, nullptr, nullptr));
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
    if (sp->resume) return RSOT_ERR_INVALID_ARG;   // the start is the network's, not a checkpoint
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
        one.absJ_start = std::fabs(li.J_pred);   // J at the start was just evaluated
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
