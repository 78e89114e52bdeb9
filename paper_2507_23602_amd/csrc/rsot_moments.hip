// Moments and maps of the entropic plan pi_qj = mu_q p_qj(psi) (Secs. 6.2, 6.3).
//
// Target side (Sec. 6.2): for every target its mass nu~_j = sum_q mu_q p_qj
// and first moment sum_q mu_q p_qj x_q; the conditional barycentre of
// Eq. barycenter_fixed_point is first_j / nu_j, and Danskin's gradient of the
// transport cost in y_j (Eq. barycenter_gradient_general) is
// 2 cs (nu~_j y_j - first_j). The kernel is the gradient pass with d more
// sums per lane: it forms the same weights w_qj from the same arguments and
// the same per-pair cutoff test, and sums w_qj (x_q - y_j) (offsets, small and
// free of the coordinates' magnitude) in FP32 per tile, scaled back to FP64
// with the tile reference; first_j = sum w (x_q - y_j) + nu~_j y_j.
//
// Point side (Sec. 6.3): for every quadrature point the barycentric map
// sum_j p_qj y_j (Eq. barycentric_map_registration) and the modal target
// argmax_j (psi_j - c_qj + eps ln nu_j) (Eq. modal_map_registration), over
// the pairs the evaluation kept. One wavefront per point tile walks the
// tile's kept target blocks (with the objective pass's chunk classes under
// the cutoff rules); p_qj = 2^(t_j - Lt_q) with Lt_q from the evaluation, the
// offsets y_j - x_q summed in FP32 per block, the argmax taken on the FP64
// exponents t_j (the decision is made in FP64, like the oracle's).
#include <algorithm>
#include <cmath>
#include <type_traits>

#include "rsot_device.h"
#include "rsot_internal.h"
#include "rsot_pairs.h"

namespace {

template <typename T>
rsot_status grow_buf(rsot_problem *p, T **ptr, size_t *cap, size_t count) {
    if (*ptr && *cap >= count) return RSOT_OK;
    if (*ptr) rsot_dev_free(p, *ptr);
    *ptr = nullptr;
    void *q = nullptr;
    const size_t c = std::max<size_t>(count + count / 4, 64);
    RSOT_TRY(rsot_dev_alloc(p, &q, c * sizeof(T)));
    *ptr = (T *)q;
    *cap = c;
    return RSOT_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// target side
// ---------------------------------------------------------------------------
// One tile of 64 points into this lane's offset sums a[k] += w (x_q[k] - y[k]).
// MASK: every pair takes the cutoff test (the tile straddles the cutoff).
template <int D, bool F64, bool MASK, typename QP, typename AP>
__device__ __forceinline__ void moment_tile(QP Q, AP qA, const double4 &rec, double G,
                                            const double *yv, double scale, double *a) {
    using Acc = typename std::conditional<F64, double, float>::type;
    Acc c[3] = {0, 0, 0};
    Acc ys[3];
#pragma unroll
    for (int k = 0; k < D; ++k) ys[k] = (Acc)yv[k];
    for (int i0 = 0; i0 < 64; i0 += CH) {
#pragma unroll
        for (int k = 0; k < CH; ++k) {
            const double4 r = ld4(Q + i0 + k);
            double v;
            bool in = true;
            if (MASK) {
                const double t = pair_exp<D>(r.x, r.y, r.z, rec);
                in = t > G - qA[i0 + k];
                v = t + r.w;
            } else {
                v = rec.w + r.w;
                v = fma(r.x, rec.x, v);
                v = fma(r.y, rec.y, v);
                if (D == 3) v = fma(r.z, rec.z, v);
            }
            Acc w;
            if (F64) w = in ? exp2(v) : 0.0;
            else w = __builtin_amdgcn_exp2f(in ? (float)v : -INFINITY);
            const double xr[3] = {r.x, r.y, r.z};
#pragma unroll
            for (int d = 0; d < D; ++d) c[d] = fma(w, (Acc)xr[d] - ys[d], c[d]);
        }
    }
#pragma unroll
    for (int d = 0; d < D; ++d) a[d] += (double)c[d] * scale;
}

template <int D, bool F64, int MODE>
__global__ __launch_bounds__(256) void k_moments(
    const double4 *__restrict__ qp, const double *__restrict__ qA,
    const double2 *__restrict__ tref, const double4 *__restrict__ trec,
    const double *__restrict__ ty, const double *__restrict__ tG,
    const int32_t *__restrict__ wi_block, const int64_t *__restrict__ wi_range,
    const int32_t *__restrict__ perm, const uint32_t *__restrict__ col_idx,
    const uint8_t *__restrict__ col_cm, int64_t n_tiles, int64_t n_blocks, int64_t n_wi,
    int64_t n_seg, int64_t seg, double *__restrict__ mpart) {
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    int64_t b, w, e0, e1;
    if (MODE == MODE_DENSE) {
        // the gradient pass's layout: each XCD sweeps its own point segments
        const int64_t nbg = (n_blocks + 3) / 4;
        const int64_t kk = blockIdx.x >> 3;
        const int64_t sgi = (kk / nbg) * 8 + (blockIdx.x & 7);
        b = (kk % nbg) * 4 + wave;
        if (sgi >= n_seg || b >= n_blocks) return;
        e0 = sgi * seg;
        e1 = std::min<int64_t>(e0 + seg, n_tiles);
        w = b * n_seg + sgi;
    } else {
        const int64_t k = xcd_run_item(wave);
        if (k >= n_wi) return;
        w = perm[k];
        b = wi_block[w];
        e0 = wi_range[2 * w];
        e1 = wi_range[2 * w + 1];
    }
    const int64_t j = b * 64 + lane;
    const double4 rec = trec[j];
    const double G = MODE == MODE_MASK ? tG[j] : 0.0;
    const double yv[3] = {ty[j * 3 + 0], ty[j * 3 + 1], ty[j * 3 + 2]};
    double a[3] = {0.0, 0.0, 0.0};
    for (int64_t e = e0; e < e1; ++e) {
        const uint32_t ent = MODE == MODE_DENSE ? (uint32_t)e : col_idx[e];
        const int64_t t = ent & ~RSOT_PARTIAL_BIT;
        const double scale = tref[t].y;
        if (MODE == MODE_MASK && (ent & RSOT_PARTIAL_BIT)) {
            moment_tile<D, F64, true>(qp + t * 64, qA + t * 64, rec, G, yv, scale, a);
        } else if (MODE == MODE_LIST && (ent & RSOT_PARTIAL_BIT)) {
            // tile rule with culling groups: this lane's chunk may be dropped
            const bool on = (col_cm[e] >> (lane >> 3)) & 1u;
            const double4 rl = make_double4(rec.x, rec.y, rec.z, on ? rec.w : -INFINITY);
            moment_tile<D, F64, false>(qp + t * 64, qA, rl, G, yv, scale, a);
        } else {
            moment_tile<D, F64, false>(qp + t * 64, qA, rec, G, yv, scale, a);
        }
    }
#pragma unroll
    for (int d = 0; d < D; ++d) mpart[(w * 64 + lane) * D + d] = a[d];
}

// per target: the items' offset sums in order, then first_j in the caller's
// coordinates and order: first = sum w (x - y) + nu~_j (y + shift)
template <int D>
__global__ __launch_bounds__(256) void k_moment_reduce(
    const double *__restrict__ mpart, const int64_t *__restrict__ wi_ptr, int64_t n_seg,
    const double *__restrict__ ty, const double *__restrict__ tnu,
    const int32_t *__restrict__ tperm, const double *__restrict__ grad, int64_t n_blocks,
    double s0, double s1, double s2, double *__restrict__ mass_out,
    double *__restrict__ first_out) {
    const int lane = threadIdx.x & 63;
    const int64_t b = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (b >= n_blocks) return;
    const int64_t j = b * 64 + lane;
    const int32_t dst = tperm[j];
    if (dst < 0) return;
    const int64_t w0 = wi_ptr ? wi_ptr[b] : b * n_seg;
    const int64_t w1 = wi_ptr ? wi_ptr[b + 1] : w0 + n_seg;
    double a[3] = {0.0, 0.0, 0.0};
    for (int64_t w = w0; w < w1; ++w)
#pragma unroll
        for (int d = 0; d < D; ++d) a[d] += mpart[(w * 64 + lane) * D + d];
    const double nut = grad[dst] + tnu[j];
    const double sh[3] = {s0, s1, s2};
    if (mass_out) mass_out[dst] = nut;
    if (first_out)
#pragma unroll
        for (int d = 0; d < D; ++d) first_out[(int64_t)dst * D + d] = a[d] + nut * (ty[j * 3 + d] + sh[d]);
}

// ---------------------------------------------------------------------------
// point side
// ---------------------------------------------------------------------------
// One block of 64 targets into this lane's sums: sw = sum w, sy[k] = sum w
// (y_j[k] - x[k]), w = 2^(t_j - Lt); and the running FP64 argmax of t_j.
// CLS: 0 skipped chunk, 1 pairs tested against the cutoff, 2 all pairs kept.
// The FP32 path reads the targets' FP32 copy Yf, the FP64 path their FP64
// coordinates Yd (3 per target).
template <int D, bool F64, typename RP, typename GP, typename YP>
__device__ __forceinline__ void map_chunk(RP T, int k0, GP G, YP Yf, const double *Yd, int cls,
                                          double x0, double x1, double x2, double A, double Lt,
                                          int64_t jbase, double &sw, double *sy, double &best,
                                          int64_t &bj) {
    using Acc = typename std::conditional<F64, double, float>::type;
    const Acc xs[3] = {(Acc)x0, (Acc)x1, (Acc)x2};
    Acc cw = 0, cy[3] = {0, 0, 0};
#pragma unroll
    for (int k = 0; k < CH; ++k) {
        const double t = pair_exp<D>(x0, x1, x2, trec_at<D>(T, k0 + k));
        const bool in = cls == PAIR_FULL || t > G[k0 + k] - A;
        Acc w;
        if (F64) w = in ? exp2(t - Lt) : 0.0;
        else w = __builtin_amdgcn_exp2f(in ? (float)(t - Lt) : -INFINITY);
        cw += w;
        Acc yy[3];
        if constexpr (F64) {
#pragma unroll
            for (int d = 0; d < 3; ++d) yy[d] = Yd[(k0 + k) * 3 + d];
        } else {
            const float4 yk = Yf[k0 + k];
            yy[0] = yk.x;
            yy[1] = yk.y;
            yy[2] = yk.z;
        }
#pragma unroll
        for (int d = 0; d < D; ++d) cy[d] = fma(w, yy[d] - xs[d], cy[d]);
        if (in && t > best) {
            best = t;
            bj = jbase + k0 + k;
        }
    }
    sw += (double)cw;
#pragma unroll
    for (int d = 0; d < D; ++d) sy[d] += (double)cy[d];
}

// The FP32 path of map_chunk. Yc holds the targets' coordinates relative to
// their block's centre c_B (FP32), so a pair adds w (y_j - c_B) with one FMA
// per coordinate and the caller subtracts (x_q - c_B) times the block's
// weight wB in FP64; the offsets stay of the block's size. The modal target
// takes the chunk's largest FP64 exponent first and looks up its index only
// when it beats the running best: the first target reaching it, as a pair-
// by-pair strict comparison finds. FULL: every pair of the chunk is kept.
template <int D, bool FULL, typename RP, typename GP>
__device__ __forceinline__ void map_chunk32(RP T, int k0, GP G, const float4 *__restrict__ Yc,
                                            double x0, double x1, double x2, double A,
                                            double Lt, int64_t jbase, double &wB, double *sy,
                                            double &best, int64_t &bj) {
    float cw = 0.0f, cy[3] = {0.0f, 0.0f, 0.0f};
    double tv[CH];
    double cmax = -INFINITY;
#pragma unroll
    for (int k = 0; k < CH; ++k) {
        const double t = pair_exp<D>(x0, x1, x2, trec_at<D>(T, k0 + k));
        const bool in = FULL || t > G[k0 + k] - A;
        tv[k] = in ? t : -INFINITY;
        cmax = fmax(cmax, tv[k]);
        const float w = __builtin_amdgcn_exp2f(in ? (float)(t - Lt) : -INFINITY);
        const float4 yk = Yc[k0 + k];
        const float yy[3] = {yk.x, yk.y, yk.z};
        cw = k == 0 ? w : cw + w;
#pragma unroll
        for (int d = 0; d < D; ++d) cy[d] = k == 0 ? w * yy[d] : fmaf(w, yy[d], cy[d]);
    }
    wB += (double)cw;
#pragma unroll
    for (int d = 0; d < D; ++d) sy[d] += (double)cy[d];
    if (cmax > best) {
        best = cmax;
#pragma unroll
        for (int k = CH - 1; k >= 0; --k)
            if (tv[k] == cmax) bj = jbase + k0 + k;
    }
}

template <int D, bool F64, int MODE>
__global__ __launch_bounds__(256) void k_maps(
    const double4 *__restrict__ qp, const double *__restrict__ qlse,
    const int32_t *__restrict__ qperm, const double4 *__restrict__ trec,
    const double *__restrict__ trec3, const double *__restrict__ tG,
    const float4 *__restrict__ tyf, const double *__restrict__ ty,
    const int32_t *__restrict__ tperm, const int64_t *__restrict__ row_ptr,
    const uint32_t *__restrict__ row_idx, const uint16_t *__restrict__ row_cm,
    const double *__restrict__ blk_lo, const double *__restrict__ blk_hi, int64_t n_tiles,
    int64_t n_blocks, double kcs, double s0, double s1, double s2,
    double *__restrict__ bary_out, int32_t *__restrict__ modal_out) {
    const int lane = threadIdx.x & 63;
    const int64_t t = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (t >= n_tiles) return;
    const int64_t q = t * 64 + lane;
    const double4 xr = qp[q];
    const double x0 = xr.x, x1 = xr.y, x2 = D == 3 ? xr.z : 0.0;
    const double A = -kcs * (x0 * x0 + x1 * x1 + x2 * x2);
    const double L = qlse[q];
    const double Lt = L * RSOT_LOG2E - A;
    double sw = 0.0, sy[3] = {0.0, 0.0, 0.0}, best = -INFINITY;
    int64_t bj = -1;
    const int64_t e0 = MODE == MODE_DENSE ? 0 : row_ptr[t];
    const int64_t e1 = MODE == MODE_DENSE ? n_blocks : row_ptr[t + 1];
    for (int64_t e = e0; e < e1; ++e) {
        const uint32_t ent = MODE == MODE_DENSE ? (uint32_t)e : row_idx[e];
        const int64_t b = ent & ~RSOT_PARTIAL_BIT;
        // chunk classes: cutoff rules as the objective pass (FP64: every
        // chunk of a straddling block tested); tile rule with groups: the
        // kept chunks whole
        uint32_t cm = 0xAAAAu;
        if (MODE == MODE_MASK && (ent & RSOT_PARTIAL_BIT)) cm = F64 ? 0x5555u : (uint32_t)row_cm[e];
        else if (MODE == MODE_LIST && (ent & RSOT_PARTIAL_BIT)) cm = row_cm[e];
        auto block = [&](auto T) {
            if constexpr (F64) {
                for (int c = 0; c < 8; ++c) {
                    const int cls = (int)((cm >> (2 * c)) & 3u);
                    if (cls == PAIR_SKIP) continue;
                    map_chunk<D, F64>(T, 8 * c, tG + b * 64, tyf + b * 64, ty + b * 64 * 3, cls,
                                      x0, x1, x2, A, Lt, b * 64, sw, sy, best, bj);
                }
            } else {
                double wB = 0.0;
                for (int c = 0; c < 8; ++c) {
                    const int cls = (int)((cm >> (2 * c)) & 3u);
                    if (cls == PAIR_SKIP) continue;
                    if (cls == PAIR_FULL)
                        map_chunk32<D, true>(T, 8 * c, tG + b * 64, tyf + b * 64, x0, x1, x2, A,
                                             Lt, b * 64, wB, sy, best, bj);
                    else
                        map_chunk32<D, false>(T, 8 * c, tG + b * 64, tyf + b * 64, x0, x1, x2, A,
                                              Lt, b * 64, wB, sy, best, bj);
                }
                const double xq[3] = {x0, x1, x2};
#pragma unroll
                for (int d = 0; d < D; ++d)
                    sy[d] = fma(-(xq[d] - 0.5 * (blk_lo[b * 3 + d] + blk_hi[b * 3 + d])), wB,
                                sy[d]);
                sw += wB;
            }
        };
        if constexpr (D == 3) block(trec + b * 64);
        else block(trec3 + b * 192);
    }
    const int32_t dst = qperm[q];
    if (dst < 0) return;
    const bool empty = !(L > -INFINITY) || !(sw > 0.0);
    const double xs[3] = {x0 + s0, x1 + s1, x2 + s2};
    if (bary_out)
#pragma unroll
        for (int d = 0; d < D; ++d)
            bary_out[(int64_t)dst * D + d] = empty ? NAN : xs[d] + sy[d] / sw;
    if (modal_out) modal_out[dst] = bj >= 0 ? tperm[bj] : -1;
}

// FP32 target coordinates relative to the centre of their block's box (the
// transport maps' offsets; 0 in the third slot for 2D)
__global__ void k_target_f32(const double *__restrict__ ty, const double *__restrict__ blk_lo,
                             const double *__restrict__ blk_hi, int dim, int64_t n_pad,
                             float4 *__restrict__ tyf) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n_pad) return;
    const int64_t b = j / 64;
    float c[3] = {0.0f, 0.0f, 0.0f};
    for (int d = 0; d < dim; ++d)
        c[d] = (float)(ty[j * 3 + d] - 0.5 * (blk_lo[b * 3 + d] + blk_hi[b * 3 + d]));
    tyf[j] = make_float4(c[0], c[1], c[2], 0.0f);
}

// ---------------------------------------------------------------------------
// ABI
// ---------------------------------------------------------------------------
namespace {

template <int D, bool F64>
void launch_moments(rsot_problem *p, int mode) {
    const int64_t n_wi = p->last_n_wi, n_seg = p->last_n_seg, seg = p->last_seg;
    unsigned grid;
    if (mode == MODE_DENSE) grid = (unsigned)(((p->n_blocks + 3) / 4) * ((n_seg + 7) / 8) * 8);
    else grid = xcd_run_grid(n_wi);
#define RSOT_MOM(M)                                                                            \
    hipLaunchKernelGGL((k_moments<D, F64, M>), dim3(grid), dim3(256), 0, p->stream, p->qp,      \
                       p->qA, p->tile_ref, p->trec, p->ty, p->tG, p->wi_block, p->wi_range,     \
                       p->wi_perm, p->col_idx, p->col_cm, p->n_tiles, p->n_blocks, n_wi, n_seg,  \
                       seg, p->mpart)
    if (mode == MODE_DENSE) RSOT_MOM(MODE_DENSE);
    else if (mode == MODE_LIST) RSOT_MOM(MODE_LIST);
    else RSOT_MOM(MODE_MASK);
#undef RSOT_MOM
}

template <int D, bool F64>
void launch_maps(rsot_problem *p, int mode, double *bary, int32_t *modal) {
    const dim3 g((unsigned)((p->n_tiles + 3) / 4));
#define RSOT_MAP(M)                                                                            \
    hipLaunchKernelGGL((k_maps<D, F64, M>), g, dim3(256), 0, p->stream, p->qp, p->qlse,         \
                       p->qperm, p->trec, p->trec3, p->tG, (const float4 *)p->tyf, p->ty,       \
                       p->tperm, p->row_ptr, p->row_idx, p->row_cm, p->blk_lo, p->blk_hi,       \
                       p->n_tiles, p->n_blocks,                                                 \
                       p->last_kcs, p->shift[0], p->shift[1], p->shift[2], bary, modal)
    if (mode == MODE_DENSE) RSOT_MAP(MODE_DENSE);
    else if (mode == MODE_LIST) RSOT_MAP(MODE_LIST);
    else RSOT_MAP(MODE_MASK);
#undef RSOT_MAP
}

}  // namespace

extern "C" rsot_status rsot_plan_moments(rsot_problem *p, double eps, const double *psi,
                                         double *mass_out, double *first_out,
                                         rsot_eval_info *info, double *kernel_ms) {
    if (!p || !psi || (!mass_out && !first_out)) return RSOT_ERR_INVALID_ARG;
    if (p->opt.cost_kind != RSOT_COST_SQEUCLID) return RSOT_ERR_INVALID_ARG;
    if (!(eps > 0.0) || !std::isfinite(eps)) return RSOT_ERR_INVALID_ARG;
    double J = 0.0;
    RSOT_TRY(rsot_eval_impl(p, eps, psi, &J, p->dgrad, info));
    const int D = p->dim, mode = p->last_mode;
    const bool f64 = rsot_pairs_fp64(p);
    RSOT_TRY(grow_buf(p, &p->mpart, &p->mpart_cap,
                      (size_t)std::max<int64_t>(p->last_n_wi, 1) * 64 * (size_t)D));
    RSOT_HIP(hipEventRecord(p->ev0, p->stream));
    if (D == 2) {
        if (f64) launch_moments<2, true>(p, mode);
        else launch_moments<2, false>(p, mode);
    } else {
        if (f64) launch_moments<3, true>(p, mode);
        else launch_moments<3, false>(p, mode);
    }
    const dim3 gblk((unsigned)((p->n_blocks + 3) / 4));
    const int64_t *wptr = mode == MODE_DENSE ? nullptr : p->wi_ptr;
    if (D == 2)
        hipLaunchKernelGGL(k_moment_reduce<2>, gblk, dim3(256), 0, p->stream, p->mpart, wptr,
                           p->last_n_seg, p->ty, p->tnu, p->tperm, p->dgrad, p->n_blocks,
                           p->shift[0], p->shift[1], p->shift[2], mass_out, first_out);
    else
        hipLaunchKernelGGL(k_moment_reduce<3>, gblk, dim3(256), 0, p->stream, p->mpart, wptr,
                           p->last_n_seg, p->ty, p->tnu, p->tperm, p->dgrad, p->n_blocks,
                           p->shift[0], p->shift[1], p->shift[2], mass_out, first_out);
    RSOT_HIP(hipGetLastError());
    RSOT_HIP(hipEventRecord(p->ev1, p->stream));
    RSOT_HIP(hipStreamSynchronize(p->stream));
    if (kernel_ms) {
        float ms = 0.0f;
        RSOT_HIP(hipEventElapsedTime(&ms, p->ev0, p->ev1));
        *kernel_ms = ms;
    }
    return RSOT_OK;
}

extern "C" rsot_status rsot_transport_maps(rsot_problem *p, double eps, const double *psi,
                                           double *bary_out, int32_t *modal_out,
                                           rsot_eval_info *info, double *kernel_ms) {
    if (!p || !psi || (!bary_out && !modal_out)) return RSOT_ERR_INVALID_ARG;
    if (p->opt.cost_kind != RSOT_COST_SQEUCLID) return RSOT_ERR_INVALID_ARG;
    if (!(eps > 0.0) || !std::isfinite(eps)) return RSOT_ERR_INVALID_ARG;
    if (!p->tyf) {
        RSOT_TRY(rsot_dev_alloc(p, (void **)&p->tyf, sizeof(float) * 4 * (size_t)p->n_pad));
        hipLaunchKernelGGL(k_target_f32, dim3((unsigned)((p->n_pad + 255) / 256)), dim3(256), 0,
                           p->stream, p->ty, p->blk_lo, p->blk_hi, p->dim, p->n_pad,
                           (float4 *)p->tyf);
        RSOT_HIP(hipGetLastError());
    }
    double J = 0.0;
    RSOT_TRY(rsot_eval_impl(p, eps, psi, &J, nullptr, info));
    const int D = p->dim, mode = p->last_mode;
    const bool f64 = rsot_pairs_fp64(p);
    RSOT_HIP(hipEventRecord(p->ev0, p->stream));
    if (D == 2) {
        if (f64) launch_maps<2, true>(p, mode, bary_out, modal_out);
        else launch_maps<2, false>(p, mode, bary_out, modal_out);
    } else {
        if (f64) launch_maps<3, true>(p, mode, bary_out, modal_out);
        else launch_maps<3, false>(p, mode, bary_out, modal_out);
    }
    RSOT_HIP(hipGetLastError());
    RSOT_HIP(hipEventRecord(p->ev1, p->stream));
    RSOT_HIP(hipStreamSynchronize(p->stream));
    if (kernel_ms) {
        float ms = 0.0f;
        RSOT_HIP(hipEventElapsedTime(&ms, p->ev0, p->ev1));
        *kernel_ms = ms;
    }
    return RSOT_OK;
}
