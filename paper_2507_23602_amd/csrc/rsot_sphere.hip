// The squared geodesic cost on the unit sphere (Sec. 6.4): the evaluation
// passes and the Riemannian barycentre step of Alg. 5.
//
// c(x, y) = cost_scale d_g(x, y)^2 with d_g the great-circle distance of
// unit vectors. The pair exponent is no longer affine in x, so each pair
// forms its squared chord s = 2 - 2 x.y (three FMAs from a lane vector
// scaled by -2; acos(t)^2 = g(2 - 2t) exactly) and d_g^2 = g(s) = s F(s) by
// a polynomial in s (F analytic for |s| < 4; degree 14 where the exponential
// is FP32, 18 where it is FP64) whose coefficients arrive pre-scaled by
// -kcs, so that z2 = B + s F'(s) is one more FMA. On the far hemisphere
// (s > 2) the antipode's squared chord u = 4 - s gives the distance
// d' = sqrt(g(u)) to -y and d_g = pi - d'. Then
//   z2_qj = B_j - kcs d_g^2,  B_j = kappa psi_j + log2 nu_j,  kcs = kappa cs
// (kappa = log2(e) / eps) in FP64. Since F >= 1 on [0, 4], B - kcs s bounds
// z2 from above: a pair whose bound lies more than 160 below the running
// maximum (objective pass) or below -160 (gradient-side passes, whose
// exponents are already normalised) has an exponential that is zero in FP32
// and below any FP64 rounding of its sum, and skips the polynomial. The same
// bound over a whole target block (objective pass: kappa max psi + log2 nu(B)
// at the least squared distance from the point to the block's box) or point
// tile (gradient side: B_j + max S' at the least squared distance from the
// target to the tile's box) skips the block or tile.
// The exponentials and their chunk sums run
// in FP32 (mixed) or FP64 as in the squared Euclidean passes, with the same
// work items, partials and merges. Target records hold {y_j, B_j}; point
// records {x_q, S'_q} with S'_q from the objective pass's merge (run with a
// zero point term, since the cost has no |x|^2 part).
#include <algorithm>
#include <cmath>
#include <type_traits>

#include "rsot_device.h"
#include "rsot_geo_poly.h"
#include "rsot_internal.h"
#include "rsot_pairs.h"

namespace {

// F(v) coefficients scaled by -kcs (degree 18 for the FP64 loop, 14 for the
// FP32-exponential loop), -1 / kcs and kcs; passed by value so that they sit
// in scalar registers
struct GeoPoly {
    double c[RSOT_GEO_DEG18 + 1];
    double neg_inv_kcs, kcs;
};

template <bool F64>
__device__ __forceinline__ double geo_F(const GeoPoly &P, double v) {
    constexpr int N = F64 ? RSOT_GEO_DEG18 : RSOT_GEO_DEG14;
    double f = P.c[N];
#pragma unroll
    for (int i = N - 1; i >= 0; --i) f = fma(f, v, P.c[i]);
    return f;
}

// -2 x.y + 2 for a lane vector xm = -2 x and unit y
__device__ __forceinline__ double chord2(const double *xm, double y0, double y1, double y2) {
    return fma(xm[0], y0, fma(xm[1], y1, fma(xm[2], y2, 2.0)));
}

// B - kcs d_g^2 for the squared chord s
template <bool F64>
__device__ __forceinline__ double sphere_z(const GeoPoly &P, double s, double B) {
    if (s <= 2.0) return fma(s, geo_F<F64>(P, s), B);
    const double u = fmax(4.0 - s, 0.0);
    const double g = u * geo_F<F64>(P, u) * P.neg_inv_kcs;
    double dp;
    if (F64) {
        dp = sqrt(g);
    } else {
        // FP32 reciprocal square root, one FP64 Newton step (relative error
        // about the square of the FP32 one)
        const double r = (double)__builtin_amdgcn_rsqf(fmaxf((float)g, 1e-30f));
        const double y = g * r;
        dp = fma(0.5 * r, fma(-y, y, g), y);
    }
    const double t = M_PI - dp;
    return fma(-P.kcs * t, t, B);
}

// H(v) = theta / sin(theta) of the logarithmic map (degree 20 for the FP64
// loop, 16 for the FP32-exponential loop), unscaled
struct LogPoly {
    double c[RSOT_LOGMAP_DEG20 + 1];
};

// theta / sin(theta) for the squared chord s of x and y: the polynomial on
// the near hemisphere; on the far one theta = pi - d' (d' from the antipode's
// chord u = 4 - s) over sin(theta) = sqrt(s u) / 2, and 0 at the antipode
// itself, where the logarithmic map is undefined
template <bool F64>
__device__ __forceinline__ double theta_over_sin(const GeoPoly &P, const LogPoly &H, double s) {
    if (s <= 2.0) {
        constexpr int N = F64 ? RSOT_LOGMAP_DEG20 : RSOT_LOGMAP_DEG16;
        double f = H.c[N];
#pragma unroll
        for (int i = N - 1; i >= 0; --i) f = fma(f, s, H.c[i]);
        return f;
    }
    const double u = fmax(4.0 - s, 0.0);
    if (!(u > 1e-300)) return 0.0;
    const double th = M_PI - sqrt(u * geo_F<F64>(P, u) * P.neg_inv_kcs);
    return 2.0 * th / sqrt(s * u);
}

LogPoly log_poly(bool f64) {
    LogPoly H{};
    const int n = f64 ? RSOT_LOGMAP_DEG20 : RSOT_LOGMAP_DEG16;
    for (int i = 0; i <= n; ++i) H.c[i] = f64 ? rsot_logmap_poly20[i] : rsot_logmap_poly16[i];
    return H;
}

// least squared distance from the point (x0, x1, x2) to the box [lo, hi]
__device__ __forceinline__ double box_dist2(const double *__restrict__ lo,
                                            const double *__restrict__ hi, double x0, double x1,
                                            double x2) {
    const double g0 = fmax(fmax(lo[0] - x0, x0 - hi[0]), 0.0);
    const double g1 = fmax(fmax(lo[1] - x1, x1 - hi[1]), 0.0);
    const double g2 = fmax(fmax(lo[2] - x2, x2 - hi[2]), 0.0);
    return fma(g0, g0, fma(g1, g1, g2 * g2));
}

GeoPoly geo_poly(bool f64, double kcs) {
    GeoPoly P{};
    const int n = f64 ? RSOT_GEO_DEG18 : RSOT_GEO_DEG14;
    for (int i = 0; i <= n; ++i) P.c[i] = -kcs * (f64 ? rsot_geo_poly18[i] : rsot_geo_poly14[i]);
    P.neg_inv_kcs = -1.0 / kcs;
    P.kcs = kcs;
    return P;
}

// target records for the sphere: {y_j, kappa psi_j + log2 nu_j}
__global__ void k_sphere_records(const double *__restrict__ ty, const double *__restrict__ tpsi,
                                 const double *__restrict__ tlog2nu,
                                 const int32_t *__restrict__ tperm, int64_t n_pad, double kappa,
                                 double4 *__restrict__ trec) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n_pad) return;
    const bool real = tperm[j] >= 0;
    trec[j] = make_double4(ty[j * 3], ty[j * 3 + 1], ty[j * 3 + 2],
                           real ? kappa * tpsi[j] + tlog2nu[j] : -INFINITY);
}

// Objective pass: lane = point, the item's target blocks in chunks of 8 with
// an exact online maximum on the point's dithered grid (as the squared
// Euclidean pass's general path). A dense item of at least 16 blocks first
// evaluates 64 probe pairs spread over its blocks: their maximum is a lower
// bound of the point's, so the running maximum starts there and far pairs
// skip from the first chunk on (the final grid value depends only on the
// true maximum).
template <bool F64, int MODE>
__global__ __launch_bounds__(256) void k_sphere_pass1(
    const double4 *__restrict__ qp, const double4 *__restrict__ trec,
    const int32_t *__restrict__ blk_cnt, const uint32_t *__restrict__ row_idx,
    const uint16_t *__restrict__ row_cm, const int32_t *__restrict__ wi_tile,
    const int64_t *__restrict__ wi_range, const int32_t *__restrict__ perm,
    const double *__restrict__ blk_lo,
    const double *__restrict__ blk_hi, const double *__restrict__ blk_lnnu,
    const double *__restrict__ blk_stat, double kappa, int64_t n_items, int64_t n_blocks,
    int64_t seg1, int64_t n_seg1, const GeoPoly P, double *__restrict__ part,
    double *__restrict__ partk) {
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    int64_t w, t, e0, e1;
    if (MODE == MODE_DENSE) {
        w = (int64_t)blockIdx.x * 4 + wave;
        if (w >= n_items) return;
        t = w / n_seg1;
        e0 = (w % n_seg1) * seg1;
        e1 = std::min<int64_t>(e0 + seg1, n_blocks);
    } else {
        const int64_t k = xcd_run_item(wave);
        if (k >= n_items) return;
        w = perm[k];
        t = wi_tile[w];
        e0 = wi_range[2 * w];
        e1 = wi_range[2 * w + 1];
    }
    const int64_t q = t * 64 + lane;
    const double4 xr = qp[q];
    const double xm[3] = {-2.0 * xr.x, -2.0 * xr.y, -2.0 * xr.z};
    const double rq = ref_offset(q);
    double m = -1e300, s = 0.0, kept = 0.0;
    if (MODE == MODE_DENSE && e1 - e0 >= 16) {
        double m0 = -INFINITY;
        for (int i = 0; i < 64; ++i) {
            const double4 r = ld4(trec + (e0 + (i * (e1 - e0)) / 64) * 64 + ((i * 37) & 63));
            m0 = fmax(m0, sphere_z<F64>(P, chord2(xm, r.x, r.y, r.z), r.w));
        }
        if (m0 > -INFINITY) m = ceil(m0 - rq) + rq;
    }
    for (int64_t e = e0; e < e1; ++e) {
        const uint32_t ent = MODE == MODE_DENSE ? (uint32_t)e : row_idx[e];
        const int64_t b = (int64_t)(ent & ~RSOT_PARTIAL_BIT);
        // tile rule with culling groups: an entry marked partial keeps only
        // the 8-target chunks whose class bits say so
        const bool part = MODE == MODE_LIST && (ent & RSOT_PARTIAL_BIT);
        const uint32_t cm = part ? (uint32_t)row_cm[e] : 0u;
        if (part) {
            const int cnt = blk_cnt[b];
            for (int c = 0; c < 8; ++c)
                if ((cm >> (2 * c)) & 2u) kept += (double)std::min(8, std::max(0, cnt - 8 * c));
        } else {
            kept += (double)blk_cnt[b];
        }
        const double ub = fma(kappa, blk_stat[b * 4], blk_lnnu[b] * RSOT_LOG2E) -
                          P.kcs * box_dist2(blk_lo + b * 3, blk_hi + b * 3, xr.x, xr.y, xr.z);
        if (ub < m - 160.0) continue;
        const double4 *T = trec + b * 64;
        for (int k0 = 0; k0 < 64; k0 += CH) {
            if (part && !((cm >> (k0 / 4)) & 2u)) continue;
            double tv[CH];
            double cm = -INFINITY;
#pragma unroll
            for (int k = 0; k < CH; ++k) {
                const double4 r = ld4(T + k0 + k);
                const double sc = chord2(xm, r.x, r.y, r.z);
                tv[k] = fma(-P.kcs, sc, r.w) < m - 160.0 ? -INFINITY : sphere_z<F64>(P, sc, r.w);
                cm = fmax(cm, tv[k]);
            }
            if (cm > m) {
                const double mn = ceil(cm - rq) + rq;
                s = ldexp(s, (int)rint(fmax(m - mn, -2000.0)));
                m = mn;
            }
            if (F64) {
                double cs = 0.0;
#pragma unroll
                for (int k = 0; k < CH; ++k) cs += exp2(tv[k] - m);
                s += cs;
            } else {
                float cs = 0.0f;
#pragma unroll
                for (int k = 0; k < CH; ++k) cs += __builtin_amdgcn_exp2f((float)(tv[k] - m));
                s += (double)cs;
            }
        }
    }
    part[w * 64 + lane] = s > 0.0 ? m + log2(s) : -INFINITY;
    partk[w * 64 + lane] = kept;
}

// item of the gradient-side kernels: the gradient pass's layouts (dense: each
// XCD sweeps its own point segments; lists: sorted items dealt in runs)
struct Item {
    int64_t b, w, e0, e1;
    bool ok;
};

template <int MODE>
__device__ __forceinline__ Item col_item(int wave, const int32_t *__restrict__ wi_block,
                                         const int64_t *__restrict__ wi_range,
                                         const int32_t *__restrict__ perm, int64_t n_tiles,
                                         int64_t n_blocks, int64_t n_wi, int64_t n_seg,
                                         int64_t seg) {
    Item it{0, 0, 0, 0, false};
    if (MODE == MODE_DENSE) {
        const int64_t nbg = (n_blocks + 3) / 4;
        const int64_t kk = blockIdx.x >> 3;
        const int64_t sgi = (kk / nbg) * 8 + (blockIdx.x & 7);
        it.b = (kk % nbg) * 4 + wave;
        if (sgi >= n_seg || it.b >= n_blocks) return it;
        it.e0 = sgi * seg;
        it.e1 = std::min<int64_t>(it.e0 + seg, n_tiles);
        it.w = it.b * n_seg + sgi;
    } else {
        const int64_t k = xcd_run_item(wave);
        if (k >= n_wi) return it;
        it.w = perm[k];
        it.b = wi_block[it.w];
        it.e0 = wi_range[2 * it.w];
        it.e1 = wi_range[2 * it.w + 1];
    }
    it.ok = true;
    return it;
}

// Gradient pass: lane = target, the item's point tiles; per tile the FP32 (or
// FP64) sum of 2^(B_j - kcs d_g^2 + S'_q) scaled back by the tile reference.
template <bool F64, int MODE>
__global__ __launch_bounds__(256) void k_sphere_pass2(
    const double4 *__restrict__ qp, const double2 *__restrict__ tref,
    const double4 *__restrict__ trec, const int32_t *__restrict__ wi_block,
    const int64_t *__restrict__ wi_range, const int32_t *__restrict__ perm,
    const uint32_t *__restrict__ col_idx, const uint8_t *__restrict__ col_cm,
    const double *__restrict__ tile_lo, const double *__restrict__ tile_hi,
    const double *__restrict__ tile_smax, int64_t n_tiles, int64_t n_blocks, int64_t n_wi,
    int64_t n_seg, int64_t seg, const GeoPoly P, double *__restrict__ gpart) {
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const Item it = col_item<MODE>(wave, wi_block, wi_range, perm, n_tiles, n_blocks, n_wi,
                                   n_seg, seg);
    if (!it.ok) return;
    const double4 rec = trec[it.b * 64 + lane];
    const double ym[3] = {-2.0 * rec.x, -2.0 * rec.y, -2.0 * rec.z};
    double acc = 0.0;
    for (int64_t e = it.e0; e < it.e1; ++e) {
        const uint32_t ent = MODE == MODE_DENSE ? (uint32_t)e : col_idx[e];
        const int64_t t = (int64_t)(ent & ~RSOT_PARTIAL_BIT);
        // culling groups: lanes of dropped 8-target chunks take no terms
        const double Bl = (MODE == MODE_LIST && (ent & RSOT_PARTIAL_BIT) &&
                           !((col_cm[e] >> (lane >> 3)) & 1u))
                              ? -INFINITY
                              : rec.w;
        if (Bl + tile_smax[t] -
                P.kcs * box_dist2(tile_lo + t * 3, tile_hi + t * 3, rec.x, rec.y, rec.z) <
            -160.0)
            continue;
        const double4 *Q = qp + t * 64;
        double a = 0.0;
        for (int i0 = 0; i0 < 64; i0 += CH) {
            if (F64) {
                double cs = 0.0;
#pragma unroll
                for (int k = 0; k < CH; ++k) {
                    const double4 r = ld4(Q + i0 + k);
                    const double sc = chord2(ym, r.x, r.y, r.z), bq = Bl + r.w;
                    if (fma(-P.kcs, sc, bq) >= -160.0) cs += exp2(sphere_z<F64>(P, sc, bq));
                }
                a += cs;
            } else {
                float cs = 0.0f;
#pragma unroll
                for (int k = 0; k < CH; ++k) {
                    const double4 r = ld4(Q + i0 + k);
                    const double sc = chord2(ym, r.x, r.y, r.z), bq = Bl + r.w;
                    if (fma(-P.kcs, sc, bq) >= -160.0)
                        cs += __builtin_amdgcn_exp2f((float)sphere_z<F64>(P, sc, bq));
                }
                a += (double)cs;
            }
        }
        acc += a * tref[t].y;
    }
    gpart[it.w * 64 + lane] = acc;
}

// Alg. 5, the sums of one step: per target j (lane) over the item's tiles,
// the plan weight w_qj = mu_q p_qj at (psi, y_plan) (the gradient pass's
// term, with its underflow skip) times the log map at the current point
// y_cur, log_y(x) = theta / sin(theta) (x - cos(theta) y) with
// cos(theta) = x.y and theta / sin(theta) from the squared chord 2 - 2 x.y,
// summed in FP64 with the weight's FP32 or FP64 exponential; and the weight.
template <bool F64, int MODE>
__global__ __launch_bounds__(256) void k_sphere_karcher(
    const double4 *__restrict__ qp, const double2 *__restrict__ tref,
    const double4 *__restrict__ trec, const int32_t *__restrict__ tperm,
    const double *__restrict__ y_cur, const int32_t *__restrict__ wi_block,
    const int64_t *__restrict__ wi_range, const int32_t *__restrict__ perm,
    const uint32_t *__restrict__ col_idx, const uint8_t *__restrict__ col_cm,
    const double *__restrict__ tile_lo, const double *__restrict__ tile_hi,
    const double *__restrict__ tile_smax, int64_t n_tiles, int64_t n_blocks, int64_t n_wi,
    int64_t n_seg, int64_t seg, const GeoPoly P, const LogPoly H, double *__restrict__ kpart) {
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const Item it = col_item<MODE>(wave, wi_block, wi_range, perm, n_tiles, n_blocks, n_wi,
                                   n_seg, seg);
    if (!it.ok) return;
    const int64_t j = it.b * 64 + lane;
    const double4 rec = trec[j];
    const double ym[3] = {-2.0 * rec.x, -2.0 * rec.y, -2.0 * rec.z};
    const int32_t src = tperm[j];
    double yc[3] = {rec.x, rec.y, rec.z};
    if (src >= 0)
        for (int k = 0; k < 3; ++k) yc[k] = y_cur[(int64_t)src * 3 + k];
    double a[4] = {0.0, 0.0, 0.0, 0.0};
    for (int64_t e = it.e0; e < it.e1; ++e) {
        const uint32_t ent = MODE == MODE_DENSE ? (uint32_t)e : col_idx[e];
        const int64_t t = (int64_t)(ent & ~RSOT_PARTIAL_BIT);
        const double Bl = (MODE == MODE_LIST && (ent & RSOT_PARTIAL_BIT) &&
                           !((col_cm[e] >> (lane >> 3)) & 1u))
                              ? -INFINITY
                              : rec.w;
        if (Bl + tile_smax[t] -
                P.kcs * box_dist2(tile_lo + t * 3, tile_hi + t * 3, rec.x, rec.y, rec.z) <
            -160.0)
            continue;
        const double4 *Q = qp + t * 64;
        double at[4] = {0.0, 0.0, 0.0, 0.0};
        for (int i = 0; i < 64; ++i) {
            const double4 r = ld4(Q + i);
            const double sc = chord2(ym, r.x, r.y, r.z), bq = Bl + r.w;
            if (fma(-P.kcs, sc, bq) < -160.0) continue;
            const double v = sphere_z<F64>(P, sc, bq);
            const double wgt = F64 ? exp2(v) : (double)__builtin_amdgcn_exp2f((float)v);
            if (!(wgt > 0.0)) continue;
            const double ct = fma(r.x, yc[0], fma(r.y, yc[1], r.z * yc[2]));
            const double wf = wgt * theta_over_sin<F64>(P, H, fma(-2.0, ct, 2.0));
            at[0] = fma(wf, fma(-ct, yc[0], r.x), at[0]);
            at[1] = fma(wf, fma(-ct, yc[1], r.y), at[1]);
            at[2] = fma(wf, fma(-ct, yc[2], r.z), at[2]);
            at[3] += wgt;
        }
        const double sc = tref[t].y;
#pragma unroll
        for (int k = 0; k < 4; ++k) a[k] += at[k] * sc;
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) kpart[(it.w * 64 + lane) * 4 + k] = a[k];
}

// One workgroup per target block: wave v sums the items v, v + 4, ... of
// the block's four-component partials, the wave sums are added in a fixed
// order; then per target delta = -2 sum w log / sum w and
// y_next = exp_{y_cur}(-alpha delta), exp_y(v) = cos|v| y + sin|v| v / |v|
__global__ __launch_bounds__(256) void k_sphere_karcher_update(
    const double *__restrict__ kpart, const int64_t *__restrict__ wi_ptr, int64_t n_seg,
    const int32_t *__restrict__ tperm, const double *__restrict__ y_cur, int64_t n_blocks,
    double alpha, double *__restrict__ y_next, double *__restrict__ step_norm,
    double *__restrict__ mass_out) {
    __shared__ double4 red[4][64];
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const int64_t b = blockIdx.x;
    if (b >= n_blocks) return;
    const int64_t j = b * 64 + lane;
    const int64_t w0 = wi_ptr ? wi_ptr[b] : b * n_seg;
    const int64_t w1 = wi_ptr ? wi_ptr[b + 1] : w0 + n_seg;
    const double4 *kp = reinterpret_cast<const double4 *>(kpart);
    double4 acc = make_double4(0.0, 0.0, 0.0, 0.0);
    for (int64_t w = w0 + wv; w < w1; w += 4) {
        const double4 v = kp[w * 64 + lane];
        acc.x += v.x;
        acc.y += v.y;
        acc.z += v.z;
        acc.w += v.w;
    }
    red[wv][lane] = acc;
    __syncthreads();
    if (wv != 0) return;
    const int32_t dst = tperm[j];
    if (dst < 0) return;
    double a[4];
    {
        const double4 r0 = red[0][lane], r1 = red[1][lane], r2 = red[2][lane], r3 = red[3][lane];
        a[0] = (r0.x + r1.x) + (r2.x + r3.x);
        a[1] = (r0.y + r1.y) + (r2.y + r3.y);
        a[2] = (r0.z + r1.z) + (r2.z + r3.z);
        a[3] = (r0.w + r1.w) + (r2.w + r3.w);
    }
    const double *yc = y_cur + (int64_t)dst * 3;
    double v[3] = {0.0, 0.0, 0.0};
    if (a[3] > 0.0)
        for (int k = 0; k < 3; ++k) v[k] = -alpha * (-2.0 * a[k] / a[3]);
    const double nv = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    for (int k = 0; k < 3; ++k)
        y_next[(int64_t)dst * 3 + k] = nv > 0.0 ? cos(nv) * yc[k] + sin(nv) * v[k] / nv : yc[k];
    if (step_norm) step_norm[dst] = alpha > 0.0 ? nv / alpha : 0.0;
    if (mass_out) mass_out[dst] = a[3];
}

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

unsigned col_grid(const rsot_problem *p, int mode, int64_t n_wi, int64_t n_seg) {
    if (mode == MODE_DENSE) return (unsigned)(((p->n_blocks + 3) / 4) * ((n_seg + 7) / 8) * 8);
    return xcd_run_grid(n_wi);
}

}  // namespace

void rsot_sphere_records(rsot_problem *p, hipStream_t st, double kappa) {
    hipLaunchKernelGGL(k_sphere_records, dim3((unsigned)((p->n_pad + 255) / 256)), dim3(256), 0,
                       st, p->ty, p->tpsi, p->tlog2nu, p->tperm, p->n_pad, kappa, p->trec);
}

void rsot_sphere_pass1(rsot_problem *p, bool f64, int mode, double kcs, int64_t n_items,
                       int64_t seg1, int64_t n_seg1) {
    const unsigned grid = mode == MODE_DENSE ? (unsigned)((n_items + 3) / 4) : xcd_run_grid(n_items);
    const GeoPoly P = geo_poly(f64, kcs);
    const double kappa = kcs / p->opt.cost_scale;
#define RSOT_SP1(F, M)                                                                         \
    hipLaunchKernelGGL((k_sphere_pass1<F, M>), dim3(grid), dim3(256), 0, p->stream, p->qp,      \
                       p->trec, p->blk_cnt, p->row_idx, p->row_cm, p->wi1_tile, p->wi1_range,    \
                       p->wi1_perm,                                                              \
                       p->blk_lo, p->blk_hi, p->blk_lnnu, p->blk_stat, kappa, n_items,           \
                       p->n_blocks, seg1, n_seg1, P, p->part1, p->part1k)
    if (mode == MODE_DENSE) {
        if (f64) RSOT_SP1(true, MODE_DENSE);
        else RSOT_SP1(false, MODE_DENSE);
    } else {
        if (f64) RSOT_SP1(true, MODE_LIST);
        else RSOT_SP1(false, MODE_LIST);
    }
#undef RSOT_SP1
}

void rsot_sphere_pass2(rsot_problem *p, bool f64, int mode, double kcs, int64_t n_wi,
                       int64_t n_seg, int64_t seg) {
    const unsigned grid = col_grid(p, mode, n_wi, n_seg);
    const GeoPoly P = geo_poly(f64, kcs);
#define RSOT_SP2(F, M)                                                                         \
    hipLaunchKernelGGL((k_sphere_pass2<F, M>), dim3(grid), dim3(256), 0, p->stream, p->qp,      \
                       p->tile_ref, p->trec, p->wi_block, p->wi_range, p->wi_perm, p->col_idx,   \
                       p->col_cm, p->tile_lo, p->tile_hi, p->tile_smax, p->n_tiles, p->n_blocks, \
                       n_wi,                                                                     \
                       n_seg, seg, P, p->gpart)
    if (mode == MODE_DENSE) {
        if (f64) RSOT_SP2(true, MODE_DENSE);
        else RSOT_SP2(false, MODE_DENSE);
    } else {
        if (f64) RSOT_SP2(true, MODE_LIST);
        else RSOT_SP2(false, MODE_LIST);
    }
#undef RSOT_SP2
}

extern "C" rsot_status rsot_sphere_karcher_step(rsot_problem *p, double eps, const double *psi,
                                                const double *y_cur, double alpha,
                                                double *y_next, double *step_norm,
                                                double *mass_out, rsot_eval_info *info,
                                                double *kernel_ms) {
    if (!p || !psi || !y_cur || !y_next) return RSOT_ERR_INVALID_ARG;
    if (p->opt.cost_kind != RSOT_COST_SPHERE) return RSOT_ERR_INVALID_ARG;
    if (!(eps > 0.0) || !std::isfinite(eps) || !(alpha >= 0.0) || !std::isfinite(alpha))
        return RSOT_ERR_INVALID_ARG;
    double J = 0.0;
    RSOT_TRY(rsot_eval_impl(p, eps, psi, &J, p->dgrad, info));
    const int mode = p->last_mode;
    const bool f64 = rsot_pairs_fp64(p);
    const int64_t n_wi = p->last_n_wi, n_seg = p->last_n_seg, seg = p->last_seg;
    RSOT_TRY(grow_buf(p, &p->mpart, &p->mpart_cap, (size_t)std::max<int64_t>(n_wi, 1) * 64 * 4));
    const GeoPoly P = geo_poly(f64, p->last_kcs);
    const LogPoly H = log_poly(f64);
    const unsigned grid = col_grid(p, mode, n_wi, n_seg);
    RSOT_HIP(hipEventRecord(p->ev0, p->stream));
#define RSOT_SK(F, M)                                                                          \
    hipLaunchKernelGGL((k_sphere_karcher<F, M>), dim3(grid), dim3(256), 0, p->stream, p->qp,    \
                       p->tile_ref, p->trec, p->tperm, y_cur, p->wi_block, p->wi_range,          \
                       p->wi_perm, p->col_idx, p->col_cm, p->tile_lo, p->tile_hi, p->tile_smax,  \
                       p->n_tiles,                                                               \
                       p->n_blocks, n_wi, n_seg, seg, P, H, p->mpart)
    if (mode == MODE_DENSE) {
        if (f64) RSOT_SK(true, MODE_DENSE);
        else RSOT_SK(false, MODE_DENSE);
    } else {
        if (f64) RSOT_SK(true, MODE_LIST);
        else RSOT_SK(false, MODE_LIST);
    }
#undef RSOT_SK
    hipLaunchKernelGGL(k_sphere_karcher_update, dim3((unsigned)p->n_blocks), dim3(256),
                       0, p->stream, p->mpart,
                       mode == MODE_DENSE ? (const int64_t *)nullptr : p->wi_ptr, n_seg, p->tperm,
                       y_cur, p->n_blocks, alpha, y_next, step_norm, mass_out);
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
