// One evaluation of J(psi) and grad J(psi) (Eqs. discretized_functional and
// discretized_gradient; Alg. 2), re-derived for CDNA wavefronts.
//
// Exponents are carried in base 2. With kappa = log2(e)/eps and cs the cost
// scale, for a point x (shifted coordinates) and a target y:
//   z2(x, y_j) = log2(e) * ((psi_j - cs|x - y_j|^2)/eps + ln nu_j)
//              = B_j + A(x) + x . Y_j
//   B_j = kappa (psi_j - cs|y_j|^2) + log2 nu_j,   Y_j = 2 kappa cs y_j,
//   A(x) = -kappa cs |x|^2.
// The expansion is formed in FP64 (full rate on CDNA), so the argument of every
// exponential carries ~1e-16 relative error before it is rounded to FP32; the
// rounded argument is then O(10) for every term that matters, which keeps the
// relative error of each weight near FP32 round-off (about |u| 2^-24 for an
// argument u, and the rounding errors of different pairs are independent).
//
// Objective pass (one wavefront = one 64-point tile, lane = point): the
// per-point log-sum-exp Lt(x) = log2 sum_j 2^(B_j + x.Y_j) is accumulated
// against an integer reference m that only grows, so rescaling the running
// sum is an exact ldexp; target records are wave-uniform and reach the
// wavefront through the scalar cache.
// Gradient pass (one wavefront = one 64-target block, lane = target): the
// target mass nu~_j = sum_q mu_q p_qj = sum_q 2^(B_j + S_q + x_q.Y_j) with
// S_q = log2 mu_q - Lt(x_q) stored by the objective pass; point records are
// wave-uniform. Each work item sums a segment of point tiles; segments are
// merged per target in a fixed order, so results are bitwise reproducible.
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>

#include "rsot_device.h"
#include "rsot_internal.h"
#include "rsot_pairs.h"

#define RSOT_SEG1_DEFAULT 256   // target blocks per objective-pass work item

// v_exp_f32 is accurate to about 1 ulp, but its error has a nonzero mean over
// arguments whose fractional parts are spread evenly (a few 1e-9 relative).
// Per-point sums inherit that mean, and J = eps sum_q mu_q L_q would pick it up
// as eps * mean * sum mu. rsot_device_exp_corr measures the mean on the device
// the library runs on, with the same instruction, and the passes divide it out
// once per point (objective) or per tile (gradient). Removing the mean needs
// the dominant arguments' fractional parts spread over the points and tiles;
// ref_offset spreads the log-sum-exp references, so this holds by
// construction even on uniform meshes, where the geometry alone would
// cluster them. What remains is zero-mean and averages out over points.

// ---------------------------------------------------------------------------
// mean error of the FP32 exponential on this device
// ---------------------------------------------------------------------------
// Each workgroup sums 2^u (v_exp_f32) / 2^u (FP64) - 1 over the FP32 arguments
// u_i = FP32(-30 (i + 1/2) / n), whose fractional parts are spread evenly.
__global__ __launch_bounds__(256) void k_exp2f_error(int64_t n, double *__restrict__ part) {
    __shared__ double red[4];
    double s = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * 256) {
        const float u = (float)(-30.0 * ((double)i + 0.5) / (double)n);
        s += (double)__builtin_amdgcn_exp2f(u) / exp2((double)u) - 1.0;
    }
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

// Measured once per device (2^24 arguments, summed in a fixed order) and kept
// for the life of the process.
rsot_status rsot_device_exp_corr(hipStream_t st, double *corr) {
    static std::mutex mu;
    static double val[64];
    static bool have[64];
    int dev = 0;
    RSOT_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) return RSOT_ERR_DEVICE;
    std::lock_guard<std::mutex> lock(mu);
    if (!have[dev]) {
        const int nwg = 256;
        const int64_t n = int64_t(1) << 24;
        double *d = nullptr;
        if (hipMalloc((void **)&d, sizeof(double) * nwg) != hipSuccess) return RSOT_ERR_OOM;
        double h[nwg];
        hipLaunchKernelGGL(k_exp2f_error, dim3(nwg), dim3(256), 0, st, n, d);
        hipError_t e = hipGetLastError();
        if (e == hipSuccess) e = hipMemcpyAsync(h, d, sizeof(h), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        (void)hipFree(d);
        if (e != hipSuccess) return RSOT_ERR_DEVICE;
        double sum = 0.0;
        for (int i = 0; i < nwg; ++i) sum += h[i];
        const double mean = sum / (double)n;
        if (!std::isfinite(mean) || std::fabs(mean) > 1e-6) return RSOT_ERR_DEVICE;
        val[dev] = 1.0 / (1.0 + mean);
        have[dev] = true;
    }
    *corr = val[dev];
    return RSOT_OK;
}

// ---------------------------------------------------------------------------
// per-target records and block statistics
// ---------------------------------------------------------------------------
template <int D>
__global__ __launch_bounds__(256) void k_prep_targets(
    const double *__restrict__ psi, const int32_t *__restrict__ tperm,
    const double *__restrict__ ty, const double *__restrict__ tnu,
    const double *__restrict__ tlog2nu, int64_t n_blocks, double kappa, double cs,
    double4 *__restrict__ trec, double *__restrict__ trec3, double *__restrict__ tpsi,
    double *__restrict__ blk_stat) {
    const int lane = threadIdx.x & 63;
    const int64_t b = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (b >= n_blocks) return;
    const int64_t j = b * 64 + lane;
    const int32_t src = tperm[j];
    const bool real = src >= 0;
    const double ps = real ? psi[src] : 0.0;
    const double y0 = ty[j * 3 + 0], y1 = ty[j * 3 + 1], y2 = D == 3 ? ty[j * 3 + 2] : 0.0;
    const double r2 = y0 * y0 + y1 * y1 + y2 * y2;
    double4 rec;
    rec.x = 2.0 * kappa * cs * y0;
    rec.y = 2.0 * kappa * cs * y1;
    rec.z = 2.0 * kappa * cs * y2;
    rec.w = real ? kappa * (ps - cs * r2) + tlog2nu[j] : -INFINITY;
    trec[j] = rec;
    if (D == 2) {
        trec3[j * 3 + 0] = rec.x;
        trec3[j * 3 + 1] = rec.y;
        trec3[j * 3 + 2] = rec.w;
    }
    tpsi[j] = ps;
    const bool fin = isfinite(ps);
    const double vmax = wave_max(real && fin ? ps : -INFINITY);
    const double vmin = wave_min(real && fin ? ps : INFINITY);
    const double pn = wave_sum(real && fin ? ps * tnu[j] : 0.0);
    const double nf = wave_sum(real && !fin ? 1.0 : 0.0);
    if (lane == 0) {
        blk_stat[b * 4 + 0] = vmax;
        blk_stat[b * 4 + 1] = vmin;
        blk_stat[b * 4 + 2] = pn;
        blk_stat[b * 4 + 3] = nf;
    }
}

// cutoff constant of the per-pair test: keep iff z2 > G_j + (per point term)
__global__ void k_target_G(const double *__restrict__ tpsi, const double *__restrict__ tlog2nu,
                           const int32_t *__restrict__ tperm, int64_t n_pad, double kappa,
                           const double *__restrict__ dscal, double *__restrict__ tG) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n_pad) return;
    const double C = dscal[SC_C];
    tG[j] = tperm[j] >= 0 ? kappa * (tpsi[j] - C) + tlog2nu[j] : INFINITY;
}

// Tile rule with culling groups of g targets (8, 16 or 32; g divides the
// 64-target block): per group the box of its real targets, ln nu(G) and the
// largest finite psi, the inputs of its bound ln U_TG. A group without a real
// target gets ln nu = -inf (never kept) and the box of its first record.
__global__ void k_group_tables(const double *__restrict__ ty, const double *__restrict__ tnu,
                               const double *__restrict__ tpsi, const int32_t *__restrict__ tperm,
                               int64_t n_groups, int g, double *__restrict__ lo,
                               double *__restrict__ hi, double *__restrict__ lnnu,
                               double *__restrict__ psimax) {
    const int64_t G = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (G >= n_groups) return;
    double l[3] = {INFINITY, INFINITY, INFINITY}, h[3] = {-INFINITY, -INFINITY, -INFINITY};
    double nu = 0.0, pm = -INFINITY;
    for (int i = 0; i < g; ++i) {
        const int64_t j = G * g + i;
        if (tperm[j] < 0) continue;
        for (int k = 0; k < 3; ++k) {
            l[k] = fmin(l[k], ty[j * 3 + k]);
            h[k] = fmax(h[k], ty[j * 3 + k]);
        }
        nu += tnu[j];
        const double ps = tpsi[j];
        if (isfinite(ps)) pm = fmax(pm, ps);
    }
    if (!(nu > 0.0))
        for (int k = 0; k < 3; ++k) l[k] = h[k] = ty[G * g * 3 + k];
    for (int k = 0; k < 3; ++k) {
        lo[G * 3 + k] = l[k];
        hi[G * 3 + k] = h[k];
    }
    lnnu[G] = nu > 0.0 ? log(nu) : -INFINITY;
    psimax[G] = pm;
}

// Single workgroup: psi statistics and the cutoff of the T1 rules.
//   GEOM (Eq. truncation_cutoff_geom): C0 + (M - m) + eps ln(eps/(nu_min tau |J|)), >= C0
//   INT  (Eq. truncation_cutoff_int):  M + eps ln(eps D/(tau |J|)), >= C0
//   PW   (Eq. cost_cutoff_delta):      M + eps ln(nu_max / delta)
__global__ __launch_bounds__(256) void k_pre_scalars(const double *__restrict__ blk_stat,
                                                     int64_t n_blocks, int rule, double eps,
                                                     double C0, double nu_min, double nu_max,
                                                     double tau, double absJ, double log_D,
                                                     double delta, double *__restrict__ dscal) {
    __shared__ double red[4][4];
    double M = -INFINITY, m = INFINITY, pn = 0.0, nf = 0.0;
    for (int64_t b = threadIdx.x; b < n_blocks; b += 256) {
        M = fmax(M, blk_stat[b * 4 + 0]);
        m = fmin(m, blk_stat[b * 4 + 1]);
        pn += blk_stat[b * 4 + 2];
        nf += blk_stat[b * 4 + 3];
    }
    M = wave_max(M);
    m = wave_min(m);
    pn = wave_sum(pn);
    nf = wave_sum(nf);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        red[w][0] = M;
        red[w][1] = m;
        red[w][2] = pn;
        red[w][3] = nf;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    for (int i = 1; i < 4; ++i) {
        M = fmax(red[0][0], red[i][0]);
        red[0][0] = M;
        red[0][1] = fmin(red[0][1], red[i][1]);
        red[0][2] += red[i][2];
        red[0][3] += red[i][3];
    }
    M = red[0][0];
    m = red[0][1];
    double C = INFINITY;
    if (rule == RSOT_TRUNC_GEOM) {
        C = C0 + (M - m) + eps * log(eps / (nu_min * tau * absJ));
        C = fmax(C, C0);
    } else if (rule == RSOT_TRUNC_INT) {
        C = M + eps * (log(eps) + log_D - log(tau * absJ));
        C = fmax(C, C0);
    } else if (rule == RSOT_TRUNC_PW) {
        C = M + eps * log(nu_max / delta);
    }
    dscal[SC_PSIMAX] = M;
    dscal[SC_PSIMIN] = m;
    dscal[SC_PSINU] = red[0][2];
    dscal[SC_NONFINITE] = red[0][3];
    dscal[SC_C] = C;
}

// ---------------------------------------------------------------------------
// culling: (tile, block) flags, transposition, CSR lists
// ---------------------------------------------------------------------------
// Class of a (point box, target box) pair under a cost cutoff C (Alg. 2 with
// I_q = {j : c < C}): skipped when even the least distance between the boxes
// reaches C, kept whole when the greatest stays below C, tested pair by pair
// otherwise. Every caller passes the point-side box first, so the row and the
// column culling classify each (tile, block) pair identically.
template <int D>
__device__ __forceinline__ uint32_t cls_cutoff(const double *pl, const double *ph,
                                               const double *tl, const double *th, double cs,
                                               double C) {
    double dmin2 = 0.0, dmax2 = 0.0;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        const double g = box_gap(pl[k], ph[k], tl[k], th[k]);
        const double f = box_far(pl[k], ph[k], tl[k], th[k]);
        dmin2 += g * g;
        dmax2 += f * f;
    }
    if (cs * dmin2 >= C) return PAIR_SKIP;
    return cs * dmax2 < C ? PAIR_FULL : PAIR_PARTIAL;
}

// Chunk mask of a (tile, block) pair that needs the per-pair test, for the
// objective pass: 2 bits per chunk of 8 targets of block b, the class of the
// chunk's box against tile t's box. (The gradient pass has no such masks: its
// lanes are the block's targets, and 8-point chunks of a straddling tile
// almost always straddle the cutoff too, so their classes would save little.)
template <int D>
__device__ __forceinline__ uint32_t chunk_mask(int64_t t, int64_t b,
                                               const double *__restrict__ tile_lo,
                                               const double *__restrict__ tile_hi,
                                               const double *__restrict__ tch_lo,
                                               const double *__restrict__ tch_hi, double cs,
                                               double C) {
    uint32_t m = 0;
    for (int c = 0; c < 8; ++c)
        m |= cls_cutoff<D>(tile_lo + t * 3, tile_hi + t * 3, tch_lo + (b * 8 + c) * 3,
                           tch_hi + (b * 8 + c) * 3, cs, C)
             << (2 * c);
    return m;
}

// Tile rule (derived from App. B), per tile T:
//   ln U_TB = ln nu(B) + (max_{j in B} psi_j - cs dmin^2(T,B)) / eps  (upper bound)
//   B* = argmax_B ln U_TB (lowest index on ties);
//   ln L_T = max_{j in B*} ln nu_j + (psi_j - cs dmax^2(T, y_j)) / eps (lower bound of S)
//   keep (T,B) iff B = B* or ln U_TB > ln L_T + ln(eta / n_blocks),
//   eta = tau |J_ref| / (eps sum mu): then J_dense - J_trunc <= tau |J_ref|.
// With the squared geodesic cost on the unit sphere the boxes bound the
// chord d; the geodesic 2 asin(d / 2) increases with it, so d^2 becomes
// (2 asin(min(1, d / 2)))^2 in every bound.
__device__ __forceinline__ double geo_of_chord2(double d2) {
    const double a = 2.0 * asin(fmin(1.0, 0.5 * sqrt(d2)));
    return a * a;
}

template <int D>
__device__ __forceinline__ double tile_lnU(const double *__restrict__ tile_lo,
                                           const double *__restrict__ tile_hi,
                                           const double *__restrict__ blk_lo,
                                           const double *__restrict__ blk_hi,
                                           const double *__restrict__ blk_lnnu,
                                           const double *__restrict__ blk_stat, int64_t t,
                                           int64_t b, double cs, double eps, bool sphere = false) {
    double dmin2 = 0.0;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        const double g = box_gap(tile_lo[t * 3 + k], tile_hi[t * 3 + k], blk_lo[b * 3 + k],
                                 blk_hi[b * 3 + k]);
        dmin2 += g * g;
    }
    if (sphere) dmin2 = geo_of_chord2(dmin2);
    return blk_lnnu[b] + (blk_stat[b * 4 + 0] - cs * dmin2) / eps;
}

// one wavefront per tile: B* and the skip threshold ln L_T + ln(eta / n_blocks)
template <int D>
__global__ __launch_bounds__(256) void k_tile_ref(
    const double *__restrict__ tile_lo, const double *__restrict__ tile_hi,
    const double *__restrict__ blk_lo, const double *__restrict__ blk_hi,
    const double *__restrict__ blk_lnnu, const double *__restrict__ blk_stat,
    const int32_t *__restrict__ blk_cnt, const double *__restrict__ ty,
    const double *__restrict__ tnu, const double *__restrict__ tpsi, int64_t n_tiles,
    int64_t n_blocks, double cs, double eps, double ln_eta_nb, int32_t *__restrict__ bstar,
    double *__restrict__ thr, int sphere) {
    const int lane = threadIdx.x & 63;
    const int64_t t = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (t >= n_tiles) return;
    double best = -INFINITY;
    int64_t bi = INT64_MAX;
    for (int64_t b = lane; b < n_blocks; b += 64) {
        const double lnU = tile_lnU<D>(tile_lo, tile_hi, blk_lo, blk_hi, blk_lnnu, blk_stat, t, b,
                                       cs, eps, sphere != 0);
        if (lnU > best) {
            best = lnU;
            bi = b;
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const double ob = __shfl_xor(best, o, 64);
        const int64_t oi = __shfl_xor(bi, o, 64);
        if (ob > best || (ob == best && oi < bi)) {
            best = ob;
            bi = oi;
        }
    }
    // no finite bound at all (only when psi is not finite: the evaluation
    // then reports it): keep nothing
    const bool found = bi != INT64_MAX;
    double lb = -INFINITY;
    if (found && lane < blk_cnt[bi]) {
        const int64_t j = bi * 64 + lane;
        double dmax2 = 0.0;
        for (int k = 0; k < D; ++k) {
            const double f = box_far_pt(tile_lo[t * 3 + k], tile_hi[t * 3 + k], ty[j * 3 + k]);
            dmax2 += f * f;
        }
        if (sphere) dmax2 = geo_of_chord2(dmax2);
        lb = log(tnu[j]) + (tpsi[j] - cs * dmax2) / eps;
    }
    const double th = wave_max(lb) + ln_eta_nb;
    if (lane == 0) {
        bstar[t] = found ? (int32_t)bi : -1;
        thr[t] = found ? th : INFINITY;
    }
}

// ln nu + v / eps > th, decided exactly as written (the division rounded
// once, then the sum) but with the division only where a product with 1/eps
// lands within a rounding band of the threshold
__device__ __forceinline__ bool bound_above(double lnnu, double v, double eps, double inv_eps,
                                            double th) {
    const double q = v * inv_eps;
    const double a = lnnu + q;
    const double band = 1e-12 * (fabs(q) + fabs(lnnu) + fabs(th) + 1.0);
    if (a > th + band) return true;
    if (a < th - band) return false;
    return lnnu + v / eps > th;
}

// ln U_TG of a culling group (the same bound with the group's tables)
template <int D>
__device__ __forceinline__ double grp_lnU(const double *__restrict__ tile_lo,
                                          const double *__restrict__ tile_hi,
                                          const double *__restrict__ glo,
                                          const double *__restrict__ ghi,
                                          const double *__restrict__ glnnu,
                                          const double *__restrict__ gpsi, int64_t t, int64_t G,
                                          double cs, double eps, bool sphere = false) {
    double dmin2 = 0.0;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        const double g = box_gap(tile_lo[t * 3 + k], tile_hi[t * 3 + k], glo[G * 3 + k],
                                 ghi[G * 3 + k]);
        dmin2 += g * g;
    }
    if (sphere) dmin2 = geo_of_chord2(dmin2);
    return glnnu[G] + (gpsi[G] - cs * dmin2) / eps;
}

// The tile rule over groups of g targets instead of blocks: G* = argmax_G
// ln U_TG (lowest index on ties), ln L_T over the targets of G*, threshold
// ln L_T + ln(eta / n_groups). One wavefront per tile.
template <int D>
__global__ __launch_bounds__(256) void k_tile_ref_grp(
    const double *__restrict__ tile_lo, const double *__restrict__ tile_hi,
    const double *__restrict__ blk_lo, const double *__restrict__ blk_hi,
    const double *__restrict__ blk_lnnu, const double *__restrict__ blk_stat,
    const double *__restrict__ glo, const double *__restrict__ ghi,
    const double *__restrict__ glnnu, const double *__restrict__ gpsi,
    const double *__restrict__ ty, const double *__restrict__ tnu,
    const double *__restrict__ tpsi, const int32_t *__restrict__ tperm, int64_t n_tiles,
    int64_t n_groups, int g, double cs, double eps, double ln_eta_ng,
    int32_t *__restrict__ gstar, double *__restrict__ thr, int sphere) {
    const int lane = threadIdx.x & 63;
    const int64_t t = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (t >= n_tiles) return;
    // A group's bound is at most its block's (less mass, no larger psi, a
    // box inside the block's), up to rounding: the block with the largest
    // bound gives a first group value gv, and only blocks whose bound reaches
    // gv (less a margin) can hold a group above it.
    const int ng = 64 / g;
    const int64_t n_blocks = n_groups / ng;
    double bmax = -INFINITY;
    int64_t bm = 0;
    for (int64_t b = lane; b < n_blocks; b += 64) {
        const double v = tile_lnU<D>(tile_lo, tile_hi, blk_lo, blk_hi, blk_lnnu, blk_stat, t, b,
                                     cs, eps, sphere != 0);
        if (v > bmax) {
            bmax = v;
            bm = b;
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const double ob = __shfl_xor(bmax, o, 64);
        const int64_t oi = __shfl_xor(bm, o, 64);
        if (ob > bmax || (ob == bmax && oi < bm)) {
            bmax = ob;
            bm = oi;
        }
    }
    double gv = -INFINITY;
    if (lane < ng)
        gv = grp_lnU<D>(tile_lo, tile_hi, glo, ghi, glnnu, gpsi, t, bm * ng + lane, cs, eps,
                        sphere != 0);
    gv = wave_max(gv);
    const double floor_v = gv - 1e-9 * (fabs(gv) + 1.0);
    double best = -INFINITY;
    int64_t bi = INT64_MAX;
    for (int64_t b = lane; b < n_blocks; b += 64) {
        const double v = tile_lnU<D>(tile_lo, tile_hi, blk_lo, blk_hi, blk_lnnu, blk_stat, t, b,
                                     cs, eps, sphere != 0);
        if (!(v >= floor_v)) continue;
        for (int i = 0; i < ng; ++i) {
            const int64_t G = b * ng + i;
            const double lnU = grp_lnU<D>(tile_lo, tile_hi, glo, ghi, glnnu, gpsi, t, G, cs, eps,
                                          sphere != 0);
            if (lnU > best) {
                best = lnU;
                bi = G;
            }
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const double ob = __shfl_xor(best, o, 64);
        const int64_t oi = __shfl_xor(bi, o, 64);
        if (ob > best || (ob == best && oi < bi)) {
            best = ob;
            bi = oi;
        }
    }
    const bool found = bi != INT64_MAX;
    double lb = -INFINITY;
    if (found && lane < g) {
        const int64_t j = bi * g + lane;
        if (tperm[j] >= 0) {
            double dmax2 = 0.0;
            for (int k = 0; k < D; ++k) {
                const double f = box_far_pt(tile_lo[t * 3 + k], tile_hi[t * 3 + k], ty[j * 3 + k]);
                dmax2 += f * f;
            }
            if (sphere) dmax2 = geo_of_chord2(dmax2);
            lb = log(tnu[j]) + (tpsi[j] - cs * dmax2) / eps;
        }
    }
    const double th = wave_max(lb) + ln_eta_ng;
    if (lane == 0) {
        gstar[t] = found ? (int32_t)bi : -1;
        thr[t] = found ? th : INFINITY;
    }
}

// Chunk bits (bit c: targets 8c..8c+7 of block b) of the groups of g targets
// of block b that the tile rule keeps for tile t.
template <int D>
__device__ __forceinline__ uint32_t group_chunks(int64_t t, int64_t b, int g,
                                                 const double *__restrict__ tile_lo,
                                                 const double *__restrict__ tile_hi,
                                                 const double *__restrict__ glo,
                                                 const double *__restrict__ ghi,
                                                 const double *__restrict__ glnnu,
                                                 const double *__restrict__ gpsi, int32_t gs,
                                                 double th, double cs, double eps,
                                                 bool sphere) {
    const int ng = 64 / g, cpg = g / 8;
    const double inv_eps = 1.0 / eps;
    double tl[3], thb[3];
#pragma unroll
    for (int k = 0; k < D; ++k) {
        tl[k] = tile_lo[t * 3 + k];
        thb[k] = tile_hi[t * 3 + k];
    }
    uint32_t m = 0;
    for (int i = 0; i < ng; ++i) {
        const int64_t G = b * ng + i;
        bool keep = G == gs;
        if (!keep) {
            double dmin2 = 0.0;
#pragma unroll
            for (int k = 0; k < D; ++k) {
                const double gp = box_gap(tl[k], thb[k], glo[G * 3 + k], ghi[G * 3 + k]);
                dmin2 += gp * gp;
            }
            if (sphere) dmin2 = geo_of_chord2(dmin2);
            keep = bound_above(glnnu[G], gpsi[G] - cs * dmin2, eps, inv_eps, th);
        }
        if (keep) m |= ((1u << cpg) - 1u) << (i * cpg);
    }
    return m;
}

// Culling of the truncated rules straight into CSR lists. Rows are tiles
// (ROWS) or target blocks; each row is cut into nseg segments of seg_len
// columns so that short lists of long rows still fill the device, and one
// wavefront handles one (row, segment), lanes over its columns.
// FILL = false classifies every pair of the segment, counts the kept entries
// into scnt and stores the classes as bits, one 64-bit word per 64 columns
// (kbits: kept, pbits: needs the per-pair test); it runs on the rows only
// (the column bits are these transposed, k_transpose_bits). FILL = true reads the words
// back and writes the entries in increasing order, from the row's start
// ptr[row] plus the counts of the row's earlier segments: the index (with
// RSOT_PARTIAL_BIT when the pair needs the per-pair test) and, for such
// entries of the rows, the chunk mask.
// TILE: the tile rule; with grp = 64 it decides per (tile, block) and kept
// pairs are whole; with culling groups of grp < 64 targets it decides per
// (tile, group): an entry keeps the chunks of its kept groups, and one that
// drops some real chunk is marked partial and carries the chunk bits (rows:
// 2-bit classes in cmask, FULL or SKIP; columns: one bit per chunk in ccm).
// The block's own bound caps its groups' bounds (a group's mass, psi and
// box distance are at most the block's), so the groups of a block whose
// bound falls below the threshold by more than a rounding margin are not
// tested. Otherwise: the cost cutoff C of the T1 rules.
template <int D, bool TILE, bool ROWS, bool FILL>
__global__ __launch_bounds__(256) void k_cull(
    const double *__restrict__ tile_lo, const double *__restrict__ tile_hi,
    const double *__restrict__ blk_lo, const double *__restrict__ blk_hi,
    const double *__restrict__ tch_lo, const double *__restrict__ tch_hi,
    const double *__restrict__ blk_lnnu, const double *__restrict__ blk_stat,
    const int32_t *__restrict__ bstar, const double *__restrict__ thr, int64_t n_tiles,
    int64_t n_blocks, int nseg, int64_t seg_len, double cs, double eps,
    const double *__restrict__ dscal, int32_t *__restrict__ scnt,
    uint64_t *__restrict__ kbits, uint64_t *__restrict__ pbits,
    const int64_t *__restrict__ ptr, uint32_t *__restrict__ idx,
    uint16_t *__restrict__ cmask, int grp, const double *__restrict__ glo,
    const double *__restrict__ ghi, const double *__restrict__ glnnu,
    const double *__restrict__ gpsi, const int32_t *__restrict__ blk_cnt,
    uint8_t *__restrict__ ccm, uint8_t *__restrict__ gm_out, const uint8_t *__restrict__ gm_in,
    int sphere) {
    const int lane = threadIdx.x & 63;
    const int64_t rs = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int64_t nrows = ROWS ? n_tiles : n_blocks, ncols = ROWS ? n_blocks : n_tiles;
    if (rs >= nrows * nseg) return;
    const int64_t r = rs / nseg;
    const int sg = (int)(rs % nseg);
    const int64_t kb = sg * seg_len, ke = std::min<int64_t>(kb + seg_len, ncols);
    const double C = TILE ? 0.0 : dscal[SC_C];
    const bool groups = TILE && grp < 64;
    int c = 0;
    int64_t base = 0;
    if (FILL) {
        base = ptr[r];
        for (int i = 0; i < sg; ++i) base += scnt[r * nseg + i];
    }
    const int64_t nwords = (ncols + 63) / 64;
    for (int64_t k0 = kb; k0 < ke; k0 += 64) {
        const int64_t k = k0 + lane;
        const int64_t t = ROWS ? r : k, b = ROWS ? k : r;
        const int64_t wi = r * nwords + k0 / 64;
        uint32_t cls = PAIR_SKIP;
        if (FILL) {
            const uint64_t kw = kbits[wi];
            const uint64_t pw = (TILE && !groups) ? 0 : pbits[wi];
            if ((kw >> lane) & 1) cls = ((pw >> lane) & 1) ? PAIR_PARTIAL : PAIR_FULL;
        } else if (k < ke) {
            if (TILE && groups) {
                uint32_t m = 0;
                if (gm_in) {
                    m = gm_in[r * ncols + k];          // the row pass's masks, transposed
                } else {
                    const int32_t gs = bstar[t];
                    const double th = thr[t];
                    const bool holds = gs >= 0 && gs / (64 / grp) == b;
                    const double lnU = tile_lnU<D>(tile_lo, tile_hi, blk_lo, blk_hi, blk_lnnu,
                                                   blk_stat, t, b, cs, eps, sphere != 0);
                    if (holds || lnU > th - 1e-9)
                        m = group_chunks<D>(t, b, grp, tile_lo, tile_hi, glo, ghi, glnnu, gpsi, gs,
                                            th, cs, eps, sphere != 0);
                    if (gm_out) gm_out[r * ncols + k] = (uint8_t)m;
                }
                if (m) {
                    const int nr = blk_cnt[b];
                    const uint32_t real = nr >= 64 ? 0xFFu : ((1u << ((nr + 7) / 8)) - 1u);
                    cls = (m & real) == real ? PAIR_FULL : PAIR_PARTIAL;
                }
            } else if (TILE) {
                const double lnU = tile_lnU<D>(tile_lo, tile_hi, blk_lo, blk_hi, blk_lnnu,
                                               blk_stat, t, b, cs, eps, sphere != 0);
                cls = (b == bstar[t] || lnU > thr[t]) ? PAIR_FULL : PAIR_SKIP;
            } else {
                cls = cls_cutoff<D>(tile_lo + t * 3, tile_hi + t * 3, blk_lo + b * 3,
                                    blk_hi + b * 3, cs, C);
            }
        }
        if (!FILL) {
            c += cls != PAIR_SKIP;
            const uint64_t kw = __ballot(cls != PAIR_SKIP);
            const uint64_t pw = __ballot(cls == PAIR_PARTIAL);
            if (lane == 0) {
                kbits[wi] = kw;
                if (!TILE || groups) pbits[wi] = pw;
            }
        } else {
            const uint64_t mask = __ballot(cls != PAIR_SKIP);
            const uint32_t below = __builtin_amdgcn_mbcnt_hi(
                (uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
            if (cls != PAIR_SKIP) {
                idx[base + below] = (uint32_t)k | (cls == PAIR_PARTIAL ? RSOT_PARTIAL_BIT : 0u);
                if (!TILE && ROWS && cls == PAIR_PARTIAL)
                    cmask[base + below] = (uint16_t)chunk_mask<D>(t, b, tile_lo, tile_hi, tch_lo,
                                                                  tch_hi, cs, C);
                if (TILE && groups && cls == PAIR_PARTIAL) {
                    const uint32_t m =
                        gm_in ? (uint32_t)gm_in[r * ncols + k]
                              : group_chunks<D>(t, b, grp, tile_lo, tile_hi, glo, ghi, glnnu,
                                                gpsi, bstar[t], thr[t], cs, eps, sphere != 0);
                    if (ROWS) {
                        uint32_t cm2 = 0;
                        for (int q = 0; q < 8; ++q)
                            if ((m >> q) & 1u) cm2 |= (uint32_t)PAIR_FULL << (2 * q);
                        cmask[base + below] = (uint16_t)cm2;
                    } else {
                        ccm[base + below] = (uint8_t)m;
                    }
                }
            }
            base += __popcll(mask);
        }
    }
    if (!FILL) {
        c = wave_sum_int(c);
        if (lane == 0) scnt[rs] = c;
    }
}

// entries of each row: the sum of its segments' counts
__global__ void k_seg_sum(const int32_t *__restrict__ scnt, int64_t nrows, int nseg,
                          int32_t *__restrict__ cnt) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nrows) return;
    int32_t c = 0;
    for (int i = 0; i < nseg; ++i) c += scnt[r * nseg + i];
    cnt[r] = c;
}

// The column culling from the row count pass's bits: both passes classify
// every (tile, block) pair with the same function of the same operands, so
// the column bits are the row bits transposed. One wavefront per 64 x 64 bit
// tile: lane l holds the row word of tile t0 + l; the ballot over lanes of
// bit j is the column word of block b0 + j. PB: the partial bits too.
template <bool PB>
__global__ __launch_bounds__(256) void k_transpose_bits(
    const uint64_t *__restrict__ rk, const uint64_t *__restrict__ rp, int64_t n_tiles,
    int64_t n_blocks, uint64_t *__restrict__ ck, uint64_t *__restrict__ cp) {
    const int lane = threadIdx.x & 63;
    const int64_t nwt = (n_tiles + 63) / 64, nwb = (n_blocks + 63) / 64;
    const int64_t wv = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (wv >= nwt * nwb) return;
    const int64_t tw = wv / nwb, bw = wv % nwb;
    const int64_t t = tw * 64 + lane;
    const uint64_t k = t < n_tiles ? rk[t * nwb + bw] : 0ull;
    const uint64_t q = (PB && t < n_tiles) ? rp[t * nwb + bw] : 0ull;
    uint64_t ko = 0, qo = 0;
    for (int j = 0; j < 64; ++j) {
        const uint64_t mk = __ballot((k >> j) & 1ull);
        if (lane == j) ko = mk;
        if (PB) {
            const uint64_t mq = __ballot((q >> j) & 1ull);
            if (lane == j) qo = mq;
        }
    }
    const int64_t b = bw * 64 + lane;
    if (b < n_blocks) {
        ck[b * nwt + tw] = ko;
        if (PB) cp[b * nwt + tw] = qo;
    }
}

// kept (tile, block) pairs per (block, segment of seg_len tiles) from the
// column bits
__global__ void k_col_seg_counts(const uint64_t *__restrict__ ck, int64_t n_tiles,
                                 int64_t n_blocks, int nseg, int64_t seg_len,
                                 int32_t *__restrict__ scnt) {
    const int64_t rs = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (rs >= n_blocks * nseg) return;
    const int64_t b = rs / nseg, sg = rs % nseg;
    const int64_t nwt = (n_tiles + 63) / 64;
    const int64_t w0 = sg * seg_len / 64;
    const int64_t w1 = std::min<int64_t>(nwt, (sg + 1) * seg_len / 64);
    int32_t c = 0;
    for (int64_t w = w0; w < w1; ++w) c += __popcll(ck[b * nwt + w]);
    scnt[rs] = c;
}

// out = in^T for a rows x cols byte matrix, through 64 x 64 tiles in LDS
// (grid: x over column tiles, y over row tiles)
__global__ __launch_bounds__(256) void k_transpose_u8(const uint8_t *__restrict__ in,
                                                      int64_t rows, int64_t cols,
                                                      uint8_t *__restrict__ out) {
    __shared__ uint8_t tb[64][65];
    const int64_t r0 = (int64_t)blockIdx.y * 64, c0 = (int64_t)blockIdx.x * 64;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    for (int i = ty; i < 64; i += 4) {
        const int64_t r = r0 + i, c = c0 + tx;
        tb[i][tx] = (r < rows && c < cols) ? in[r * cols + c] : (uint8_t)0;
    }
    __syncthreads();
    for (int i = ty; i < 64; i += 4) {
        const int64_t c = c0 + i, r = r0 + tx;
        if (c < cols && r < rows) out[c * rows + r] = tb[tx][i];
    }
}

// bounding boxes of consecutive groups of 8 elements (coordinates with the
// given stride), for the chunk masks
__global__ void k_chunk_boxes(const double *__restrict__ x, int stride, int64_t n_chunks,
                              double *__restrict__ lo, double *__restrict__ hi) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n_chunks) return;
    for (int k = 0; k < 3; ++k) {
        double a = INFINITY, b = -INFINITY;
        for (int i = 0; i < 8; ++i) {
            const double v = x[(c * 8 + i) * stride + k];
            a = fmin(a, v);
            b = fmax(b, v);
        }
        lo[c * 3 + k] = a;
        hi[c * 3 + k] = b;
    }
}

// one wavefront per row: number of non-skipped entries
__global__ __launch_bounds__(256) void k_count_rows(const uint8_t *__restrict__ flags,
                                                    int64_t nrows, int64_t ncols,
                                                    int32_t *__restrict__ cnt) {
    const int lane = threadIdx.x & 63;
    const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (r >= nrows) return;
    int c = 0;
    for (int64_t k = lane; k < ncols; k += 64) c += flags[r * ncols + k] != PAIR_SKIP;
    c = wave_sum_int(c);
    if (lane == 0) cnt[r] = c;
}

// one wavefront per row: kept column indices in increasing order
__global__ __launch_bounds__(256) void k_fill_rows(const uint8_t *__restrict__ flags,
                                                   int64_t nrows, int64_t ncols,
                                                   const int64_t *__restrict__ ptr,
                                                   uint32_t *__restrict__ idx) {
    const int lane = threadIdx.x & 63;
    const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (r >= nrows) return;
    int64_t base = ptr[r];
    for (int64_t k0 = 0; k0 < ncols; k0 += 64) {
        const int64_t k = k0 + lane;
        const uint8_t f = k < ncols ? flags[r * ncols + k] : PAIR_SKIP;
        const uint64_t mask = __ballot(f != PAIR_SKIP);
        const uint32_t below = __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                                        __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
        if (f != PAIR_SKIP)
            idx[base + below] = (uint32_t)k | (f == PAIR_PARTIAL ? RSOT_PARTIAL_BIT : 0u);
        base += __popcll(mask);
    }
}

// Single workgroup exclusive scan: ptr[0..n] from cnt[0..n-1]; ptr[n] = total.
// With seg > 0 the scanned quantity is ceil(cnt / seg) (work items per block).
__global__ __launch_bounds__(1024) void k_scan(const int32_t *__restrict__ cnt, int64_t n,
                                               int seg, int64_t *__restrict__ ptr,
                                               double *__restrict__ total_out) {
    __shared__ int64_t sums[1024];
    const int tid = threadIdx.x;
    const int64_t chunk = (n + 1023) / 1024;
    const int64_t a = std::min<int64_t>(n, tid * chunk), b = std::min<int64_t>(n, a + chunk);
    int64_t loc = 0;
    for (int64_t i = a; i < b; ++i) loc += seg > 0 ? (cnt[i] + seg - 1) / seg : cnt[i];
    sums[tid] = loc;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        int64_t v = tid >= off ? sums[tid - off] : 0;
        __syncthreads();
        sums[tid] += v;
        __syncthreads();
    }
    int64_t run = sums[tid] - loc;
    for (int64_t i = a; i < b; ++i) {
        ptr[i] = run;
        run += seg > 0 ? (cnt[i] + seg - 1) / seg : cnt[i];
    }
    if (tid == 1023) {
        ptr[n] = sums[1023];
        *total_out = (double)sums[1023];
    }
}

// The same exclusive prefix sums for long arrays, over pieces of 1024
// entries in three launches: each piece's sum (k_scan_piece), the scan of
// the piece sums in one workgroup (k_scan_top), then each piece's own scan
// offset by its piece's prefix (k_scan_apply). psum holds
// ceil(n / 1024) entries.
__device__ __forceinline__ int64_t scan_term(const int32_t *__restrict__ cnt, int64_t i,
                                             int64_t n, int seg) {
    if (i >= n) return 0;
    const int64_t c = cnt[i];
    return seg > 0 ? (c + seg - 1) / seg : c;
}

// inclusive scan of v over the 1024 threads of the workgroup; *total gets the
// workgroup's sum (wsum: 16 entries of shared memory)
__device__ __forceinline__ int64_t group_scan_1024(int64_t v, int64_t *wsum, int64_t *total) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int64_t t = __shfl_up(v, o, 64);
        if (lane >= o) v += t;
    }
    if (lane == 63) wsum[w] = v;
    __syncthreads();
    if (w == 0) {
        int64_t s = lane < 16 ? wsum[lane] : 0;
#pragma unroll
        for (int o = 1; o < 16; o <<= 1) {
            const int64_t t = __shfl_up(s, o, 64);
            if (lane >= o) s += t;
        }
        if (lane < 16) wsum[lane] = s;
    }
    __syncthreads();
    const int64_t r = v + (w > 0 ? wsum[w - 1] : 0);
    *total = wsum[15];
    __syncthreads();
    return r;
}

__global__ __launch_bounds__(1024) void k_scan_piece(const int32_t *__restrict__ cnt, int64_t n,
                                                     int seg, int64_t *__restrict__ psum) {
    __shared__ int64_t wsum[16];
    const int64_t i = (int64_t)blockIdx.x * 1024 + threadIdx.x;
    int64_t total = 0;
    (void)group_scan_1024(scan_term(cnt, i, n, seg), wsum, &total);
    if (threadIdx.x == 0) psum[blockIdx.x] = total;
}

// one workgroup: psum (np entries) becomes its exclusive prefix sums;
// ptr[n] and *total_out get the total
__global__ __launch_bounds__(1024) void k_scan_top(int64_t *__restrict__ psum, int64_t np,
                                                   int64_t *__restrict__ ptr, int64_t n,
                                                   double *__restrict__ total_out) {
    __shared__ int64_t wsum[16];
    int64_t carry = 0;
    for (int64_t base = 0; base < np; base += 1024) {
        const int64_t i = base + threadIdx.x;
        const int64_t v = i < np ? psum[i] : 0;
        int64_t total = 0;
        const int64_t inc = group_scan_1024(v, wsum, &total);
        if (i < np) psum[i] = carry + inc - v;
        carry += total;
    }
    if (threadIdx.x == 0) {
        ptr[n] = carry;
        *total_out = (double)carry;
    }
}

__global__ __launch_bounds__(1024) void k_scan_apply(const int32_t *__restrict__ cnt, int64_t n,
                                                     int seg, const int64_t *__restrict__ psum,
                                                     int64_t *__restrict__ ptr) {
    __shared__ int64_t wsum[16];
    const int64_t i = (int64_t)blockIdx.x * 1024 + threadIdx.x;
    const int64_t v = scan_term(cnt, i, n, seg);
    int64_t total = 0;
    const int64_t inc = group_scan_1024(v, wsum, &total);
    if (i < n) ptr[i] = psum[blockIdx.x] + inc - v;
}

// exclusive prefix sums of cnt (or of ceil(cnt / seg) when seg > 0) into
// ptr[0..n], the total also into *total_out; psum: ceil(n / 1024) entries
static void launch_scan(hipStream_t st, const int32_t *cnt, int64_t n, int seg, int64_t *ptr,
                        double *total_out, int64_t *psum) {
    if (n <= 4096) {
        hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, st, cnt, n, seg, ptr, total_out);
        return;
    }
    const int64_t np = (n + 1023) / 1024;
    hipLaunchKernelGGL(k_scan_piece, dim3((unsigned)np), dim3(1024), 0, st, cnt, n, seg, psum);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(1024), 0, st, psum, np, ptr, n, total_out);
    hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)np), dim3(1024), 0, st, cnt, n, seg, psum,
                       ptr);
}

// work items of the gradient pass: block b owns ceil(len_b / seg) segments of
// its column list
__global__ void k_fill_work(const int64_t *__restrict__ col_ptr, const int64_t *__restrict__ wi_ptr,
                            int64_t n_blocks, int seg, int32_t *__restrict__ wi_block,
                            int64_t *__restrict__ wi_range) {
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= n_blocks) return;
    const int64_t c0 = col_ptr[b], c1 = col_ptr[b + 1];
    int64_t w = wi_ptr[b];
    for (int64_t s = c0; s < c1; s += seg, ++w) {
        wi_block[w] = (int32_t)b;
        wi_range[2 * w] = s;
        wi_range[2 * w + 1] = std::min<int64_t>(c1, s + seg);
    }
}

// sort keys of work items: the item's first list entry (a block or tile index)
__global__ void k_item_keys(const int64_t *__restrict__ wi_range, const uint32_t *__restrict__ idx,
                            int64_t n, int32_t *__restrict__ key, int32_t *__restrict__ val) {
    const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (w >= n) return;
    key[w] = (int32_t)(idx[wi_range[2 * w]] & ~RSOT_PARTIAL_BIT);
    val[w] = (int32_t)w;
}

// ---------------------------------------------------------------------------
// objective pass
// ---------------------------------------------------------------------------
// Accumulates one 64-target block into the running (m, s) of this lane's
// point: s = sum 2^(t_j - m). m is an online maximum on the grid
// k + rq (k integer); when a chunk's max exceeds it, s is rescaled by an exact
// power of two. Exact for any first value of m (m = -1e300: no reference yet).
// MASK: only targets with t_j > G_j - A (c < C) enter, and are counted.
template <int D, bool F64, bool MASK, typename RP, typename GP>
__device__ __forceinline__ void lse_chunk(RP T, int k0, GP G, double x0, double x1, double x2,
                                          double A, double rq, double &m, double &s,
                                          double &kept) {
    {
        double tv[CH];
        double cm = -INFINITY;
#pragma unroll
        for (int k = 0; k < CH; ++k) {
            double v = pair_exp<D>(x0, x1, x2, trec_at<D>(T, k0 + k));
            if (MASK) {
                const bool in = v > G[k0 + k] - A;
                v = in ? v : -INFINITY;
                kept += in ? 1.0 : 0.0;
            }
            tv[k] = v;
            cm = fmax(cm, v);
        }
        if (cm > m) {
            const double mn = ceil(cm - rq) + rq;
            s = ldexp(s, (int)rint(fmax(m - mn, -2000.0)));
            m = mn;
        }
        if (F64) {
            double cs = exp2(tv[0] - m);
#pragma unroll
            for (int k = 1; k < CH; ++k) cs += exp2(tv[k] - m);
            s += cs;
        } else {
            float cs = __builtin_amdgcn_exp2f((float)(tv[0] - m));
#pragma unroll
            for (int k = 1; k < CH; ++k) cs += __builtin_amdgcn_exp2f((float)(tv[k] - m));
            s += (double)cs;
        }
    }
}

template <int D, bool F64, bool MASK, typename RP, typename GP>
__device__ __forceinline__ void lse_block(RP T, GP G, double x0, double x1, double x2, double A,
                                          double rq, double &m, double &s, double &kept) {
    for (int k0 = 0; k0 < 64; k0 += CH)
        lse_chunk<D, F64, MASK>(T, k0, G, x0, x1, x2, A, rq, m, s, kept);
}

// Mixed-precision fast path for a chunk of 8 targets whose pairs are all
// kept: the reference m enters the FMA chain's initial value (B_j - m), so
// each pair costs the FP64 argument, one rounding, one v_exp_f32 and one FP32
// add. m starts at ceil(t) of the first target of the item (kept under the
// dense and tile rules), so there m <= max_j t_j + 1 always. The reference
// must also stay close to the running maximum: the FP32-rounded argument
// u = t - m carries an absolute error ~|u| 2^-24, so the largest terms need
// |u| < 1. A chunk whose FP32 sum exceeds 2 and whose largest u is positive
// raises m by ceil of that u and is recomputed from the FP64 records; without
// the trigger every u < 1. Spurious triggers (several terms just below the
// reference) cost the max over the chunk only.
template <int D, typename RP>
__device__ __forceinline__ void lse_chunk_fast(RP T, int k0, double x0, double x1, double x2,
                                               double &m, double &s) {
    float u[CH];
    float cs = 0.0f;
#pragma unroll
    for (int k = 0; k < CH; ++k) {
        const double4 r = trec_at<D>(T, k0 + k);
        double v = r.w - m;
        v = fma(x0, r.x, v);
        v = fma(x1, r.y, v);
        if (D == 3) v = fma(x2, r.z, v);
        u[k] = (float)v;
        const float e = __builtin_amdgcn_exp2f(u[k]);
        cs = k == 0 ? e : cs + e;
    }
    if (!(cs <= 2.0f)) {
        float mx = u[0];
#pragma unroll
        for (int k = 1; k < CH; ++k) mx = fmaxf(mx, u[k]);
        if (mx > 0.0f) {
            const double dm = ceil((double)mx);
            s = ldexp(s, -(int)fmin(dm, 2000.0));
            m += dm;
            cs = 0.0f;
#pragma unroll
            for (int k = 0; k < CH; ++k) {
                const double4 r = trec_at<D>(T, k0 + k);
                double v = r.w - m;
                v = fma(x0, r.x, v);
                v = fma(x1, r.y, v);
                if (D == 3) v = fma(x2, r.z, v);
                const float e = __builtin_amdgcn_exp2f((float)v);
                cs = k == 0 ? e : cs + e;
            }
        }
    }
    s += (double)cs;
}

template <int D, typename RP>
__device__ __forceinline__ void lse_block_fast(RP T, double x0, double x1, double x2, double &m,
                                               double &s) {
    for (int k0 = 0; k0 < 64; k0 += CH) lse_chunk_fast<D>(T, k0, x0, x1, x2, m, s);
}

// c + (in ? 1 : 0) as one add with carry: the lane mask of the predicate is
// the carry input. Left to itself the compiler packs the eight predicates of
// a chunk into a byte and counts its bits, about 2.5 instructions a pair.
__device__ __forceinline__ int add_pred(int c, bool in) {
    const uint64_t m = __builtin_amdgcn_ballot_w64(in);
    asm("v_addc_co_u32 %0, vcc, 0, %0, %1" : "+v"(c) : "s"(m) : "vcc");
    return c;
}

// The same for a chunk that straddles the cutoff of a T1 rule: each pair
// takes the test t_j > G_j - A (c < C), failing pairs enter as 2^-inf = 0;
// kept pairs are counted. The chunk's records and cutoff constants are taken
// in two halves of 4 targets, so that it holds fewer scalar registers than
// the fast chunk. On a trigger the kept FP32 arguments are shifted by the
// integer dm: exact for the terms near the new reference (Sterbenz), and for
// the others an error of the size their argument's rounding already has.
template <int D, typename RP, typename GP>
__device__ __forceinline__ void lse_chunk_mask(RP T, int k0, GP G, double x0, double x1,
                                               double x2, double A, double &m, double &s,
                                               double &kept) {
    float u[CH];
    float cs = 0.0f;
    int kc = 0;
#pragma unroll
    for (int k = 0; k < CH; ++k) {
        const double t = pair_exp<D>(x0, x1, x2, trec_at<D>(T, k0 + k));
        const bool in = t > G[k0 + k] - A;
        kc = add_pred(kc, in);
        u[k] = in ? (float)(t - m) : -INFINITY;
        const float e = __builtin_amdgcn_exp2f(u[k]);
        cs = k == 0 ? e : cs + e;
    }
    if (!(cs <= 2.0f)) {
        float mx = u[0];
#pragma unroll
        for (int k = 1; k < CH; ++k) mx = fmaxf(mx, u[k]);
        if (mx > 0.0f) {
            const double dm = ceil((double)mx);
            s = ldexp(s, -(int)fmin(dm, 2000.0));
            m += dm;
            cs = 0.0f;
            const float fdm = (float)dm;
#pragma unroll
            for (int k = 0; k < CH; ++k) {
                const float e = __builtin_amdgcn_exp2f(u[k] - fdm);
                cs = k == 0 ? e : cs + e;
            }
        }
    }
    s += (double)cs;
    kept += (double)kc;
}

// Objective pass, one work item = (tile, segment of its block list): per
// lane the partial log2-sum-exp of t_j = B_j + x.Y_j over the segment's
// targets, and the number of pairs it summed. Rows of very different length
// (a tile far from every target keeps many blocks) are split into segments,
// so no wavefront carries a whole long row.
// Under the cutoff rules (MODE_MASK), a block kept whole runs the fast path;
// a block that straddles the cutoff runs its 8-target chunks by their class
// in the entry's chunk mask: skipped, fast, or tested pair by pair. There the
// first reference comes from a target that may lie beyond the cutoff; if it
// then exceeds every kept term by more than 60 (the lane's sum ends below
// 2^-60), FP32 exponentials of kept terms may have underflowed: the lane is
// marked in redo[w], and k_pass1_redo sums it again with the exact online
// maximum.
template <int D, bool F64, int MODE, typename RP, typename R3, typename GP, typename CP,
          typename IP, typename MP>
__device__ __forceinline__ void pass1_item(const double4 *__restrict__ qp, RP trec, R3 trec3,
                                           GP tG, CP blk_cnt, IP row_idx, MP row_cm, int64_t t,
                                           int64_t e0, int64_t e1, double kcs, int64_t w, int lane,
                                           double *__restrict__ part, double *__restrict__ partk,
                                           uint64_t *__restrict__ redo) {
    const int64_t q = t * 64 + lane;
    const double4 xr = qp[q];
    const double x0 = xr.x, x1 = xr.y, x2 = D == 3 ? xr.z : 0.0;
    const double A = -kcs * (x0 * x0 + x1 * x1 + x2 * x2);
    const double rq = ref_offset(q);
    double m = -1e300, s = 0.0, kept = 0.0;
    constexpr bool FAST = !F64;
    if (FAST && e1 > e0) {
        // reference from the first target of the first block (under the tile
        // rule with groups: of its first kept chunk), a kept target
        const uint32_t ent0 = MODE == MODE_DENSE ? (uint32_t)e0 : row_idx[e0];
        const int64_t b0 = (int64_t)(ent0 & ~RSOT_PARTIAL_BIT);
        int k0 = 0;
        if (MODE == MODE_LIST && (ent0 & RSOT_PARTIAL_BIT)) {
            const uint32_t cm0 = row_cm[e0];
            while (k0 < 56 && !((cm0 >> (k0 / 4)) & 2u)) k0 += 8;
        }
        double4 r;
        if constexpr (D == 3) r = trec_at<D>(trec + b0 * 64, k0);
        else r = trec_at<D>(trec3 + b0 * 192, k0);
        m = ceil(pair_exp<D>(x0, x1, x2, r) - rq) + rq;
    }
    // the next list entry is read one block ahead, and the block's pair
    // count before its pairs, so neither load waits at a block boundary
    uint32_t ent_next = MODE == MODE_DENSE ? (uint32_t)e0 : (e1 > e0 ? row_idx[e0] : 0u);
    for (int64_t e = e0; e < e1; ++e) {
        const uint32_t ent = ent_next;
        if (MODE == MODE_DENSE) ent_next = (uint32_t)(e + 1);
        else if (e + 1 < e1) ent_next = row_idx[e + 1];
        const int64_t b = ent & ~RSOT_PARTIAL_BIT;
        auto block = [&](auto T) {
            if (MODE == MODE_LIST && (ent & RSOT_PARTIAL_BIT)) {
                // tile rule with groups: the kept 8-target chunks only
                const uint32_t cm = row_cm[e];
                const int cnt = blk_cnt[b];
                for (int c = 0; c < 8; ++c) {
                    if (!((cm >> (2 * c)) & 2u)) continue;
                    if (FAST) lse_chunk_fast<D>(T, 8 * c, x0, x1, x2, m, s);
                    else lse_chunk<D, F64, false>(T, 8 * c, tG, x0, x1, x2, A, rq, m, s, kept);
                    kept += (double)std::min(8, std::max(0, cnt - 8 * c));
                }
            } else if (MODE == MODE_MASK && (ent & RSOT_PARTIAL_BIT)) {
                if (!FAST) {
                    lse_block<D, F64, true>(T, tG + b * 64, x0, x1, x2, A, rq, m, s, kept);
                } else {
                    const uint32_t cm = row_cm[e];
                    const int cnt = blk_cnt[b];
                    for (int c = 0; c < 8; ++c) {
                        const uint32_t k = (cm >> (2 * c)) & 3u;
                        if (k == PAIR_FULL) {
                            lse_chunk_fast<D>(T, 8 * c, x0, x1, x2, m, s);
                            kept += (double)std::min(8, std::max(0, cnt - 8 * c));
                        } else if (k == PAIR_PARTIAL) {
                            lse_chunk_mask<D>(T, 8 * c, tG + b * 64, x0, x1, x2, A, m, s, kept);
                        }
                    }
                }
            } else {
                const double cnt = (double)blk_cnt[b];
                if (FAST) lse_block_fast<D>(T, x0, x1, x2, m, s);
                else lse_block<D, F64, false>(T, tG, x0, x1, x2, A, rq, m, s, kept);
                kept += cnt;
            }
        };
        if constexpr (D == 3) block(trec + b * 64);
        else block(trec3 + b * 192);
    }
    if constexpr (MODE == MODE_MASK && FAST) {
        const uint64_t lanes = __ballot(kept > 0.0 && !(s >= 0x1p-60));
        if (lane == 0) redo[w] = lanes;
    }
    part[w * 64 + lane] = s > 0.0 ? m + log2(s) : -INFINITY;
    partk[w * 64 + lane] = kept;
}

// Objective pass under the cutoff rules (mixed precision): items in the order
// of their first target block, dealt to the XCDs in runs. With the kept
// count taken as an add with carry the kernel holds 43 vector registers
// (eight waves per SIMD); the compiler's own count, the predicates packed
// into bytes, needed 72.
template <int D>
__global__ __launch_bounds__(256) void k_pass1_cut(
    const double4 *__restrict__ qp, const double4 *__restrict__ trec,
    const double *__restrict__ trec3, const double *__restrict__ tG,
    const int32_t *__restrict__ blk_cnt, const uint32_t *__restrict__ row_idx,
    const uint16_t *__restrict__ row_cm, const int32_t *__restrict__ wi_tile,
    const int64_t *__restrict__ wi_range, const int32_t *__restrict__ perm, int64_t n_items,
    double kcs, double *__restrict__ part, double *__restrict__ partk,
    uint64_t *__restrict__ redo) {
    const int lane = threadIdx.x & 63;
    const int64_t k = xcd_run_item(__builtin_amdgcn_readfirstlane(threadIdx.x >> 6));
    if (k >= n_items) return;
    const int64_t w = perm[k];
    pass1_item<D, false, MODE_MASK>(qp, trec, trec3, tG, blk_cnt, row_idx, row_cm, wi_tile[w],
                                    wi_range[2 * w], wi_range[2 * w + 1], kcs, w, lane, part,
                                    partk, redo);
}

// The marked lanes of objective-pass items under the cutoff rules, summed
// again with the exact online maximum (lse_block, every straddling pair
// tested). One wavefront per item; items with no marked lane return at once.
template <int D>
__global__ __launch_bounds__(256) void k_pass1_redo(
    const double4 *__restrict__ qp, const double4 *__restrict__ trec,
    const double *__restrict__ trec3, const double *__restrict__ tG,
    const int32_t *__restrict__ blk_cnt, const uint32_t *__restrict__ row_idx,
    const int32_t *__restrict__ wi_tile, const int64_t *__restrict__ wi_range, int64_t n_items,
    double kcs, const uint64_t *__restrict__ redo, double *__restrict__ part,
    double *__restrict__ partk) {
    const int lane = threadIdx.x & 63;
    const int64_t w = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (w >= n_items) return;
    const uint64_t lanes = redo[w];
    if (!lanes) return;
    const int64_t t = wi_tile[w], e0 = wi_range[2 * w], e1 = wi_range[2 * w + 1];
    const int64_t q = t * 64 + lane;
    const double4 xr = qp[q];
    const double x0 = xr.x, x1 = xr.y, x2 = D == 3 ? xr.z : 0.0;
    const double A = -kcs * (x0 * x0 + x1 * x1 + x2 * x2);
    const double rq = ref_offset(q);
    double m = -1e300, s = 0.0, kept = 0.0;
    for (int64_t e = e0; e < e1; ++e) {
        const uint32_t ent = row_idx[e];
        const int64_t b = ent & ~RSOT_PARTIAL_BIT;
        auto block = [&](auto T) {
            if (ent & RSOT_PARTIAL_BIT) {
                lse_block<D, false, true>(T, tG + b * 64, x0, x1, x2, A, rq, m, s, kept);
            } else {
                lse_block<D, false, false>(T, tG, x0, x1, x2, A, rq, m, s, kept);
                kept += (double)blk_cnt[b];
            }
        };
        if constexpr (D == 3) block(trec + b * 64);
        else block(trec3 + b * 192);
    }
    if ((lanes >> lane) & 1) {
        part[w * 64 + lane] = s > 0.0 ? m + log2(s) : -INFINITY;
        partk[w * 64 + lane] = kept;
    }
}

template <int D, bool F64, int MODE>
__global__ __launch_bounds__(256) void k_pass1(
    const double4 *__restrict__ qp, const double4 *__restrict__ trec,
    const double *__restrict__ trec3, const double *__restrict__ tG,
    const int32_t *__restrict__ blk_cnt, const uint32_t *__restrict__ row_idx,
    const uint16_t *__restrict__ row_cm, const int32_t *__restrict__ wi_tile,
    const int64_t *__restrict__ wi_range, const int32_t *__restrict__ perm, int64_t n_items,
    int64_t n_blocks, int64_t seg1, int64_t n_seg1, double kcs, double *__restrict__ part,
    double *__restrict__ partk, uint64_t *__restrict__ redo) {
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
        // items in the order of their first target block, dealt to the XCDs
        // in runs of that order
        const int64_t k = xcd_run_item(wave);
        if (k >= n_items) return;
        w = perm[k];
        t = wi_tile[w];
        e0 = wi_range[2 * w];
        e1 = wi_range[2 * w + 1];
    }
    pass1_item<D, F64, MODE>(qp, trec, trec3, tG, blk_cnt, row_idx, row_cm, t, e0, e1, kcs, w,
                             lane, part, partk, redo);
}

// One wavefront per tile: merge the tile's partial log-sum-exps (FP64) into
// Lt = log2 sum_j 2^(B_j + x.Y_j) (lcorr = log2 of the exponential's mean
// correction), L_q = (Lt + A_q) ln 2, and the tile's objective, ln D,
// kept-pair and empty-point partials. For the gradient pass: the tile's
// reference R_T = ceil(max_q log2 mu_q - r_T) + r_T (r_T = ref_offset(T)),
// S_q = log2 mu_q - Lt - R_T, so that the argument log2(mu_q p_qj) - R_T of a
// dominant term is O(1) however small mu_q is, and tile_ref[T] =
// {R_T, 2^R_T corr} to scale the tile's sums back.
__global__ __launch_bounds__(256) void k_pass1_combine(
    double4 *__restrict__ qp, const double *__restrict__ qmu, const double *__restrict__ qlog2mu,
    const int32_t *__restrict__ qperm, const double *__restrict__ part,
    const double *__restrict__ partk, const int64_t *__restrict__ wi_ptr, int64_t n_seg1,
    int64_t n_tiles, double kcs, int want_A, double lcorr, double corr,
    double *__restrict__ qA, double *__restrict__ qlse, int32_t *__restrict__ qkept,
    double2 *__restrict__ tile_ref, double *__restrict__ tile_part,
    double *__restrict__ tile_smax) {
    const int lane = threadIdx.x & 63;
    const int64_t t = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (t >= n_tiles) return;
    const int64_t q = t * 64 + lane;
    const int64_t w0 = wi_ptr ? wi_ptr[t] : t * n_seg1;
    const int64_t w1 = wi_ptr ? wi_ptr[t + 1] : w0 + n_seg1;
    double mx = -INFINITY, kept = 0.0;
    for (int64_t w = w0; w < w1; ++w) {
        mx = fmax(mx, part[w * 64 + lane]);
        kept += partk[w * 64 + lane];
    }
    double sum = 0.0;
    if (mx > -INFINITY)
        for (int64_t w = w0; w < w1; ++w) sum += exp2(part[w * 64 + lane] - mx);
    const double4 xr = qp[q];
    const double A = -kcs * (xr.x * xr.x + xr.y * xr.y + xr.z * xr.z);
    const bool real = qperm[q] >= 0;
    const bool empty = !(mx > -INFINITY);
    const double Lt = empty ? -INFINITY : mx + log2(sum) + lcorr;
    const double lm = qlog2mu[q];
    const double lmax = wave_max(real && !empty ? lm : -INFINITY);
    const double rT = ref_offset(t);
    const double RT = lmax > -INFINITY ? ceil(lmax - rT) + rT : 0.0;
    const double S = empty ? -INFINITY : lm - Lt - RT;
    reinterpret_cast<double *>(qp)[q * 4 + 3] = S;
    if (want_A) qA[q] = A;
    const double L2 = Lt + A;
    qlse[q] = empty ? -INFINITY : L2 * RSOT_LN2;
    qkept[q] = real ? (int32_t)kept : 0;
    const double jp = (real && !empty) ? qmu[q] * L2 : 0.0;
    const double dl = (real && !empty && lm > -INFINITY) ? (lm - L2) * RSOT_LN2 : -INFINITY;
    const double js = wave_sum(jp);
    const double dm = wave_max(dl);
    const double ds = wave_sum(dm > -INFINITY ? exp(dl - dm) : 0.0);
    const double ks = wave_sum(real ? kept : 0.0);
    const double es = wave_sum(real && empty ? 1.0 : 0.0);
    if (tile_smax) {
        const double sm = wave_max(real && !empty ? S : -INFINITY);
        if (lane == 0) tile_smax[t] = sm;
    }
    if (lane == 0) {
        tile_ref[t] = make_double2(RT, exp2(RT) * corr);
        tile_part[t * 4 + 0] = js;
        tile_part[t * 4 + 1] = dm > -INFINITY ? dm + log(ds) : -INFINITY;
        tile_part[t * 4 + 2] = ks;
        tile_part[t * 4 + 3] = es;
    }
}

// ---------------------------------------------------------------------------
// gradient pass
// ---------------------------------------------------------------------------
// Sum over 8 points (a chunk of a tile) of 2^(B + S'_q + x_q.Y) for this
// lane's target, S'_q = log2 mu_q - Lt_q - R_T carried in the point records.
// MASK (cutoff rules): only pairs with t > G - A_q enter, t = B + x_q.Y formed
// as in the objective pass (pair_exp), A_q from qA; both passes then decide
// every pair's membership on the same FP64 operands.
template <int D, bool F64, bool MASK, typename QP, typename AP>
__device__ __forceinline__ double mass_chunk(QP Q, int i0, AP qA, double Y0, double Y1,
                                             double Y2, double B, double G) {
    const double4 rec = make_double4(Y0, Y1, Y2, B);
    if (F64) {
        double cs = 0.0;
#pragma unroll
        for (int k = 0; k < CH; ++k) {
            const double4 r = ld4(Q + i0 + k);
            double v;
            if (MASK) {
                const double t = pair_exp<D>(r.x, r.y, r.z, rec);
                v = t > G - qA[i0 + k] ? t + r.w : -INFINITY;
            } else {
                v = B + r.w;
                v = fma(r.x, Y0, v);
                v = fma(r.y, Y1, v);
                if (D == 3) v = fma(r.z, Y2, v);
            }
            const double e = exp2(v);
            cs = k == 0 ? e : cs + e;
        }
        return cs;
    } else {
        float cs = 0.0f;
#pragma unroll
        for (int k = 0; k < CH; ++k) {
            const double4 r = ld4(Q + i0 + k);
            float u;
            if (MASK) {
                const double t = pair_exp<D>(r.x, r.y, r.z, rec);
                u = (float)(t + r.w);
                u = t > G - qA[i0 + k] ? u : -INFINITY;
            } else {
                double v = B + r.w;
                v = fma(r.x, Y0, v);
                v = fma(r.y, Y1, v);
                if (D == 3) v = fma(r.z, Y2, v);
                u = (float)v;
            }
            const float e = __builtin_amdgcn_exp2f(u);
            cs = k == 0 ? e : cs + e;
        }
        return (double)cs;
    }
}

template <int D, bool F64, typename QP>
__device__ __forceinline__ double mass_tile(QP Q, double Y0, double Y1, double Y2, double B) {
    double acc = 0.0;
    for (int i0 = 0; i0 < 64; i0 += CH)
        acc += mass_chunk<D, F64, false>(Q, i0, (const double *)nullptr, Y0, Y1, Y2, B, 0.0);
    return acc;
}

// Gradient pass, one work item = (target block, segment of its tile list).
// Under the cutoff rules a tile that straddles the cutoff runs its 8-point
// chunks by their class in the entry's chunk mask (FP64: every pair tested).
// Under the tile rule with culling groups, an entry that keeps only some of
// the block's 8-target chunks carries their bits: the other lanes' terms
// enter as 2^-inf = 0.
template <int D, bool F64, int MODE, typename QP, typename AP, typename IP, typename RP,
          typename CP>
__device__ __forceinline__ void pass2_item(QP qp, AP qA, RP tref, const double4 *__restrict__ trec,
                                           const double *__restrict__ tG, IP col_idx, CP col_cm,
                                           int64_t b, int64_t e0, int64_t e1, int64_t w, int lane,
                                           double *__restrict__ gpart) {
    const int64_t j = b * 64 + lane;
    const double4 rec = trec[j];
    const double G = MODE == MODE_MASK ? tG[j] : 0.0;
    double acc = 0.0;
    uint32_t ent_next = MODE == MODE_DENSE ? (uint32_t)e0 : (e1 > e0 ? col_idx[e0] : 0u);
    for (int64_t e = e0; e < e1; ++e) {
        const uint32_t ent = ent_next;
        if (MODE == MODE_DENSE) ent_next = (uint32_t)(e + 1);
        else if (e + 1 < e1) ent_next = col_idx[e + 1];
        const int64_t t = ent & ~RSOT_PARTIAL_BIT;
        const auto Q = qp + t * 64;
        const double scale = tref[t].y;
        if (MODE == MODE_MASK && (ent & RSOT_PARTIAL_BIT)) {
            double a = 0.0;
            for (int i0 = 0; i0 < 64; i0 += CH)
                a += mass_chunk<D, F64, true>(Q, i0, qA + t * 64, rec.x, rec.y, rec.z, rec.w, G);
            acc += a * scale;
        } else if (MODE == MODE_LIST && (ent & RSOT_PARTIAL_BIT)) {
            const double Bl = ((col_cm[e] >> (lane >> 3)) & 1u) ? rec.w : -INFINITY;
            acc += mass_tile<D, F64>(Q, rec.x, rec.y, rec.z, Bl) * scale;
        } else {
            acc += mass_tile<D, F64>(Q, rec.x, rec.y, rec.z, rec.w) * scale;
        }
    }
    gpart[w * 64 + lane] = acc;
}

template <int D, bool F64, int MODE>
__global__ __launch_bounds__(256) void k_pass2(
    const double4 *__restrict__ qp, const double *__restrict__ qA,
    const double2 *__restrict__ tref, const double4 *__restrict__ trec,
    const double *__restrict__ tG, const int32_t *__restrict__ wi_block,
    const int64_t *__restrict__ wi_range, const int32_t *__restrict__ perm,
    const uint32_t *__restrict__ col_idx, const uint8_t *__restrict__ col_cm, int64_t n_tiles,
    int64_t n_blocks, int64_t n_wi, int64_t n_seg, int64_t seg, double *__restrict__ gpart) {
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    int64_t b, w, e0, e1;
    if (MODE == MODE_DENSE) {
        // Workgroup i is dispatched to XCD i % 8. Each XCD sweeps its own
        // point segments (s = 8k + xcd), all block groups of one segment
        // before the next, so the segment's point records stay in that XCD's
        // L2 while every target block reads them. The four wavefronts of a
        // workgroup share the segment.
        const int64_t nbg = (n_blocks + 3) / 4;
        const int64_t kk = blockIdx.x >> 3;
        const int64_t sgi = (kk / nbg) * 8 + (blockIdx.x & 7);
        b = (kk % nbg) * 4 + wave;
        if (sgi >= n_seg || b >= n_blocks) return;
        e0 = sgi * seg;
        e1 = std::min<int64_t>(e0 + seg, n_tiles);
        w = b * n_seg + sgi;
    } else {
        // items in the order of their first point tile, dealt to the XCDs in
        // runs of that order: items that read the same point records share
        // that XCD's L2
        const int64_t k = xcd_run_item(wave);
        if (k >= n_wi) return;
        w = perm[k];
        b = wi_block[w];
        e0 = wi_range[2 * w];
        e1 = wi_range[2 * w + 1];
    }
    pass2_item<D, F64, MODE>(qp, qA, tref, trec, tG, col_idx, col_cm, b, e0, e1, w, lane, gpart);
}

// ---------------------------------------------------------------------------
// batched evaluation: one launch per pass over many problems
// ---------------------------------------------------------------------------
// Work descriptor of one problem in a batch (device memory).
struct BatchDesc {
    int dim, mode;
    int64_t n_tiles, n_blocks;
    const double4 *qp;
    const double *qA;
    const double2 *tile_ref;
    const double4 *trec;
    const double *trec3;
    const double *tG;
    const int32_t *blk_cnt;
    const uint32_t *row_idx;
    const uint16_t *row_cm;
    const int32_t *wi1_tile;
    const int64_t *wi1_range;
    const int32_t *wi1_perm;
    int64_t n_items1, seg1, n_seg1;
    double kcs;
    double *part1, *part1k;
    const uint32_t *col_idx;
    const uint8_t *col_cm;
    const int32_t *wi_block;
    const int64_t *wi_range;
    const int32_t *wi_perm;
    int64_t n_wi, n_seg, seg;
    double *gpart;
};

// position k of the problem owning group item g: begin[k] <= g < begin[k+1]
__device__ inline int owner(const int64_t *__restrict__ begin, int n, uint64_t g) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if ((uint64_t)begin[mid] <= g) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// A pointer read from a descriptor, made wave-uniform and marked read-only
// (constant address space) so its loads can go through the scalar cache.
template <typename T>
__device__ __forceinline__ const RSOT_CAS T *uniform_const(const T *p) {
    return (const RSOT_CAS T *)uniform_u64((uint64_t)p);
}

// Objective pass of every problem of one (dimension, rule) group of the
// batch, one launch: the group's items (problems in decreasing cost order,
// each problem's items in its own sorted order) are numbered consecutively
// and dealt to the XCDs in runs as in the single-problem passes; each wave
// finds its item's problem by binary search and runs the same item body.
template <int D, int MODE>
__global__ __launch_bounds__(256) void k_pass1_batched(const BatchDesc *__restrict__ descs,
                                                       const int32_t *__restrict__ order,
                                                       const int64_t *__restrict__ begin, int n) {
    const int lane = threadIdx.x & 63;
    const uint64_t g = (uint64_t)xcd_run_item(__builtin_amdgcn_readfirstlane(threadIdx.x >> 6));
    if (g >= (uint64_t)begin[n]) return;
    const int k = owner(begin, n, g);
    const BatchDesc &d = descs[order[k]];
    const int64_t v = (int64_t)(g - (uint64_t)begin[k]);
    int64_t t, e0, e1, w;
    if (MODE == MODE_DENSE) {
        // consecutive items share the block segment (target records)
        const int64_t s1 = v / d.n_tiles;
        t = v % d.n_tiles;
        e0 = s1 * d.seg1;
        e1 = std::min<int64_t>(e0 + d.seg1, d.n_blocks);
        w = t * d.n_seg1 + s1;
    } else {
        w = uniform_const(d.wi1_perm)[v];
        t = uniform_const(d.wi1_tile)[w];
        e0 = uniform_const(d.wi1_range)[2 * w];
        e1 = uniform_const(d.wi1_range)[2 * w + 1];
    }
    pass1_item<D, false, MODE>(d.qp, uniform_const(d.trec), uniform_const(d.trec3),
                               uniform_const(d.tG), uniform_const(d.blk_cnt),
                               uniform_const(d.row_idx), uniform_const(d.row_cm), t, e0, e1,
                               d.kcs, w, lane, d.part1, d.part1k, (uint64_t *)nullptr);
}

template <int D, int MODE>
__global__ __launch_bounds__(256) void k_pass2_batched(const BatchDesc *__restrict__ descs,
                                                       const int32_t *__restrict__ order,
                                                       const int64_t *__restrict__ begin, int n) {
    const int lane = threadIdx.x & 63;
    const uint64_t g = (uint64_t)xcd_run_item(__builtin_amdgcn_readfirstlane(threadIdx.x >> 6));
    if (g >= (uint64_t)begin[n]) return;
    const int k = owner(begin, n, g);
    const BatchDesc &d = descs[order[k]];
    const int64_t v = (int64_t)(g - (uint64_t)begin[k]);
    int64_t b, e0, e1, w;
    if (MODE == MODE_DENSE) {
        // consecutive items share the point segment (point records)
        const int64_t sgi = v / d.n_blocks;
        b = v % d.n_blocks;
        e0 = sgi * d.seg;
        e1 = std::min<int64_t>(e0 + d.seg, d.n_tiles);
        w = b * d.n_seg + sgi;
    } else {
        w = uniform_const(d.wi_perm)[v];
        b = uniform_const(d.wi_block)[w];
        e0 = uniform_const(d.wi_range)[2 * w];
        e1 = uniform_const(d.wi_range)[2 * w + 1];
    }
    pass2_item<D, false, MODE>(uniform_const(d.qp), uniform_const(d.qA),
                               uniform_const(d.tile_ref), d.trec, d.tG,
                               uniform_const(d.col_idx), uniform_const(d.col_cm), b, e0, e1, w,
                               lane, d.gpart);
}

// per target: merge the work-item partials in order, un-permute, norms
// One workgroup per target block: wave v sums the block's item partials
// v, v + 4, v + 8, ... in four interleaved accumulators (so that many loads
// are in flight however many items a block has), the four wave sums are
// added in a fixed order, and wave 0 writes the gradient and the block's
// norm partials.
__global__ __launch_bounds__(256) void k_grad_reduce(
    const double *__restrict__ gpart, const int64_t *__restrict__ wi_ptr, int64_t n_seg,
    const double *__restrict__ tnu, const int32_t *__restrict__ tperm, int64_t n_blocks,
    const double *__restrict__ dscal, double *__restrict__ grad_out,
    double *__restrict__ blk_gpart) {
    __shared__ double red[4][64];
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const int64_t b = blockIdx.x;
    if (b >= n_blocks) return;
    const int64_t j = b * 64 + lane;
    const int64_t w0 = wi_ptr ? wi_ptr[b] : b * n_seg;
    const int64_t w1 = wi_ptr ? wi_ptr[b + 1] : w0 + n_seg;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    int64_t w = w0 + wv;
    for (; w + 12 < w1; w += 16)
#pragma unroll
        for (int k = 0; k < 4; ++k) acc[k] += gpart[(w + 4 * k) * 64 + lane];
    if (w < w1) acc[0] += gpart[w * 64 + lane];
    if (w + 4 < w1) acc[1] += gpart[(w + 4) * 64 + lane];
    if (w + 8 < w1) acc[2] += gpart[(w + 8) * 64 + lane];
    red[wv][lane] = (acc[0] + acc[1]) + (acc[2] + acc[3]);
    __syncthreads();
    if (wv != 0) return;
    const double nut = (red[0][lane] + red[1][lane]) + (red[2][lane] + red[3][lane]);
    const double g = nut - tnu[j];
    const int32_t dst = tperm[j];
    const bool ok = dscal[SC_NONFINITE] == 0.0;
    if (dst >= 0 && ok && grad_out) grad_out[dst] = g;
    const double a = dst >= 0 ? fabs(g) : 0.0;
    const double s1 = wave_sum(a);
    const double mx = wave_max(a);
    if (lane == 0) {
        blk_gpart[b * 2 + 0] = s1;
        blk_gpart[b * 2 + 1] = mx;
    }
}

// single workgroup: evaluation statistics (kept pairs, empty points, ln D,
// gradient norms), each summed in a fixed order
__global__ __launch_bounds__(256) void k_finalize(const double *__restrict__ tile_part,
                                                  int64_t n_tiles,
                                                  const double *__restrict__ blk_gpart,
                                                  int64_t n_blocks, int have_grad,
                                                  double *__restrict__ dscal) {
    __shared__ double red[4][6];
    const int w = threadIdx.x >> 6;
    const bool l0 = (threadIdx.x & 63) == 0;
    double kp = 0.0, em = 0.0, dmx = -INFINITY;
    for (int64_t t = threadIdx.x; t < n_tiles; t += 256) {
        dmx = fmax(dmx, tile_part[t * 4 + 1]);
        kp += tile_part[t * 4 + 2];
        em += tile_part[t * 4 + 3];
    }
    kp = wave_sum(kp);
    em = wave_sum(em);
    dmx = wave_max(dmx);
    if (l0) {
        red[w][0] = kp;
        red[w][1] = em;
        red[w][2] = dmx;
    }
    __syncthreads();
    const double dall = fmax(fmax(red[0][2], red[1][2]), fmax(red[2][2], red[3][2]));
    double dsum = 0.0;
    if (dall > -INFINITY)
        for (int64_t t = threadIdx.x; t < n_tiles; t += 256) {
            const double v = tile_part[t * 4 + 1];
            dsum += v > -INFINITY ? exp(v - dall) : 0.0;
        }
    double g1 = 0.0, gi = 0.0;
    if (have_grad)
        for (int64_t b = threadIdx.x; b < n_blocks; b += 256) {
            g1 += blk_gpart[b * 2 + 0];
            gi = fmax(gi, blk_gpart[b * 2 + 1]);
        }
    dsum = wave_sum(dsum);
    g1 = wave_sum(g1);
    gi = wave_max(gi);
    if (l0) {
        red[w][3] = dsum;
        red[w][4] = g1;
        red[w][5] = gi;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    double ks = 0.0, es = 0.0, ds = 0.0, gs = 0.0, gm = 0.0;
    for (int i = 0; i < 4; ++i) {
        ks += red[i][0];
        es += red[i][1];
        ds += red[i][3];
        gs += red[i][4];
        gm = fmax(gm, red[i][5]);
    }
    dscal[SC_KEPT] = ks;
    dscal[SC_EMPTY] = es;
    dscal[SC_LOGD] = dall > -INFINITY ? dall + log(ds) : -INFINITY;
    dscal[SC_GL1] = gs;
    dscal[SC_GLINF] = gm;
}

// J = eps ln2 sum_q mu_q L2_q - sum_j psi_j nu_j (Alg. 2, last two lines);
// kept in its own single-workgroup kernel so the sum order is fixed.
__global__ __launch_bounds__(256) void k_objective(const double *__restrict__ tile_part,
                                                   int64_t n_tiles, double eps,
                                                   double *__restrict__ dscal) {
    __shared__ double red[4];
    double js = 0.0;
    for (int64_t t = threadIdx.x; t < n_tiles; t += 256) js += tile_part[t * 4 + 0];
    js = wave_sum(js);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = js;
    __syncthreads();
    if (threadIdx.x != 0) return;
    const double s = (red[0] + red[1]) + (red[2] + red[3]);
    dscal[SC_SUM_L2] = s;
    dscal[SC_J] = eps * RSOT_LN2 * s - dscal[SC_PSINU];
}

// ---------------------------------------------------------------------------
// driver
// ---------------------------------------------------------------------------
template <typename T>
static rsot_status grow(rsot_problem *p, T **ptr, size_t *cap, size_t count) {
    if (*ptr && *cap >= count) return RSOT_OK;
    if (*ptr) rsot_dev_free(p, *ptr);
    *ptr = nullptr;
    void *q = nullptr;
    size_t c = std::max<size_t>(count + count / 4, 64);
    RSOT_TRY(rsot_dev_alloc(p, &q, c * sizeof(T)));
    *ptr = (T *)q;
    *cap = c;
    return RSOT_OK;
}

struct Pass1Work {
    int64_t n_items, seg1, n_seg1;
};

// log2 of the exponential's mean correction, and the correction, for the
// precision the pair loops run in
static double pass_lcorr(const rsot_problem *p, bool f64) { return f64 ? 0.0 : std::log2(p->exp_corr); }
static double pass_corr(const rsot_problem *p, bool f64) { return f64 ? 1.0 : p->exp_corr; }

template <int D, bool F64, int MODE>
static void launch_pass1(rsot_problem *p, double kcs, const Pass1Work &pw) {
    const unsigned grid = MODE == MODE_DENSE ? (unsigned)((pw.n_items + 3) / 4)
                                             : xcd_run_grid(pw.n_items);
    if (MODE == MODE_MASK && !F64)
        hipLaunchKernelGGL(k_pass1_cut<D>, dim3(grid), dim3(256), 0, p->stream, p->qp, p->trec,
                           p->trec3, p->tG, p->blk_cnt, p->row_idx, p->row_cm, p->wi1_tile,
                           p->wi1_range, p->wi1_perm, pw.n_items, kcs, p->part1, p->part1k,
                           p->redo1);
    else
        hipLaunchKernelGGL((k_pass1<D, F64, MODE>), dim3(grid), dim3(256), 0, p->stream, p->qp,
                           p->trec, p->trec3, p->tG, p->blk_cnt, p->row_idx, p->row_cm,
                           p->wi1_tile, p->wi1_range, p->wi1_perm, pw.n_items, p->n_blocks,
                           pw.seg1, pw.n_seg1, kcs, p->part1, p->part1k, p->redo1);
    if (MODE == MODE_MASK && !F64)
        hipLaunchKernelGGL(k_pass1_redo<D>, dim3((unsigned)((pw.n_items + 3) / 4)), dim3(256), 0,
                           p->stream, p->qp, p->trec, p->trec3, p->tG, p->blk_cnt, p->row_idx,
                           p->wi1_tile, p->wi1_range, pw.n_items, kcs, p->redo1, p->part1,
                           p->part1k);
    hipLaunchKernelGGL(k_pass1_combine, dim3((unsigned)((p->n_tiles + 3) / 4)), dim3(256), 0,
                       p->stream, p->qp, p->qmu, p->qlog2mu, p->qperm, p->part1, p->part1k,
                       MODE == MODE_DENSE ? (const int64_t *)nullptr : p->wi1_ptr, pw.n_seg1,
                       p->n_tiles, kcs, MODE == MODE_MASK ? 1 : 0, pass_lcorr(p, F64),
                       pass_corr(p, F64), p->qA, p->qlse, p->qkept, p->tile_ref, p->tile_part,
                       p->tile_smax);
}

template <int D, bool F64, int MODE>
static void launch_pass2(rsot_problem *p, int64_t n_wi, int64_t n_seg, int64_t seg) {
    unsigned grid;
    if (MODE == MODE_DENSE)
        grid = (unsigned)(((p->n_blocks + 3) / 4) * ((n_seg + 7) / 8) * 8);
    else
        grid = xcd_run_grid(n_wi);
    hipLaunchKernelGGL((k_pass2<D, F64, MODE>), dim3(grid), dim3(256), 0, p->stream, p->qp, p->qA,
                       p->tile_ref, p->trec, p->tG, p->wi_block, p->wi_range, p->wi_perm, p->col_idx,
                       p->col_cm, p->n_tiles, p->n_blocks, n_wi, n_seg, seg, p->gpart);
}

template <int D, bool F64>
static void launch_passes(rsot_problem *p, int mode, bool grad, double kcs, int64_t n_wi,
                          int64_t n_seg, int64_t seg, const Pass1Work &pw) {
    if (mode == MODE_DENSE) launch_pass1<D, F64, MODE_DENSE>(p, kcs, pw);
    else if (mode == MODE_LIST) launch_pass1<D, F64, MODE_LIST>(p, kcs, pw);
    else launch_pass1<D, F64, MODE_MASK>(p, kcs, pw);
    (void)hipEventRecord(p->ev_mid, p->stream);
    if (!grad) return;
    if (mode == MODE_DENSE) launch_pass2<D, F64, MODE_DENSE>(p, n_wi, n_seg, seg);
    else if (mode == MODE_LIST) launch_pass2<D, F64, MODE_LIST>(p, n_wi, n_seg, seg);
    else launch_pass2<D, F64, MODE_MASK>(p, n_wi, n_seg, seg);
}

// The squared geodesic cost on the sphere: its own pair kernels, the shared
// merge (with no point term: the cost has no |x|^2 part) and reductions.
static void launch_passes_sphere(rsot_problem *p, bool f64, int mode, bool grad, double kcs,
                                 int64_t n_wi, int64_t n_seg, int64_t seg, const Pass1Work &pw) {
    rsot_sphere_pass1(p, f64, mode, kcs, pw.n_items, pw.seg1, pw.n_seg1);
    hipLaunchKernelGGL(k_pass1_combine, dim3((unsigned)((p->n_tiles + 3) / 4)), dim3(256), 0,
                       p->stream, p->qp, p->qmu, p->qlog2mu, p->qperm, p->part1, p->part1k,
                       mode == MODE_DENSE ? (const int64_t *)nullptr : p->wi1_ptr, pw.n_seg1,
                       p->n_tiles, 0.0, 0, pass_lcorr(p, f64), pass_corr(p, f64), p->qA,
                       p->qlse, p->qkept, p->tile_ref, p->tile_part, p->tile_smax);
    (void)hipEventRecord(p->ev_mid, p->stream);
    if (grad) rsot_sphere_pass2(p, f64, mode, kcs, n_wi, n_seg, seg);
}

// Segments per row: enough (row, segment) wavefronts to fill the device
// (16,384), each segment at least 64 columns.
static void cull_segments(int64_t nrows, int64_t ncols, int *nseg, int64_t *seg_len) {
    const int64_t want = std::max<int64_t>(1, (16384 + nrows - 1) / nrows);
    const int64_t most = std::max<int64_t>(1, (ncols + 63) / 64);
    const int64_t ns = std::min(want, most);
    int64_t len = (ncols + ns - 1) / ns;
    len = (len + 63) / 64 * 64;
    *seg_len = len;
    *nseg = (int)((ncols + len - 1) / len);
}

// Culling group of the tile rule: targets per group (64 = whole blocks)
static int tile_group(const rsot_problem *p) {
    return p->opt.tile_group > 0 ? (int)p->opt.tile_group : RSOT_TILE_GROUP_DEFAULT;
}

// Buffers of the culling step: list pointers and counts; for the tile rule
// the per-tile B* and threshold, and with culling groups the group tables;
// for the cutoff rules the boxes of 8-target chunks (made once).
static rsot_status ensure_cull_buffers(rsot_problem *p, bool tile_rule, hipStream_t st) {
    if (!p->row_ptr) {
        RSOT_TRY(rsot_dev_alloc(p, (void **)&p->row_ptr, sizeof(int64_t) * (p->n_tiles + 1)));
        RSOT_TRY(rsot_dev_alloc(p, (void **)&p->col_ptr, sizeof(int64_t) * (p->n_blocks + 1)));
        RSOT_TRY(rsot_dev_alloc(p, (void **)&p->wi_ptr, sizeof(int64_t) * (p->n_blocks + 1)));
        RSOT_TRY(rsot_dev_alloc(p, (void **)&p->wi1_ptr, sizeof(int64_t) * (p->n_tiles + 1)));
        RSOT_TRY(rsot_dev_alloc(p, (void **)&p->row_cnt, sizeof(int32_t) * p->n_tiles));
        RSOT_TRY(rsot_dev_alloc(p, (void **)&p->col_cnt, sizeof(int32_t) * p->n_blocks));
        const int64_t np = (std::max(p->n_tiles, p->n_blocks) + 1023) / 1024;
        RSOT_TRY(rsot_dev_alloc(p, (void **)&p->scan_tmp, sizeof(int64_t) * np));
        int ns = 1;
        int64_t len = 0;
        cull_segments(p->n_tiles, p->n_blocks, &ns, &len);
        RSOT_TRY(rsot_dev_alloc(p, (void **)&p->row_scnt, sizeof(int32_t) * p->n_tiles * ns));
        cull_segments(p->n_blocks, p->n_tiles, &ns, &len);
        RSOT_TRY(rsot_dev_alloc(p, (void **)&p->col_scnt, sizeof(int32_t) * p->n_blocks * ns));
        const size_t rw = (size_t)p->n_tiles * (size_t)((p->n_blocks + 63) / 64);
        const size_t cw = (size_t)p->n_blocks * (size_t)((p->n_tiles + 63) / 64);
        RSOT_TRY(rsot_dev_alloc(p, (void **)&p->row_kbits, sizeof(uint64_t) * rw));
        RSOT_TRY(rsot_dev_alloc(p, (void **)&p->col_kbits, sizeof(uint64_t) * cw));
    }
    const bool groups = tile_rule && tile_group(p) < 64;
    if ((!tile_rule || groups) && !p->row_pbits) {
        const size_t rw = (size_t)p->n_tiles * (size_t)((p->n_blocks + 63) / 64);
        const size_t cw = (size_t)p->n_blocks * (size_t)((p->n_tiles + 63) / 64);
        RSOT_TRY(rsot_dev_alloc(p, (void **)&p->row_pbits, sizeof(uint64_t) * rw));
        RSOT_TRY(rsot_dev_alloc(p, (void **)&p->col_pbits, sizeof(uint64_t) * cw));
    }
    if (tile_rule && !p->tile_bstar) {
        RSOT_TRY(rsot_dev_alloc(p, (void **)&p->tile_bstar, sizeof(int32_t) * p->n_tiles));
        RSOT_TRY(rsot_dev_alloc(p, (void **)&p->tile_thr, sizeof(double) * p->n_tiles));
    }
    // the group masks of every (tile, block) pair and their transpose, when
    // both fit in 4 GiB (else every culling pass recomputes them)
    if (groups && !p->gmask && !p->gmask_tried) {
        p->gmask_tried = 1;
        const size_t nf = (size_t)p->n_tiles * (size_t)p->n_blocks;
        if (2 * nf <= ((size_t)1 << 32) &&
            rsot_dev_alloc(p, (void **)&p->gmask, nf) == RSOT_OK) {
            if (rsot_dev_alloc(p, (void **)&p->gmaskT, nf) == RSOT_OK) {
                p->gmask_ok = 1;
            } else {
                rsot_dev_free(p, p->gmask);
                p->gmask = nullptr;
            }
        }
    }
    if (groups && !p->grp_lo) {       // sized for the smallest group, 8 targets
        const int64_t ng = p->n_pad / 8;
        RSOT_TRY(rsot_dev_alloc(p, (void **)&p->grp_lo, sizeof(double) * 3 * ng));
        RSOT_TRY(rsot_dev_alloc(p, (void **)&p->grp_hi, sizeof(double) * 3 * ng));
        RSOT_TRY(rsot_dev_alloc(p, (void **)&p->grp_lnnu, sizeof(double) * ng));
        RSOT_TRY(rsot_dev_alloc(p, (void **)&p->grp_psi, sizeof(double) * ng));
    }
    if (!tile_rule && !p->tch_lo) {
        const int64_t ntc = p->n_pad / 8;
        RSOT_TRY(rsot_dev_alloc(p, (void **)&p->tch_lo, sizeof(double) * 3 * ntc));
        RSOT_TRY(rsot_dev_alloc(p, (void **)&p->tch_hi, sizeof(double) * 3 * ntc));
        hipLaunchKernelGGL(k_chunk_boxes, dim3((unsigned)((ntc + 255) / 256)), dim3(256), 0, st,
                           p->ty, 3, ntc, p->tch_lo, p->tch_hi);
        RSOT_HIP(hipGetLastError());
    }
    return RSOT_OK;
}

// culling into the row (tile) or column (target block) lists: count or fill
static void launch_cull(rsot_problem *p, hipStream_t st, int D, bool tile_rule, bool rows,
                        bool fill, double eps) {
    const int64_t nrows = rows ? p->n_tiles : p->n_blocks;
    int nseg = 1;
    int64_t seg_len = 0;
    cull_segments(nrows, rows ? p->n_blocks : p->n_tiles, &nseg, &seg_len);
    const dim3 g((unsigned)((nrows * nseg + 3) / 4));
    const double cs = p->opt.cost_scale;
    int32_t *cnt = rows ? p->row_scnt : p->col_scnt;
    const int64_t *ptr = rows ? p->row_ptr : p->col_ptr;
    uint32_t *idx = rows ? p->row_idx : p->col_idx;
    uint16_t *cm = rows ? p->row_cm : nullptr;
    uint64_t *kb = rows ? p->row_kbits : p->col_kbits;
    uint64_t *pb = rows ? p->row_pbits : p->col_pbits;
    const int grp = tile_rule ? tile_group(p) : 64;
    // tile rule with groups and stored masks: the row count pass writes them,
    // every other pass reads them (the column passes the transposed copy)
    const bool masks = tile_rule && grp < 64 && p->gmask_ok;
    uint8_t *gm_out = (masks && rows && !fill) ? p->gmask : nullptr;
    const uint8_t *gm_in = !masks ? nullptr : (rows ? (fill ? p->gmask : nullptr) : p->gmaskT);
#define RSOT_CULL(DD, TT, RR, FF)                                                              \
    hipLaunchKernelGGL((k_cull<DD, TT, RR, FF>), g, dim3(256), 0, st, p->tile_lo, p->tile_hi,    \
                       p->blk_lo, p->blk_hi, p->tch_lo, p->tch_hi,                               \
                       p->blk_lnnu, p->blk_stat, p->tile_bstar, p->tile_thr, p->n_tiles,         \
                       p->n_blocks, nseg, seg_len, cs, eps, p->dscal, cnt, kb, pb, ptr, idx, cm, \
                       grp, p->grp_lo, p->grp_hi, p->grp_lnnu, p->grp_psi, p->blk_cnt,          \
                       rows ? nullptr : p->col_cm, gm_out, gm_in,                                \
                       p->opt.cost_kind == RSOT_COST_SPHERE ? 1 : 0)
#define RSOT_CULL_F(DD, TT, RR)                                                                \
    do {                                                                                        \
        if (fill) RSOT_CULL(DD, TT, RR, true);                                                  \
        else RSOT_CULL(DD, TT, RR, false);                                                      \
    } while (0)
#define RSOT_CULL_R(DD, TT)                                                                    \
    do {                                                                                        \
        if (rows) RSOT_CULL_F(DD, TT, true);                                                    \
        else RSOT_CULL_F(DD, TT, false);                                                        \
    } while (0)
    if (D == 2) {
        if (tile_rule) RSOT_CULL_R(2, true);
        else RSOT_CULL_R(2, false);
    } else {
        if (tile_rule) RSOT_CULL_R(3, true);
        else RSOT_CULL_R(3, false);
    }
#undef RSOT_CULL_R
#undef RSOT_CULL_F
#undef RSOT_CULL
    if (!fill)
        hipLaunchKernelGGL(k_seg_sum, dim3((unsigned)((nrows + 255) / 256)), dim3(256), 0, st, cnt,
                           nrows, nseg, rows ? p->row_cnt : p->col_cnt);
    if (gm_out)
        hipLaunchKernelGGL(k_transpose_u8,
                           dim3((unsigned)((p->n_blocks + 63) / 64), (unsigned)((p->n_tiles + 63) / 64)),
                           dim3(256), 0, st, p->gmask, p->n_tiles, p->n_blocks, p->gmaskT);
}

// The column count pass: the row count pass's bits transposed, then the
// kept pairs per (block, segment of its tiles) and per block.
static void launch_col_counts(rsot_problem *p, hipStream_t st, bool tile_rule) {
    const bool pb = !tile_rule || tile_group(p) < 64;
    const int64_t waves = ((p->n_tiles + 63) / 64) * ((p->n_blocks + 63) / 64);
    const dim3 g((unsigned)((waves + 3) / 4));
    if (pb)
        hipLaunchKernelGGL(k_transpose_bits<true>, g, dim3(256), 0, st, p->row_kbits,
                           p->row_pbits, p->n_tiles, p->n_blocks, p->col_kbits, p->col_pbits);
    else
        hipLaunchKernelGGL(k_transpose_bits<false>, g, dim3(256), 0, st, p->row_kbits,
                           (const uint64_t *)nullptr, p->n_tiles, p->n_blocks, p->col_kbits,
                           (uint64_t *)nullptr);
    int nseg = 1;
    int64_t seg_len = 0;
    cull_segments(p->n_blocks, p->n_tiles, &nseg, &seg_len);
    const int64_t nrs = p->n_blocks * nseg;
    hipLaunchKernelGGL(k_col_seg_counts, dim3((unsigned)((nrs + 255) / 256)), dim3(256), 0, st,
                       p->col_kbits, p->n_tiles, p->n_blocks, nseg, seg_len, p->col_scnt);
    hipLaunchKernelGGL(k_seg_sum, dim3((unsigned)((p->n_blocks + 255) / 256)), dim3(256), 0, st,
                       p->col_scnt, p->n_blocks, nseg, p->col_cnt);
}

// One evaluation in stages, so that a batch of problems can share host
// synchronisations and batched launches:
//   plan_begin  target records, psi statistics, cutoff, culling and counts
//   plan_lists  (after a sync when culling ran) list and work-item fills
//   plan_passes objective + gradient passes of this problem alone
//   plan_finish gradient merge, J, statistics, copy of the scalars to host
//   plan_result (after a sync) outputs and problem state
struct EvalPlan {
    rsot_problem *p = nullptr;
    hipStream_t st = nullptr;
    double eps = 0, kappa = 0, kcs = 0;
    const double *psi = nullptr;
    double *grad = nullptr;
    int rule = 0, mode = MODE_DENSE, dense_fallback = 0;
    bool culled = false;
    int64_t n_wi = 0, n_seg = 1, seg = 1;
    Pass1Work pw{0, 0, 1};
    int64_t seg1_cfg = RSOT_SEG1_DEFAULT;
    int group = 64;                     // culling group of the tile rule
};

static rsot_status plan_begin(EvalPlan &e) {
    rsot_problem *p = e.p;
    const hipStream_t st = e.st;
    const int D = p->dim;
    const double cs = p->opt.cost_scale, eps = e.eps;
    e.kappa = RSOT_LOG2E / eps;
    e.kcs = e.kappa * cs;
    e.rule = p->opt.truncation;
    if ((e.rule == RSOT_TRUNC_GEOM || e.rule == RSOT_TRUNC_TILE || e.rule == RSOT_TRUNC_INT) &&
        !(p->absJ_ref > 0.0)) {
        e.rule = RSOT_TRUNC_DENSE;
        e.dense_fallback = 1;
    }
    if (e.rule == RSOT_TRUNC_INT && !p->have_D) {
        e.rule = RSOT_TRUNC_DENSE;
        e.dense_fallback = 1;
    }
    if (e.rule == RSOT_TRUNC_GEOM || e.rule == RSOT_TRUNC_INT) {
        const hipStream_t keep = p->stream;
        p->stream = st;
        rsot_status s = rsot_compute_covering_cost(p);
        p->stream = keep;
        RSOT_TRY(s);
    }
    RSOT_HIP(hipEventRecord(p->ev0, st));
    const dim3 gblk((unsigned)((p->n_blocks + 3) / 4));
    const dim3 gtile((unsigned)((p->n_tiles + 3) / 4));
    if (D == 2)
        hipLaunchKernelGGL(k_prep_targets<2>, gblk, dim3(256), 0, st, e.psi, p->tperm, p->ty,
                           p->tnu, p->tlog2nu, p->n_blocks, e.kappa, cs, p->trec, p->trec3,
                           p->tpsi, p->blk_stat);
    else
        hipLaunchKernelGGL(k_prep_targets<3>, gblk, dim3(256), 0, st, e.psi, p->tperm, p->ty,
                           p->tnu, p->tlog2nu, p->n_blocks, e.kappa, cs, p->trec, p->trec3,
                           p->tpsi, p->blk_stat);
    if (p->opt.cost_kind == RSOT_COST_SPHERE) rsot_sphere_records(p, st, e.kappa);
    hipLaunchKernelGGL(k_pre_scalars, dim3(1), dim3(256), 0, st, p->blk_stat, p->n_blocks, e.rule,
                       eps, p->C0 < 0 ? 0.0 : p->C0, p->nu_min, p->nu_max, p->opt.tau,
                       p->absJ_ref, p->log_D_prev, p->opt.delta_thr, p->dscal);
    const int64_t seg_cfg = p->opt.seg_tiles;
    e.seg1_cfg = p->opt.seg_blocks > 0 ? p->opt.seg_blocks : RSOT_SEG1_DEFAULT;
    if (e.rule == RSOT_TRUNC_DENSE) {
        e.mode = MODE_DENSE;
        // Dense rows all have n_blocks entries: by default one work item per
        // tile, split only when the tiles alone cannot fill the device.
        if (p->opt.seg_blocks <= 0) {
            const int64_t want_items = 8192;
            const int64_t nseg = std::max<int64_t>(1, (want_items + p->n_tiles - 1) / p->n_tiles);
            e.seg1_cfg = (p->n_blocks + nseg - 1) / nseg;
        }
        e.pw.seg1 = std::min<int64_t>(e.seg1_cfg, p->n_blocks);
        e.pw.n_seg1 = (p->n_blocks + e.pw.seg1 - 1) / e.pw.seg1;
        e.pw.n_items = p->n_tiles * e.pw.n_seg1;
        // default: segments of at most 512 tiles (1 MB of point records, kept
        // in one XCD's L2), and at least 32,768 work items in all
        int64_t n_seg = std::max<int64_t>((p->n_tiles + 511) / 512,
                                          (32768 + p->n_blocks - 1) / p->n_blocks);
        if (seg_cfg > 0) n_seg = (p->n_tiles + seg_cfg - 1) / seg_cfg;
        n_seg = std::min<int64_t>(n_seg, p->n_tiles);
        e.seg = (p->n_tiles + n_seg - 1) / n_seg;
        e.n_seg = (p->n_tiles + e.seg - 1) / e.seg;
        e.n_wi = p->n_blocks * e.n_seg;
        return RSOT_OK;
    }
    const bool tile_rule = e.rule == RSOT_TRUNC_TILE;
    RSOT_TRY(ensure_cull_buffers(p, tile_rule, st));
    e.culled = true;
    e.mode = tile_rule ? MODE_LIST : MODE_MASK;
    const int grp = tile_rule ? tile_group(p) : 64;
    e.group = grp;
    if (tile_rule && grp < 64) {
        const int64_t ng = p->n_pad / grp;
        const double ln_eta_ng = std::log(p->opt.tau * p->absJ_ref / (eps * p->sum_mu)) -
                                 std::log((double)ng);
        hipLaunchKernelGGL(k_group_tables, dim3((unsigned)((ng + 255) / 256)), dim3(256), 0, st,
                           p->ty, p->tnu, p->tpsi, p->tperm, ng, grp, p->grp_lo, p->grp_hi,
                           p->grp_lnnu, p->grp_psi);
        if (D == 2)
            hipLaunchKernelGGL(k_tile_ref_grp<2>, gtile, dim3(256), 0, st, p->tile_lo, p->tile_hi,
                               p->blk_lo, p->blk_hi, p->blk_lnnu, p->blk_stat, p->grp_lo, p->grp_hi, p->grp_lnnu, p->grp_psi, p->ty, p->tnu,
                               p->tpsi, p->tperm, p->n_tiles, ng, grp, cs, eps, ln_eta_ng,
                               p->tile_bstar, p->tile_thr,
                               p->opt.cost_kind == RSOT_COST_SPHERE ? 1 : 0);
        else
            hipLaunchKernelGGL(k_tile_ref_grp<3>, gtile, dim3(256), 0, st, p->tile_lo, p->tile_hi,
                               p->blk_lo, p->blk_hi, p->blk_lnnu, p->blk_stat, p->grp_lo, p->grp_hi, p->grp_lnnu, p->grp_psi, p->ty, p->tnu,
                               p->tpsi, p->tperm, p->n_tiles, ng, grp, cs, eps, ln_eta_ng,
                               p->tile_bstar, p->tile_thr,
                               p->opt.cost_kind == RSOT_COST_SPHERE ? 1 : 0);
    } else if (tile_rule) {
        const double ln_eta_nb = std::log(p->opt.tau * p->absJ_ref / (eps * p->sum_mu)) -
                                 std::log((double)p->n_blocks);
        if (D == 2)
            hipLaunchKernelGGL(k_tile_ref<2>, gtile, dim3(256), 0, st, p->tile_lo, p->tile_hi,
                               p->blk_lo, p->blk_hi, p->blk_lnnu, p->blk_stat, p->blk_cnt, p->ty,
                               p->tnu, p->tpsi, p->n_tiles, p->n_blocks, cs, eps, ln_eta_nb,
                               p->tile_bstar, p->tile_thr, 0);
        else
            hipLaunchKernelGGL(k_tile_ref<3>, gtile, dim3(256), 0, st, p->tile_lo, p->tile_hi,
                               p->blk_lo, p->blk_hi, p->blk_lnnu, p->blk_stat, p->blk_cnt, p->ty,
                               p->tnu, p->tpsi, p->n_tiles, p->n_blocks, cs, eps, ln_eta_nb,
                               p->tile_bstar, p->tile_thr,
                               p->opt.cost_kind == RSOT_COST_SPHERE ? 1 : 0);
    } else {
        hipLaunchKernelGGL(k_target_G, dim3((unsigned)((p->n_pad + 255) / 256)), dim3(256), 0, st,
                           p->tpsi, p->tlog2nu, p->tperm, p->n_pad, e.kappa, p->dscal, p->tG);
    }
    launch_cull(p, st, D, tile_rule, true, false, eps);
    launch_col_counts(p, st, tile_rule);
    e.seg = seg_cfg > 0 ? seg_cfg : 64;
    launch_scan(st, p->row_cnt, p->n_tiles, 0, p->row_ptr, p->dscal + SC_ROWTOT, p->scan_tmp);
    launch_scan(st, p->col_cnt, p->n_blocks, 0, p->col_ptr, p->dscal + SC_COLTOT, p->scan_tmp);
    launch_scan(st, p->col_cnt, p->n_blocks, (int)e.seg, p->wi_ptr, p->dscal + SC_NWI,
                p->scan_tmp);
    launch_scan(st, p->row_cnt, p->n_tiles, (int)e.seg1_cfg, p->wi1_ptr, p->dscal + SC_NWI1,
                p->scan_tmp);
    RSOT_HIP(hipGetLastError());
    RSOT_HIP(hipMemcpyAsync(p->hscal, p->dscal, sizeof(double) * SC_COUNT, hipMemcpyDeviceToHost,
                            st));
    return RSOT_OK;
}

// processing order of n work items: item numbers sorted (stable radix sort)
// by the first entry of their list range
static rsot_status order_items(rsot_problem *p, hipStream_t st, const int64_t *range,
                               const uint32_t *idx, int64_t n, int64_t n_keys, int32_t **perm,
                               size_t *perm_cap) {
    if (n <= 0) return RSOT_OK;
    if (n > INT32_MAX) return RSOT_ERR_INVALID_ARG;
    RSOT_TRY(grow(p, perm, perm_cap, (size_t)n));
    size_t cap = p->sort_cap, cap2 = p->sort_cap, cap3 = p->sort_cap;
    RSOT_TRY(grow(p, &p->sort_key, &cap, (size_t)n));
    RSOT_TRY(grow(p, &p->sort_key2, &cap2, (size_t)n));
    RSOT_TRY(grow(p, &p->sort_val, &cap3, (size_t)n));
    p->sort_cap = std::min(cap, std::min(cap2, cap3));
    hipLaunchKernelGGL(k_item_keys, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, range,
                       idx, n, p->sort_key, p->sort_val);
    int bits = 1;
    while (bits < 31 && (int64_t(1) << bits) < n_keys) ++bits;
    size_t tmp_bytes = 0;
    RSOT_HIP(hipcub::DeviceRadixSort::SortPairs(nullptr, tmp_bytes, p->sort_key, p->sort_key2,
                                                p->sort_val, *perm, (int)n, 0, bits, st));
    RSOT_TRY(grow(p, (char **)&p->sort_tmp, &p->sort_tmp_cap, tmp_bytes));
    RSOT_HIP(hipcub::DeviceRadixSort::SortPairs(p->sort_tmp, tmp_bytes, p->sort_key, p->sort_key2,
                                                p->sort_val, *perm, (int)n, 0, bits, st));
    return RSOT_OK;
}

// after plan_begin's stream work completed (only needed when culled)
static rsot_status plan_lists(EvalPlan &e) {
    rsot_problem *p = e.p;
    const hipStream_t st = e.st;
    const bool grad = e.grad != nullptr;
    if (e.culled) {
        if (p->hscal[SC_NONFINITE] != 0.0) return RSOT_ERR_NONFINITE;
        const int64_t rtot = (int64_t)p->hscal[SC_ROWTOT];
        const int64_t ctot = (int64_t)p->hscal[SC_COLTOT];
        e.n_wi = (int64_t)p->hscal[SC_NWI];
        size_t cap_r = p->list_cap, cap_c = p->list_cap, cap_rm = p->list_cap;
        const size_t want = (size_t)std::max<int64_t>(std::max(rtot, ctot), 1);
        RSOT_TRY(grow(p, &p->row_idx, &cap_r, want));
        RSOT_TRY(grow(p, &p->col_idx, &cap_c, want));
        RSOT_TRY(grow(p, &p->row_cm, &cap_rm, want));
        p->list_cap = std::min(std::min(cap_r, cap_c), cap_rm);
        if (e.group < 64) RSOT_TRY(grow(p, &p->col_cm, &p->col_cm_cap, want));
        size_t cap_b = p->wi_cap, cap_rg = p->wi_cap;
        RSOT_TRY(grow(p, &p->wi_block, &cap_b, (size_t)std::max<int64_t>(e.n_wi, 1)));
        RSOT_TRY(grow(p, &p->wi_range, &cap_rg, (size_t)std::max<int64_t>(2 * e.n_wi, 2)));
        p->wi_cap = std::min(cap_b, cap_rg / 2);
        e.pw.n_items = (int64_t)p->hscal[SC_NWI1];
        e.pw.seg1 = e.seg1_cfg;
        size_t cap_t = p->wi1_cap, cap_tr = p->wi1_cap;
        RSOT_TRY(grow(p, &p->wi1_tile, &cap_t, (size_t)std::max<int64_t>(e.pw.n_items, 1)));
        RSOT_TRY(grow(p, &p->wi1_range, &cap_tr, (size_t)std::max<int64_t>(2 * e.pw.n_items, 2)));
        p->wi1_cap = std::min(cap_t, cap_tr / 2);
        const dim3 gblk((unsigned)((p->n_blocks + 3) / 4));
        const dim3 gtile((unsigned)((p->n_tiles + 3) / 4));
        launch_cull(p, st, p->dim, e.mode == MODE_LIST, true, true, e.eps);
        launch_cull(p, st, p->dim, e.mode == MODE_LIST, false, true, e.eps);
        hipLaunchKernelGGL(k_fill_work, dim3((unsigned)((p->n_blocks + 255) / 256)), dim3(256), 0,
                           st, p->col_ptr, p->wi_ptr, p->n_blocks, (int)e.seg, p->wi_block,
                           p->wi_range);
        hipLaunchKernelGGL(k_fill_work, dim3((unsigned)((p->n_tiles + 255) / 256)), dim3(256), 0,
                           st, p->row_ptr, p->wi1_ptr, p->n_tiles, (int)e.seg1_cfg, p->wi1_tile,
                           p->wi1_range);
        RSOT_HIP(hipGetLastError());
        RSOT_TRY(order_items(p, st, p->wi1_range, p->row_idx, e.pw.n_items, p->n_blocks,
                             &p->wi1_perm, &p->perm1_cap));
        if (grad)
            RSOT_TRY(order_items(p, st, p->wi_range, p->col_idx, e.n_wi, p->n_tiles, &p->wi_perm,
                                 &p->perm_cap));
    }
    size_t c1 = p->part1_cap, c2 = p->part1_cap;
    RSOT_TRY(grow(p, &p->part1, &c1, (size_t)std::max<int64_t>(e.pw.n_items, 1) * 64));
    RSOT_TRY(grow(p, &p->part1k, &c2, (size_t)std::max<int64_t>(e.pw.n_items, 1) * 64));
    p->part1_cap = std::min(c1, c2);
    if (e.mode == MODE_MASK)
        RSOT_TRY(grow(p, &p->redo1, &p->redo1_cap, (size_t)std::max<int64_t>(e.pw.n_items, 1)));
    if (grad) RSOT_TRY(grow(p, &p->gpart, &p->gpart_cap, (size_t)std::max<int64_t>(e.n_wi, 1) * 64));
    return RSOT_OK;
}

static void plan_passes(EvalPlan &e) {
    rsot_problem *p = e.p;
    const hipStream_t keep = p->stream;
    p->stream = e.st;
    const bool f64 = rsot_pairs_fp64(p);
    const bool grad = e.grad != nullptr;
    (void)hipEventRecord(p->ev_p1, e.st);
    if (p->opt.cost_kind == RSOT_COST_SPHERE) {
        launch_passes_sphere(p, f64, e.mode, grad, e.kcs, e.n_wi, e.n_seg, e.seg, e.pw);
    } else if (p->dim == 2) {
        if (f64) launch_passes<2, true>(p, e.mode, grad, e.kcs, e.n_wi, e.n_seg, e.seg, e.pw);
        else launch_passes<2, false>(p, e.mode, grad, e.kcs, e.n_wi, e.n_seg, e.seg, e.pw);
    } else {
        if (f64) launch_passes<3, true>(p, e.mode, grad, e.kcs, e.n_wi, e.n_seg, e.seg, e.pw);
        else launch_passes<3, false>(p, e.mode, grad, e.kcs, e.n_wi, e.n_seg, e.seg, e.pw);
    }
    (void)hipEventRecord(p->ev_p2, e.st);
    p->stream = keep;
}

static rsot_status plan_finish(EvalPlan &e) {
    rsot_problem *p = e.p;
    const hipStream_t st = e.st;
    const bool grad = e.grad != nullptr;
    if (grad)
        hipLaunchKernelGGL(k_grad_reduce, dim3((unsigned)p->n_blocks), dim3(256), 0, st, p->gpart,
                           e.mode == MODE_DENSE ? (const int64_t *)nullptr : p->wi_ptr, e.n_seg,
                           p->tnu, p->tperm, p->n_blocks, p->dscal, e.grad, p->blk_gpart);
    hipLaunchKernelGGL(k_objective, dim3(1), dim3(256), 0, st, p->tile_part, p->n_tiles, e.eps,
                       p->dscal);
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(256), 0, st, p->tile_part, p->n_tiles,
                       p->blk_gpart, p->n_blocks, grad ? 1 : 0, p->dscal);
    RSOT_HIP(hipGetLastError());
    RSOT_HIP(hipEventRecord(p->ev1, st));
    RSOT_HIP(hipMemcpyAsync(p->hscal, p->dscal, sizeof(double) * SC_COUNT, hipMemcpyDeviceToHost,
                            st));
    return RSOT_OK;
}

static rsot_status plan_result(EvalPlan &e, bool timed_passes, double *J_out,
                               rsot_eval_info *info) {
    rsot_problem *p = e.p;
    const bool grad = e.grad != nullptr;
    const double *h = p->hscal;
    if (h[SC_NONFINITE] != 0.0) return RSOT_ERR_NONFINITE;
    float ms = 0.0f, ms_pre = 0.0f, ms_passes = 0.0f, ms_p1 = 0.0f, ms_p2 = 0.0f;
    RSOT_HIP(hipEventElapsedTime(&ms, p->ev0, p->ev1));
    if (timed_passes) {
        RSOT_HIP(hipEventElapsedTime(&ms_pre, p->ev0, p->ev_p1));
        RSOT_HIP(hipEventElapsedTime(&ms_passes, p->ev_p1, p->ev_p2));
        RSOT_HIP(hipEventElapsedTime(&ms_p1, p->ev_p1, p->ev_mid));
        RSOT_HIP(hipEventElapsedTime(&ms_p2, p->ev_mid, p->ev_p2));
    }
    *J_out = h[SC_J];
    if (e.rule == RSOT_TRUNC_INT || p->opt.truncation == RSOT_TRUNC_INT) {
        p->log_D_prev = h[SC_LOGD];
        p->have_D = 1;
    }
    if (e.dense_fallback && p->absJ_ref <= 0.0) p->absJ_ref = std::fabs(h[SC_J]);
    p->last_eval_valid = 1;
    p->last_mode = e.mode;
    p->last_group = e.group;
    p->last_n_wi = e.n_wi;
    p->last_n_seg = e.n_seg;
    p->last_seg = e.seg;
    p->last_kcs = e.kcs;
    if (info) {
        const int rule = e.rule;
        info->total_pairs = p->nq * p->n;
        info->kept_pairs = (int64_t)h[SC_KEPT];
        info->n_empty_qp = (int64_t)h[SC_EMPTY];
        info->cutoff = (rule == RSOT_TRUNC_GEOM || rule == RSOT_TRUNC_INT || rule == RSOT_TRUNC_PW)
                           ? h[SC_C]
                           : 0.0;
        info->absJ_ref = p->absJ_ref;
        info->log_D = h[SC_LOGD];
        info->grad_l1 = grad ? h[SC_GL1] : 0.0;
        info->grad_linf = grad ? h[SC_GLINF] : 0.0;
        info->kernel_ms = ms;
        info->setup_ms = ms_pre;
        info->passes_ms = ms_passes;
        info->pass1_ms = ms_p1;
        info->pass2_ms = grad ? ms_p2 : 0.0;
        info->dense_fallback = e.dense_fallback;
        info->fp64_pairs = rsot_pairs_fp64(p) ? 1 : 0;
    }
    return RSOT_OK;
}

rsot_status rsot_eval_impl(rsot_problem *p, double eps, const double *psi, double *J_out,
                           double *grad_out, rsot_eval_info *info) {
    EvalPlan e;
    e.p = p;
    e.st = p->stream;
    e.eps = eps;
    e.psi = psi;
    e.grad = grad_out;
    RSOT_TRY(plan_begin(e));
    if (e.culled) RSOT_HIP(hipStreamSynchronize(e.st));
    RSOT_TRY(plan_lists(e));
    plan_passes(e);
    RSOT_TRY(plan_finish(e));
    RSOT_HIP(hipStreamSynchronize(e.st));
    return plan_result(e, true, J_out, info);
}

// Dense evaluation with the work-item partials in caller-provided device
// memory (scratch, scratch_bytes) instead of the problem's own buffers. The
// segmentation is the default one when its partials fit; otherwise one
// objective-pass item per tile and as many gradient-pass point segments as
// fit (never more than the default). Allocates nothing.
rsot_status rsot_eval_dense_in(rsot_problem *p, double eps, const double *psi, double *J_out,
                               double *grad_out, rsot_eval_info *info, double *scratch,
                               size_t scratch_bytes) {
    if (p->opt.truncation != RSOT_TRUNC_DENSE) return RSOT_ERR_INVALID_ARG;
    EvalPlan e;
    e.p = p;
    e.st = p->stream;
    e.eps = eps;
    e.psi = psi;
    e.grad = grad_out;
    RSOT_TRY(plan_begin(e));
    const bool grad = grad_out != nullptr;
    const size_t cap = scratch_bytes / sizeof(double);
    auto need = [&]() {
        return (size_t)e.pw.n_items * 128 + (grad ? (size_t)e.n_wi * 64 : 0);
    };
    if (need() > cap) {
        e.pw.seg1 = p->n_blocks;
        e.pw.n_seg1 = 1;
        e.pw.n_items = p->n_tiles;
        const size_t used1 = (size_t)p->n_tiles * 128;
        if (grad) {
            const size_t left = cap > used1 ? cap - used1 : 0;
            int64_t n_seg = (int64_t)(left / ((size_t)p->n_blocks * 64));
            if (n_seg < 1) return RSOT_ERR_OOM;
            n_seg = std::min(n_seg, e.n_seg);
            e.seg = (p->n_tiles + n_seg - 1) / n_seg;
            e.n_seg = (p->n_tiles + e.seg - 1) / e.seg;
            e.n_wi = p->n_blocks * e.n_seg;
        }
        if (need() > cap) return RSOT_ERR_OOM;
    }
    double *keep1 = p->part1, *keep1k = p->part1k, *keepg = p->gpart;
    p->part1 = scratch;
    p->part1k = scratch + (size_t)e.pw.n_items * 64;
    p->gpart = scratch + (size_t)e.pw.n_items * 128;
    plan_passes(e);
    const rsot_status s = plan_finish(e);
    p->part1 = keep1;
    p->part1k = keep1k;
    p->gpart = keepg;
    RSOT_TRY(s);
    RSOT_HIP(hipStreamSynchronize(e.st));
    return plan_result(e, true, J_out, info);
}

extern "C" rsot_status rsot_dual_eval(rsot_problem *p, double eps, const double *psi,
                                      double *J_out, double *grad_out, rsot_eval_info *info) {
    if (!p || !psi || !J_out) return RSOT_ERR_INVALID_ARG;
    if (!(eps > 0.0) || !std::isfinite(eps)) return RSOT_ERR_INVALID_ARG;
    return rsot_eval_impl(p, eps, psi, J_out, grad_out, info);
}

// Batched evaluation: every problem's preparation and culling, one host
// synchronisation, one launch per pass for the problems that run
// mixed precision with the dense or tile rule (others run their own passes in
// the same stream), one final synchronisation. Work goes on ps[0]'s stream.
extern "C" rsot_status rsot_dual_eval_batched(rsot_problem *const *ps, int n, const double *eps,
                                              const double *const *psi, double *J_out,
                                              double *const *grad_out, rsot_eval_info *infos,
                                              double *batch_ms) {
    if (!ps || n < 1 || !eps || !psi || !J_out) return RSOT_ERR_INVALID_ARG;
    for (int i = 0; i < n; ++i)
        if (!ps[i] || !psi[i] || !(eps[i] > 0.0) || !std::isfinite(eps[i]))
            return RSOT_ERR_INVALID_ARG;
    rsot_problem *p0 = ps[0];
    const hipStream_t st = p0->stream;
    std::vector<EvalPlan> plans((size_t)n);
    RSOT_HIP(hipEventRecord(p0->ev_b0, st));
    bool any_cull = false;
    for (int i = 0; i < n; ++i) {
        EvalPlan &e = plans[(size_t)i];
        e.p = ps[i];
        e.st = st;
        e.eps = eps[i];
        e.psi = psi[i];
        e.grad = grad_out ? grad_out[i] : nullptr;
        RSOT_TRY(plan_begin(e));
        any_cull = any_cull || e.culled;
    }
    if (any_cull) RSOT_HIP(hipStreamSynchronize(st));
    for (int i = 0; i < n; ++i) RSOT_TRY(plan_lists(plans[(size_t)i]));

    // problems for the batched kernels, in decreasing order of work
    std::vector<BatchDesc> descs;
    std::vector<int> members;
    std::vector<double> cost;
    for (int i = 0; i < n; ++i) {
        EvalPlan &e = plans[(size_t)i];
        rsot_problem *p = e.p;
        const bool batchable = !rsot_pairs_fp64(p) && p->opt.cost_kind == RSOT_COST_SQEUCLID &&
                               (e.mode == MODE_DENSE || e.mode == MODE_LIST);
        if (!batchable) {
            plan_passes(e);
            continue;
        }
        BatchDesc d{};
        d.dim = p->dim;
        d.mode = e.mode;
        d.n_tiles = p->n_tiles;
        d.n_blocks = p->n_blocks;
        d.qp = p->qp;
        d.qA = p->qA;
        d.tile_ref = p->tile_ref;
        d.trec = p->trec;
        d.trec3 = p->trec3;
        d.tG = p->tG;
        d.blk_cnt = p->blk_cnt;
        d.row_idx = p->row_idx;
        d.row_cm = p->row_cm;
        d.wi1_tile = p->wi1_tile;
        d.wi1_range = p->wi1_range;
        d.wi1_perm = p->wi1_perm;
        d.n_items1 = e.pw.n_items;
        d.seg1 = e.pw.seg1;
        d.n_seg1 = e.pw.n_seg1;
        d.kcs = e.kcs;
        d.part1 = p->part1;
        d.part1k = p->part1k;
        d.col_idx = p->col_idx;
        d.col_cm = p->col_cm;
        d.wi_block = p->wi_block;
        d.wi_range = p->wi_range;
        d.wi_perm = p->wi_perm;
        d.n_wi = e.grad ? e.n_wi : 0;
        d.n_seg = e.n_seg;
        d.seg = e.seg;
        d.gpart = p->gpart;
        descs.push_back(d);
        members.push_back(i);
        cost.push_back((double)(e.culled ? p->hscal[SC_ROWTOT] : (double)p->n_tiles * p->n_blocks));
    }
    const int nb = (int)descs.size();
    if (nb > 0) {
        // group members by (dimension, rule): one launch per pass and group
        // and pass; within a group, problems in decreasing order of work
        std::vector<int32_t> order((size_t)nb);
        for (int k = 0; k < nb; ++k) order[(size_t)k] = k;
        auto gkey = [&](int k) { return descs[(size_t)k].dim * 4 + descs[(size_t)k].mode; };
        std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
            if (gkey(a) != gkey(b)) return gkey(a) < gkey(b);
            return cost[(size_t)a] > cost[(size_t)b];
        });
        std::vector<int> gstart;
        for (int k = 0; k < nb; ++k)
            if (k == 0 || gkey(order[(size_t)k]) != gkey(order[(size_t)k - 1])) gstart.push_back(k);
        gstart.push_back(nb);
        const int ng = (int)gstart.size() - 1;
        // per group: item offsets of its problems (count + 1 entries each)
        std::vector<int64_t> begin1, begin2;
        std::vector<size_t> goff;
        for (int gi = 0; gi < ng; ++gi) {
            goff.push_back(begin1.size());
            int64_t a1 = 0, a2 = 0;
            for (int k = gstart[(size_t)gi]; k < gstart[(size_t)gi + 1]; ++k) {
                begin1.push_back(a1);
                begin2.push_back(a2);
                const BatchDesc &d = descs[(size_t)order[(size_t)k]];
                a1 += d.n_items1;
                a2 += d.n_wi;
            }
            begin1.push_back(a1);
            begin2.push_back(a2);
        }
        const size_t nbeg = begin1.size();
        const size_t s_desc = (sizeof(BatchDesc) * nb + 255) & ~size_t(255);
        const size_t s_ord = (sizeof(int32_t) * nb + 255) & ~size_t(255);
        const size_t s_beg = (sizeof(int64_t) * nbeg + 255) & ~size_t(255);
        const size_t bytes = s_desc + s_ord + 2 * s_beg + 256;
        size_t cap = p0->batch_cap;
        RSOT_TRY(grow(p0, &p0->batch_buf, &cap, bytes));
        p0->batch_cap = cap;
        char *base = p0->batch_buf;
        BatchDesc *d_desc = (BatchDesc *)base;
        int32_t *d_order = (int32_t *)(base + s_desc);
        int64_t *d_b1 = (int64_t *)(base + s_desc + s_ord);
        int64_t *d_b2 = (int64_t *)(base + s_desc + s_ord + s_beg);
        const size_t stage_bytes = s_desc + s_ord + 2 * s_beg;
        std::vector<char> stage(stage_bytes);
        std::memcpy(stage.data(), descs.data(), sizeof(BatchDesc) * nb);
        std::memcpy(stage.data() + s_desc, order.data(), sizeof(int32_t) * nb);
        std::memcpy(stage.data() + s_desc + s_ord, begin1.data(), sizeof(int64_t) * nbeg);
        std::memcpy(stage.data() + s_desc + s_ord + s_beg, begin2.data(), sizeof(int64_t) * nbeg);
        RSOT_HIP(hipMemcpyAsync(base, stage.data(), stage_bytes, hipMemcpyHostToDevice, st));
        for (int k = 0; k < nb; ++k) (void)hipEventRecord(ps[members[(size_t)k]]->ev_p1, st);
        for (int gi = 0; gi < ng; ++gi) {
            const int k0 = gstart[(size_t)gi], cnt = gstart[(size_t)gi + 1] - k0;
            const BatchDesc &d0 = descs[(size_t)order[(size_t)k0]];
            const int32_t *o = d_order + k0;
            const int64_t *b1 = d_b1 + goff[(size_t)gi];
            const unsigned grid = xcd_run_grid(begin1[goff[(size_t)gi] + (size_t)cnt]);
            if (grid == 0) continue;
            if (d0.dim == 3 && d0.mode == MODE_DENSE)
                hipLaunchKernelGGL((k_pass1_batched<3, MODE_DENSE>), dim3(grid), dim3(256), 0, st, d_desc, o, b1, cnt);
            else if (d0.dim == 3)
                hipLaunchKernelGGL((k_pass1_batched<3, MODE_LIST>), dim3(grid), dim3(256), 0, st, d_desc, o, b1, cnt);
            else if (d0.mode == MODE_DENSE)
                hipLaunchKernelGGL((k_pass1_batched<2, MODE_DENSE>), dim3(grid), dim3(256), 0, st, d_desc, o, b1, cnt);
            else
                hipLaunchKernelGGL((k_pass1_batched<2, MODE_LIST>), dim3(grid), dim3(256), 0, st, d_desc, o, b1, cnt);
        }
        for (int k = 0; k < nb; ++k) {
            EvalPlan &e = plans[(size_t)members[(size_t)k]];
            rsot_problem *p = e.p;
            hipLaunchKernelGGL(k_pass1_combine, dim3((unsigned)((p->n_tiles + 3) / 4)), dim3(256),
                               0, st, p->qp, p->qmu, p->qlog2mu, p->qperm, p->part1, p->part1k,
                               e.mode == MODE_DENSE ? (const int64_t *)nullptr : p->wi1_ptr,
                               e.pw.n_seg1, p->n_tiles, e.kcs, 0, pass_lcorr(p, false),
                               pass_corr(p, false), p->qA, p->qlse, p->qkept, p->tile_ref,
                               p->tile_part, p->tile_smax);
        }
        for (int gi = 0; gi < ng; ++gi) {
            const int k0 = gstart[(size_t)gi], cnt = gstart[(size_t)gi + 1] - k0;
            if (begin2[goff[(size_t)gi] + (size_t)cnt] == 0) continue;
            const BatchDesc &d0 = descs[(size_t)order[(size_t)k0]];
            const int32_t *o = d_order + k0;
            const int64_t *b2 = d_b2 + goff[(size_t)gi];
            const unsigned grid = xcd_run_grid(begin2[goff[(size_t)gi] + (size_t)cnt]);
            if (d0.dim == 3 && d0.mode == MODE_DENSE)
                hipLaunchKernelGGL((k_pass2_batched<3, MODE_DENSE>), dim3(grid), dim3(256), 0, st, d_desc, o, b2, cnt);
            else if (d0.dim == 3)
                hipLaunchKernelGGL((k_pass2_batched<3, MODE_LIST>), dim3(grid), dim3(256), 0, st, d_desc, o, b2, cnt);
            else if (d0.mode == MODE_DENSE)
                hipLaunchKernelGGL((k_pass2_batched<2, MODE_DENSE>), dim3(grid), dim3(256), 0, st, d_desc, o, b2, cnt);
            else
                hipLaunchKernelGGL((k_pass2_batched<2, MODE_LIST>), dim3(grid), dim3(256), 0, st, d_desc, o, b2, cnt);
        }
        RSOT_HIP(hipGetLastError());
        // the host staging buffer must outlive the asynchronous copy
        RSOT_HIP(hipStreamSynchronize(st));
        for (int k = 0; k < nb; ++k) (void)hipEventRecord(ps[members[(size_t)k]]->ev_p2, st);
    }
    for (int i = 0; i < n; ++i) RSOT_TRY(plan_finish(plans[(size_t)i]));
    RSOT_HIP(hipEventRecord(p0->ev_b1, st));
    RSOT_HIP(hipStreamSynchronize(st));
    rsot_status status = RSOT_OK;
    for (int i = 0; i < n; ++i) {
        rsot_status s = plan_result(plans[(size_t)i], false, &J_out[i], infos ? &infos[i] : nullptr);
        if (s != RSOT_OK && status == RSOT_OK) status = s;
    }
    if (batch_ms) {
        float ms = 0.0f;
        RSOT_HIP(hipEventElapsedTime(&ms, p0->ev_b0, p0->ev_b1));
        *batch_ms = ms;
    }
    return status;
}

__global__ void k_unpermute_lse(const double *__restrict__ qlse, const int32_t *__restrict__ qperm,
                                int64_t nq_pad, double *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nq_pad) return;
    const int32_t d = qperm[i];
    if (d >= 0) out[d] = qlse[i];
}

__global__ void k_unpermute_i32(const int32_t *__restrict__ v, const int32_t *__restrict__ perm,
                                int64_t n_pad, int32_t *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_pad) return;
    const int32_t d = perm[i];
    if (d >= 0) out[d] = v[i];
}

extern "C" rsot_status rsot_get_kept_counts(rsot_problem *p, int32_t *counts_out) {
    if (!p || !counts_out || !p->last_eval_valid) return RSOT_ERR_INVALID_ARG;
    hipLaunchKernelGGL(k_unpermute_i32, dim3((unsigned)((p->nq_pad + 255) / 256)), dim3(256), 0,
                       p->stream, p->qkept, p->qperm, p->nq_pad, counts_out);
    RSOT_HIP(hipGetLastError());
    RSOT_HIP(hipStreamSynchronize(p->stream));
    return RSOT_OK;
}

__global__ void k_fill_u8(uint8_t *__restrict__ out, int64_t n, uint8_t v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = v;
}

// one thread per tile row: its list entries into the (tile, block) matrix
__global__ void k_scatter_keep(const int64_t *__restrict__ row_ptr,
                               const uint32_t *__restrict__ row_idx, int64_t n_tiles,
                               int64_t n_blocks, uint8_t *__restrict__ out) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_tiles) return;
    for (int64_t e = row_ptr[t]; e < row_ptr[t + 1]; ++e) {
        const uint32_t ent = row_idx[e];
        out[t * n_blocks + (ent & ~RSOT_PARTIAL_BIT)] =
            (ent & RSOT_PARTIAL_BIT) ? PAIR_PARTIAL : PAIR_FULL;
    }
}

extern "C" rsot_status rsot_get_tile_keep(rsot_problem *p, uint8_t *keep_out) {
    if (!p || !keep_out || !p->last_eval_valid) return RSOT_ERR_INVALID_ARG;
    const int64_t nf = p->n_tiles * p->n_blocks;
    const bool dense = p->last_mode == MODE_DENSE;
    hipLaunchKernelGGL(k_fill_u8, dim3((unsigned)((nf + 255) / 256)), dim3(256), 0, p->stream,
                       keep_out, nf, (uint8_t)(dense ? PAIR_FULL : PAIR_SKIP));
    if (!dense)
        hipLaunchKernelGGL(k_scatter_keep, dim3((unsigned)((p->n_tiles + 255) / 256)), dim3(256),
                           0, p->stream, p->row_ptr, p->row_idx, p->n_tiles, p->n_blocks,
                           keep_out);
    RSOT_HIP(hipGetLastError());
    RSOT_HIP(hipStreamSynchronize(p->stream));
    return RSOT_OK;
}

// one thread per tile row: per kept entry the bits of its 8-target chunks
// whose pairs entered the sum (cutoff rules: every chunk not skipped; FP64
// cutoff rules test every chunk of a straddling block)
__global__ void k_scatter_chunks(const int64_t *__restrict__ row_ptr,
                                 const uint32_t *__restrict__ row_idx,
                                 const uint16_t *__restrict__ row_cm, int64_t n_tiles,
                                 int64_t n_blocks, int all_tested, uint8_t *__restrict__ out) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_tiles) return;
    for (int64_t e = row_ptr[t]; e < row_ptr[t + 1]; ++e) {
        const uint32_t ent = row_idx[e];
        uint32_t m = 0xFFu;
        if ((ent & RSOT_PARTIAL_BIT) && !all_tested) {
            const uint32_t cm = row_cm[e];
            m = 0;
            for (int c = 0; c < 8; ++c)
                if ((cm >> (2 * c)) & 3u) m |= 1u << c;
        }
        out[t * n_blocks + (ent & ~RSOT_PARTIAL_BIT)] = (uint8_t)m;
    }
}

extern "C" rsot_status rsot_get_tile_chunk_keep(rsot_problem *p, uint8_t *mask_out) {
    if (!p || !mask_out || !p->last_eval_valid) return RSOT_ERR_INVALID_ARG;
    const int64_t nf = p->n_tiles * p->n_blocks;
    const bool dense = p->last_mode == MODE_DENSE;
    hipLaunchKernelGGL(k_fill_u8, dim3((unsigned)((nf + 255) / 256)), dim3(256), 0, p->stream,
                       mask_out, nf, (uint8_t)(dense ? 0xFF : 0));
    if (!dense)
        hipLaunchKernelGGL(k_scatter_chunks, dim3((unsigned)((p->n_tiles + 255) / 256)), dim3(256),
                           0, p->stream, p->row_ptr, p->row_idx, p->row_cm, p->n_tiles,
                           p->n_blocks, (p->last_mode == MODE_MASK && rsot_pairs_fp64(p)) ? 1 : 0,
                           mask_out);
    RSOT_HIP(hipGetLastError());
    RSOT_HIP(hipStreamSynchronize(p->stream));
    return RSOT_OK;
}

__global__ void k_target_slots(const int32_t *__restrict__ tperm, int64_t n_pad,
                               int32_t *__restrict__ slot) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_pad) return;
    const int32_t src = tperm[i];
    if (src >= 0) slot[src] = (int32_t)i;
}

extern "C" rsot_status rsot_get_target_slots(rsot_problem *p, int32_t *slot_out) {
    if (!p || !slot_out) return RSOT_ERR_INVALID_ARG;
    hipLaunchKernelGGL(k_target_slots, dim3((unsigned)((p->n_pad + 255) / 256)), dim3(256), 0,
                       p->stream, p->tperm, p->n_pad, slot_out);
    RSOT_HIP(hipGetLastError());
    RSOT_HIP(hipStreamSynchronize(p->stream));
    return RSOT_OK;
}

extern "C" rsot_status rsot_get_lse(rsot_problem *p, double *L_out) {
    if (!p || !L_out || !p->last_eval_valid) return RSOT_ERR_INVALID_ARG;
    hipLaunchKernelGGL(k_unpermute_lse, dim3((unsigned)((p->nq_pad + 255) / 256)), dim3(256), 0,
                       p->stream, p->qlse, p->qperm, p->nq_pad, L_out);
    RSOT_HIP(hipGetLastError());
    RSOT_HIP(hipStreamSynchronize(p->stream));
    return RSOT_OK;
}

// ---------------------------------------------------------------------------
// softmax potential refinement (Eq. softmax_refinement_formula)
//   psi_k = -eps ln sum_q mu_q exp(-L_q) exp(-c(x_q, y_k)/eps)
// with L_q the log-sum-exp of the coarse targets at the current points. In
// base 2 the summand is 2^(B_k + S_q + x_q.Y_k) with B_k = -kappa cs |y_k|^2,
// Y_k = 2 kappa cs y_k and S_q = log2 mu_q - Lt_q from the objective pass, so
// the gradient pass's loop applies with fine-target records; the terms span
// far more than FP32's range at small eps, so the sum is a log-sum-exp.
// ---------------------------------------------------------------------------

// fine-target records (psi = 0, nu = 1) and block boxes
__global__ __launch_bounds__(256) void k_refine_targets(
    const double *__restrict__ yf, const int32_t *__restrict__ order, int64_t nf, int64_t nf_pad,
    int dim, double s0, double s1, double s2, double kappa, double cs,
    double4 *__restrict__ rec, int32_t *__restrict__ fperm, double *__restrict__ fy,
    double *__restrict__ blo, double *__restrict__ bhi, int32_t *__restrict__ bcnt) {
    const int lane = threadIdx.x & 63;
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t b = j / 64;
    if (b * 64 >= nf_pad) return;
    const bool real = j < nf;
    const int32_t src = order[real ? j : nf - 1];
    const double y0 = yf[(int64_t)src * dim + 0] - s0;
    const double y1 = yf[(int64_t)src * dim + 1] - s1;
    const double y2 = dim == 3 ? yf[(int64_t)src * dim + 2] - s2 : 0.0;
    double4 r;
    r.x = 2.0 * kappa * cs * y0;
    r.y = 2.0 * kappa * cs * y1;
    r.z = 2.0 * kappa * cs * y2;
    r.w = real ? -kappa * cs * (y0 * y0 + y1 * y1 + y2 * y2) : -INFINITY;
    rec[j] = r;
    fperm[j] = real ? src : -1;
    fy[j * 3 + 0] = y0;
    fy[j * 3 + 1] = y1;
    fy[j * 3 + 2] = y2;
    const double v[3] = {y0, y1, y2};
    for (int k = 0; k < 3; ++k) {
        const double a = wave_min(v[k]), c = wave_max(v[k]);
        if (lane == 0) {
            blo[b * 3 + k] = a;
            bhi[b * 3 + k] = c;
        }
    }
    const double n = wave_sum(real ? 1.0 : 0.0);
    if (lane == 0) bcnt[b] = (int32_t)n;
}

// Culling for the refinement, one wavefront per fine block F:
//   ln U_TF = ln D_T - cs dmin^2(T,F)/eps bounds the tile's contribution to
//   every target of F (D_T = sum_{q in T} mu_q e^{-L_q});
//   T* = argmax_T ln U_TF; L_F = min_{k in F} max_{q in T*} (ln mu_q - L_q -
//   c(x_q,y_k)/eps) bounds every target's kept sum from below;
//   keep (T,F) iff T = T* or ln U_TF > L_F + ln(eta / n_tiles).
// Neglected mass <= eta * kept mass, so psi_k moves by at most eps ln(1+eta).
template <int D>
__global__ __launch_bounds__(256) void k_flags_refine(
    const double *__restrict__ tile_lo, const double *__restrict__ tile_hi,
    const double *__restrict__ tile_part, const double4 *__restrict__ qp,
    const double *__restrict__ qlog2mu, const double *__restrict__ qlse,
    const double *__restrict__ fblo, const double *__restrict__ fbhi,
    const int32_t *__restrict__ fbcnt, const double *__restrict__ fy, int64_t n_tiles,
    int64_t n_fblocks, double cs, double eps, double ln_eta_nt, uint8_t *__restrict__ flags_cm) {
    const int lane = threadIdx.x & 63;
    const int64_t F = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (F >= n_fblocks) return;
    double fl[3], fh[3];
    for (int k = 0; k < 3; ++k) {
        fl[k] = fblo[F * 3 + k];
        fh[k] = fbhi[F * 3 + k];
    }
    double best = -INFINITY;
    int64_t bt = INT64_MAX;
    for (int64_t t = lane; t < n_tiles; t += 64) {
        double dmin2 = 0.0;
        for (int k = 0; k < D; ++k) {
            const double g = box_gap(tile_lo[t * 3 + k], tile_hi[t * 3 + k], fl[k], fh[k]);
            dmin2 += g * g;
        }
        const double lnU = tile_part[t * 4 + 1] - cs * dmin2 / eps;
        if (lnU > best) {
            best = lnU;
            bt = t;
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const double ob = __shfl_xor(best, o, 64);
        const int64_t oi = __shfl_xor(bt, o, 64);
        if (ob > best || (ob == best && oi < bt)) {
            best = ob;
            bt = oi;
        }
    }
    double lb = INFINITY;
    if (bt != INT64_MAX && lane < fbcnt[F]) {
        const int64_t k = F * 64 + lane;
        const double y0 = fy[k * 3], y1 = fy[k * 3 + 1], y2 = fy[k * 3 + 2];
        double mx = -INFINITY;
        for (int i = 0; i < 64; ++i) {
            const int64_t q = bt * 64 + i;
            const double lq = qlse[q];
            const double lm = qlog2mu[q];
            if (!(lq > -INFINITY) || !(lm > -INFINITY)) continue;
            const double4 r = qp[q];
            const double e0 = r.x - y0, e1 = r.y - y1, e2 = D == 3 ? r.z - y2 : 0.0;
            const double v = lm * RSOT_LN2 - lq - cs * (e0 * e0 + e1 * e1 + e2 * e2) / eps;
            mx = fmax(mx, v);
        }
        lb = mx;
    }
    const double thr = wave_min(lb) + ln_eta_nt;
    for (int64_t t = lane; t < n_tiles; t += 64) {
        double dmin2 = 0.0;
        for (int k = 0; k < D; ++k) {
            const double g = box_gap(tile_lo[t * 3 + k], tile_hi[t * 3 + k], fl[k], fh[k]);
            dmin2 += g * g;
        }
        const double lnU = tile_part[t * 4 + 1] - cs * dmin2 / eps;
        flags_cm[F * n_tiles + t] = (t == bt || lnU > thr) ? PAIR_FULL : PAIR_SKIP;
    }
}

// one 64-point tile into a lane's running (m, s): s = sum 2^(v - m), m an
// integer that only grows (the objective pass's scheme, transposed)
template <int D, bool F64>
__device__ __forceinline__ void lse_tile(const double4 *__restrict__ Q, double Y0, double Y1,
                                         double Y2, double B, double rk, double &m, double &s) {
    for (int i0 = 0; i0 < 64; i0 += CH) {
        double tv[CH];
        double cm = -INFINITY;
#pragma unroll
        for (int k = 0; k < CH; ++k) {
            const double4 r = ld4(Q + i0 + k);
            double v = B + r.w;
            v = fma(r.x, Y0, v);
            v = fma(r.y, Y1, v);
            if (D == 3) v = fma(r.z, Y2, v);
            tv[k] = v;
            cm = fmax(cm, v);
        }
        if (cm > m) {
            const double mn = ceil(cm - rk) + rk;
            s = ldexp(s, (int)rint(fmax(m - mn, -2000.0)));
            m = mn;
        }
        if (F64) {
            double cs = exp2(tv[0] - m);
#pragma unroll
            for (int k = 1; k < CH; ++k) cs += exp2(tv[k] - m);
            s += cs;
        } else {
            float cs = __builtin_amdgcn_exp2f((float)(tv[0] - m));
#pragma unroll
            for (int k = 1; k < CH; ++k) cs += __builtin_amdgcn_exp2f((float)(tv[k] - m));
            s += (double)cs;
        }
    }
}

// per work item and lane: log2 of the partial sum (or -inf)
template <int D, bool F64>
__global__ __launch_bounds__(256) void k_pass2_lse(
    const double4 *__restrict__ qp, const double2 *__restrict__ tref,
    const double4 *__restrict__ frec, const int32_t *__restrict__ wi_block,
    const int64_t *__restrict__ wi_range, const uint32_t *__restrict__ col_idx, int64_t n_wi,
    double *__restrict__ out) {
    const int lane = threadIdx.x & 63;
    const int64_t w =
        xcd_group((n_wi + 3) / 4) * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (w >= n_wi) return;
    const int64_t F = wi_block[w];
    const double4 rec = frec[F * 64 + lane];
    const double rk = ref_offset(F * 64 + lane);
    double m = -1e300, s = 0.0;
    for (int64_t e = wi_range[2 * w]; e < wi_range[2 * w + 1]; ++e) {
        const int64_t t = col_idx[e] & ~RSOT_PARTIAL_BIT;
        // the point records carry S_q - R_T; R_T returns through B
        lse_tile<D, F64>(qp + t * 64, rec.x, rec.y, rec.z, rec.w + tref[t].x, rk, m, s);
    }
    out[w * 64 + lane] = s > 0.0 ? m + log2(s) : -INFINITY;
}

__global__ __launch_bounds__(256) void k_refine_reduce(const double *__restrict__ part,
                                                       const int64_t *__restrict__ wi_ptr,
                                                       const int32_t *__restrict__ fperm,
                                                       int64_t n_fblocks, double eps, double lcorr,
                                                       double *__restrict__ psi_out) {
    const int lane = threadIdx.x & 63;
    const int64_t F = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (F >= n_fblocks) return;
    const int64_t w0 = wi_ptr[F], w1 = wi_ptr[F + 1];
    double mx = -INFINITY;
    for (int64_t w = w0; w < w1; ++w) mx = fmax(mx, part[w * 64 + lane]);
    double s = 0.0;
    if (mx > -INFINITY)
        for (int64_t w = w0; w < w1; ++w) s += exp2(part[w * 64 + lane] - mx);
    const int32_t dst = fperm[F * 64 + lane];
    if (dst >= 0) psi_out[dst] = -eps * RSOT_LN2 * (mx + log2(s) + lcorr);
}

rsot_status rsot_refine_impl(rsot_problem *p, double eps, const double *psi_coarse,
                             int64_t nf, const double *yf, double eta, double *psi_out) {
    if (p->opt.cost_kind != RSOT_COST_SQEUCLID) return RSOT_ERR_INVALID_ARG;
    // 1. coarse log-sum-exp L_q at the current points (objective pass only)
    double J = 0.0;
    rsot_eval_info info{};
    RSOT_TRY(rsot_eval_impl(p, eps, psi_coarse, &J, nullptr, &info));
    // 2. fine targets: Morton order, records, block boxes
    int32_t *order = nullptr;
    RSOT_TRY(rsot_morton_order(p, yf, nf, &order));
    const int64_t nf_pad = (nf + 63) / 64 * 64, nfb = nf_pad / 64;
    const double kappa = RSOT_LOG2E / eps, cs = p->opt.cost_scale;
    std::vector<void *> tmp;
    auto A = [&](size_t bytes) -> void * {
        void *q = nullptr;
        if (rsot_dev_alloc(p, &q, bytes) != RSOT_OK) return nullptr;
        tmp.push_back(q);
        return q;
    };
    auto cleanup = [&]() {
        for (void *q : tmp) rsot_dev_free(p, q);
        rsot_dev_free(p, order);
    };
    double4 *frec = (double4 *)A(sizeof(double4) * nf_pad);
    int32_t *fperm = (int32_t *)A(sizeof(int32_t) * nf_pad);
    double *fy = (double *)A(sizeof(double) * nf_pad * 3);
    double *fblo = (double *)A(sizeof(double) * nfb * 3);
    double *fbhi = (double *)A(sizeof(double) * nfb * 3);
    int32_t *fbcnt = (int32_t *)A(sizeof(int32_t) * nfb);
    uint8_t *flags = (uint8_t *)A((size_t)nfb * (size_t)p->n_tiles);
    int32_t *cnt = (int32_t *)A(sizeof(int32_t) * nfb);
    int64_t *cptr = (int64_t *)A(sizeof(int64_t) * (nfb + 1));
    int64_t *wptr = (int64_t *)A(sizeof(int64_t) * (nfb + 1));
    if (!frec || !fperm || !fy || !fblo || !fbhi || !fbcnt || !flags || !cnt || !cptr || !wptr) {
        cleanup();
        return RSOT_ERR_OOM;
    }
    hipLaunchKernelGGL(k_refine_targets, dim3((unsigned)(nf_pad / 64)), dim3(64), 0, p->stream,
                       yf, order, nf, nf_pad, p->dim, p->shift[0], p->shift[1], p->shift[2], kappa,
                       cs, frec, fperm, fy, fblo, fbhi, fbcnt);
    // 3. culling and lists
    const double ln_eta_nt = std::log(eta) - std::log((double)p->n_tiles);
    const dim3 gfb((unsigned)((nfb + 3) / 4));
    if (p->dim == 2)
        hipLaunchKernelGGL(k_flags_refine<2>, gfb, dim3(256), 0, p->stream, p->tile_lo,
                           p->tile_hi, p->tile_part, p->qp, p->qlog2mu, p->qlse, fblo, fbhi,
                           fbcnt, fy, p->n_tiles, nfb, cs, eps, ln_eta_nt, flags);
    else
        hipLaunchKernelGGL(k_flags_refine<3>, gfb, dim3(256), 0, p->stream, p->tile_lo,
                           p->tile_hi, p->tile_part, p->qp, p->qlog2mu, p->qlse, fblo, fbhi,
                           fbcnt, fy, p->n_tiles, nfb, cs, eps, ln_eta_nt, flags);
    hipLaunchKernelGGL(k_count_rows, gfb, dim3(256), 0, p->stream, flags, nfb, p->n_tiles, cnt);
    const int seg = 64;
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, p->stream, cnt, nfb, 0, cptr,
                       p->dscal + SC_COLTOT);
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, p->stream, cnt, nfb, seg, wptr,
                       p->dscal + SC_NWI);
    RSOT_HIP(hipGetLastError());
    RSOT_HIP(hipMemcpyAsync(p->hscal, p->dscal, sizeof(double) * SC_COUNT, hipMemcpyDeviceToHost,
                            p->stream));
    RSOT_HIP(hipStreamSynchronize(p->stream));
    const int64_t ctot = (int64_t)p->hscal[SC_COLTOT], n_wi = (int64_t)p->hscal[SC_NWI];
    uint32_t *cidx = (uint32_t *)A(sizeof(uint32_t) * std::max<int64_t>(ctot, 1));
    int32_t *wblk = (int32_t *)A(sizeof(int32_t) * std::max<int64_t>(n_wi, 1));
    int64_t *wrng = (int64_t *)A(sizeof(int64_t) * 2 * std::max<int64_t>(n_wi, 1));
    double *part = (double *)A(sizeof(double) * 64 * std::max<int64_t>(n_wi, 1));
    if (!cidx || !wblk || !wrng || !part) {
        cleanup();
        return RSOT_ERR_OOM;
    }
    hipLaunchKernelGGL(k_fill_rows, gfb, dim3(256), 0, p->stream, flags, nfb, p->n_tiles, cptr,
                       cidx);
    hipLaunchKernelGGL(k_fill_work, dim3((unsigned)((nfb + 255) / 256)), dim3(256), 0, p->stream,
                       cptr, wptr, nfb, seg, wblk, wrng);
    // 4. log-sum-exp gradient-pass loop and merge
    const dim3 gw(xcd_grid((n_wi + 3) / 4));
    const bool f64 = rsot_pairs_fp64(p);
    const double2 *tref = p->tile_ref;
    if (p->dim == 2) {
        if (f64) hipLaunchKernelGGL((k_pass2_lse<2, true>), gw, dim3(256), 0, p->stream, p->qp, tref, frec, wblk, wrng, cidx, n_wi, part);
        else hipLaunchKernelGGL((k_pass2_lse<2, false>), gw, dim3(256), 0, p->stream, p->qp, tref, frec, wblk, wrng, cidx, n_wi, part);
    } else {
        if (f64) hipLaunchKernelGGL((k_pass2_lse<3, true>), gw, dim3(256), 0, p->stream, p->qp, tref, frec, wblk, wrng, cidx, n_wi, part);
        else hipLaunchKernelGGL((k_pass2_lse<3, false>), gw, dim3(256), 0, p->stream, p->qp, tref, frec, wblk, wrng, cidx, n_wi, part);
    }
    hipLaunchKernelGGL(k_refine_reduce, gfb, dim3(256), 0, p->stream, part, wptr, fperm, nfb, eps,
                       pass_lcorr(p, f64), psi_out);
    RSOT_HIP(hipGetLastError());
    RSOT_HIP(hipStreamSynchronize(p->stream));
    p->last_refine_pairs = ctot * 64 * 64;
    cleanup();
    return RSOT_OK;
}

extern "C" rsot_status rsot_softmax_refine(rsot_problem *p, double eps, const double *psi_coarse,
                                           int64_t n_fine, const double *y_fine,
                                           double *psi_fine_out) {
    if (!p || !psi_coarse || !y_fine || !psi_fine_out || n_fine <= 0) return RSOT_ERR_INVALID_ARG;
    if (!(eps > 0.0) || !std::isfinite(eps)) return RSOT_ERR_INVALID_ARG;
    return rsot_refine_impl(p, eps, psi_coarse, n_fine, y_fine, 1e-12, psi_fine_out);
}

// ---------------------------------------------------------------------------
// autotuner: work granularity of both passes, by timing the live problem
// ---------------------------------------------------------------------------
// Coordinate search: objective-pass segment (target blocks per work item),
// then gradient-pass segment (point tiles per work item), each candidate
// timed as the best of `reps` evaluations with HIP events. The problem keeps
// the fastest pair; the default configuration's time is reported beside it.
static rsot_status time_config(rsot_problem *p, double eps, const double *psi, int sb, int stl,
                               int grp, int reps, double *ms_out) {
    p->opt.seg_blocks = sb;
    p->opt.seg_tiles = stl;
    p->opt.tile_group = grp;
    double best = INFINITY, J = 0.0;
    rsot_eval_info info{};
    for (int r = 0; r < reps; ++r) {
        RSOT_TRY(rsot_eval_impl(p, eps, psi, &J, p->dgrad, &info));
        best = std::min(best, info.kernel_ms);
    }
    *ms_out = best;
    return RSOT_OK;
}

extern "C" rsot_status rsot_autotune(rsot_problem *p, double eps, const double *psi, int reps,
                                     int *seg_blocks_out, int *seg_tiles_out,
                                     int *tile_group_out, double *best_ms_out,
                                     double *default_ms_out) {
    if (!p || !psi || !(eps > 0.0) || reps < 1) return RSOT_ERR_INVALID_ARG;
    static const int GR[] = {64, 32, 16, 8};
    static const int SB[] = {64, 128, 256, 512, 1024};
    static const int ST[] = {16, 32, 64, 128, 256, 512, 1024, 4096};
    const rsot_options keep = p->opt;
    double J = 0.0;
    rsot_eval_info info{};
    RSOT_TRY(rsot_eval_impl(p, eps, psi, &J, p->dgrad, &info));   // state (|J_ref|), warm-up
    double t_def = 0.0;
    rsot_status s = time_config(p, eps, psi, 0, 0, 0, reps, &t_def);
    int best_sb = 0, best_st = 0, best_gr = 0;
    double best = t_def;
    // culling group first (tile rule only): it sets the lists the segments cut
    if (p->opt.truncation == RSOT_TRUNC_TILE) {
        for (int gr : GR) {
            if (s != RSOT_OK) break;
            double t = 0.0;
            s = time_config(p, eps, psi, 0, 0, gr, reps, &t);
            if (s == RSOT_OK && t < best) {
                best = t;
                best_gr = gr;
            }
        }
    }
    for (int sb : SB) {
        if (s != RSOT_OK) break;
        double t = 0.0;
        s = time_config(p, eps, psi, sb, best_st, best_gr, reps, &t);
        if (s == RSOT_OK && t < best) {
            best = t;
            best_sb = sb;
        }
    }
    for (int st : ST) {
        if (s != RSOT_OK) break;
        double t = 0.0;
        s = time_config(p, eps, psi, best_sb, st, best_gr, reps, &t);
        if (s == RSOT_OK && t < best) {
            best = t;
            best_st = st;
        }
    }
    p->opt = keep;
    if (s != RSOT_OK) return s;
    p->opt.seg_blocks = best_sb;
    p->opt.seg_tiles = best_st;
    p->opt.tile_group = best_gr;
    if (seg_blocks_out) *seg_blocks_out = best_sb;
    if (seg_tiles_out) *seg_tiles_out = best_st;
    if (tile_group_out) *tile_group_out = best_gr;
    if (best_ms_out) *best_ms_out = best;
    if (default_ms_out) *default_ms_out = t_def;
    return RSOT_OK;
}

extern "C" rsot_status rsot_set_tuning(rsot_problem *p, int seg_blocks, int seg_tiles,
                                       int tile_group) {
    if (!p || seg_blocks < 0 || seg_tiles < 0) return RSOT_ERR_INVALID_ARG;
    if (tile_group != 0 && tile_group != 8 && tile_group != 16 && tile_group != 32 &&
        tile_group != 64)
        return RSOT_ERR_INVALID_ARG;
    p->opt.seg_blocks = seg_blocks;
    p->opt.seg_tiles = seg_tiles;
    p->opt.tile_group = tile_group;
    return RSOT_OK;
}
