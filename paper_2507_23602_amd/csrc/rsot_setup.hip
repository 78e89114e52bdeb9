// Problem setup: validation, spatial sort into 64-point tiles and 64-target
// blocks, per-tile / per-block bounding boxes, covering cost.
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <limits>

#include "rsot_device.h"
#include "rsot_internal.h"

// ---------------------------------------------------------------------------
// allocation with the optional memory cap
// ---------------------------------------------------------------------------
rsot_status rsot_dev_alloc(rsot_problem *p, void **ptr, size_t bytes) {
    if (bytes == 0) bytes = 256;
    bytes = (bytes + 255) & ~size_t(255);
    if (p->opt.mem_limit_bytes > 0 && p->bytes + bytes > (size_t)p->opt.mem_limit_bytes)
        return RSOT_ERR_OOM;
    void *q = nullptr;
    if (hipMalloc(&q, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return RSOT_ERR_OOM;
    }
    p->allocs.push_back(q);
    p->alloc_bytes.push_back(bytes);
    p->bytes += bytes;
    *ptr = q;
    return RSOT_OK;
}

void rsot_dev_free(rsot_problem *p, void *ptr) {
    if (!ptr) return;
    for (size_t i = 0; i < p->allocs.size(); ++i) {
        if (p->allocs[i] == ptr) {
            (void)hipFree(ptr);
            p->bytes -= p->alloc_bytes[i];
            p->allocs.erase(p->allocs.begin() + i);
            p->alloc_bytes.erase(p->alloc_bytes.begin() + i);
            return;
        }
    }
}

template <typename T>
static rsot_status dalloc(rsot_problem *p, T **ptr, size_t count) {
    void *q = nullptr;
    RSOT_TRY(rsot_dev_alloc(p, &q, count * sizeof(T)));
    *ptr = (T *)q;
    return RSOT_OK;
}

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------
// Per-workgroup statistics of a point set: bounding box, mass sum, number of
// non-finite values, number of masses below the allowed minimum.
struct PointStats {
    double lo[3], hi[3];
    double wsum, wmin, wmax, w2sum;
    double nonfinite, badmass;
    double unitdev;             // max | |v|^2 - 1 | (3D rows)
};

__global__ __launch_bounds__(256) void k_point_stats(const double *__restrict__ x,
                                                     const double *__restrict__ w, int64_t n,
                                                     int dim, int strict_positive,
                                                     PointStats *__restrict__ part) {
    __shared__ PointStats red[4];
    PointStats s;
    for (int k = 0; k < 3; ++k) {
        s.lo[k] = INFINITY;
        s.hi[k] = -INFINITY;
    }
    s.wsum = 0;
    s.w2sum = 0;
    s.wmin = INFINITY;
    s.wmax = -INFINITY;
    s.nonfinite = 0;
    s.badmass = 0;
    s.unitdev = 0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        if (dim == 3) {
            const double r2 = x[i * 3] * x[i * 3] + x[i * 3 + 1] * x[i * 3 + 1] +
                              x[i * 3 + 2] * x[i * 3 + 2];
            s.unitdev = fmax(s.unitdev, fabs(r2 - 1.0));
        }
        for (int k = 0; k < dim; ++k) {
            double v = x[i * dim + k];
            if (!isfinite(v)) {
                s.nonfinite += 1;
                continue;
            }
            s.lo[k] = fmin(s.lo[k], v);
            s.hi[k] = fmax(s.hi[k], v);
        }
        double m = w[i];
        if (!isfinite(m)) {
            s.nonfinite += 1;
            continue;
        }
        if (strict_positive ? !(m > 0.0) : !(m >= 0.0)) s.badmass += 1;
        s.wsum += m;
        s.w2sum += m * m;
        s.wmin = fmin(s.wmin, m);
        s.wmax = fmax(s.wmax, m);
    }
    for (int k = 0; k < 3; ++k) {
        s.lo[k] = wave_min(s.lo[k]);
        s.hi[k] = wave_max(s.hi[k]);
    }
    s.wsum = wave_sum(s.wsum);
    s.w2sum = wave_sum(s.w2sum);
    s.wmin = wave_min(s.wmin);
    s.wmax = wave_max(s.wmax);
    s.nonfinite = wave_sum(s.nonfinite);
    s.badmass = wave_sum(s.badmass);
    s.unitdev = wave_max(s.unitdev);
    const int wv = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) red[wv] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        PointStats r = red[0];
        for (int i = 1; i < 4; ++i) {
            for (int k = 0; k < 3; ++k) {
                r.lo[k] = fmin(r.lo[k], red[i].lo[k]);
                r.hi[k] = fmax(r.hi[k], red[i].hi[k]);
            }
            r.wsum += red[i].wsum;
            r.w2sum += red[i].w2sum;
            r.wmin = fmin(r.wmin, red[i].wmin);
            r.wmax = fmax(r.wmax, red[i].wmax);
            r.nonfinite += red[i].nonfinite;
            r.badmass += red[i].badmass;
            r.unitdev = fmax(r.unitdev, red[i].unitdev);
        }
        part[blockIdx.x] = r;
    }
}

// single workgroup: fold the per-workgroup partials in index order
__global__ __launch_bounds__(64) void k_point_stats_final(const PointStats *__restrict__ part,
                                                          int np, PointStats *__restrict__ out) {
    if (threadIdx.x != 0) return;
    PointStats r = part[0];
    for (int i = 1; i < np; ++i) {
        for (int k = 0; k < 3; ++k) {
            r.lo[k] = fmin(r.lo[k], part[i].lo[k]);
            r.hi[k] = fmax(r.hi[k], part[i].hi[k]);
        }
        r.wsum += part[i].wsum;
        r.w2sum += part[i].w2sum;
        r.wmin = fmin(r.wmin, part[i].wmin);
        r.wmax = fmax(r.wmax, part[i].wmax);
        r.nonfinite += part[i].nonfinite;
        r.badmass += part[i].badmass;
        r.unitdev = fmax(r.unitdev, part[i].unitdev);
    }
    *out = r;
}

__global__ void k_fill_value(double *__restrict__ v, int64_t n, double val) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) v[i] = val;
}

__device__ inline uint32_t spread2(uint32_t v) {  // 16 bits -> even positions
    v &= 0xffffu;
    v = (v | (v << 8)) & 0x00ff00ffu;
    v = (v | (v << 4)) & 0x0f0f0f0fu;
    v = (v | (v << 2)) & 0x33333333u;
    v = (v | (v << 1)) & 0x55555555u;
    return v;
}
__device__ inline uint32_t spread3(uint32_t v) {  // 10 bits -> every third position
    v &= 0x3ffu;
    v = (v | (v << 16)) & 0x030000ffu;
    v = (v | (v << 8)) & 0x0300f00fu;
    v = (v | (v << 4)) & 0x030c30c3u;
    v = (v | (v << 2)) & 0x09249249u;
    return v;
}

// Morton key of each point on a uniform grid over [lo, hi]
__global__ void k_morton(const double *__restrict__ x, int64_t n, int dim, double lo0, double lo1,
                         double lo2, double inv0, double inv1, double inv2,
                         uint32_t *__restrict__ keys, int32_t *__restrict__ idx) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double lo[3] = {lo0, lo1, lo2};
    const double inv[3] = {inv0, inv1, inv2};
    const double cells = dim == 2 ? 65535.0 : 1023.0;
    uint32_t c[3] = {0, 0, 0};
    for (int k = 0; k < dim; ++k) {
        double t = (x[i * dim + k] - lo[k]) * inv[k] * cells;
        t = fmin(fmax(t, 0.0), cells);
        c[k] = (uint32_t)t;
    }
    keys[i] = dim == 2 ? (spread2(c[0]) | (spread2(c[1]) << 1))
                       : (spread3(c[0]) | (spread3(c[1]) << 1) | (spread3(c[2]) << 2));
    idx[i] = (int32_t)i;
}

// gather points into sorted, padded slots
__global__ void k_gather_points(const double *__restrict__ x, const double *__restrict__ mu,
                                const int32_t *__restrict__ order, int64_t nq, int64_t nq_pad,
                                int dim, double s0, double s1, double s2,
                                double4 *__restrict__ qp, double *__restrict__ qmu,
                                double *__restrict__ qlog2mu, int32_t *__restrict__ qperm) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= nq_pad) return;
    const bool real = i < nq;
    const int32_t src = order[real ? i : nq - 1];
    double4 r;
    r.x = x[(int64_t)src * dim + 0] - s0;
    r.y = x[(int64_t)src * dim + 1] - s1;
    r.z = dim == 3 ? x[(int64_t)src * dim + 2] - s2 : 0.0;
    r.w = 0.0;
    qp[i] = r;
    const double m = real ? mu[src] : 0.0;
    qmu[i] = m;
    qlog2mu[i] = m > 0.0 ? log2(m) : -INFINITY;
    qperm[i] = real ? src : -1;
}

__global__ void k_gather_targets(const double *__restrict__ y, const double *__restrict__ nu,
                                 const int32_t *__restrict__ order, int64_t n, int64_t n_pad,
                                 int dim, double s0, double s1, double s2,
                                 double *__restrict__ ty, double *__restrict__ tnu,
                                 double *__restrict__ tlog2nu, int32_t *__restrict__ tperm) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n_pad) return;
    const bool real = i < n;
    const int32_t src = order[real ? i : n - 1];
    ty[i * 3 + 0] = y[(int64_t)src * dim + 0] - s0;
    ty[i * 3 + 1] = y[(int64_t)src * dim + 1] - s1;
    ty[i * 3 + 2] = dim == 3 ? y[(int64_t)src * dim + 2] - s2 : 0.0;
    const double v = real ? nu[src] : 0.0;
    tnu[i] = v;
    tlog2nu[i] = real ? log2(v) : -INFINITY;
    tperm[i] = real ? src : -1;
}

// one wavefront per 64-point tile: bounding box and number of real points
__global__ __launch_bounds__(256) void k_tile_boxes(const double4 *__restrict__ qp,
                                                    const int32_t *__restrict__ qperm,
                                                    int64_t n_tiles, double *__restrict__ lo,
                                                    double *__restrict__ hi,
                                                    int32_t *__restrict__ cnt) {
    const int lane = threadIdx.x & 63;
    const int64_t t = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (t >= n_tiles) return;
    const int64_t q = t * 64 + lane;
    const double4 r = qp[q];
    const double v[3] = {r.x, r.y, r.z};
    for (int k = 0; k < 3; ++k) {
        double a = wave_min(v[k]);
        double b = wave_max(v[k]);
        if (lane == 0) {
            lo[t * 3 + k] = a;
            hi[t * 3 + k] = b;
        }
    }
    double c = wave_sum(qperm[q] >= 0 ? 1.0 : 0.0);
    if (lane == 0) cnt[t] = (int32_t)c;
}

__global__ __launch_bounds__(256) void k_block_boxes(const double *__restrict__ ty,
                                                     const double *__restrict__ tnu,
                                                     const int32_t *__restrict__ tperm,
                                                     int64_t n_blocks, double *__restrict__ lo,
                                                     double *__restrict__ hi,
                                                     double *__restrict__ bnu,
                                                     double *__restrict__ blnnu,
                                                     int32_t *__restrict__ cnt) {
    const int lane = threadIdx.x & 63;
    const int64_t b = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (b >= n_blocks) return;
    const int64_t j = b * 64 + lane;
    for (int k = 0; k < 3; ++k) {
        double v = ty[j * 3 + k];
        double a = wave_min(v);
        double c = wave_max(v);
        if (lane == 0) {
            lo[b * 3 + k] = a;
            hi[b * 3 + k] = c;
        }
    }
    double m = wave_sum(tnu[j]);
    double c = wave_sum(tperm[j] >= 0 ? 1.0 : 0.0);
    if (lane == 0) {
        bnu[b] = m;
        blnnu[b] = log(m);
        cnt[b] = (int32_t)c;
    }
}

// Covering cost, one wavefront per tile: the nearest target of every point
// lies in a block whose least box distance to the tile is at most
// min_B (greatest box distance), so only those blocks are scanned.
template <int D>
__global__ __launch_bounds__(256) void k_covering(const double4 *__restrict__ qp,
                                                  const int32_t *__restrict__ qperm,
                                                  const double *__restrict__ ty,
                                                  const double *__restrict__ tile_lo,
                                                  const double *__restrict__ tile_hi,
                                                  const double *__restrict__ blk_lo,
                                                  const double *__restrict__ blk_hi,
                                                  const int32_t *__restrict__ blk_cnt,
                                                  int64_t n_tiles, int64_t n_blocks,
                                                  double *__restrict__ tile_best) {
    const int lane = threadIdx.x & 63;
    const int64_t t = blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (t >= n_tiles) return;
    double tl[3], th[3];
    for (int k = 0; k < 3; ++k) {
        tl[k] = tile_lo[t * 3 + k];
        th[k] = tile_hi[t * 3 + k];
    }
    double ub = INFINITY;
    for (int64_t b = lane; b < n_blocks; b += 64) {
        double s = 0;
        for (int k = 0; k < D; ++k) {
            double g = box_far(tl[k], th[k], blk_lo[b * 3 + k], blk_hi[b * 3 + k]);
            s += g * g;
        }
        ub = fmin(ub, s);
    }
    ub = wave_min(ub);
    const double4 r = qp[t * 64 + lane];
    const double x[3] = {r.x, r.y, r.z};
    double best = INFINITY;
    for (int64_t b = 0; b < n_blocks; ++b) {
        double s = 0;
        for (int k = 0; k < D; ++k) {
            double g = box_gap(tl[k], th[k], blk_lo[b * 3 + k], blk_hi[b * 3 + k]);
            s += g * g;
        }
        if (s > ub) continue;
        const int cnt = blk_cnt[b];
        for (int k = 0; k < cnt; ++k) {
            const double *yy = ty + (b * 64 + k) * 3;
            double d2 = 0;
            for (int c = 0; c < D; ++c) {
                double e = x[c] - yy[c];
                d2 += e * e;
            }
            best = fmin(best, d2);
        }
    }
    if (qperm[t * 64 + lane] < 0) best = 0.0;
    best = wave_max(best);
    if (lane == 0) tile_best[t] = best;
}

__global__ __launch_bounds__(256) void k_max_final(const double *__restrict__ v, int64_t n,
                                                   double *__restrict__ out) {
    __shared__ double red[4];
    double m = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 256) m = fmax(m, v[i]);
    m = wave_max(m);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) *out = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
static rsot_status point_stats(rsot_problem *p, const double *x, const double *w, int64_t n,
                               int strict, PointStats *out) {
    const int nwg = (int)std::min<int64_t>(1024, (n + 255) / 256);
    PointStats *part = nullptr, *fin = nullptr;
    RSOT_TRY(dalloc(p, &part, nwg));
    RSOT_TRY(dalloc(p, &fin, 1));
    hipLaunchKernelGGL(k_point_stats, dim3(nwg), dim3(256), 0, p->stream, x, w, n, p->dim, strict,
                       part);
    hipLaunchKernelGGL(k_point_stats_final, dim3(1), dim3(64), 0, p->stream, part, nwg, fin);
    RSOT_HIP(hipMemcpyAsync(out, fin, sizeof(PointStats), hipMemcpyDeviceToHost, p->stream));
    RSOT_HIP(hipStreamSynchronize(p->stream));
    rsot_dev_free(p, part);
    rsot_dev_free(p, fin);
    return RSOT_OK;
}

static rsot_status sort_points(rsot_problem *p, const double *x, int64_t n, const PointStats &st,
                               int32_t **order_out) {
    uint32_t *keys = nullptr, *keys2 = nullptr;
    int32_t *idx = nullptr, *idx2 = nullptr;
    RSOT_TRY(dalloc(p, &keys, n));
    RSOT_TRY(dalloc(p, &keys2, n));
    RSOT_TRY(dalloc(p, &idx, n));
    RSOT_TRY(dalloc(p, &idx2, n));
    double inv[3] = {0, 0, 0};
    for (int k = 0; k < p->dim; ++k) {
        double ext = st.hi[k] - st.lo[k];
        inv[k] = ext > 0 ? 1.0 / ext : 0.0;
    }
    hipLaunchKernelGGL(k_morton, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, p->stream, x, n,
                       p->dim, st.lo[0], st.lo[1], p->dim == 3 ? st.lo[2] : 0.0, inv[0], inv[1],
                       inv[2], keys, idx);
    size_t tmp_bytes = 0;
    RSOT_HIP(hipcub::DeviceRadixSort::SortPairs(nullptr, tmp_bytes, keys, keys2, idx, idx2, (int)n,
                                                0, 32, p->stream));
    void *tmp = nullptr;
    RSOT_TRY(rsot_dev_alloc(p, &tmp, tmp_bytes));
    RSOT_HIP(hipcub::DeviceRadixSort::SortPairs(tmp, tmp_bytes, keys, keys2, idx, idx2, (int)n, 0,
                                                32, p->stream));
    RSOT_HIP(hipStreamSynchronize(p->stream));
    rsot_dev_free(p, tmp);
    rsot_dev_free(p, keys);
    rsot_dev_free(p, keys2);
    rsot_dev_free(p, idx);
    *order_out = idx2;
    return RSOT_OK;
}

static rsot_status create_impl(rsot_problem *p, const double *x, const double *mu,
                               const double *y, const double *nu) {
    const int64_t nq = p->nq, n = p->n;
    const double *dx = x, *dmu = mu, *dy = y, *dnu = nu;
    double *tx = nullptr, *tmu = nullptr, *tyy = nullptr, *tnu = nullptr;
    if (!p->opt.inputs_on_device) {
        RSOT_TRY(dalloc(p, &tx, nq * p->dim));
        RSOT_TRY(dalloc(p, &tmu, nq));
        RSOT_TRY(dalloc(p, &tyy, n * p->dim));
        RSOT_TRY(dalloc(p, &tnu, n));
        RSOT_HIP(hipMemcpyAsync(tx, x, sizeof(double) * nq * p->dim, hipMemcpyHostToDevice,
                                p->stream));
        RSOT_HIP(hipMemcpyAsync(tmu, mu, sizeof(double) * nq, hipMemcpyHostToDevice, p->stream));
        RSOT_HIP(hipMemcpyAsync(tyy, y, sizeof(double) * n * p->dim, hipMemcpyHostToDevice,
                                p->stream));
        RSOT_HIP(hipMemcpyAsync(tnu, nu, sizeof(double) * n, hipMemcpyHostToDevice, p->stream));
        dx = tx;
        dmu = tmu;
        dy = tyy;
        dnu = tnu;
    }
    PointStats sq, st;
    RSOT_TRY(point_stats(p, dx, dmu, nq, 0, &sq));
    RSOT_TRY(point_stats(p, dy, dnu, n, 1, &st));
    if (sq.nonfinite > 0 || st.nonfinite > 0) return RSOT_ERR_NONFINITE;
    if (sq.badmass > 0 || st.badmass > 0 || !(sq.wsum > 0.0)) return RSOT_ERR_INVALID_ARG;
    p->sum_mu = sq.wsum;
    p->sum_mu2 = sq.w2sum;
    p->sum_nu = st.wsum;
    RSOT_TRY(rsot_device_exp_corr(p->stream, &p->exp_corr));
    p->nu_min = st.wmin;
    p->nu_max = st.wmax;
    // the sphere cost needs unit vectors (and keeps them unshifted)
    if (p->opt.cost_kind == RSOT_COST_SPHERE && (sq.unitdev > 1e-9 || st.unitdev > 1e-9))
        return RSOT_ERR_INVALID_ARG;
    for (int k = 0; k < 3; ++k)
        p->shift[k] = (k < p->dim && p->opt.cost_kind == RSOT_COST_SQEUCLID)
                          ? 0.5 * (st.lo[k] + st.hi[k])
                          : 0.0;

    int32_t *qorder = nullptr, *torder = nullptr;
    RSOT_TRY(sort_points(p, dx, nq, sq, &qorder));
    RSOT_TRY(sort_points(p, dy, n, st, &torder));

    p->nq_pad = (nq + 63) / 64 * 64;
    p->n_pad = (n + 63) / 64 * 64;
    p->n_tiles = p->nq_pad / 64;
    p->n_blocks = p->n_pad / 64;
    RSOT_TRY(dalloc(p, &p->qp, p->nq_pad));
    RSOT_TRY(dalloc(p, &p->qmu, p->nq_pad));
    RSOT_TRY(dalloc(p, &p->qlog2mu, p->nq_pad));
    RSOT_TRY(dalloc(p, &p->qA, p->nq_pad));
    RSOT_TRY(dalloc(p, &p->qlse, p->nq_pad));
    RSOT_TRY(dalloc(p, &p->qkept, p->nq_pad));
    RSOT_TRY(dalloc(p, &p->qperm, p->nq_pad));
    RSOT_TRY(dalloc(p, &p->tile_lo, p->n_tiles * 3));
    RSOT_TRY(dalloc(p, &p->tile_hi, p->n_tiles * 3));
    RSOT_TRY(dalloc(p, &p->tile_cnt, p->n_tiles));
    RSOT_TRY(dalloc(p, &p->tile_part, p->n_tiles * 4));
    RSOT_TRY(dalloc(p, &p->tile_ref, p->n_tiles));
    if (p->opt.cost_kind == RSOT_COST_SPHERE) RSOT_TRY(dalloc(p, &p->tile_smax, p->n_tiles));
    RSOT_TRY(dalloc(p, &p->ty, p->n_pad * 3));
    RSOT_TRY(dalloc(p, &p->tnu, p->n_pad));
    RSOT_TRY(dalloc(p, &p->tlog2nu, p->n_pad));
    RSOT_TRY(dalloc(p, &p->tperm, p->n_pad));
    RSOT_TRY(dalloc(p, &p->trec, p->n_pad));
    if (p->dim == 2) RSOT_TRY(dalloc(p, &p->trec3, p->n_pad * 3));
    RSOT_TRY(dalloc(p, &p->tG, p->n_pad));
    RSOT_TRY(dalloc(p, &p->tpsi, p->n_pad));
    RSOT_TRY(dalloc(p, &p->blk_lo, p->n_blocks * 3));
    RSOT_TRY(dalloc(p, &p->blk_hi, p->n_blocks * 3));
    RSOT_TRY(dalloc(p, &p->blk_nu, p->n_blocks));
    RSOT_TRY(dalloc(p, &p->blk_lnnu, p->n_blocks));
    RSOT_TRY(dalloc(p, &p->blk_cnt, p->n_blocks));
    RSOT_TRY(dalloc(p, &p->blk_stat, p->n_blocks * 4));
    RSOT_TRY(dalloc(p, &p->blk_gpart, p->n_blocks * 2));
    RSOT_TRY(dalloc(p, &p->dscal, 64));
    RSOT_TRY(dalloc(p, &p->dpsi, p->n));
    RSOT_TRY(dalloc(p, &p->dgrad, p->n));
    RSOT_TRY(dalloc(p, &p->i64tmp, 64));
    RSOT_HIP(hipHostMalloc((void **)&p->hscal, sizeof(double) * 64, hipHostMallocDefault));
    RSOT_HIP(hipHostMalloc((void **)&p->hpsi, sizeof(double) * p->n, hipHostMallocDefault));
    RSOT_HIP(hipHostMalloc((void **)&p->hgrad, sizeof(double) * p->n, hipHostMallocDefault));

    hipLaunchKernelGGL(k_gather_points, dim3((unsigned)((p->nq_pad + 255) / 256)), dim3(256), 0,
                       p->stream, dx, dmu, qorder, nq, p->nq_pad, p->dim, p->shift[0],
                       p->shift[1], p->shift[2], p->qp, p->qmu, p->qlog2mu, p->qperm);
    hipLaunchKernelGGL(k_gather_targets, dim3((unsigned)((p->n_pad + 255) / 256)), dim3(256), 0,
                       p->stream, dy, dnu, torder, n, p->n_pad, p->dim, p->shift[0], p->shift[1],
                       p->shift[2], p->ty, p->tnu, p->tlog2nu, p->tperm);
    hipLaunchKernelGGL(k_tile_boxes, dim3((unsigned)((p->n_tiles + 3) / 4)), dim3(256), 0,
                       p->stream, p->qp, p->qperm, p->n_tiles, p->tile_lo, p->tile_hi,
                       p->tile_cnt);
    hipLaunchKernelGGL(k_block_boxes, dim3((unsigned)((p->n_blocks + 3) / 4)), dim3(256), 0,
                       p->stream, p->ty, p->tnu, p->tperm, p->n_blocks, p->blk_lo, p->blk_hi,
                       p->blk_nu, p->blk_lnnu, p->blk_cnt);
    RSOT_HIP(hipGetLastError());
    RSOT_HIP(hipStreamSynchronize(p->stream));
    rsot_dev_free(p, qorder);
    rsot_dev_free(p, torder);
    if (tx) {
        rsot_dev_free(p, tx);
        rsot_dev_free(p, tmu);
        rsot_dev_free(p, tyy);
        rsot_dev_free(p, tnu);
    }
    RSOT_HIP(hipEventCreate(&p->ev0));
    RSOT_HIP(hipEventCreate(&p->ev1));
    RSOT_HIP(hipEventCreate(&p->ev_p1));
    RSOT_HIP(hipEventCreate(&p->ev_mid));
    RSOT_HIP(hipEventCreate(&p->ev_p2));
    RSOT_HIP(hipEventCreate(&p->ev_b0));
    RSOT_HIP(hipEventCreate(&p->ev_b1));
    return RSOT_OK;
}

// Morton order of n device points (dim of the problem) over their own box;
// *order_out (device, n int32) is allocated here and owned by the caller.
rsot_status rsot_morton_order(rsot_problem *p, const double *x, int64_t n, int32_t **order_out) {
    const int nwg = (int)std::min<int64_t>(1024, (n + 255) / 256);
    PointStats *part = nullptr, *fin = nullptr;
    RSOT_TRY(dalloc(p, &part, nwg));
    RSOT_TRY(dalloc(p, &fin, 1));
    double *ones = nullptr;
    RSOT_TRY(dalloc(p, &ones, n));
    hipLaunchKernelGGL(k_fill_value, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, p->stream,
                       ones, n, 1.0);
    hipLaunchKernelGGL(k_point_stats, dim3(nwg), dim3(256), 0, p->stream, x, ones, n, p->dim, 0,
                       part);
    hipLaunchKernelGGL(k_point_stats_final, dim3(1), dim3(64), 0, p->stream, part, nwg, fin);
    PointStats st;
    RSOT_HIP(hipMemcpyAsync(&st, fin, sizeof(PointStats), hipMemcpyDeviceToHost, p->stream));
    RSOT_HIP(hipStreamSynchronize(p->stream));
    rsot_dev_free(p, part);
    rsot_dev_free(p, fin);
    rsot_dev_free(p, ones);
    if (st.nonfinite > 0) return RSOT_ERR_NONFINITE;
    return sort_points(p, x, n, st, order_out);
}

rsot_status rsot_compute_covering_cost(rsot_problem *p) {
    if (p->C0 >= 0) return RSOT_OK;
    double *tb = nullptr;
    RSOT_TRY(dalloc(p, &tb, p->n_tiles));
    const dim3 grid((unsigned)((p->n_tiles + 3) / 4));
    if (p->dim == 2)
        hipLaunchKernelGGL(k_covering<2>, grid, dim3(256), 0, p->stream, p->qp, p->qperm, p->ty,
                           p->tile_lo, p->tile_hi, p->blk_lo, p->blk_hi, p->blk_cnt, p->n_tiles,
                           p->n_blocks, tb);
    else
        hipLaunchKernelGGL(k_covering<3>, grid, dim3(256), 0, p->stream, p->qp, p->qperm, p->ty,
                           p->tile_lo, p->tile_hi, p->blk_lo, p->blk_hi, p->blk_cnt, p->n_tiles,
                           p->n_blocks, tb);
    hipLaunchKernelGGL(k_max_final, dim3(1), dim3(256), 0, p->stream, tb, p->n_tiles,
                       p->dscal + SC_C0);
    RSOT_HIP(hipGetLastError());
    RSOT_HIP(hipMemcpyAsync(p->hscal + SC_C0, p->dscal + SC_C0, sizeof(double),
                            hipMemcpyDeviceToHost, p->stream));
    RSOT_HIP(hipStreamSynchronize(p->stream));
    p->C0 = p->opt.cost_scale * p->hscal[SC_C0];
    rsot_dev_free(p, tb);
    return RSOT_OK;
}

// ---------------------------------------------------------------------------
// ABI
// ---------------------------------------------------------------------------
extern "C" void rsot_options_default(rsot_options *opt) {
    if (!opt) return;
    std::memset(opt, 0, sizeof(*opt));
    opt->cost_scale = 0.5;
    opt->precision = RSOT_PREC_MIXED;
    opt->truncation = RSOT_TRUNC_DENSE;
    opt->tau = 1e-12;
    opt->delta_thr = 1e-12;
    opt->fp64_below_points = 16384;
    opt->tile_group = 0;
}

extern "C" const char *rsot_status_string(rsot_status s) {
    switch (s) {
    case RSOT_OK: return "ok";
    case RSOT_ERR_INVALID_ARG: return "invalid argument";
    case RSOT_ERR_NONFINITE: return "non-finite input";
    case RSOT_ERR_UNBALANCED: return "unbalanced masses";
    case RSOT_ERR_DEVICE: return "device error";
    case RSOT_ERR_OOM: return "out of device memory";
    case RSOT_ERR_LINESEARCH: return "line search failed";
    case RSOT_ERR_NOT_CONVERGED: return "not converged";
    case RSOT_ERR_CANCELLED: return "cancelled";
    }
    return "unknown status";
}

static bool options_valid(const rsot_options &o) {
    if (!(o.cost_scale > 0.0) || !std::isfinite(o.cost_scale)) return false;
    if (o.precision != RSOT_PREC_MIXED && o.precision != RSOT_PREC_FP64) return false;
    if (o.truncation < RSOT_TRUNC_DENSE || o.truncation > RSOT_TRUNC_TILE) return false;
    if (!(o.tau > 0.0) || !(o.delta_thr > 0.0)) return false;
    if (o.seg_tiles < 0 || o.seg_blocks < 0 || o.mem_limit_bytes < 0) return false;
    if (o.fp64_below_points < 0) return false;
    if (o.tile_group != 0 && o.tile_group != 8 && o.tile_group != 16 && o.tile_group != 32 &&
        o.tile_group != 64)
        return false;
    if (o.cost_kind != RSOT_COST_SQEUCLID && o.cost_kind != RSOT_COST_SPHERE) return false;
    if (o.cost_kind == RSOT_COST_SPHERE && o.truncation != RSOT_TRUNC_DENSE &&
        o.truncation != RSOT_TRUNC_TILE)
        return false;
    return true;
}

extern "C" rsot_status rsot_problem_create(int dim, int64_t n_quad, const double *x,
                                           const double *mu, int64_t n_target, const double *y,
                                           const double *nu, const rsot_options *opt,
                                           void *hip_stream, rsot_problem **out) {
    if (!out) return RSOT_ERR_INVALID_ARG;
    *out = nullptr;
    if (dim != 2 && dim != 3) return RSOT_ERR_INVALID_ARG;
    if (n_quad <= 0 || n_target <= 0 || !x || !mu || !y || !nu) return RSOT_ERR_INVALID_ARG;
    if (n_quad > (int64_t)INT32_MAX - 64 || n_target > (int64_t)INT32_MAX - 64)
        return RSOT_ERR_INVALID_ARG;
    rsot_options o;
    rsot_options_default(&o);
    if (opt) o = *opt;
    if (!options_valid(o)) return RSOT_ERR_INVALID_ARG;
    if (o.cost_kind == RSOT_COST_SPHERE && dim != 3) return RSOT_ERR_INVALID_ARG;
    rsot_problem *p = new (std::nothrow) rsot_problem();
    if (!p) return RSOT_ERR_OOM;
    p->dim = dim;
    p->nq = n_quad;
    p->n = n_target;
    p->opt = o;
    p->stream = (hipStream_t)hip_stream;
    rsot_status s = create_impl(p, x, mu, y, nu);
    if (s != RSOT_OK) {
        rsot_problem_destroy(p);
        return s;
    }
    *out = p;
    return RSOT_OK;
}

extern "C" void rsot_problem_destroy(rsot_problem *p) {
    if (!p) return;
    (void)hipStreamSynchronize(p->stream);
    for (void *a : p->allocs) (void)hipFree(a);
    if (p->hscal) (void)hipHostFree(p->hscal);
    if (p->hpsi) (void)hipHostFree(p->hpsi);
    if (p->hgrad) (void)hipHostFree(p->hgrad);
    if (p->ev0) (void)hipEventDestroy(p->ev0);
    if (p->ev1) (void)hipEventDestroy(p->ev1);
    if (p->ev_p1) (void)hipEventDestroy(p->ev_p1);
    if (p->ev_mid) (void)hipEventDestroy(p->ev_mid);
    if (p->ev_p2) (void)hipEventDestroy(p->ev_p2);
    if (p->ev_b0) (void)hipEventDestroy(p->ev_b0);
    if (p->ev_b1) (void)hipEventDestroy(p->ev_b1);
    delete p;
}

extern "C" rsot_status rsot_problem_sizes(const rsot_problem *p, int *dim, int64_t *n_quad,
                                          int64_t *n_target) {
    if (!p) return RSOT_ERR_INVALID_ARG;
    if (dim) *dim = p->dim;
    if (n_quad) *n_quad = p->nq;
    if (n_target) *n_target = p->n;
    return RSOT_OK;
}

extern "C" rsot_status rsot_set_truncation(rsot_problem *p, int truncation, double tau,
                                           double delta_thr) {
    if (!p) return RSOT_ERR_INVALID_ARG;
    rsot_options o = p->opt;
    o.truncation = truncation;
    o.tau = tau;
    o.delta_thr = delta_thr;
    if (!options_valid(o)) return RSOT_ERR_INVALID_ARG;
    p->opt = o;
    p->have_D = 0;
    return RSOT_OK;
}

extern "C" rsot_status rsot_set_precision(rsot_problem *p, int precision) {
    if (!p) return RSOT_ERR_INVALID_ARG;
    if (precision != RSOT_PREC_MIXED && precision != RSOT_PREC_FP64) return RSOT_ERR_INVALID_ARG;
    p->opt.precision = precision;
    return RSOT_OK;
}

// MIXED problems run the FP64 pair loop when both their effective number of
// points is below opt.fp64_below_points (too few for the FP32 exponentials'
// per-point errors to average below 1e-9 of J) and their pair count is below
// 2^27 (where the FP64 loop costs well under a millisecond). Larger problems
// with concentrated masses keep the FP32 loop: there the error of J is the
// per-point one averaged over n_eff points, 1.5e-7 eps sum(mu) / sqrt(n_eff).
bool rsot_pairs_fp64(const rsot_problem *p) {
    if (p->opt.precision == RSOT_PREC_FP64) return true;
    const double n_eff = p->sum_mu2 > 0.0 ? p->sum_mu * p->sum_mu / p->sum_mu2 : 0.0;
    return n_eff < (double)p->opt.fp64_below_points && (double)p->nq * (double)p->n < 0x1p27;
}

extern "C" rsot_status rsot_set_reference(rsot_problem *p, double absJ_ref) {
    if (!p || !(absJ_ref >= 0.0) || !std::isfinite(absJ_ref)) return RSOT_ERR_INVALID_ARG;
    p->absJ_ref = absJ_ref;
    return RSOT_OK;
}

extern "C" rsot_status rsot_covering_cost(rsot_problem *p, double *C0_out) {
    if (!p || !C0_out) return RSOT_ERR_INVALID_ARG;
    if (p->opt.cost_kind != RSOT_COST_SQEUCLID) return RSOT_ERR_INVALID_ARG;
    RSOT_TRY(rsot_compute_covering_cost(p));
    *C0_out = p->C0;
    return RSOT_OK;
}

__global__ void k_partition(const int32_t *__restrict__ perm, int64_t npad,
                            int32_t *__restrict__ out) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= npad) return;
    int32_t src = perm[i];
    if (src >= 0) out[src] = (int32_t)(i / 64);
}

extern "C" rsot_status rsot_get_partition(rsot_problem *p, int32_t *tile_of_point,
                                          int32_t *block_of_target, int64_t *n_tiles,
                                          int64_t *n_blocks) {
    if (!p) return RSOT_ERR_INVALID_ARG;
    if (tile_of_point)
        hipLaunchKernelGGL(k_partition, dim3((unsigned)((p->nq_pad + 255) / 256)), dim3(256), 0,
                           p->stream, p->qperm, p->nq_pad, tile_of_point);
    if (block_of_target)
        hipLaunchKernelGGL(k_partition, dim3((unsigned)((p->n_pad + 255) / 256)), dim3(256), 0,
                           p->stream, p->tperm, p->n_pad, block_of_target);
    RSOT_HIP(hipGetLastError());
    RSOT_HIP(hipStreamSynchronize(p->stream));
    if (n_tiles) *n_tiles = p->n_tiles;
    if (n_blocks) *n_blocks = p->n_blocks;
    return RSOT_OK;
}
