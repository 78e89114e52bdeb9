// Target-set hierarchy by k-means coarsening (Sec. 5.2): level l-1 is a
// k-means clustering of the points of level l; each cluster becomes one point
// at its centroid (mean of the member points) carrying the summed mass of its
// members, so every level keeps the total mass. Levels are built from the
// finest down.
//
// GPU Lloyd iterations: initial centroids are means of consecutive groups of
// points in Morton order; the assignment step finds the exact nearest centroid
// through a uniform grid over the centroids, scanning rings of cells until the
// unscanned region is provably farther than the best candidate (ties go to
// the lowest centroid index); the update step sorts points by cluster (stable
// radix sort) and averages each cluster's members in index order. No atomics
// on floating point: results are reproducible.
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <cmath>
#include <vector>

#include "rsot_device.h"
#include "rsot_internal.h"

namespace {

struct Ctx {
    hipStream_t stream;
    std::vector<void *> mem;
    ~Ctx() {
        for (void *p : mem) (void)hipFree(p);
    }
    template <typename T>
    T *alloc(size_t n) {
        void *p = nullptr;
        if (hipMalloc(&p, std::max<size_t>(n, 1) * sizeof(T)) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
        mem.push_back(p);
        return (T *)p;
    }
};

__global__ void k_iota(int32_t *v, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) v[i] = (int32_t)i;
}

// Morton key on a 1024^3 / 65536^2 grid over [lo, lo + ext]
__global__ void k_keys(const double *__restrict__ y, int64_t n, int dim, double l0, double l1,
                       double l2, double inv, uint32_t *__restrict__ keys) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double lo[3] = {l0, l1, l2};
    const double cells = dim == 2 ? 65535.0 : 1023.0;
    uint32_t c[3] = {0, 0, 0};
    for (int k = 0; k < dim; ++k) {
        double t = (y[i * dim + k] - lo[k]) * inv * cells;
        c[k] = (uint32_t)fmin(fmax(t, 0.0), cells);
    }
    uint32_t key = 0;
    const int bits = dim == 2 ? 16 : 10;
    for (int b = bits - 1; b >= 0; --b)
        for (int k = dim - 1; k >= 0; --k) key = (key << 1) | ((c[k] >> b) & 1u);
    keys[i] = key;
}

// initial centroid c: mean of points order[c*n/k, (c+1)*n/k)
__global__ void k_init_centroids(const double *__restrict__ y, const int32_t *__restrict__ order,
                                 int64_t n, int64_t k, int dim, double *__restrict__ cen) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= k) return;
    const int64_t a = c * n / k, b = (c + 1) * n / k;
    double s[3] = {0, 0, 0};
    for (int64_t i = a; i < b; ++i)
        for (int d = 0; d < dim; ++d) s[d] += y[(int64_t)order[i] * dim + d];
    for (int d = 0; d < dim; ++d) cen[c * dim + d] = s[d] / (double)(b - a);
}

struct Grid {
    double lo[3];
    double h;
    int g[3];
};

__device__ inline int64_t cell_of(const Grid &G, const double *p, int dim, int c[3]) {
    int64_t id = 0;
    for (int d = dim - 1; d >= 0; --d) {
        int v = (int)floor((p[d] - G.lo[d]) / G.h);
        v = min(max(v, 0), G.g[d] - 1);
        c[d] = v;
        id = id * G.g[d] + v;
    }
    return id;
}

__global__ void k_cell_keys(const double *__restrict__ cen, int64_t k, int dim, Grid G,
                            int32_t *__restrict__ key) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= k) return;
    int c[3];
    key[i] = (int32_t)cell_of(G, cen + i * dim, dim, c);
}

// cell_start[cell .. ] from centroids sorted by cell: start = first position
__global__ void k_cell_ranges(const int32_t *__restrict__ skey, int64_t k, int64_t ncell,
                              int32_t *__restrict__ start) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i > k) return;
    // positions where the key changes open every cell in (prev, cur]
    const int64_t prev = i == 0 ? -1 : skey[i - 1];
    const int64_t cur = i == k ? ncell : skey[i];
    for (int64_t c = prev + 1; c <= cur; ++c) start[c] = (int32_t)i;
}

// exact nearest centroid: rings of cells until the unscanned region is
// farther than the best candidate
__global__ void k_assign(const double *__restrict__ y, int64_t n, int dim, Grid G,
                         const double *__restrict__ cen, const int32_t *__restrict__ sidx,
                         const int32_t *__restrict__ start, int32_t *__restrict__ assign) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double *p = y + i * dim;
    int c[3] = {0, 0, 0};
    (void)cell_of(G, p, dim, c);
    double best = INFINITY;
    int32_t bi = INT32_MAX;
    const int gmax = max(G.g[0], max(G.g[1], dim == 3 ? G.g[2] : 0));
    for (int r = 0; r <= gmax; ++r) {
        const int z0 = dim == 3 ? -r : 0, z1 = dim == 3 ? r : 0;
        for (int dz = z0; dz <= z1; ++dz)
            for (int dy = -r; dy <= r; ++dy)
                for (int dx = -r; dx <= r; ++dx) {
                    const int ring = max(abs(dx), max(abs(dy), abs(dz)));
                    if (ring != r) continue;
                    const int cx = c[0] + dx, cy = c[1] + dy, cz = c[2] + dz;
                    if (cx < 0 || cy < 0 || cx >= G.g[0] || cy >= G.g[1]) continue;
                    if (dim == 3 && (cz < 0 || cz >= G.g[2])) continue;
                    const int64_t cell =
                        dim == 3 ? ((int64_t)cz * G.g[1] + cy) * G.g[0] + cx
                                 : (int64_t)cy * G.g[0] + cx;
                    for (int32_t s = start[cell]; s < start[cell + 1]; ++s) {
                        const int32_t j = sidx[s];
                        double d2 = 0.0;
                        for (int d = 0; d < dim; ++d) {
                            const double e = p[d] - cen[(int64_t)j * dim + d];
                            d2 += e * e;
                        }
                        if (d2 < best || (d2 == best && j < bi)) {
                            best = d2;
                            bi = j;
                        }
                    }
                }
        const double reach = r * G.h;
        if (bi != INT32_MAX && best <= reach * reach) break;
    }
    assign[i] = bi;
}

// per cluster: first member position in the cluster-sorted order
__global__ void k_cluster_ranges(const int32_t *__restrict__ skey, int64_t n, int64_t k,
                                 int32_t *__restrict__ start) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i > n) return;
    const int64_t prev = i == 0 ? -1 : skey[i - 1];
    const int64_t cur = i == n ? k : skey[i];
    for (int64_t c = prev + 1; c <= cur; ++c) start[c] = (int32_t)i;
}

// centroid = mean of members (empty cluster keeps its centroid), mass = sum
__global__ void k_update(const double *__restrict__ y, const double *__restrict__ w,
                         const int32_t *__restrict__ sidx, const int32_t *__restrict__ start,
                         int64_t k, int dim, double *__restrict__ cen, double *__restrict__ mass,
                         int32_t *__restrict__ count) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= k) return;
    double s[3] = {0, 0, 0}, m = 0.0;
    const int32_t a = start[c], b = start[c + 1];
    for (int32_t t = a; t < b; ++t) {
        const int64_t i = sidx[t];
        for (int d = 0; d < dim; ++d) s[d] += y[i * dim + d];
        m += w[i];
    }
    if (b > a)
        for (int d = 0; d < dim; ++d) cen[c * dim + d] = s[d] / (double)(b - a);
    mass[c] = m;
    count[c] = b - a;
}

__global__ void k_compact(const double *__restrict__ cen, const double *__restrict__ mass,
                          const int32_t *__restrict__ count, const int32_t *__restrict__ pos,
                          int64_t k, int dim, double *__restrict__ yo, double *__restrict__ mo) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= k || count[c] == 0) return;
    const int32_t o = pos[c];
    for (int d = 0; d < dim; ++d) yo[(int64_t)o * dim + d] = cen[c * dim + d];
    mo[o] = mass[c];
}

__global__ void k_parent(const int32_t *__restrict__ assign, const int32_t *__restrict__ pos,
                         int64_t n, int32_t *__restrict__ parent) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) parent[i] = pos[assign[i]];
}

__global__ void k_nonempty_prefix(const int32_t *__restrict__ count, int64_t k,
                                  int32_t *__restrict__ pos, int64_t *__restrict__ total) {
    // single thread: k is at most a few 1e5 and this runs once per level
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    int32_t o = 0;
    for (int64_t c = 0; c < k; ++c) {
        pos[c] = o;
        o += count[c] > 0;
    }
    *total = o;
}

unsigned nb(int64_t n) { return (unsigned)((n + 255) / 256); }

template <typename K>
rsot_status sort_pairs(Ctx &ctx, const K *kin, K *kout, const int32_t *vin, int32_t *vout,
                       int64_t n, int bits) {
    size_t bytes = 0;
    RSOT_HIP(hipcub::DeviceRadixSort::SortPairs(nullptr, bytes, kin, kout, vin, vout, (int)n, 0,
                                                bits, ctx.stream));
    void *tmp = ctx.alloc<char>(bytes);
    if (!tmp) return RSOT_ERR_OOM;
    RSOT_HIP(hipcub::DeviceRadixSort::SortPairs(tmp, bytes, kin, kout, vin, vout, (int)n, 0, bits,
                                                ctx.stream));
    return RSOT_OK;
}

int bits_for(int64_t v) {
    int b = 1;
    while ((int64_t(1) << b) <= v && b < 31) ++b;
    return b;
}

// one coarsening step: n points (y, w) -> k clusters written to (yo, wo)
rsot_status kmeans_level(Ctx &ctx, int dim, int64_t n, const double *y, const double *w,
                         int64_t k, uint64_t seed, int iters, double *yo, double *wo,
                         int32_t *parent, int64_t *k_out) {
    (void)seed;
    // bounding box on the host (one copy; setup-time)
    std::vector<double> hy((size_t)n * dim);
    RSOT_HIP(hipMemcpyAsync(hy.data(), y, sizeof(double) * n * dim, hipMemcpyDeviceToHost,
                            ctx.stream));
    RSOT_HIP(hipStreamSynchronize(ctx.stream));
    double lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
    for (int d = 0; d < dim; ++d) {
        lo[d] = INFINITY;
        hi[d] = -INFINITY;
    }
    for (int64_t i = 0; i < n; ++i)
        for (int d = 0; d < dim; ++d) {
            lo[d] = std::min(lo[d], hy[i * dim + d]);
            hi[d] = std::max(hi[d], hy[i * dim + d]);
        }
    double ext = 0.0;
    for (int d = 0; d < dim; ++d) ext = std::max(ext, hi[d] - lo[d]);
    if (!(ext > 0.0)) ext = 1.0;

    uint32_t *keys = ctx.alloc<uint32_t>(n), *keys2 = ctx.alloc<uint32_t>(n);
    int32_t *idx = ctx.alloc<int32_t>(n), *order = ctx.alloc<int32_t>(n);
    double *cen = ctx.alloc<double>(k * dim), *mass = ctx.alloc<double>(k);
    int32_t *count = ctx.alloc<int32_t>(k), *assign = ctx.alloc<int32_t>(n);
    int32_t *assign2 = ctx.alloc<int32_t>(n), *pidx = ctx.alloc<int32_t>(n);
    int32_t *sorted_pts = ctx.alloc<int32_t>(n), *cstart = ctx.alloc<int32_t>(k + 1);
    int32_t *ckey = ctx.alloc<int32_t>(k), *ckey2 = ctx.alloc<int32_t>(k);
    int32_t *cidx = ctx.alloc<int32_t>(k), *cidx2 = ctx.alloc<int32_t>(k);
    int32_t *pos = ctx.alloc<int32_t>(k);
    int64_t *tot = ctx.alloc<int64_t>(1);
    if (!keys || !keys2 || !idx || !order || !cen || !mass || !count || !assign || !assign2 ||
        !pidx || !sorted_pts || !cstart || !ckey || !ckey2 || !cidx || !cidx2 || !pos || !tot)
        return RSOT_ERR_OOM;
    hipLaunchKernelGGL(k_keys, dim3(nb(n)), dim3(256), 0, ctx.stream, y, n, dim, lo[0], lo[1],
                       lo[2], 1.0 / ext, keys);
    hipLaunchKernelGGL(k_iota, dim3(nb(n)), dim3(256), 0, ctx.stream, idx, n);
    RSOT_TRY(sort_pairs(ctx, keys, keys2, idx, order, n, 32));
    hipLaunchKernelGGL(k_init_centroids, dim3(nb(k)), dim3(256), 0, ctx.stream, y, order, n, k,
                       dim, cen);

    // grid: about two centroids per cell
    Grid G;
    double vol = 1.0;
    for (int d = 0; d < dim; ++d) vol *= std::max(hi[d] - lo[d], 1e-12 * ext);
    G.h = std::pow(2.0 * vol / (double)k, 1.0 / dim);
    // at most 4096^2 / 256^3 cells: widen the cells of flat point sets
    const double gmax_axis = dim == 2 ? 4096.0 : 256.0;
    for (int d = 0; d < dim; ++d) G.h = std::max(G.h, (hi[d] - lo[d]) / gmax_axis);
    if (!(G.h > 0.0)) G.h = 1.0;
    int64_t ncell = 1;
    for (int d = 0; d < 3; ++d) {
        G.lo[d] = d < dim ? lo[d] : 0.0;
        G.g[d] = d < dim ? std::max(1, (int)std::ceil((hi[d] - lo[d]) / G.h)) : 1;
        G.g[d] = std::min(G.g[d], (int)gmax_axis);
        ncell *= G.g[d];
    }
    int32_t *start = ctx.alloc<int32_t>(ncell + 1);
    if (!start) return RSOT_ERR_OOM;
    hipLaunchKernelGGL(k_iota, dim3(nb(n)), dim3(256), 0, ctx.stream, pidx, n);
    for (int it = 0; it <= iters; ++it) {
        hipLaunchKernelGGL(k_cell_keys, dim3(nb(k)), dim3(256), 0, ctx.stream, cen, k, dim, G,
                           ckey);
        hipLaunchKernelGGL(k_iota, dim3(nb(k)), dim3(256), 0, ctx.stream, cidx, k);
        RSOT_TRY(sort_pairs(ctx, ckey, ckey2, cidx, cidx2, k, bits_for(ncell)));
        hipLaunchKernelGGL(k_cell_ranges, dim3(nb(k + 1)), dim3(256), 0, ctx.stream, ckey2, k,
                           ncell, start);
        hipLaunchKernelGGL(k_assign, dim3(nb(n)), dim3(256), 0, ctx.stream, y, n, dim, G, cen,
                           cidx2, start, assign);
        RSOT_TRY(sort_pairs(ctx, assign, assign2, pidx, sorted_pts, n, bits_for(k)));
        hipLaunchKernelGGL(k_cluster_ranges, dim3(nb(n + 1)), dim3(256), 0, ctx.stream, assign2,
                           n, k, cstart);
        hipLaunchKernelGGL(k_update, dim3(nb(k)), dim3(256), 0, ctx.stream, y, w, sorted_pts,
                           cstart, k, dim, cen, mass, count);
        RSOT_HIP(hipGetLastError());
    }
    hipLaunchKernelGGL(k_nonempty_prefix, dim3(1), dim3(64), 0, ctx.stream, count, k, pos, tot);
    hipLaunchKernelGGL(k_compact, dim3(nb(k)), dim3(256), 0, ctx.stream, cen, mass, count, pos, k,
                       dim, yo, wo);
    if (parent)
        hipLaunchKernelGGL(k_parent, dim3(nb(n)), dim3(256), 0, ctx.stream, assign, pos, n, parent);
    RSOT_HIP(hipGetLastError());
    RSOT_HIP(hipMemcpyAsync(k_out, tot, sizeof(int64_t), hipMemcpyDeviceToHost, ctx.stream));
    RSOT_HIP(hipStreamSynchronize(ctx.stream));
    return RSOT_OK;
}

}  // namespace

extern "C" rsot_status rsot_target_hierarchy(int dim, int64_t n, const double *y, const double *nu,
                                             int n_levels, const int64_t *n_per_level,
                                             int lloyd_iters, uint64_t seed, void *hip_stream,
                                             double *const *y_levels, double *const *nu_levels,
                                             int32_t *const *parent_levels, int64_t *n_out) {
    if ((dim != 2 && dim != 3) || n <= 0 || !y || !nu || n_levels < 1 || !n_per_level ||
        !y_levels || !nu_levels || !n_out || lloyd_iters < 0)
        return RSOT_ERR_INVALID_ARG;
    if (n_per_level[n_levels - 1] != n) return RSOT_ERR_INVALID_ARG;
    for (int l = 0; l + 1 < n_levels; ++l)
        if (n_per_level[l] <= 0 || n_per_level[l] > n_per_level[l + 1]) return RSOT_ERR_INVALID_ARG;
    for (int l = 0; l < n_levels; ++l)
        if (!y_levels[l] || !nu_levels[l]) return RSOT_ERR_INVALID_ARG;
    Ctx ctx;
    ctx.stream = (hipStream_t)hip_stream;
    // finest level is the input
    RSOT_HIP(hipMemcpyAsync(y_levels[n_levels - 1], y, sizeof(double) * n * dim,
                            hipMemcpyDeviceToDevice, ctx.stream));
    RSOT_HIP(hipMemcpyAsync(nu_levels[n_levels - 1], nu, sizeof(double) * n,
                            hipMemcpyDeviceToDevice, ctx.stream));
    n_out[n_levels - 1] = n;
    for (int l = n_levels - 2; l >= 0; --l) {
        const int64_t nf = n_out[l + 1];
        const int64_t k = std::min<int64_t>(n_per_level[l], nf);
        RSOT_TRY(kmeans_level(ctx, dim, nf, y_levels[l + 1], nu_levels[l + 1], k, seed + l,
                              lloyd_iters, y_levels[l], nu_levels[l],
                              parent_levels ? parent_levels[l + 1] : nullptr, &n_out[l]));
    }
    return RSOT_OK;
}
