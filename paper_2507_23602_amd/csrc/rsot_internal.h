// Internal declarations of librsot (not part of the ABI).
//
// Data layout in device memory (all library-owned):
//   points  : spatially sorted (Morton order of a grid over their bounding
//             box), padded to a multiple of 64 so that one 64-point tile is one
//             wavefront. qp[q] = {x0, x1, x2, S_q} (x2 = 0 in 2D; S_q is the
//             per-point constant of the gradient pass, rewritten by every
//             objective pass). Padding points copy the last real point and
//             carry mu = 0.
//   targets : sorted the same way, padded to a multiple of 64 (one 64-target
//             block per wavefront in the gradient pass); padding targets
//             carry nu = 0 (log2 nu = -inf), so they add nothing.
//   Coordinates are shifted by the centre of the target bounding box (the
//   cost only depends on x - y).
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>
#include <cmath>
#include <cstdint>
#include <vector>

#include "../../include/rsot.h"

#define RSOT_WAVE 64
#define RSOT_TILE 64
#define RSOT_BLOCK 64

// flag values of a (tile, block) pair after culling
enum : uint8_t { PAIR_SKIP = 0, PAIR_PARTIAL = 1, PAIR_FULL = 2 };
// list entries: index, with the top bit set when the pair needs the per-pair
// cutoff test
#define RSOT_PARTIAL_BIT 0x80000000u
// targets per culling group of the tile rule when opt.tile_group is 0
#define RSOT_TILE_GROUP_DEFAULT 64

struct rsot_problem {
    int dim = 0;
    int64_t nq = 0, n = 0;
    int64_t nq_pad = 0, n_pad = 0;
    int64_t n_tiles = 0, n_blocks = 0;
    rsot_options opt{};
    hipStream_t stream = nullptr;
    double shift[3] = {0, 0, 0};
    double sum_mu = 0, sum_nu = 0, nu_min = 0, nu_max = 0;
    double sum_mu2 = 0;          // sum of mu_q^2: (sum mu)^2 / sum_mu2 = effective point count
    double exp_corr = 1.0;       // 1 / (1 + mean relative error of v_exp_f32), this device

    // allocations (for cleanup and the memory cap)
    std::vector<void *> allocs;
    std::vector<size_t> alloc_bytes;
    size_t bytes = 0;

    // points
    double4 *qp = nullptr;       // [nq_pad] {x0,x1,x2,S}
    double *qmu = nullptr;       // [nq_pad]
    double *qlog2mu = nullptr;   // [nq_pad]
    double *qA = nullptr;        // [nq_pad] A_q = -kappa cs |x_q|^2 (per-pair cutoff test)
    double *qlse = nullptr;      // [nq_pad] L_q (natural log)
    int32_t *qkept = nullptr;    // [nq_pad] |I_q|: targets summed at the point (last evaluation)
    int32_t *qperm = nullptr;    // [nq_pad] sorted slot -> caller index (-1 pad)
    double *tile_lo = nullptr;   // [n_tiles*3]
    double *tile_hi = nullptr;   // [n_tiles*3]
    int32_t *tile_cnt = nullptr; // [n_tiles] real points per tile

    // targets
    double *ty = nullptr;        // [n_pad*3] shifted coordinates (AoS, 3 per target)
    double *tnu = nullptr;       // [n_pad]
    double *tlog2nu = nullptr;   // [n_pad]
    int32_t *tperm = nullptr;    // [n_pad]
    double4 *trec = nullptr;     // [n_pad] per evaluation {Y0,Y1,Y2,B}
    double *trec3 = nullptr;     // [3 n_pad] d = 2: the same records packed {Y0,Y1,B}
    double *tG = nullptr;        // [n_pad] per evaluation cutoff constant
    double *tpsi = nullptr;      // [n_pad] sorted psi (per evaluation)
    double *blk_lo = nullptr;    // [n_blocks*3]
    double *blk_hi = nullptr;
    double *blk_nu = nullptr;    // [n_blocks] block mass
    double *blk_lnnu = nullptr;  // [n_blocks] ln of the block mass
    int32_t *blk_cnt = nullptr;  // [n_blocks] real targets per block
    double *blk_stat = nullptr;  // [n_blocks*4] per evaluation: psimax, psimin, psi.nu, nonfinite

    // per-evaluation partials and scalars
    double *tile_part = nullptr; // [n_tiles*4] sum mu L2, logD part, kept, empty
    double2 *tile_ref = nullptr; // [n_tiles] gradient-pass reference {R_T, 2^R_T * corr}
    double *tile_smax = nullptr; // [n_tiles] sphere cost: max over the tile of S'_q, the
                                 // gradient-side bound of whole-tile skips
    double *blk_gpart = nullptr; // [n_blocks*2] |g|_1, |g|_inf per block
    double *dscal = nullptr;     // [32] device scalars
    double *hscal = nullptr;     // [32] pinned host copy
    double *hpsi = nullptr;      // pinned host staging (n)
    double *hgrad = nullptr;     // pinned host staging (n)
    double *dpsi = nullptr;      // device staging for solve (n)
    double *dgrad = nullptr;     // device staging for solve (n)

    // gradient pass work items and partials
    double *gpart = nullptr;     // [n_wi*64]
    size_t gpart_cap = 0;
    int32_t *wi_block = nullptr; // list mode: block of each work item
    int64_t *wi_range = nullptr; // list mode: [start,end) into the column list
    int64_t *wi_ptr = nullptr;   // [n_blocks+1] first work item of each block
    size_t wi_cap = 0;

    // objective pass work items (tile, segment of its block list) and partials
    int32_t *wi1_tile = nullptr;
    int64_t *wi1_range = nullptr;
    int64_t *wi1_ptr = nullptr;  // [n_tiles+1]
    size_t wi1_cap = 0;
    // processing order of the work items of the truncated rules: item numbers
    // sorted by their first entry (first target block of an objective-pass
    // item, first point tile of a gradient-pass item), so items that read the
    // same records run close together; partials stay at the item's own index
    int32_t *wi1_perm = nullptr, *wi_perm = nullptr;
    int32_t *sort_key = nullptr, *sort_key2 = nullptr, *sort_val = nullptr;
    size_t perm1_cap = 0, perm_cap = 0, sort_cap = 0;
    void *sort_tmp = nullptr;
    size_t sort_tmp_cap = 0;
    double *part1 = nullptr;     // [items*64] partial log2-sum-exp
    double *part1k = nullptr;    // [items*64] kept pairs
    size_t part1_cap = 0;
    uint64_t *redo1 = nullptr;   // [items] cutoff rules: lanes to sum again exactly
    size_t redo1_cap = 0;

    // culling (truncated rules): CSR lists of kept (tile, block) pairs by tile
    // (rows) and by block (columns), built directly from box tests
    int64_t *row_ptr = nullptr;  // [n_tiles+1]
    int64_t *col_ptr = nullptr;  // [n_blocks+1]
    int32_t *row_cnt = nullptr;  // [n_tiles]
    int32_t *col_cnt = nullptr;  // [n_blocks]
    int64_t *scan_tmp = nullptr; // [ceil(max(n_tiles, n_blocks) / 1024)] piece sums of the scans
    int32_t *row_scnt = nullptr; // kept entries per (tile, segment of its blocks)
    int32_t *col_scnt = nullptr; // kept entries per (block, segment of its tiles)
    // culling classes of the count pass, read back by the fill pass: one bit
    // per (tile, block) pair, row-major by tile (row_*) and by block (col_*);
    // kbits = kept, pbits = needs the per-pair test
    uint64_t *row_kbits = nullptr, *row_pbits = nullptr;
    uint64_t *col_kbits = nullptr, *col_pbits = nullptr;
    uint32_t *row_idx = nullptr; // kept entries per tile
    uint32_t *col_idx = nullptr; // kept entries per block
    uint16_t *row_cm = nullptr;  // chunk classes of row entries that keep part of a block
    int32_t *tile_bstar = nullptr; // tile rule: B* (or G*, with groups) of each tile
    // tile rule with culling groups below 64 targets: per group of the last
    // evaluation the box of its real targets, ln nu(G) and max psi; and the
    // chunk bits of the column entries that keep only some of their chunks
    double *grp_lo = nullptr, *grp_hi = nullptr, *grp_lnnu = nullptr, *grp_psi = nullptr;
    uint8_t *col_cm = nullptr;
    size_t col_cm_cap = 0;
    // group masks (chunk bits) of every (tile, block) pair, row-major by tile,
    // and their transpose, written by the row count pass and read by the
    // other culling passes; only when both fit (gmask_ok)
    uint8_t *gmask = nullptr, *gmaskT = nullptr;
    int gmask_ok = 0, gmask_tried = 0;
    int last_group = 64;         // culling group of the last evaluation (64: blocks)
    double *tile_thr = nullptr;  // tile rule: skip threshold of each tile
    double *tch_lo = nullptr, *tch_hi = nullptr;   // [n_pad/8*3] boxes of 8-target chunks
    size_t list_cap = 0;
    int64_t *i64tmp = nullptr;   // small scratch for counts

    // state
    double C0 = -1.0;            // covering cost (lazy)
    double absJ_ref = 0.0;       // |J| for the cutoff rules (0 = unknown)
    double log_D_prev = 0.0;     // ln D of the previous evaluation (INT rule)
    int have_D = 0;
    int last_eval_valid = 0;
    int last_mode = 0;           // pair-loop mode of the last evaluation (dense, list, mask)
    // work decomposition of the last evaluation's gradient pass (the plan
    // moments follow it): items, point segments per block and their length
    int64_t last_n_wi = 0, last_n_seg = 1, last_seg = 1;
    double last_kcs = 0.0;       // kappa * cost_scale of the last evaluation
    double *mpart = nullptr;     // plan moments: per-item partial first moments
    size_t mpart_cap = 0;
    float *tyf = nullptr;        // transport maps: FP32 target coordinates less their block's box centre {y0, y1, y2, 0}
    int64_t last_refine_pairs = 0;   // (tile, fine block) pairs x 64 x 64 of the last refinement
    hipEvent_t ev0 = nullptr, ev1 = nullptr, ev_p1 = nullptr, ev_mid = nullptr, ev_p2 = nullptr;
    hipEvent_t ev_b0 = nullptr, ev_b1 = nullptr;   // batched call
    char *batch_buf = nullptr;                      // batched call: descriptors, order, item offsets
    size_t batch_cap = 0;
};

// ---- helpers --------------------------------------------------------------
rsot_status rsot_dev_alloc(rsot_problem *p, void **ptr, size_t bytes);
void rsot_dev_free(rsot_problem *p, void *ptr);

#define RSOT_HIP(call)                                                    \
    do {                                                                  \
        hipError_t e_ = (call);                                           \
        if (e_ != hipSuccess) return RSOT_ERR_DEVICE;                     \
    } while (0)

#define RSOT_TRY(call)                                                    \
    do {                                                                  \
        rsot_status s_ = (call);                                          \
        if (s_ != RSOT_OK) return s_;                                     \
    } while (0)

// Morton order of n device points (problem's dim); caller frees *order_out
rsot_status rsot_morton_order(rsot_problem *p, const double *x, int64_t n, int32_t **order_out);

// kernels launched from the evaluation driver
rsot_status rsot_compute_covering_cost(rsot_problem *p);
rsot_status rsot_eval_impl(rsot_problem *p, double eps, const double *psi_dev, double *J_out,
                           double *grad_dev, rsot_eval_info *info);

// true when the pair loops run in FP64: FP64 precision, or MIXED precision on a
// problem whose effective number of points is below opt.fp64_below_points
bool rsot_pairs_fp64(const rsot_problem *p);

// the squared geodesic cost on the sphere (rsot_sphere.hip): target records,
// objective-pass and gradient-pass pair kernels on the evaluation's items
void rsot_sphere_records(rsot_problem *p, hipStream_t st, double kappa);
void rsot_sphere_pass1(rsot_problem *p, bool f64, int mode, double kcs, int64_t n_items,
                       int64_t seg1, int64_t n_seg1);
void rsot_sphere_pass2(rsot_problem *p, bool f64, int mode, double kcs, int64_t n_wi,
                       int64_t n_seg, int64_t seg);

// 1 / (1 + mean relative error of the FP32 exponential instruction) on the
// current device, measured once per device (rsot_eval.hip)
rsot_status rsot_device_exp_corr(hipStream_t st, double *corr);

// dense evaluation with the work-item partials in caller-provided device
// memory; allocates nothing (rsot_eval.hip)
rsot_status rsot_eval_dense_in(rsot_problem *p, double eps, const double *psi, double *J_out,
                               double *grad_out, rsot_eval_info *info, double *scratch,
                               size_t scratch_bytes);

rsot_status rsot_refine_impl(rsot_problem *p, double eps, const double *psi_coarse, int64_t nf,
                             const double *yf, double eta, double *psi_out);

// device scalar slots
enum {
    SC_J = 0,        // J
    SC_SUM_L2,       // sum_q mu_q L2_q
    SC_LOGD,         // ln D
    SC_KEPT,         // kept pairs
    SC_EMPTY,        // empty points
    SC_PSIMAX,
    SC_PSIMIN,
    SC_PSINU,        // sum psi nu
    SC_NONFINITE,    // count of non-finite psi
    SC_GL1,
    SC_GLINF,
    SC_C,            // cutoff used
    SC_C0,
    SC_ROWTOT,       // total row entries (culling)
    SC_COLTOT,
    SC_NWI,          // work items of the gradient pass
    SC_NWI1,         // work items of the objective pass
    SC_COUNT
};
