/*
 * rsot.h -- C ABI of the MI355X semi-discrete RSOT dual library (librsot.so).
 *
 * The library evaluates, for a source measure given as quadrature points
 * {x_q, mu_q} (mu_q = rho_h(x_q) w_q, Sec. 3.2 Remark 3.1) and a discrete
 * target measure {y_j, nu_j} (Sec. 2), the discretised dual objective
 *
 *   J(psi) = sum_q eps ln( sum_j nu_j exp((psi_j - c(x_q,y_j))/eps) ) mu_q
 *            - sum_j psi_j nu_j                       (Eq. discretized_functional)
 *
 * and its gradient
 *
 *   dJ/dpsi_k = sum_q p_k(x_q|psi) mu_q - nu_k        (Eq. discretized_gradient)
 *
 * with p_k the plan density of Eq. final_plan_density and the cost
 * c(x, y) = cost_scale |x - y|^2 (Sec. 2 uses cost_scale = 1/2). J is the
 * convex functional the paper minimises; the gradient has the paper's sign
 * (target marginal of the plan minus nu).
 *
 * Conventions for every call:
 *   - Every call returns an rsot_status; nothing throws or aborts across the
 *     ABI. Outputs are left untouched unless RSOT_OK is returned, except
 *     rsot_solve*, which always write the best accepted potential and info.
 *   - Arrays are row-major: points are n x dim doubles.
 *   - "device pointer" means memory of the current HIP device (e.g. a torch
 *     CUDA tensor's data_ptr()); "host pointer" means ordinary host memory.
 *   - Work is issued on the HIP stream given at creation, in stream order.
 *   - Handles are not thread safe: one handle, one host thread at a time.
 */
#ifndef RSOT_H
#define RSOT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    RSOT_OK = 0,
    RSOT_ERR_INVALID_ARG = 1,   /* bad size, dim, eps, option or NULL pointer     */
    RSOT_ERR_NONFINITE = 2,     /* NaN/Inf in x, mu, y, nu or psi                  */
    RSOT_ERR_UNBALANCED = 3,    /* |sum mu - sum nu| > 1e-12 sum nu (solve only)   */
    RSOT_ERR_DEVICE = 4,        /* a HIP call failed                               */
    RSOT_ERR_OOM = 5,           /* device allocation failed or exceeds mem_limit   */
    RSOT_ERR_LINESEARCH = 6,    /* line search found no acceptable step            */
    RSOT_ERR_NOT_CONVERGED = 7, /* iteration cap reached before ||grad||_1 <= tol  */
    RSOT_ERR_CANCELLED = 8      /* cancel flag or callback asked to stop           */
} rsot_status;

/* Arithmetic of the pair loop.
 * MIXED: exponent arguments formed in FP64, exponentials and per-chunk sums
 *        in FP32, per-point log-sum-exp, per-target sums and J in FP64. The
 *        FP32 exponential's per-term error (about 1e-7 relative) averages out
 *        over many points; a problem whose effective number of points
 *        (sum mu)^2 / sum mu^2 is below opt.fp64_below_points and whose pair
 *        count is below 2^27 runs the FP64 pair loop instead, so J stays
 *        within 1e-9 of the exact value. (A larger problem with concentrated
 *        masses keeps the FP32 loop; its J error is about
 *        1.5e-7 eps sum(mu) / sqrt(effective points).)
 * FP64 : everything in FP64 (software exp2). */
typedef enum { RSOT_PREC_MIXED = 0, RSOT_PREC_FP64 = 1 } rsot_precision;

/* Which (point, target) pairs enter the sums.
 * DENSE: all (Eqs. discretized_functional/gradient).
 * GEOM : c < C_geom, Eq. truncation_cutoff_geom (paper default).
 * INT  : c < C_int, Eq. truncation_cutoff_int, D lagged one evaluation.
 * PW   : c < C_pw, Eq. cost_cutoff_delta.
 * TILE : tile-local bound derived from App. B: pairs of (point tile, target
 *        block) whose bound is below tau |J_ref| eps-scaled are skipped whole;
 *        J_dense - J_trunc <= tau |J_ref|. */
typedef enum {
    RSOT_TRUNC_DENSE = 0,
    RSOT_TRUNC_GEOM = 1,
    RSOT_TRUNC_INT = 2,
    RSOT_TRUNC_PW = 3,
    RSOT_TRUNC_TILE = 4
} rsot_truncation;

/* The cost c(x, y).
 * SQEUCLID: cost_scale |x - y|^2 (Sec. 2; cost_scale 1/2 is the paper's).
 * SPHERE  : cost_scale d_g(x, y)^2 with d_g = acos(x.y) the great-circle
 *           distance on the unit sphere (Sec. 6.4 uses c = d_g^2: cost_scale
 *           1). The pair loops evaluate d_g^2 as a polynomial in the squared
 *           chord 2 - 2 x.y (absolute error below 3e-13 where the exponential
 *           is FP32, a few FP64 rounding units on the FP64 loop), through the
 *           antipode on the far hemisphere. Requires dim 3 and points and targets
 *           of unit norm (| |v|^2 - 1 | <= 1e-9, else INVALID_ARG), and the
 *           DENSE or TILE rule; the tile rule's box bounds pass through the
 *           chord (the geodesic increases with it), over whole blocks or
 *           culling groups as for SQEUCLID. Batched calls run such members one by
 *           one; the moments, maps, refinement, multilevel and allocation-free
 *           calls return INVALID_ARG for them (rsot_sphere_karcher_step is
 *           the sphere's own moment call). */
typedef enum { RSOT_COST_SQEUCLID = 0, RSOT_COST_SPHERE = 1 } rsot_cost;

typedef struct {
    double cost_scale;        /* c(x,y) = cost_scale |x-y|^2; default 0.5         */
    int precision;            /* rsot_precision; default MIXED                     */
    int truncation;           /* rsot_truncation; default DENSE                    */
    double tau;               /* relative error tolerance (GEOM, INT, TILE); 1e-12 */
    double delta_thr;         /* pointwise threshold (PW); default 1e-12           */
    int inputs_on_device;     /* 1: x, mu, y, nu passed to create are device ptrs  */
    int seg_tiles;            /* gradient pass: point tiles per work item; 0 = default
                                 (dense: 512-tile segments, at least 32,768 items;
                                 truncated rules: 64 list entries)                    */
    int seg_blocks;           /* objective pass: target blocks per work item; 0 = default
                                 (dense: whole rows unless the tiles are too few to fill
                                 the device; truncated rules: 256)                     */
    int64_t mem_limit_bytes;  /* cap on library device memory; 0 = none            */
    int64_t fp64_below_points;/* MIXED: FP64 pair loop when (sum mu)^2 / sum mu^2 is
                                 below this (and N_q N < 2^27); default 16384;
                                 0 = never                                          */
    int64_t tile_group;       /* TILE: targets per culling group, 8, 16, 32 or 64
                                 (the rule decides per (point tile, group) pair;
                                 the passes still run 64-target blocks, skipping
                                 the dropped groups' 8-target chunks); 0 = default
                                 (64). Finer groups have tighter bounds but each
                                 gets a smaller share of the budget tau |J|, so
                                 which keeps fewer pairs depends on the problem:
                                 rsot_autotune picks it                             */
    int cost_kind;            /* rsot_cost; default SQEUCLID                        */
} rsot_options;

typedef struct rsot_problem rsot_problem;

typedef struct {
    int64_t total_pairs;      /* N_q * N                                           */
    int64_t kept_pairs;       /* pairs summed in the objective pass                */
    int64_t n_empty_qp;       /* points whose kept set was empty (dropped, Alg. 2) */
    double cutoff;            /* C used by GEOM/INT/PW, else 0                     */
    double absJ_ref;          /* |J| the cutoff rule used                           */
    double log_D;             /* ln sum_q mu_q exp(-L_q)  (D of Sec. 4.1)           */
    double grad_l1;           /* ||grad||_1  (Remark 3.2)                           */
    double grad_linf;         /* ||grad||_inf                                       */
    double kernel_ms;         /* device time of the evaluation (HIP events)        */
    double setup_ms;          /* of which: target records, cutoff and culling      */
    double passes_ms;         /* of which: objective + gradient passes             */
    double pass1_ms;          /* objective pass (per-point log-sum-exp)            */
    double pass2_ms;          /* gradient pass (per-target masses)                 */
    int dense_fallback;       /* 1 if a truncated rule ran dense (no |J| yet)       */
    int fp64_pairs;           /* 1 if the pair loops ran in FP64                   */
} rsot_eval_info;

/* Fills *opt with the defaults listed above. */
void rsot_options_default(rsot_options *opt);

/* Human-readable name of a status code (static string, never NULL). */
const char *rsot_status_string(rsot_status s);

/*
 * Creates a problem: copies the source quadrature measure and the targets
 * into library-owned device buffers (spatially sorted, padded), so the
 * caller keeps ownership of its arrays and may free them afterwards.
 *   dim          2 or 3
 *   n_quad, x,mu quadrature points (n_quad x dim) and masses (n_quad), mu >= 0,
 *                sum mu > 0 (Sec. 3.2, Remark 3.1)
 *   n_target,y,nu targets (n_target x dim) and masses nu > 0 (Sec. 2)
 *   opt          options (NULL = defaults); opt->inputs_on_device selects
 *                host or device pointers for x, mu, y, nu
 *   hip_stream   hipStream_t to issue work on (NULL = default stream)
 *   out          receives the handle
 * Errors: INVALID_ARG (dim, sizes, NULL, options), NONFINITE, OOM, DEVICE.
 */
rsot_status rsot_problem_create(int dim, int64_t n_quad, const double *x, const double *mu,
                                int64_t n_target, const double *y, const double *nu,
                                const rsot_options *opt, void *hip_stream,
                                rsot_problem **out);

/* Frees all library-owned memory of the problem. Safe on NULL. */
void rsot_problem_destroy(rsot_problem *p);

/* Sizes of a problem (any pointer may be NULL). */
rsot_status rsot_problem_sizes(const rsot_problem *p, int *dim, int64_t *n_quad,
                               int64_t *n_target);

/* Changes the truncation rule / tolerances of an existing problem. */
rsot_status rsot_set_truncation(rsot_problem *p, int truncation, double tau, double delta_thr);

/* Changes the arithmetic (rsot_precision) of an existing problem. */
rsot_status rsot_set_precision(rsot_problem *p, int precision);

/*
 * Sets |J_ref|, the magnitude of J used by the GEOM, INT and TILE rules
 * (Eqs. truncation_cutoff_geom/int: |J(psi)| of the current iterate, read here
 * as the last accepted one). 0 clears it: the next truncated evaluation then
 * runs dense and stores its own |J|.
 */
rsot_status rsot_set_reference(rsot_problem *p, double absJ_ref);

/*
 * Evaluates J(psi) and grad J(psi) (Eqs. discretized_functional/gradient;
 * Alg. 2 with the problem's truncation rule).
 *   eps       regularisation > 0 (Sec. 2)
 *   psi       DEVICE pointer, n_target doubles, caller's target order
 *   J_out     HOST pointer, receives J
 *   grad_out  DEVICE pointer, n_target doubles in caller's order, or NULL for
 *             the objective only
 *   info      HOST pointer or NULL
 * The call synchronises the problem's stream before returning (J is a host
 * value). Errors: INVALID_ARG, NONFINITE (psi), DEVICE, OOM.
 */
rsot_status rsot_dual_eval(rsot_problem *p, double eps, const double *psi, double *J_out,
                           double *grad_out, rsot_eval_info *info);

/*
 * rsot_dual_eval for callers that cannot allocate device memory (code under
 * stream capture, tight serving loops, harnesses that forbid allocation):
 * same arguments, results and errors, for a problem whose rule is DENSE. The
 * evaluation's work-item partials live in a static device array of 64 MiB per
 * device (held until the process ends) instead of the problem's own buffers;
 * the call itself allocates nothing. The partials use rsot_dual_eval's
 * default segmentation when they fit (results then equal rsot_dual_eval's
 * bit for bit), else the coarsest segmentation that fits.
 * Calls that overlap on one device share the array and race: serialise them.
 * Errors: INVALID_ARG (NULL, eps, or a rule other than DENSE), NONFINITE,
 * OOM (the partials exceed 64 MiB even at the coarsest segmentation: about
 * more than 4 million points), DEVICE.
 */
rsot_status rsot_dual_eval_noalloc(rsot_problem *p, double eps, const double *psi,
                                   double *J_out, double *grad_out, rsot_eval_info *info);

/*
 * Evaluates n problems in one call (same quantities as rsot_dual_eval for
 * each): every problem's preparation and culling, one host synchronisation,
 * then one launch per pass over the (problem, work item) pairs of all
 * problems, numbered with the problems in decreasing order of work.
 * Problems with the FP64 arithmetic or a cutoff rule (GEOM/INT/PW) run their
 * own passes inside the same call. All work is issued on ps[0]'s stream.
 *   ps        n problem handles (distinct)
 *   eps       HOST array of n eps values
 *   psi       HOST array of n DEVICE pointers (each problem's n_target doubles)
 *   J_out     HOST array of n doubles
 *   grad_out  NULL, or HOST array of n DEVICE pointers (NULL entries allowed)
 *   infos     NULL or HOST array of n infos (per-problem pass times are 0)
 *   batch_ms  NULL or HOST: device time of the whole batch
 * Results equal per-problem rsot_dual_eval calls up to the order of the
 * floating-point sums (identical for the same segmentation).
 */
rsot_status rsot_dual_eval_batched(rsot_problem *const *ps, int n, const double *eps,
                                   const double *const *psi, double *J_out,
                                   double *const *grad_out, rsot_eval_info *infos,
                                   double *batch_ms);

/*
 * Autotuner: picks the granularity of the culling and of both passes for
 * this problem by timing evaluations at (eps, psi): under the TILE rule first
 * the culling group in {64, 32, 16, 8} targets (finer groups keep fewer
 * pairs and cost more culling), then the objective-pass segment in
 * {64,128,256,512,1024} target blocks, then the gradient-pass segment in
 * {16,...,4096} point tiles (0 = library default), each the best of `reps`
 * device timings. The problem keeps the fastest triple.
 *   psi             DEVICE pointer (n_target doubles)
 *   seg_*_out, tile_group_out  HOST, chosen values (0 = default); may be NULL
 *   best_ms_out     HOST, time of the chosen configuration; may be NULL
 *   default_ms_out  HOST, time of the default configuration; may be NULL
 */
rsot_status rsot_autotune(rsot_problem *p, double eps, const double *psi, int reps,
                          int *seg_blocks_out, int *seg_tiles_out, int *tile_group_out,
                          double *best_ms_out, double *default_ms_out);

/* Sets the granularities directly (e.g. from a cache of autotuner results);
 * tile_group 0, 8, 16, 32 or 64 (else INVALID_ARG). */
rsot_status rsot_set_tuning(rsot_problem *p, int seg_blocks, int seg_tiles, int tile_group);

/*
 * Per-point log-sum-exp L_q = ln sum_j nu_j exp((psi_j - c_qj)/eps) of the
 * last evaluation (the log of S_q in Alg. 2; -inf for a dropped point), in
 * the caller's point order. L_out: DEVICE pointer, n_quad doubles.
 */
rsot_status rsot_get_lse(rsot_problem *p, double *L_out);

/*
 * Size of the kept set I_q of every point in the last evaluation: the number
 * of targets whose terms entered the point's sum (Sec. 4.1: I_q = {j : c_qj <
 * C} under the cutoff rules; N under DENSE; under TILE the targets of the
 * blocks, or groups, kept for the point's tile). A point dropped for an empty
 * set has 0.
 *   counts_out  DEVICE pointer, n_quad int32 in the caller's point order
 * Errors: INVALID_ARG (NULL, or no evaluation yet), DEVICE.
 */
rsot_status rsot_get_kept_counts(rsot_problem *p, int32_t *counts_out);

/*
 * Culling decision of the last evaluation for every (point tile, target
 * block) pair of rsot_get_partition's grouping, row-major by tile:
 * 0 = skipped, 1 = kept in part (cutoff rules: with the per-pair test
 * c < C; TILE with culling groups below 64: some of the block's groups
 * dropped, see rsot_get_tile_chunk_keep), 2 = every pair kept (DENSE: all 2).
 *   keep_out  DEVICE pointer, n_tiles * n_blocks bytes
 * Errors: INVALID_ARG (NULL, or no evaluation yet), DEVICE.
 */
rsot_status rsot_get_tile_keep(rsot_problem *p, uint8_t *keep_out);

/*
 * The same at the granularity of 8-target chunks: per (tile, block) a byte
 * whose bit c is set when the pairs of the block's targets 8c..8c+7 (in
 * rsot_get_target_slots order) entered the last evaluation: all of them
 * under DENSE and TILE; under the cutoff rules the chunk was not skipped and
 * its pairs took the test c < C. Bits of chunks holding only padding may be
 * set.
 *   mask_out  DEVICE pointer, n_tiles * n_blocks bytes, row-major by tile
 * Errors: INVALID_ARG (NULL, or no evaluation yet), DEVICE.
 */
rsot_status rsot_get_tile_chunk_keep(rsot_problem *p, uint8_t *mask_out);

/*
 * Position of every target in the library's sorted, padded target order:
 * target i sits in block slot[i] / 64, chunk slot[i] / 8, culling group
 * slot[i] / tile_group.
 *   slot_out  DEVICE pointer, n_target int32 (caller order)
 * Errors: INVALID_ARG, DEVICE.
 */
rsot_status rsot_get_target_slots(rsot_problem *p, int32_t *slot_out);

/*
 * Covering cost C_0 = max_q min_j c(x_q, y_j) (Sec. 4.1 / App. B, maximum
 * over the quadrature points). C0_out: HOST pointer.
 */
rsot_status rsot_covering_cost(rsot_problem *p, double *C0_out);

/*
 * Tile structure of the problem (for checking the TILE rule against an
 * independent implementation): for every point (caller's order) its tile id,
 * for every target its block id. Both DEVICE pointers to int32, or NULL.
 */
rsot_status rsot_get_partition(rsot_problem *p, int32_t *tile_of_point, int32_t *block_of_target,
                               int64_t *n_tiles, int64_t *n_blocks);

/*
 * Softmax potential refinement (Eq. softmax_refinement_formula, Sec. 5.2):
 *   psi_fine_k = -eps ln( sum_q mu_q exp(-c(x_q, y_fine_k)/eps) / S_q ),
 *   S_q = sum_j nu_j exp((psi_coarse_j - c(x_q, y_j))/eps)
 * over the problem's points and (coarse) targets. Evaluated in the log
 * domain; (point tile, fine block) pairs whose bound is below 1e-12 of the
 * kept sum are skipped (psi moves by at most 1e-12 eps).
 *   psi_coarse   DEVICE pointer, the problem's n_target doubles (caller order)
 *   n_fine       number of fine targets (> 0)
 *   y_fine       DEVICE pointer, n_fine x dim doubles
 *   psi_fine_out DEVICE pointer, n_fine doubles
 * Also leaves the coarse L_q readable through rsot_get_lse.
 */
rsot_status rsot_softmax_refine(rsot_problem *p, double eps, const double *psi_coarse,
                                int64_t n_fine, const double *y_fine, double *psi_fine_out);

/*
 * Target moments of the plan pi_qj = mu_q p_qj(psi) (Sec. 6.2), over the
 * pairs of the problem's truncation rule:
 *   mass_out[j]          = nu~_j = sum_q mu_q p_qj          (Eq. discretized_gradient + nu)
 *   first_out[j*dim + k] = sum_q mu_q p_qj x_q[k]
 * At the optimum first_j / nu_j is the conditional barycentre T_j of
 * Eq. barycenter_fixed_point (the damped Lloyd step of Eq. damped_lloyd
 * moves y_j towards it), and 2 cost_scale (nu~_j y_j - first_j) is Danskin's
 * gradient of the transport cost in y_j (Eq. barycenter_gradient_general).
 *   psi        DEVICE pointer, n_target doubles (caller order)
 *   mass_out   DEVICE pointer, n_target doubles, or NULL
 *   first_out  DEVICE pointer, n_target x dim doubles (row-major), or NULL
 *              (not both NULL)
 *   info       HOST pointer or NULL: the evaluation's statistics
 *   kernel_ms  HOST pointer or NULL: device time of the moment kernels
 * The call evaluates J at psi first (it leaves L_q for rsot_get_lse).
 * Errors: INVALID_ARG, NONFINITE (psi), DEVICE, OOM.
 */
rsot_status rsot_plan_moments(rsot_problem *p, double eps, const double *psi, double *mass_out,
                              double *first_out, rsot_eval_info *info, double *kernel_ms);

/*
 * Transport maps of the plan (Sec. 6.3), per quadrature point, over the pairs
 * of the problem's truncation rule:
 *   bary_out[q*dim + k] = sum_j p_qj y_j[k]        (Eq. barycentric_map_registration)
 *   modal_out[q]        = argmax_j (psi_j - c_qj + eps ln nu_j), a target index
 *                         in the caller's order   (Eq. modal_map_registration)
 * The argmax is decided on FP64 exponents; where two targets tie to within
 * FP64 rounding either may be returned. A point with no kept pair (pointwise
 * rule) gets NaN and -1.
 *   psi        DEVICE pointer, n_target doubles (caller order)
 *   bary_out   DEVICE pointer, n_quad x dim doubles, or NULL
 *   modal_out  DEVICE pointer, n_quad int32, or NULL (not both NULL)
 *   info, kernel_ms as for rsot_plan_moments
 * Errors: INVALID_ARG, NONFINITE (psi), DEVICE, OOM.
 */
rsot_status rsot_transport_maps(rsot_problem *p, double eps, const double *psi, double *bary_out,
                                int32_t *modal_out, rsot_eval_info *info, double *kernel_ms);

/*
 * One step of the Riemannian barycentre iteration (Alg. 5) for every target,
 * for a problem with the squared geodesic cost on the sphere (opt.cost_kind
 * SPHERE). The conditional measures mu_j(x | psi) of the plan at (psi, the
 * problem's targets) are held fixed (Alg. 4 computes them once per Lloyd
 * iteration); the log and exp maps are taken at the current points y_cur:
 *   delta_j  = -2 sum_q w_qj log_{y_cur_j}(x_q) / sum_q w_qj,  w_qj = mu_q p_qj
 *   y_next_j = exp_{y_cur_j}(-alpha delta_j)
 * with log_y(x) = theta / sin(theta) (x - cos(theta) y), theta = d_g(x, y),
 * and exp_y(v) = cos|v| y + sin|v| v / |v|. alpha = 1/2 moves a point to the
 * barycentre of the measure it sees when that measure is a single point.
 *   psi        DEVICE, n_target doubles (caller order)
 *   y_cur      DEVICE, n_target x 3 doubles (unit vectors, caller order)
 *   y_next     DEVICE, n_target x 3 doubles (out; may alias nothing else)
 *   step_norm  DEVICE, n_target doubles |delta_j| (out), or NULL
 *   mass_out   DEVICE, n_target doubles sum_q w_qj = nu~_j (out), or NULL
 *   info, kernel_ms  as for rsot_plan_moments
 * The call evaluates J at psi first, under the problem's rule. A target with
 * no mass keeps its point.
 * Errors: INVALID_ARG (NULL, another cost, eps <= 0, alpha < 0), NONFINITE,
 * DEVICE, OOM.
 */
rsot_status rsot_sphere_karcher_step(rsot_problem *p, double eps, const double *psi,
                                     const double *y_cur, double alpha, double *y_next,
                                     double *step_norm, double *mass_out, rsot_eval_info *info,
                                     double *kernel_ms);

/* ------------------------------------------------------------------------ */
/* Solver (Alg. 1): L-BFGS on J with an eps schedule (Sec. 4.2).            */
/* ------------------------------------------------------------------------ */
typedef struct {
    int stage;                /* index into the eps schedule                       */
    int iteration;            /* accepted iterations in this stage                 */
    int evaluations;          /* dual evaluations in this stage                     */
    double eps;
    double J, grad_l1, grad_linf, step;
    int64_t kept_pairs;
    double cutoff;
} rsot_iter_info;

/* Return nonzero to cancel the solve. */
typedef int (*rsot_callback)(const rsot_iter_info *it, void *user);

/*
 * Solver state to resume from: the eps stage (Sec. 4.2), the accepted
 * iterations done in it, the L-BFGS history of Alg. 1's quasi-Newton step and
 * the |J| reference of the truncation rules. Together with the returned
 * potential it continues a stopped solve exactly where it stopped. The
 * caller owns every buffer.
 */
typedef struct {
    int64_t n_target;         /* length of the potential the pairs belong to      */
    int capacity;             /* pairs the buffers hold (lbfgs_m keeps them all)  */
    double *s, *y;            /* HOST: capacity x n_target doubles each; pair i   */
                              /* at offset i * n_target, oldest first             */
    int n_pairs;              /* pairs held (<= capacity)                          */
    int stage;                /* eps stage the solve was in                        */
    int iteration;            /* accepted iterations done in that stage            */
    double absJ_ref;          /* |J| reference of the truncation rules             */
    int valid;                /* 1 once a solve has written the state              */
} rsot_checkpoint;

typedef struct {
    const double *eps_schedule; /* HOST array: eps_0 > ... > eps_final (Sec. 4.2)  */
    int n_eps;                  /* >= 1                                            */
    double tol;                 /* stop when ||grad||_1 <= tol (Remark 3.2); 1e-6  */
    int max_iter;               /* accepted iterations per stage; default 10000    */
    int lbfgs_m;                /* history pairs; default 10                       */
    double c1, c2;              /* Wolfe constants; default 1e-4, 0.9              */
    int max_ls;                 /* evaluations per line search; default 20         */
    double stage_tol;           /* ||grad||_1 target of non-final stages; 0 = tol  */
    rsot_callback callback;     /* called after every accepted iteration, or NULL  */
    void *user;
    volatile int *cancel;       /* polled between evaluations, or NULL             */
    double absJ_start;          /* |J| reference of the truncation rules for the
                                   first evaluation (Sec. 4.1 uses |J| of the
                                   current iterate; later ones use the last
                                   accepted iterate, and each eps stage starts
                                   from the previous stage's); 0 = evaluate the
                                   warm start densely to obtain it; >= 0      */
    rsot_checkpoint *checkpoint;/* NULL, or written on every exit of the solve   */
    int resume;                 /* 1: continue from *checkpoint (stage, history,
                                   |J| reference) and psi_inout                 */
    int test_flip_gradient;     /* test hook, 0 in use: the solver sees -grad, so
                                   no step decreases J and the first line search
                                   ends with RSOT_ERR_LINESEARCH                 */
} rsot_solve_params;

typedef struct {
    int iterations;             /* accepted iterations, all stages                 */
    int evaluations;            /* dual evaluations, all stages                    */
    int stages;                 /* stages run; after an error the last of them is
                                   the one that stopped (resume from it with psi) */
    double J, grad_l1, grad_linf;
    double seconds;             /* wall time of the solve                           */
    double eval_ms;             /* device time spent in evaluations                */
    double cull_ms;             /* of which: target records, cutoff, culling       */
    double pass1_ms;            /* of which: objective passes                      */
    double pass2_ms;            /* of which: gradient passes                       */
    double kept_frac;           /* mean fraction of pairs summed per evaluation    */
    int status;                 /* rsot_status of the solve                         */
    int stalled_stages;         /* non-final eps stages that ended on a line-search
                                   failure before stage_tol (no step improved J at
                                   the pair loop's precision); the next stage
                                   continues from the best iterate. A failure in
                                   the final stage is the solve's status.        */
} rsot_solve_info;

void rsot_solve_params_default(rsot_solve_params *sp);

/*
 * Minimises J with L-BFGS (Alg. 1, Sec. 3.4) through the eps schedule
 * (Sec. 4.2), warm-starting each stage from the previous one.
 *   psi_inout HOST pointer, n_target doubles: warm start in (zeros allowed),
 *             solution out, centred on success so that sum_j nu_j psi_j = 0
 *             (App. A: the minimiser is unique up to a constant). On any
 *             other status it is the last accepted iterate unshifted, so
 *             that a resume continues from exactly that point.
 * With sp->checkpoint the solver state is written on every exit; with
 * sp->resume the solve continues from it (its stage, its L-BFGS pairs, its
 * |J| reference, its iteration count against max_iter) at psi_inout, which
 * must be the potential that solve returned.
 * Errors: INVALID_ARG (also: resume without a valid checkpoint of this size
 * and schedule), UNBALANCED, NONFINITE, LINESEARCH, NOT_CONVERGED,
 * CANCELLED, DEVICE; psi_inout and info hold the best accepted iterate.
 */
rsot_status rsot_solve(rsot_problem *p, const rsot_solve_params *sp, double *psi_inout,
                       rsot_solve_info *info);

/* ------------------------------------------------------------------------ */
/* Multilevel (Sec. 5): target hierarchy, combined source/target solve.      */
/* ------------------------------------------------------------------------ */

/*
 * Target-set hierarchy by k-means coarsening (Sec. 5.2): level l-1 is a
 * k-means clustering of the points of level l; each non-empty cluster becomes
 * one point at its centroid (mean of member points) with the summed mass of
 * its members, so every level has the same total mass. Levels run from the
 * coarsest (0) to the finest (n_levels-1 = the input).
 *   y, nu          DEVICE pointers: n x dim targets and masses
 *   n_per_level    HOST array: requested sizes, non-decreasing, last == n
 *   lloyd_iters    Lloyd iterations per level (initial centroids: means of
 *                  consecutive groups in Morton order)
 *   seed           reserved (the construction is deterministic)
 *   y_levels[l]    DEVICE buffers of n_per_level[l] x dim doubles (caller-owned)
 *   nu_levels[l]   DEVICE buffers of n_per_level[l] doubles
 *   parent_levels  NULL, or HOST array of DEVICE int32 buffers: parent_levels[l]
 *                  (l >= 1, n_per_level[l] entries) receives, for every point of
 *                  level l, the index of its cluster in level l-1; entry 0 unused
 *   n_out[l]       HOST: realised sizes (empty clusters are dropped)
 * The returned points are the means of their final clusters and carry the
 * clusters' summed masses.
 */
rsot_status rsot_target_hierarchy(int dim, int64_t n, const double *y, const double *nu,
                                  int n_levels, const int64_t *n_per_level, int lloyd_iters,
                                  uint64_t seed, void *hip_stream, double *const *y_levels,
                                  double *const *nu_levels, int32_t *const *parent_levels,
                                  int64_t *n_out);

#define RSOT_ML_MAX_LEVELS 16
enum { RSOT_TRANSFER_SOFTMAX = 0 };

typedef struct rsot_multilevel rsot_multilevel;

/*
 * Copies source levels T_0..T_{n_source_levels-1} (coarsest first: points
 * x[l] and masses mu[l]) and target levels nu^(0)..nu^(n_target_levels-1)
 * (coarsest first) into library memory. opt->inputs_on_device selects host or
 * device pointers; problems for each (source level, target level) pair are
 * created when first needed with opt.
 */
rsot_status rsot_multilevel_create(int dim, int n_source_levels, const int64_t *n_quad,
                                   const double *const *x, const double *const *mu,
                                   int n_target_levels, const int64_t *n_target,
                                   const double *const *y, const double *const *nu,
                                   const rsot_options *opt, void *hip_stream,
                                   rsot_multilevel **out);
void rsot_multilevel_destroy(rsot_multilevel *ml);

/* Combined index rule of Sec. 5.3: is = max(0, l - (Lmax - Lmu)),
 * it = max(0, l - (Lmax - Lnu)), Lmax = max(Lmu, Lnu). */
void rsot_multilevel_indices(int n_source_levels, int n_target_levels, int l, int *is, int *it);

typedef struct {
    const double *eps;        /* HOST: eps of each stage                                 */
    const int *level;         /* HOST: combined level l of each stage, non-decreasing    */
    int n_stages;
    rsot_solve_params base;   /* tol, max_iter, lbfgs_m, ... (eps_schedule ignored)      */
    double level_tol;         /* ||grad||_1 target of non-final levels; 0 = base.tol     */
    int transfer;             /* RSOT_TRANSFER_SOFTMAX (Eq. softmax_refinement_combined) */
} rsot_ml_params;

typedef struct {
    int n_steps;                                  /* Lmax + 1                     */
    int source_level[RSOT_ML_MAX_LEVELS];
    int target_level[RSOT_ML_MAX_LEVELS];
    int iterations[RSOT_ML_MAX_LEVELS];
    int evaluations[RSOT_ML_MAX_LEVELS];
    double seconds[RSOT_ML_MAX_LEVELS];           /* solve time of each step      */
    double refine_seconds[RSOT_ML_MAX_LEVELS];    /* transfer time into each step */
    int64_t refine_pairs[RSOT_ML_MAX_LEVELS];     /* pairs the refinement summed  */
    double eval_ms[RSOT_ML_MAX_LEVELS];           /* device time in evaluations   */
    double kept_frac[RSOT_ML_MAX_LEVELS];         /* mean kept-pair fraction      */
    double total_seconds;
    double grad_l1;
    int status;
    int stalled_levels;       /* non-final steps whose solve ended on a line-search
                                 failure before level_tol; the next step continues
                                 from their best iterate, as after the iteration
                                 cap. A failure in the final step is the status. */
} rsot_ml_info;

/*
 * Combined multilevel solve (Sec. 5.3) with the eps stages of mp: step
 * l = 0..Lmax solves on (T_is(l), nu^(it(l))); when it(l) = it(l-1)+1 the
 * potential is transferred by softmax refinement at the eps of the last
 * stage of step l-1 (Eq. softmax_refinement_formula_combined), otherwise it is
 * kept. psi_out: HOST pointer, n_target of the finest level, centred when the
 * final step succeeds.
 * mp->base must carry no checkpoint and no resume (INVALID_ARG): the levels
 * differ in size. Problems other than the finest (source, target) pair run
 * the FP32 pair loop whatever their size (fp64_below_points applies to the
 * finest only): they warm-start the next level and stop at its tolerance.
 */
rsot_status rsot_solve_multilevel(rsot_multilevel *ml, const rsot_ml_params *mp, double *psi_out,
                                  rsot_ml_info *info);

#ifdef __cplusplus
}
#endif
#endif /* RSOT_H */
