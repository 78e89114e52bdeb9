/*
 * rsot_oracle.c -- plain FP64 CPU oracle for the semi-discrete RSOT dual.
 *
 * TEST INFRASTRUCTURE ONLY. This file is the slow, obviously correct checker
 * the HIP library is compared against. Only tests, the smoke check and the
 * benchmark's CPU-baseline leg may load it. It shares no code, header, table
 * or constant with the HIP library.
 *
 * Notation (Sec. 2, Sec. 3.3): targets y_j with masses nu_j, potential psi_j,
 * quadrature points x_q with masses mu_q = rho_h(x_q) w_q, cost
 * c(x, y) = cost_scale * |x - y|^2 (the paper's canonical cost has
 * cost_scale = 1/2), regularisation eps.
 *
 *   z_qj   = (psi_j - c(x_q, y_j)) / eps + ln nu_j
 *   L_q    = ln sum_j exp(z_qj)                  (log of S_q in Alg. 2)
 *   J      = eps sum_q mu_q L_q - sum_j psi_j nu_j          (Eq. discretized_functional)
 *   dJ/dpsi_k = sum_q mu_q exp(z_qk - L_q) - nu_k           (Eq. discretized_gradient)
 *
 * Alg. 2 forms S_q = exp(L_q) directly; the oracle keeps it in log form
 * (max-shifted sum), which is the same number without underflow at small eps.
 *
 * Truncation (Sec. 4.1): with a cutoff C > 0 the sums run over
 * I_q = { j : c(x_q, y_j) < C } only (strict), and a point with empty I_q
 * contributes nothing (the S_q > 0 test of Alg. 2).
 *
 * Every function is plain loops over doubles with libm exp/log; OpenMP splits
 * the quadrature points over threads, each with its own gradient array, and
 * the thread arrays are summed in thread order.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static int oracle_threads(int want)
{
#ifdef _OPENMP
    if (want > 0) return want;
    return omp_get_max_threads();
#else
    (void)want;
    return 1;
#endif
}

/* c(x, y) = cost_scale * |x - y|^2  (Sec. 2: c(x, y_j) = 1/2 |x - y_j|^2) */
static double cost(int d, const double *x, const double *y, double cost_scale)
{
    double s = 0.0;
    for (int k = 0; k < d; ++k) {
        double t = x[k] - y[k];
        s += t * t;
    }
    return cost_scale * s;
}

/*
 * Dual objective and gradient, dense (cutoff <= 0 or infinite) or truncated
 * with the rule I_q = { j : c_qj < cutoff } (Alg. 2).
 *
 * x: nq*d row-major, mu: nq, y: n*d row-major, nu: n, psi: n.
 * Outputs: *J_out; grad_out (n, may be NULL); L_out (nq, may be NULL; gets
 * L_q, or -INFINITY for a point with empty I_q); *kept_out = sum_q |I_q|;
 * *nempty_out = number of points with empty I_q.
 * Returns 0, or -1 on invalid arguments / allocation failure.
 */
int oracle_dual_eval(int d, int64_t nq, const double *x, const double *mu,
                     int64_t n, const double *y, const double *nu,
                     const double *psi, double eps, double cost_scale,
                     double cutoff, int nthreads,
                     double *J_out, double *grad_out, double *L_out,
                     int64_t *kept_out, int64_t *nempty_out)
{
    if (d < 1 || nq < 0 || n < 1 || !(eps > 0.0)) return -1;
    const int truncated = (cutoff > 0.0 && isfinite(cutoff));
    const int T = oracle_threads(nthreads);

    double *lognu = (double *)malloc(sizeof(double) * (size_t)n);
    double *gpart = (double *)calloc((size_t)T * (size_t)n, sizeof(double));
    double *Jpart = (double *)calloc((size_t)T, sizeof(double));
    int64_t *kpart = (int64_t *)calloc((size_t)T, sizeof(int64_t));
    int64_t *epart = (int64_t *)calloc((size_t)T, sizeof(int64_t));
    if (!lognu || !gpart || !Jpart || !kpart || !epart) {
        free(lognu); free(gpart); free(Jpart); free(kpart); free(epart);
        return -1;
    }
    for (int64_t j = 0; j < n; ++j) lognu[j] = log(nu[j]);

#pragma omp parallel num_threads(T)
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        double *z = (double *)malloc(sizeof(double) * (size_t)n);
        char *in = (char *)malloc((size_t)n);
        double *g = gpart + (size_t)tid * (size_t)n;
        double Jt = 0.0;
        int64_t kt = 0, et = 0;
#pragma omp for schedule(static)
        for (int64_t q = 0; q < nq; ++q) {
            const double *xq = x + q * d;
            /* membership and exponents z_qj */
            double zmax = -INFINITY;
            int64_t cnt = 0;
            for (int64_t j = 0; j < n; ++j) {
                double c = cost(d, xq, y + j * d, cost_scale);
                in[j] = (char)(!truncated || c < cutoff);
                if (!in[j]) continue;
                z[j] = (psi[j] - c) / eps + lognu[j];
                if (z[j] > zmax) zmax = z[j];
                ++cnt;
            }
            if (cnt == 0) {               /* S_q = 0: point skipped (Alg. 2) */
                ++et;
                if (L_out) L_out[q] = -INFINITY;
                continue;
            }
            kt += cnt;
            /* L_q = log sum_j exp(z_qj), max-shifted */
            double s = 0.0;
            for (int64_t j = 0; j < n; ++j)
                if (in[j]) s += exp(z[j] - zmax);
            double L = zmax + log(s);
            if (L_out) L_out[q] = L;
            Jt += eps * L * mu[q];
            /* gradient scatter: mu_q * T_qj / S_q */
            if (grad_out)
                for (int64_t j = 0; j < n; ++j)
                    if (in[j]) g[j] += mu[q] * exp(z[j] - L);
        }
        Jpart[tid] = Jt;
        kpart[tid] = kt;
        epart[tid] = et;
        free(z);
        free(in);
    }

    double J = 0.0;
    int64_t kept = 0, nempty = 0;
    for (int t = 0; t < T; ++t) {
        J += Jpart[t];
        kept += kpart[t];
        nempty += epart[t];
    }
    for (int64_t j = 0; j < n; ++j) J -= psi[j] * nu[j];
    if (grad_out) {
        for (int64_t j = 0; j < n; ++j) {
            double s = 0.0;
            for (int t = 0; t < T; ++t) s += gpart[(size_t)t * (size_t)n + j];
            grad_out[j] = s - nu[j];
        }
    }
    *J_out = J;
    if (kept_out) *kept_out = kept;
    if (nempty_out) *nempty_out = nempty;
    free(lognu); free(gpart); free(Jpart); free(kpart); free(epart);
    return 0;
}

/*
 * Covering cost C_0 = max_q min_j c(x_q, y_j) (Sec. 4.1, App. B), with the
 * maximum over the quadrature points (the only points the discrete functional
 * sees). Brute force.
 */
double oracle_covering_cost(int d, int64_t nq, const double *x, int64_t n,
                            const double *y, double cost_scale, int nthreads)
{
    const int T = oracle_threads(nthreads);
    double best = 0.0;
#pragma omp parallel for num_threads(T) reduction(max : best) schedule(static)
    for (int64_t q = 0; q < nq; ++q) {
        double m = INFINITY;
        for (int64_t j = 0; j < n; ++j) {
            double c = cost(d, x + q * d, y + j * d, cost_scale);
            if (c < m) m = c;
        }
        if (m > best) best = m;
    }
    return best;
}

/*
 * Kept-set sizes of a cost cutoff (Sec. 4.1): kept_out[q] = |I_q| =
 * #{ j : c(x_q, y_j) < cutoff }, brute force. near_out (may be NULL) counts
 * the targets with |c(x_q, y_j) - cutoff| <= rel_band * cutoff: the pairs whose
 * membership another, equally exact evaluation order of the cost may decide
 * the other way.
 */
int oracle_kept_counts(int d, int64_t nq, const double *x, int64_t n, const double *y,
                       double cost_scale, double cutoff, double rel_band, int nthreads,
                       int32_t *kept_out, int32_t *near_out)
{
    if (d < 1 || nq < 0 || n < 1 || !kept_out || !(rel_band >= 0.0)) return -1;
    const int T = oracle_threads(nthreads);
#pragma omp parallel for num_threads(T) schedule(static)
    for (int64_t q = 0; q < nq; ++q) {
        int32_t k = 0, m = 0;
        for (int64_t j = 0; j < n; ++j) {
            double c = cost(d, x + q * d, y + j * d, cost_scale);
            if (c < cutoff) ++k;
            if (fabs(c - cutoff) <= rel_band * fabs(cutoff)) ++m;
        }
        kept_out[q] = k;
        if (near_out) near_out[q] = m;
    }
    return 0;
}

/* Geometric cutoff (Eq. truncation_cutoff_geom, App. B):
 * C = C_0 + (M - m) + eps ln(eps / (nu_min tau |J|)), and C >= C_0. */
double oracle_cutoff_geom(double C0, double M, double m, double nu_min,
                          double tau, double absJ, double eps)
{
    double C = C0 + (M - m) + eps * log(eps / (nu_min * tau * absJ));
    return C > C0 ? C : C0;
}

/* Integral cutoff (Eq. truncation_cutoff_int), D from the previous
 * evaluation: C = M + eps ln(eps D / (tau |J|)), kept >= C_0. */
double oracle_cutoff_int(double C0, double M, double D, double tau,
                         double absJ, double eps)
{
    double C = M + eps * log(eps * D / (tau * absJ));
    return C > C0 ? C : C0;
}

/* Pointwise cutoff (Eq. cost_cutoff_delta): C = M + eps ln(nu_max / delta). */
double oracle_cutoff_pw(double M, double nu_max, double delta_thr, double eps)
{
    return M + eps * log(nu_max / delta_thr);
}

/*
 * D = sum_q mu_q / S_trunc(x_q) = sum_q mu_q exp(-L_q) (the integrated inverse
 * of the truncated sum in Eq. truncation_cutoff_int), from per-point L_q;
 * points with L_q = -inf (empty I_q) are left out.
 */
double oracle_integral_D(int64_t nq, const double *mu, const double *L)
{
    double D = 0.0;
    for (int64_t q = 0; q < nq; ++q)
        if (isfinite(L[q])) D += mu[q] * exp(-L[q]);
    return D;
}

/*
 * Softmax potential refinement (Eq. softmax_refinement_formula):
 *   psi_k = -eps ln sum_q mu_q exp(-c(x_q, y_k)/eps) / S_q^coarse
 *         = -eps LSE_q( ln mu_q - L_q - c(x_q, y_k)/eps ),
 * where L_q = ln S_q^coarse comes from the coarse targets and potential
 * (Eq. phi_from_psi_coarse). Points with mu_q = 0 contribute nothing.
 */
int oracle_softmax_refine(int d, int64_t nq, const double *x, const double *mu,
                          const double *L, int64_t nf, const double *yf,
                          double eps, double cost_scale, int nthreads,
                          double *psi_out)
{
    const int T = oracle_threads(nthreads);
#pragma omp parallel for num_threads(T) schedule(static)
    for (int64_t k = 0; k < nf; ++k) {
        double vmax = -INFINITY;
        for (int64_t q = 0; q < nq; ++q) {
            if (!(mu[q] > 0.0)) continue;
            double v = log(mu[q]) - L[q] - cost(d, x + q * d, yf + k * d, cost_scale) / eps;
            if (v > vmax) vmax = v;
        }
        double s = 0.0;
        for (int64_t q = 0; q < nq; ++q) {
            if (!(mu[q] > 0.0)) continue;
            double v = log(mu[q]) - L[q] - cost(d, x + q * d, yf + k * d, cost_scale) / eps;
            s += exp(v - vmax);
        }
        psi_out[k] = -eps * (vmax + log(s));
    }
    return 0;
}

/*
 * Tile-local error-controlled truncation (derived from App. B's bound).
 *
 * The quadrature points come grouped into tiles (tile_of[q]) and the targets
 * into blocks (block_of[j]); both groupings are data. With bounding boxes of
 * each tile and block, for every pair (T, B):
 *   ln U_TB = ln nu(B) + (Psi_B - cost_scale dmin^2(T,B)) / eps
 * bounds every term of block B at every point of T from above
 * (Psi_B = max_{j in B} psi_j, nu(B) = sum_{j in B} nu_j, dmin = least
 * distance between the two boxes). For each tile a reference target j_T gives
 *   ln L_T = ln nu_jT + (psi_jT - cost_scale dmax^2(T, y_jT)) / eps,
 * a lower bound of the truncated sum at every point of T (dmax = greatest
 * distance from the tile box to y_jT). j_T is chosen as: B* = the block of
 * largest ln U_TB (lowest index on ties), then the target of B* with the
 * largest ln nu_j + (psi_j - cost_scale dmax^2(T, y_j))/eps (lowest index on
 * ties). A pair (T, B) is skipped iff B != B* and
 *   ln U_TB <= ln L_T + ln(eta / n_blocks),  eta = tau |J_ref| / (eps sum mu),
 * so the neglected sum at any x in T is at most eta * S_trunc(x), and App. B's
 * chain ln(1 + z) <= z gives J_dense - J_trunc <= eps eta sum mu = tau |J_ref|.
 * All pairs inside kept (T, B) are summed.
 *
 * keep_out (n_tiles * n_blocks, row-major by tile, may be NULL) receives the
 * kept flags. Then the same quantities as oracle_dual_eval over the kept pairs.
 */
int oracle_dual_eval_tile(int d, int64_t nq, const double *x, const double *mu,
                          int64_t n, const double *y, const double *nu,
                          const double *psi, double eps, double cost_scale,
                          const int32_t *tile_of, int64_t n_tiles,
                          const int32_t *block_of, int64_t n_blocks,
                          double tau, double absJ_ref, int nthreads,
                          double *J_out, double *grad_out, double *L_out,
                          int64_t *kept_out, uint8_t *keep_out)
{
    if (d < 1 || d > 3 || n_tiles < 1 || n_blocks < 1) return -1;
    double *tlo = (double *)malloc(sizeof(double) * (size_t)n_tiles * 3);
    double *thi = (double *)malloc(sizeof(double) * (size_t)n_tiles * 3);
    double *blo = (double *)malloc(sizeof(double) * (size_t)n_blocks * 3);
    double *bhi = (double *)malloc(sizeof(double) * (size_t)n_blocks * 3);
    double *bpsi = (double *)malloc(sizeof(double) * (size_t)n_blocks);
    double *bnu = (double *)malloc(sizeof(double) * (size_t)n_blocks);
    uint8_t *keep = (uint8_t *)calloc((size_t)n_tiles * (size_t)n_blocks, 1);
    if (!tlo || !thi || !blo || !bhi || !bpsi || !bnu || !keep) return -1;
    double summu = 0.0;
    for (int64_t q = 0; q < nq; ++q) summu += mu[q];

    for (int64_t t = 0; t < n_tiles * 3; ++t) { tlo[t] = INFINITY; thi[t] = -INFINITY; }
    for (int64_t b = 0; b < n_blocks * 3; ++b) { blo[b] = INFINITY; bhi[b] = -INFINITY; }
    for (int64_t b = 0; b < n_blocks; ++b) { bpsi[b] = -INFINITY; bnu[b] = 0.0; }
    for (int64_t q = 0; q < nq; ++q) {
        int64_t t = tile_of[q];
        for (int k = 0; k < d; ++k) {
            double v = x[q * d + k];
            if (v < tlo[t * 3 + k]) tlo[t * 3 + k] = v;
            if (v > thi[t * 3 + k]) thi[t * 3 + k] = v;
        }
    }
    for (int64_t j = 0; j < n; ++j) {
        int64_t b = block_of[j];
        for (int k = 0; k < d; ++k) {
            double v = y[j * d + k];
            if (v < blo[b * 3 + k]) blo[b * 3 + k] = v;
            if (v > bhi[b * 3 + k]) bhi[b * 3 + k] = v;
        }
        if (psi[j] > bpsi[b]) bpsi[b] = psi[j];
        bnu[b] += nu[j];
    }
    const double ln_eta_over_nb = log(tau * absJ_ref / (eps * summu)) - log((double)n_blocks);
    const int T = oracle_threads(nthreads);

#pragma omp parallel for num_threads(T) schedule(static)
    for (int64_t t = 0; t < n_tiles; ++t) {
        if (!(tlo[t * 3] <= thi[t * 3])) continue;      /* empty tile */
        /* upper bounds ln U_TB and the best block B* */
        int64_t bstar = -1;
        double ubest = -INFINITY;
        double *lnU = (double *)malloc(sizeof(double) * (size_t)n_blocks);
        for (int64_t b = 0; b < n_blocks; ++b) {
            lnU[b] = -INFINITY;
            if (!(bnu[b] > 0.0)) continue;              /* empty block */
            double dmin2 = 0.0;
            for (int k = 0; k < d; ++k) {
                double gap = 0.0;
                if (blo[b * 3 + k] > thi[t * 3 + k]) gap = blo[b * 3 + k] - thi[t * 3 + k];
                else if (tlo[t * 3 + k] > bhi[b * 3 + k]) gap = tlo[t * 3 + k] - bhi[b * 3 + k];
                dmin2 += gap * gap;
            }
            lnU[b] = log(bnu[b]) + (bpsi[b] - cost_scale * dmin2) / eps;
            if (lnU[b] > ubest) { ubest = lnU[b]; bstar = b; }
        }
        /* reference target in B*: largest lower bound over the tile box */
        double lnL = -INFINITY;
        for (int64_t j = 0; j < n; ++j) {
            if (block_of[j] != bstar) continue;
            double dmax2 = 0.0;
            for (int k = 0; k < d; ++k) {
                double a = fabs(y[j * d + k] - tlo[t * 3 + k]);
                double c = fabs(y[j * d + k] - thi[t * 3 + k]);
                double m = a > c ? a : c;
                dmax2 += m * m;
            }
            double lb = log(nu[j]) + (psi[j] - cost_scale * dmax2) / eps;
            if (lb > lnL) lnL = lb;
        }
        for (int64_t b = 0; b < n_blocks; ++b) {
            if (!(bnu[b] > 0.0)) continue;
            int skip = (b != bstar) && (lnU[b] <= lnL + ln_eta_over_nb);
            keep[t * n_blocks + b] = (uint8_t)!skip;
        }
        free(lnU);
    }

    /* evaluation over kept pairs */
    double *lognu = (double *)malloc(sizeof(double) * (size_t)n);
    double *gpart = (double *)calloc((size_t)T * (size_t)n, sizeof(double));
    double *Jpart = (double *)calloc((size_t)T, sizeof(double));
    int64_t *kpart = (int64_t *)calloc((size_t)T, sizeof(int64_t));
    for (int64_t j = 0; j < n; ++j) lognu[j] = log(nu[j]);
#pragma omp parallel num_threads(T)
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        double *z = (double *)malloc(sizeof(double) * (size_t)n);
        char *in = (char *)malloc((size_t)n);
        double *g = gpart + (size_t)tid * (size_t)n;
        double Jt = 0.0;
        int64_t kt = 0;
#pragma omp for schedule(static)
        for (int64_t q = 0; q < nq; ++q) {
            const uint8_t *row = keep + (size_t)tile_of[q] * (size_t)n_blocks;
            double zmax = -INFINITY;
            int64_t cnt = 0;
            for (int64_t j = 0; j < n; ++j) {
                in[j] = row[block_of[j]];
                if (!in[j]) continue;
                z[j] = (psi[j] - cost(d, x + q * d, y + j * d, cost_scale)) / eps + lognu[j];
                if (z[j] > zmax) zmax = z[j];
                ++cnt;
            }
            kt += cnt;
            double s = 0.0;
            for (int64_t j = 0; j < n; ++j)
                if (in[j]) s += exp(z[j] - zmax);
            double L = zmax + log(s);
            if (L_out) L_out[q] = L;
            Jt += eps * L * mu[q];
            if (grad_out)
                for (int64_t j = 0; j < n; ++j)
                    if (in[j]) g[j] += mu[q] * exp(z[j] - L);
        }
        Jpart[tid] = Jt;
        kpart[tid] = kt;
        free(z);
        free(in);
    }
    double J = 0.0;
    int64_t kept = 0;
    for (int t = 0; t < T; ++t) { J += Jpart[t]; kept += kpart[t]; }
    for (int64_t j = 0; j < n; ++j) J -= psi[j] * nu[j];
    if (grad_out)
        for (int64_t j = 0; j < n; ++j) {
            double s = 0.0;
            for (int t = 0; t < T; ++t) s += gpart[(size_t)t * (size_t)n + j];
            grad_out[j] = s - nu[j];
        }
    *J_out = J;
    if (kept_out) *kept_out = kept;
    if (keep_out) memcpy(keep_out, keep, (size_t)n_tiles * (size_t)n_blocks);
    free(tlo); free(thi); free(blo); free(bhi); free(bpsi); free(bnu); free(keep);
    free(lognu); free(gpart); free(Jpart); free(kpart);
    return 0;
}

/*
 * Pair membership shared by the plan-moment and map functions: all pairs; or
 * (keep != NULL) the pairs whose (tile_of[q], block_of[j]) entry of the
 * row-major n_tiles x n_blocks keep matrix is nonzero (the tile rule); and,
 * with a finite cutoff > 0, only pairs with c_qj < cutoff (Sec. 4.1).
 */
static int pair_kept(const uint8_t *keep, const int32_t *tile_of, const int32_t *block_of,
                     int64_t n_blocks, int64_t q, int64_t j, double c, double cutoff)
{
    if (cutoff > 0.0 && isfinite(cutoff) && !(c < cutoff)) return 0;
    if (!keep) return 1;
    return keep[(int64_t)tile_of[q] * n_blocks + block_of[j]] != 0;
}

/*
 * Moments of the plan pi_qj = mu_q p_qj(psi) over the targets (Sec. 6.2):
 *   mass_out[j]       = sum_q mu_q p_qj                 (= nu~_j, Eq. discretized_gradient)
 *   first_out[j*d+k]  = sum_q mu_q p_qj x_q[k]          (the integral in Eq. barycenter_fixed_point;
 *                                                        T_j = first_j / nu_j)
 * with p_qj = nu_j exp((psi_j - c_qj)/eps) / S_q over the kept pairs. Plain
 * loops: per point its log-sum-exp, then its weights scattered to the
 * targets; per-thread arrays summed in thread order. Either output may be NULL.
 */
int oracle_plan_moments(int d, int64_t nq, const double *x, const double *mu,
                        int64_t n, const double *y, const double *nu,
                        const double *psi, double eps, double cost_scale,
                        const int32_t *tile_of, const int32_t *block_of,
                        int64_t n_blocks, const uint8_t *keep, double cutoff, int nthreads,
                        double *mass_out, double *first_out)
{
    if (d < 1 || nq < 0 || n < 1 || !(eps > 0.0)) return -1;
    const int T = oracle_threads(nthreads);
    const size_t per = (size_t)n * (size_t)(d + 1);
    double *part = (double *)calloc((size_t)T * per, sizeof(double));
    if (!part) return -1;
#pragma omp parallel num_threads(T)
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        double *z = (double *)malloc(sizeof(double) * (size_t)n);
        double *acc = part + (size_t)tid * per;
#pragma omp for schedule(static)
        for (int64_t q = 0; q < nq; ++q) {
            double zmax = -INFINITY;
            for (int64_t j = 0; j < n; ++j) {
                z[j] = -INFINITY;
                const double c = cost(d, x + q * d, y + j * d, cost_scale);
                if (!pair_kept(keep, tile_of, block_of, n_blocks, q, j, c, cutoff)) continue;
                z[j] = (psi[j] - c) / eps + log(nu[j]);
                if (z[j] > zmax) zmax = z[j];
            }
            if (!(zmax > -INFINITY)) continue;
            double s = 0.0;
            for (int64_t j = 0; j < n; ++j) s += exp(z[j] - zmax);
            const double L = zmax + log(s);
            for (int64_t j = 0; j < n; ++j) {
                if (!(z[j] > -INFINITY)) continue;
                const double w = mu[q] * exp(z[j] - L);
                acc[j * (d + 1)] += w;
                for (int k = 0; k < d; ++k) acc[j * (d + 1) + 1 + k] += w * x[q * d + k];
            }
        }
        free(z);
    }
    for (int64_t j = 0; j < n; ++j) {
        double m = 0.0, f[3] = {0.0, 0.0, 0.0};
        for (int t = 0; t < T; ++t) {
            const double *a = part + (size_t)t * per + (size_t)j * (d + 1);
            m += a[0];
            for (int k = 0; k < d && k < 3; ++k) f[k] += a[1 + k];
        }
        if (mass_out) mass_out[j] = m;
        if (first_out)
            for (int k = 0; k < d && k < 3; ++k) first_out[j * d + k] = f[k];
    }
    free(part);
    return 0;
}

/*
 * Transport maps of the plan (Sec. 6.3), per quadrature point:
 *   bary_out[q*d+k] = sum_j p_qj y_j[k]               (Eq. barycentric_map_registration)
 *   modal_out[q]    = argmax_j (psi_j - c_qj + eps ln nu_j)   (Eq. modal_map_registration;
 *                     the lowest index on ties; -1 for a point with no kept pair)
 *   val_out[q]      = that maximum (may be NULL)
 * over the kept pairs. Either output may be NULL.
 */
int oracle_transport_maps(int d, int64_t nq, const double *x, int64_t n, const double *y,
                          const double *nu, const double *psi, double eps,
                          double cost_scale, const int32_t *tile_of,
                          const int32_t *block_of, int64_t n_blocks,
                          const uint8_t *keep, double cutoff, int nthreads, double *bary_out,
                          int32_t *modal_out, double *val_out)
{
    if (d < 1 || nq < 0 || n < 1 || !(eps > 0.0) || d > 3) return -1;
    const int T = oracle_threads(nthreads);
#pragma omp parallel num_threads(T)
    {
        double *z = (double *)malloc(sizeof(double) * (size_t)n);
#pragma omp for schedule(static)
        for (int64_t q = 0; q < nq; ++q) {
            double zmax = -INFINITY, vmax = -INFINITY;
            int64_t jbest = -1;
            for (int64_t j = 0; j < n; ++j) {
                z[j] = -INFINITY;
                const double c = cost(d, x + q * d, y + j * d, cost_scale);
                if (!pair_kept(keep, tile_of, block_of, n_blocks, q, j, c, cutoff)) continue;
                z[j] = (psi[j] - c) / eps + log(nu[j]);
                if (z[j] > zmax) zmax = z[j];
                const double v = psi[j] - c + eps * log(nu[j]);
                if (v > vmax) {
                    vmax = v;
                    jbest = j;
                }
            }
            if (modal_out) modal_out[q] = (int32_t)jbest;
            if (val_out) val_out[q] = vmax;
            if (!bary_out) continue;
            double s = 0.0, b[3] = {0.0, 0.0, 0.0};
            if (zmax > -INFINITY)
                for (int64_t j = 0; j < n; ++j) {
                    if (!(z[j] > -INFINITY)) continue;
                    const double w = exp(z[j] - zmax);
                    s += w;
                    for (int k = 0; k < d; ++k) b[k] += w * y[j * d + k];
                }
            for (int k = 0; k < d; ++k) bary_out[q * d + k] = s > 0.0 ? b[k] / s : NAN;
        }
        free(z);
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Squared geodesic cost on the unit sphere (Sec. 6.4, Algs. 4-5)           */
/* ------------------------------------------------------------------------ */

/* c(x, y) = cost_scale * d_g(x, y)^2, d_g = arccos(x . y) for unit vectors
 * (the great-circle distance; Sec. 6.4 uses c = d_g^2) */
static double sphere_angle(const double *x, const double *y)
{
    double t = x[0] * y[0] + x[1] * y[1] + x[2] * y[2];
    if (t > 1.0) t = 1.0;
    if (t < -1.0) t = -1.0;
    return acos(t);
}

static double sphere_cost(const double *x, const double *y, double cost_scale)
{
    double a = sphere_angle(x, y);
    return cost_scale * a * a;
}

/*
 * Dual objective and gradient with the squared geodesic cost on the unit
 * sphere, dense (Eqs. discretized_functional, discretized_gradient with
 * c = cost_scale d_g^2). x: nq x 3 unit vectors, y: n x 3 unit vectors; the
 * rest as oracle_dual_eval.
 */
int oracle_dual_eval_sphere(int64_t nq, const double *x, const double *mu, int64_t n,
                            const double *y, const double *nu, const double *psi,
                            double eps, double cost_scale, int nthreads, double *J_out,
                            double *grad_out, double *L_out)
{
    if (nq < 0 || n < 1 || !(eps > 0.0)) return -1;
    const int T = oracle_threads(nthreads);
    double *gpart = (double *)calloc((size_t)T * (size_t)n, sizeof(double));
    double *Jpart = (double *)calloc((size_t)T, sizeof(double));
    if (!gpart || !Jpart) { free(gpart); free(Jpart); return -1; }
#pragma omp parallel num_threads(T)
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        double *z = (double *)malloc(sizeof(double) * (size_t)n);
        double *g = gpart + (size_t)tid * (size_t)n;
        double Jt = 0.0;
#pragma omp for schedule(static)
        for (int64_t q = 0; q < nq; ++q) {
            double zmax = -INFINITY;
            for (int64_t j = 0; j < n; ++j) {
                z[j] = (psi[j] - sphere_cost(x + q * 3, y + j * 3, cost_scale)) / eps + log(nu[j]);
                if (z[j] > zmax) zmax = z[j];
            }
            double s = 0.0;
            for (int64_t j = 0; j < n; ++j) s += exp(z[j] - zmax);
            double L = zmax + log(s);
            if (L_out) L_out[q] = L;
            Jt += eps * L * mu[q];
            if (grad_out)
                for (int64_t j = 0; j < n; ++j) g[j] += mu[q] * exp(z[j] - L);
        }
        Jpart[tid] = Jt;
        free(z);
    }
    double J = 0.0;
    for (int t = 0; t < T; ++t) J += Jpart[t];
    for (int64_t j = 0; j < n; ++j) J -= psi[j] * nu[j];
    if (grad_out)
        for (int64_t j = 0; j < n; ++j) {
            double s = 0.0;
            for (int t = 0; t < T; ++t) s += gpart[(size_t)t * (size_t)n + j];
            grad_out[j] = s - nu[j];
        }
    *J_out = J;
    free(gpart); free(Jpart);
    return 0;
}

/* geodesic length of a chord of Euclidean length d on the unit sphere */
static double chord_to_angle(double d)
{
    double h = 0.5 * d;
    if (h > 1.0) h = 1.0;
    return 2.0 * asin(h);
}

/*
 * The tile rule of oracle_dual_eval_tile with the squared geodesic cost. The
 * boxes are axis-aligned boxes of the unit vectors in R^3; the geodesic
 * distance increases with the chord, so the least chord between two boxes
 * gives a lower bound of the cost, cost_scale (2 asin(dmin / 2))^2, and the
 * largest chord from a target to a tile box an upper bound. Everything else
 * (U_TB, B*, L_T, the threshold ln L_T + ln(eta / n_blocks)) as there.
 */
int oracle_dual_eval_tile_sphere(int64_t nq, const double *x, const double *mu, int64_t n,
                                 const double *y, const double *nu, const double *psi,
                                 double eps, double cost_scale, const int32_t *tile_of,
                                 int64_t n_tiles, const int32_t *block_of, int64_t n_blocks,
                                 double tau, double absJ_ref, int nthreads, double *J_out,
                                 double *grad_out, double *L_out, int64_t *kept_out,
                                 uint8_t *keep_out)
{
    if (n_tiles < 1 || n_blocks < 1 || n < 1 || !(eps > 0.0)) return -1;
    double *tlo = (double *)malloc(sizeof(double) * (size_t)n_tiles * 3);
    double *thi = (double *)malloc(sizeof(double) * (size_t)n_tiles * 3);
    double *blo = (double *)malloc(sizeof(double) * (size_t)n_blocks * 3);
    double *bhi = (double *)malloc(sizeof(double) * (size_t)n_blocks * 3);
    double *bpsi = (double *)malloc(sizeof(double) * (size_t)n_blocks);
    double *bnu = (double *)malloc(sizeof(double) * (size_t)n_blocks);
    uint8_t *keep = (uint8_t *)calloc((size_t)n_tiles * (size_t)n_blocks, 1);
    if (!tlo || !thi || !blo || !bhi || !bpsi || !bnu || !keep) return -1;
    double summu = 0.0;
    for (int64_t q = 0; q < nq; ++q) summu += mu[q];
    for (int64_t t = 0; t < n_tiles * 3; ++t) { tlo[t] = INFINITY; thi[t] = -INFINITY; }
    for (int64_t b = 0; b < n_blocks * 3; ++b) { blo[b] = INFINITY; bhi[b] = -INFINITY; }
    for (int64_t b = 0; b < n_blocks; ++b) { bpsi[b] = -INFINITY; bnu[b] = 0.0; }
    for (int64_t q = 0; q < nq; ++q) {
        int64_t t = tile_of[q];
        for (int k = 0; k < 3; ++k) {
            double v = x[q * 3 + k];
            if (v < tlo[t * 3 + k]) tlo[t * 3 + k] = v;
            if (v > thi[t * 3 + k]) thi[t * 3 + k] = v;
        }
    }
    for (int64_t j = 0; j < n; ++j) {
        int64_t b = block_of[j];
        for (int k = 0; k < 3; ++k) {
            double v = y[j * 3 + k];
            if (v < blo[b * 3 + k]) blo[b * 3 + k] = v;
            if (v > bhi[b * 3 + k]) bhi[b * 3 + k] = v;
        }
        if (psi[j] > bpsi[b]) bpsi[b] = psi[j];
        bnu[b] += nu[j];
    }
    const double ln_eta_over_nb = log(tau * absJ_ref / (eps * summu)) - log((double)n_blocks);
    const int T = oracle_threads(nthreads);
#pragma omp parallel for num_threads(T) schedule(static)
    for (int64_t t = 0; t < n_tiles; ++t) {
        if (!(tlo[t * 3] <= thi[t * 3])) continue;
        int64_t bstar = -1;
        double ubest = -INFINITY;
        double *lnU = (double *)malloc(sizeof(double) * (size_t)n_blocks);
        for (int64_t b = 0; b < n_blocks; ++b) {
            lnU[b] = -INFINITY;
            if (!(bnu[b] > 0.0)) continue;
            double dmin2 = 0.0;
            for (int k = 0; k < 3; ++k) {
                double gap = 0.0;
                if (blo[b * 3 + k] > thi[t * 3 + k]) gap = blo[b * 3 + k] - thi[t * 3 + k];
                else if (tlo[t * 3 + k] > bhi[b * 3 + k]) gap = tlo[t * 3 + k] - bhi[b * 3 + k];
                dmin2 += gap * gap;
            }
            double a = chord_to_angle(sqrt(dmin2));
            lnU[b] = log(bnu[b]) + (bpsi[b] - cost_scale * a * a) / eps;
            if (lnU[b] > ubest) { ubest = lnU[b]; bstar = b; }
        }
        double lnL = -INFINITY;
        for (int64_t j = 0; j < n; ++j) {
            if (block_of[j] != bstar) continue;
            double dmax2 = 0.0;
            for (int k = 0; k < 3; ++k) {
                double a = fabs(y[j * 3 + k] - tlo[t * 3 + k]);
                double c = fabs(y[j * 3 + k] - thi[t * 3 + k]);
                double m = a > c ? a : c;
                dmax2 += m * m;
            }
            double a = chord_to_angle(sqrt(dmax2));
            double lb = log(nu[j]) + (psi[j] - cost_scale * a * a) / eps;
            if (lb > lnL) lnL = lb;
        }
        for (int64_t b = 0; b < n_blocks; ++b) {
            if (!(bnu[b] > 0.0)) continue;
            int skip = (b != bstar) && (lnU[b] <= lnL + ln_eta_over_nb);
            keep[t * n_blocks + b] = (uint8_t)!skip;
        }
        free(lnU);
    }
    double *gpart = (double *)calloc((size_t)T * (size_t)n, sizeof(double));
    double *Jpart = (double *)calloc((size_t)T, sizeof(double));
    int64_t *kpart = (int64_t *)calloc((size_t)T, sizeof(int64_t));
#pragma omp parallel num_threads(T)
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        double *z = (double *)malloc(sizeof(double) * (size_t)n);
        char *in = (char *)malloc((size_t)n);
        double *g = gpart + (size_t)tid * (size_t)n;
        double Jt = 0.0;
        int64_t kt = 0;
#pragma omp for schedule(static)
        for (int64_t q = 0; q < nq; ++q) {
            const uint8_t *row = keep + (size_t)tile_of[q] * (size_t)n_blocks;
            double zmax = -INFINITY;
            for (int64_t j = 0; j < n; ++j) {
                in[j] = row[block_of[j]];
                if (!in[j]) continue;
                z[j] = (psi[j] - sphere_cost(x + q * 3, y + j * 3, cost_scale)) / eps + log(nu[j]);
                if (z[j] > zmax) zmax = z[j];
                ++kt;
            }
            double s = 0.0;
            for (int64_t j = 0; j < n; ++j)
                if (in[j]) s += exp(z[j] - zmax);
            double L = zmax + log(s);
            if (L_out) L_out[q] = L;
            Jt += eps * L * mu[q];
            if (grad_out)
                for (int64_t j = 0; j < n; ++j)
                    if (in[j]) g[j] += mu[q] * exp(z[j] - L);
        }
        Jpart[tid] = Jt;
        kpart[tid] = kt;
        free(z);
        free(in);
    }
    double J = 0.0;
    int64_t kept = 0;
    for (int t = 0; t < T; ++t) { J += Jpart[t]; kept += kpart[t]; }
    for (int64_t j = 0; j < n; ++j) J -= psi[j] * nu[j];
    if (grad_out)
        for (int64_t j = 0; j < n; ++j) {
            double s = 0.0;
            for (int t = 0; t < T; ++t) s += gpart[(size_t)t * (size_t)n + j];
            grad_out[j] = s - nu[j];
        }
    *J_out = J;
    if (kept_out) *kept_out = kept;
    if (keep_out) memcpy(keep_out, keep, (size_t)n_tiles * (size_t)n_blocks);
    free(tlo); free(thi); free(blo); free(bhi); free(bpsi); free(bnu); free(keep);
    free(gpart); free(Jpart); free(kpart);
    return 0;
}

/*
 * One step of the Riemannian barycentre iteration (Alg. 5) for every target,
 * with the conditional measures mu_j(x | psi) of the plan at (psi, y_plan)
 * held fixed (Alg. 4 computes them once per Lloyd iteration):
 *   w_qj   = mu_q p_qj(psi, y_plan)                 (the plan, Eq. final_plan_density)
 *   log_y(x) = theta / sin(theta) (x - cos(theta) y),  theta = d_g(x, y)
 *   delta_j = -2 sum_q w_qj log_{y_j}(x_q) / sum_q w_qj     (gradient of the
 *             expected squared distance on the tangent space at y_j)
 *   y_next_j = exp_{y_j}(-alpha delta_j),  exp_y(v) = cos|v| y + sin|v| v / |v|
 * at the current points y_cur. Outputs y_next (n x 3), step_norm[j] = |delta_j|,
 * mass_out[j] = sum_q w_qj (may be NULL). A target with no mass keeps its point.
 */
int oracle_sphere_karcher_step(int64_t nq, const double *x, const double *mu, int64_t n,
                               const double *y_plan, const double *nu, const double *psi,
                               double eps, double cost_scale, const double *y_cur,
                               double alpha, int nthreads, double *y_next,
                               double *step_norm, double *mass_out)
{
    if (nq < 0 || n < 1 || !(eps > 0.0)) return -1;
    const int T = oracle_threads(nthreads);
    double *acc = (double *)calloc((size_t)T * (size_t)n * 4, sizeof(double));
    if (!acc) return -1;
#pragma omp parallel num_threads(T)
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        double *z = (double *)malloc(sizeof(double) * (size_t)n);
        double *a = acc + (size_t)tid * (size_t)n * 4;
#pragma omp for schedule(static)
        for (int64_t q = 0; q < nq; ++q) {
            const double *xq = x + q * 3;
            double zmax = -INFINITY;
            for (int64_t j = 0; j < n; ++j) {
                z[j] = (psi[j] - sphere_cost(xq, y_plan + j * 3, cost_scale)) / eps + log(nu[j]);
                if (z[j] > zmax) zmax = z[j];
            }
            double s = 0.0;
            for (int64_t j = 0; j < n; ++j) s += exp(z[j] - zmax);
            const double L = zmax + log(s);
            for (int64_t j = 0; j < n; ++j) {
                const double w = mu[q] * exp(z[j] - L);
                const double *yc = y_cur + j * 3;
                const double th = sphere_angle(xq, yc);
                const double ct = cos(th);
                const double f = th > 0.0 ? th / sin(th) : 1.0;
                for (int k = 0; k < 3; ++k) a[j * 4 + k] += w * f * (xq[k] - ct * yc[k]);
                a[j * 4 + 3] += w;
            }
        }
        free(z);
    }
    for (int64_t j = 0; j < n; ++j) {
        double lg[3] = {0.0, 0.0, 0.0}, m = 0.0;
        for (int t = 0; t < T; ++t) {
            const double *a = acc + ((size_t)t * (size_t)n + (size_t)j) * 4;
            for (int k = 0; k < 3; ++k) lg[k] += a[k];
            m += a[3];
        }
        const double *yc = y_cur + j * 3;
        double v[3] = {0.0, 0.0, 0.0};
        if (m > 0.0)
            for (int k = 0; k < 3; ++k) v[k] = -alpha * (-2.0 * lg[k] / m);
        const double nv = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
        for (int k = 0; k < 3; ++k)
            y_next[j * 3 + k] = nv > 0.0 ? cos(nv) * yc[k] + sin(nv) * v[k] / nv : yc[k];
        step_norm[j] = alpha > 0.0 ? nv / alpha : 0.0;
        if (mass_out) mass_out[j] = m;
    }
    free(acc);
    return 0;
}
