/* Driver for the sanitizer run of the CPU oracle (test infrastructure): every
 * entry point on small ragged inputs in 2D and 3D, dense and truncated; prints
 * a checksum line per call. Built and run by tests/test_oracle_sanitized.py
 * with AddressSanitizer and UndefinedBehaviorSanitizer. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int oracle_dual_eval(int d, int64_t nq, const double *x, const double *mu, int64_t n,
                     const double *y, const double *nu, const double *psi, double eps,
                     double cost_scale, double cutoff, int nthreads, double *J_out,
                     double *grad_out, double *L_out, int64_t *kept_out, int64_t *nempty_out);
double oracle_covering_cost(int d, int64_t nq, const double *x, int64_t n, const double *y,
                            double cost_scale, int nthreads);
int oracle_kept_counts(int d, int64_t nq, const double *x, int64_t n, const double *y,
                       double cost_scale, double cutoff, double rel_band, int nthreads,
                       int32_t *kept_out, int32_t *near_out);
int oracle_plan_moments(int d, int64_t nq, const double *x, const double *mu, int64_t n,
                        const double *y, const double *nu, const double *psi, double eps,
                        double cost_scale, const int32_t *tile_of, const int32_t *block_of,
                        int64_t n_blocks, const uint8_t *keep, double cutoff, int nthreads,
                        double *mass_out, double *first_out);
int oracle_transport_maps(int d, int64_t nq, const double *x, int64_t n, const double *y,
                          const double *nu, const double *psi, double eps, double cost_scale,
                          const int32_t *tile_of, const int32_t *block_of, int64_t n_blocks,
                          const uint8_t *keep, double cutoff, int nthreads, double *bary_out,
                          int32_t *modal_out, double *val_out);
double oracle_cutoff_geom(double C0, double M, double m, double nu_min, double tau,
                          double absJ, double eps);
double oracle_cutoff_int(double C0, double M, double D, double tau, double absJ, double eps);
double oracle_cutoff_pw(double M, double nu_max, double delta_thr, double eps);
double oracle_integral_D(int64_t nq, const double *mu, const double *L);
int oracle_softmax_refine(int d, int64_t nq, const double *x, const double *mu, const double *L,
                          int64_t nf, const double *yf, double eps, double cost_scale,
                          int nthreads, double *psi_out);
int oracle_dual_eval_tile(int d, int64_t nq, const double *x, const double *mu, int64_t n,
                          const double *y, const double *nu, const double *psi, double eps,
                          double cost_scale, const int32_t *tile_of, int64_t n_tiles,
                          const int32_t *block_of, int64_t n_blocks, double tau,
                          double absJ_ref, int nthreads, double *J_out, double *grad_out,
                          double *L_out, int64_t *kept_out, uint8_t *keep_out);

static uint64_t state = 88172645463325252ull;
static double unif(void) {  /* xorshift64 */
    state ^= state << 13;
    state ^= state >> 7;
    state ^= state << 17;
    return (double)(state >> 11) * (1.0 / 9007199254740992.0);
}

static double *alloc_fill(int64_t n, double lo, double hi) {
    double *a = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i) a[i] = lo + (hi - lo) * unif();
    return a;
}

static void run(int d, int64_t nq, int64_t n, double eps) {
    double *x = alloc_fill(nq * d, 0.0, 1.0), *mu = alloc_fill(nq, 0.5, 1.5);
    double *y = alloc_fill(n * d, -0.1, 1.1), *nu = alloc_fill(n, 0.5, 1.5);
    double *psi = alloc_fill(n, -0.02, 0.02);
    double sm = 0.0, sn = 0.0, M = -INFINITY, m = INFINITY, numin = INFINITY, numax = 0.0;
    for (int64_t q = 0; q < nq; ++q) sm += mu[q];
    for (int64_t j = 0; j < n; ++j) sn += nu[j];
    for (int64_t q = 0; q < nq; ++q) mu[q] /= sm;
    for (int64_t j = 0; j < n; ++j) {
        nu[j] /= sn;
        M = fmax(M, psi[j]);
        m = fmin(m, psi[j]);
        numin = fmin(numin, nu[j]);
        numax = fmax(numax, nu[j]);
    }
    double J = 0.0, *g = alloc_fill(n, 0, 0), *L = alloc_fill(nq, 0, 0);
    int64_t kept = 0, nempty = 0;
    int rc = oracle_dual_eval(d, nq, x, mu, n, y, nu, psi, eps, 0.5, INFINITY, 3, &J, g, L, &kept,
                              &nempty);
    double gs = 0.0;
    for (int64_t j = 0; j < n; ++j) gs += g[j];
    printf("dense d=%d nq=%ld n=%ld rc=%d J=%.15e sum_g=%.3e kept=%ld\n", d, (long)nq, (long)n,
           rc, J, gs, (long)kept);
    const double C0 = oracle_covering_cost(d, nq, x, n, y, 0.5, 2);
    const double Cg = oracle_cutoff_geom(C0, M, m, numin, 1e-8, fabs(J), eps);
    const double D = oracle_integral_D(nq, mu, L);
    const double Ci = oracle_cutoff_int(C0, M, D, 1e-8, fabs(J), eps);
    const double Cp = oracle_cutoff_pw(M, numax, 1e-6, eps);
    const double cuts[3] = {Cg, Ci, Cp};
    for (int k = 0; k < 3; ++k) {
        double Jt = 0.0;
        rc = oracle_dual_eval(d, nq, x, mu, n, y, nu, psi, eps, 0.5, cuts[k], 2, &Jt, g, L, &kept,
                              &nempty);
        printf("cut %d C=%.6e rc=%d J=%.15e kept=%ld empty=%ld\n", k, cuts[k], rc, Jt,
               (long)kept, (long)nempty);
    }
    /* tile rule on a ragged partition: tiles of 5 points, blocks of 3 targets */
    const int64_t nt = (nq + 4) / 5, nb = (n + 2) / 3;
    int32_t *tof = (int32_t *)malloc(sizeof(int32_t) * (size_t)nq);
    int32_t *bof = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    for (int64_t q = 0; q < nq; ++q) tof[q] = (int32_t)(q / 5);
    for (int64_t j = 0; j < n; ++j) bof[j] = (int32_t)(j / 3);
    uint8_t *keep = (uint8_t *)malloc((size_t)(nt * nb));
    double Jtile = 0.0;
    rc = oracle_dual_eval_tile(d, nq, x, mu, n, y, nu, psi, eps, 0.5, tof, nt, bof, nb, 1e-10,
                               fabs(J), 2, &Jtile, g, L, &kept, keep);
    printf("tile rc=%d J=%.15e kept=%ld\n", rc, Jtile, (long)kept);
    /* kept-set sizes at a cutoff */
    int32_t *kq = (int32_t *)malloc(sizeof(int32_t) * (size_t)nq);
    int32_t *nr = (int32_t *)malloc(sizeof(int32_t) * (size_t)nq);
    rc = oracle_kept_counts(d, nq, x, n, y, 0.5, 0.05, 1e-12, 2, kq, nr);
    long ks = 0;
    for (int64_t q = 0; q < nq; ++q) ks += kq[q] + nr[q];
    printf("counts rc=%d sum=%ld\n", rc, ks);
    free(kq); free(nr);
    /* plan moments and maps, dense and over the tile rule's kept pairs */
    double *mass = alloc_fill(n, 0, 0), *first = alloc_fill(n * d, 0, 0);
    double *bary = alloc_fill(nq * d, 0, 0), *mval = alloc_fill(nq, 0, 0);
    int32_t *modal = (int32_t *)malloc(sizeof(int32_t) * (size_t)nq);
    for (int pass = 0; pass < 2; ++pass) {
        const uint8_t *kp = pass ? keep : NULL;
        rc = oracle_plan_moments(d, nq, x, mu, n, y, nu, psi, eps, 0.5, tof, bof, nb, kp,
                                 pass ? 0.05 : INFINITY, 2, mass, first);
        printf("moments rc=%d mass0=%.15e\n", rc, mass[0]);
        rc = oracle_transport_maps(d, nq, x, n, y, nu, psi, eps, 0.5, tof, bof, nb, kp,
                                   pass ? 0.05 : INFINITY, 2, bary, modal, mval);
        printf("maps rc=%d modal0=%d\n", rc, (int)modal[0]);
    }
    free(mass); free(first); free(bary); free(mval); free(modal);
    /* softmax refinement onto 7 fine targets */
    double *yf = alloc_fill(7 * d, 0.0, 1.0), *pf = alloc_fill(7, 0, 0);
    oracle_dual_eval(d, nq, x, mu, n, y, nu, psi, eps, 0.5, INFINITY, 1, &J, NULL, L, &kept,
                     &nempty);
    rc = oracle_softmax_refine(d, nq, x, mu, L, 7, yf, eps, 0.5, 2, pf);
    printf("refine rc=%d psi0=%.15e\n", rc, pf[0]);
    free(x); free(mu); free(y); free(nu); free(psi); free(g); free(L);
    free(tof); free(bof); free(keep); free(yf); free(pf);
}

int oracle_dual_eval_sphere(int64_t nq, const double *x, const double *mu, int64_t n,
                            const double *y, const double *nu, const double *psi, double eps,
                            double cost_scale, int nthreads, double *J_out, double *grad_out,
                            double *L_out);
int oracle_dual_eval_tile_sphere(int64_t nq, const double *x, const double *mu, int64_t n,
                                 const double *y, const double *nu, const double *psi,
                                 double eps, double cost_scale, const int32_t *tile_of,
                                 int64_t n_tiles, const int32_t *block_of, int64_t n_blocks,
                                 double tau, double absJ_ref, int nthreads, double *J_out,
                                 double *grad_out, double *L_out, int64_t *kept_out,
                                 uint8_t *keep_out);
int oracle_sphere_karcher_step(int64_t nq, const double *x, const double *mu, int64_t n,
                               const double *y_plan, const double *nu, const double *psi,
                               double eps, double cost_scale, const double *y_cur,
                               double alpha, int nthreads, double *y_next, double *step_norm,
                               double *mass_out);

/* unit vectors for the sphere functions */
static void normalise_rows(double *v, int64_t n)
{
    for (int64_t i = 0; i < n; ++i) {
        double s = sqrt(v[i * 3] * v[i * 3] + v[i * 3 + 1] * v[i * 3 + 1] + v[i * 3 + 2] * v[i * 3 + 2]);
        for (int k = 0; k < 3; ++k) v[i * 3 + k] /= s;
    }
}

static void run_sphere(int64_t nq, int64_t n, double eps)
{
    double *x = alloc_fill(nq * 3, -1.0, 1.0), *y = alloc_fill(n * 3, -1.0, 1.0);
    normalise_rows(x, nq);
    normalise_rows(y, n);
    double *mu = alloc_fill(nq, 0.5, 1.5), *nu = alloc_fill(n, 0.5, 1.5);
    double *psi = alloc_fill(n, -eps, eps), *g = alloc_fill(n, 0, 0), *L = alloc_fill(nq, 0, 0);
    double J = 0.0;
    int rc = oracle_dual_eval_sphere(nq, x, mu, n, y, nu, psi, eps, 1.0, 2, &J, g, L);
    printf("sphere rc=%d J=%.15e\n", rc, J);
    int64_t nt = (nq + 7) / 8, nb = (n + 3) / 4, kept = 0;
    int32_t *tof = (int32_t *)malloc(sizeof(int32_t) * (size_t)nq);
    int32_t *bof = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    for (int64_t q = 0; q < nq; ++q) tof[q] = (int32_t)(q / 8);
    for (int64_t j = 0; j < n; ++j) bof[j] = (int32_t)(j / 4);
    uint8_t *keep = (uint8_t *)malloc((size_t)(nt * nb));
    double Jt = 0.0;
    rc = oracle_dual_eval_tile_sphere(nq, x, mu, n, y, nu, psi, eps, 1.0, tof, nt, bof, nb, 1e-8,
                                      fabs(J), 2, &Jt, g, L, &kept, keep);
    printf("sphere tile rc=%d J=%.15e kept=%ld\n", rc, Jt, (long)kept);
    double *yn = alloc_fill(n * 3, 0, 0), *st = alloc_fill(n, 0, 0), *ms = alloc_fill(n, 0, 0);
    rc = oracle_sphere_karcher_step(nq, x, mu, n, y, nu, psi, eps, 1.0, y, 0.5, 2, yn, st, ms);
    printf("karcher rc=%d y0=%.15e step0=%.15e\n", rc, yn[0], st[0]);
    free(x); free(y); free(mu); free(nu); free(psi); free(g); free(L); free(tof); free(bof);
    free(keep); free(yn); free(st); free(ms);
}

int main(void) {
    run_sphere(37, 11, 0.05);
    run_sphere(1, 1, 0.1);
    run(2, 37, 11, 0.03);
    run(3, 29, 17, 0.05);
    run(2, 1, 1, 0.1);
    run(3, 64, 65, 0.01);
    return 0;
}
