// Combined multilevel solve (Sec. 5.3) with an eps schedule (Sec. 4.2).
//
// Source levels T_0..T_Lmu (coarsest first) and target levels nu^(0)..nu^(Lnu)
// are copied into library memory at creation. Step l = 0..Lmax, Lmax =
// max(Lmu, Lnu), solves on (T_is(l), nu^(it(l))) with
//   is(l) = max(0, l - (Lmax - Lmu)),  it(l) = max(0, l - (Lmax - Lnu)).
// Between steps the potential is transferred by softmax refinement (Eq.
// softmax_refinement_formula_combined: coarse targets and potential, current
// source level) when it(l) = it(l-1) + 1, and kept (injection) otherwise.
// Each step runs the eps stages the caller assigns to it, warm-starting each
// from the previous one.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <map>
#include <vector>

#include "rsot_internal.h"

struct rsot_multilevel {
    int dim = 0;
    rsot_options opt{};
    hipStream_t stream = nullptr;
    std::vector<int64_t> nq, nt;
    std::vector<double *> x, mu, y, nu;      // device copies
    std::map<std::pair<int, int>, rsot_problem *> probs;
    ~rsot_multilevel() {
        for (auto &kv : probs) rsot_problem_destroy(kv.second);
        for (double *p : x) (void)hipFree(p);
        for (double *p : mu) (void)hipFree(p);
        for (double *p : y) (void)hipFree(p);
        for (double *p : nu) (void)hipFree(p);
    }
    rsot_status get(int is, int it, rsot_problem **out) {
        auto key = std::make_pair(is, it);
        auto f = probs.find(key);
        if (f != probs.end()) {
            *out = f->second;
            return RSOT_OK;
        }
        rsot_options o = opt;
        o.inputs_on_device = 1;
        // a coarser (source, target) pair only warm-starts the next level and
        // stops at the level tolerance: it keeps the FP32 pair loop whatever
        // its size (the FP64 loop for small problems measured a third slower
        // on the blob family's coarsest level, with the same iterations)
        if (is != (int)nq.size() - 1 || it != (int)nt.size() - 1) o.fp64_below_points = 0;
        rsot_problem *p = nullptr;
        RSOT_TRY(rsot_problem_create(dim, nq[is], x[is], mu[is], nt[it], y[it], nu[it], &o,
                                     stream, &p));
        probs[key] = p;
        *out = p;
        return RSOT_OK;
    }
};

static rsot_status copy_in(const double *src, size_t count, int on_dev, hipStream_t s,
                           double **dst) {
    if (hipMalloc((void **)dst, std::max<size_t>(count, 1) * sizeof(double)) != hipSuccess) {
        (void)hipGetLastError();
        return RSOT_ERR_OOM;
    }
    RSOT_HIP(hipMemcpyAsync(*dst, src, count * sizeof(double),
                            on_dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s));
    return RSOT_OK;
}

extern "C" rsot_status rsot_multilevel_create(int dim, int n_source_levels, const int64_t *n_quad,
                                              const double *const *x, const double *const *mu,
                                              int n_target_levels, const int64_t *n_target,
                                              const double *const *y, const double *const *nu,
                                              const rsot_options *opt, void *hip_stream,
                                              rsot_multilevel **out) {
    if (!out) return RSOT_ERR_INVALID_ARG;
    *out = nullptr;
    if ((dim != 2 && dim != 3) || n_source_levels < 1 || n_target_levels < 1 || !n_quad || !x ||
        !mu || !n_target || !y || !nu || n_source_levels > RSOT_ML_MAX_LEVELS ||
        n_target_levels > RSOT_ML_MAX_LEVELS)
        return RSOT_ERR_INVALID_ARG;
    rsot_options o;
    rsot_options_default(&o);
    if (opt) o = *opt;
    if (o.cost_kind != RSOT_COST_SQEUCLID) return RSOT_ERR_INVALID_ARG;   // refinement is Euclidean
    auto *ml = new (std::nothrow) rsot_multilevel();
    if (!ml) return RSOT_ERR_OOM;
    ml->dim = dim;
    ml->opt = o;
    ml->stream = (hipStream_t)hip_stream;
    rsot_status s = RSOT_OK;
    for (int l = 0; l < n_source_levels && s == RSOT_OK; ++l) {
        if (n_quad[l] <= 0 || !x[l] || !mu[l]) s = RSOT_ERR_INVALID_ARG;
        double *a = nullptr, *b = nullptr;
        if (s == RSOT_OK) s = copy_in(x[l], (size_t)n_quad[l] * dim, o.inputs_on_device, ml->stream, &a);
        if (s == RSOT_OK) s = copy_in(mu[l], (size_t)n_quad[l], o.inputs_on_device, ml->stream, &b);
        ml->x.push_back(a);
        ml->mu.push_back(b);
        ml->nq.push_back(n_quad[l]);
    }
    for (int l = 0; l < n_target_levels && s == RSOT_OK; ++l) {
        if (n_target[l] <= 0 || !y[l] || !nu[l]) s = RSOT_ERR_INVALID_ARG;
        double *a = nullptr, *b = nullptr;
        if (s == RSOT_OK) s = copy_in(y[l], (size_t)n_target[l] * dim, o.inputs_on_device, ml->stream, &a);
        if (s == RSOT_OK) s = copy_in(nu[l], (size_t)n_target[l], o.inputs_on_device, ml->stream, &b);
        ml->y.push_back(a);
        ml->nu.push_back(b);
        ml->nt.push_back(n_target[l]);
    }
    if (s == RSOT_OK && hipStreamSynchronize(ml->stream) != hipSuccess) s = RSOT_ERR_DEVICE;
    if (s != RSOT_OK) {
        delete ml;
        return s;
    }
    *out = ml;
    return RSOT_OK;
}

extern "C" void rsot_multilevel_destroy(rsot_multilevel *ml) { delete ml; }

extern "C" void rsot_multilevel_indices(int n_source_levels, int n_target_levels, int l,
                                        int *is, int *it) {
    const int Lmu = n_source_levels - 1, Lnu = n_target_levels - 1;
    const int Lmax = std::max(Lmu, Lnu);
    if (is) *is = std::max(0, l - (Lmax - Lmu));
    if (it) *it = std::max(0, l - (Lmax - Lnu));
}

extern "C" rsot_status rsot_solve_multilevel(rsot_multilevel *ml, const rsot_ml_params *mp,
                                             double *psi_out, rsot_ml_info *info) {
    if (!ml || !mp || !psi_out || !mp->eps || !mp->level || mp->n_stages < 1)
        return RSOT_ERR_INVALID_ARG;
    if (mp->base.checkpoint || mp->base.resume) return RSOT_ERR_INVALID_ARG;  // per level n differs
    const int ns = (int)ml->nq.size(), nt = (int)ml->nt.size();
    const int Lmax = std::max(ns, nt) - 1;
    for (int k = 0; k < mp->n_stages; ++k) {
        if (mp->level[k] < 0 || mp->level[k] > Lmax) return RSOT_ERR_INVALID_ARG;
        if (k > 0 && mp->level[k] < mp->level[k - 1]) return RSOT_ERR_INVALID_ARG;
        if (!(mp->eps[k] > 0.0)) return RSOT_ERR_INVALID_ARG;
    }
    rsot_ml_info inf{};
    inf.n_steps = Lmax + 1;
    const auto t0 = std::chrono::steady_clock::now();
    auto now = [] { return std::chrono::steady_clock::now(); };
    auto secs = [](std::chrono::steady_clock::time_point a, std::chrono::steady_clock::time_point b) {
        return std::chrono::duration<double>(b - a).count();
    };

    int it_prev = -1, is_prev = -1;
    double eps_prev = mp->eps[0];
    double absJ_prev = 0.0;
    std::vector<double> psi;
    double *d_a = nullptr, *d_b = nullptr;
    rsot_status status = RSOT_OK;
    int stage = 0;
    for (int l = 0; l <= Lmax && status == RSOT_OK; ++l) {
        int is = 0, it = 0;
        rsot_multilevel_indices(ns, nt, l, &is, &it);
        inf.source_level[l] = is;
        inf.target_level[l] = it;
        const auto tr0 = now();
        if (l == 0) {
            psi.assign((size_t)ml->nt[it], 0.0);
        } else if (it == it_prev + 1 && mp->transfer == RSOT_TRANSFER_SOFTMAX) {
            // softmax refinement: previous targets and potential on the current source
            rsot_problem *pr = nullptr;
            status = ml->get(is, it_prev, &pr);
            if (status != RSOT_OK) break;
            (void)hipFree(d_a);
            (void)hipFree(d_b);
            d_a = d_b = nullptr;
            if (hipMalloc((void **)&d_a, sizeof(double) * psi.size()) != hipSuccess ||
                hipMalloc((void **)&d_b, sizeof(double) * ml->nt[it]) != hipSuccess) {
                status = RSOT_ERR_OOM;
                break;
            }
            (void)hipMemcpy(d_a, psi.data(), sizeof(double) * psi.size(), hipMemcpyHostToDevice);
            status = rsot_refine_impl(pr, eps_prev, d_a, ml->nt[it], ml->y[it], 1e-12, d_b);
            if (status != RSOT_OK) break;
            psi.assign((size_t)ml->nt[it], 0.0);
            (void)hipMemcpy(psi.data(), d_b, sizeof(double) * psi.size(), hipMemcpyDeviceToHost);
            inf.refine_pairs[l] = pr->last_refine_pairs;
        } else if (it == it_prev + 1) {
            // injection fallback: the potential of the nearest coarse target
            status = RSOT_ERR_INVALID_ARG;
            break;
        }
        inf.refine_seconds[l] = l > 0 ? secs(tr0, now()) : 0.0;
        (void)is_prev;
        // the eps stages of this level
        std::vector<double> eps_l;
        while (stage < mp->n_stages && mp->level[stage] == l) eps_l.push_back(mp->eps[stage++]);
        const auto ts0 = now();
        if (!eps_l.empty()) {
            rsot_problem *p = nullptr;
            status = ml->get(is, it, &p);
            if (status != RSOT_OK) break;
            rsot_solve_params sp = mp->base;
            sp.eps_schedule = eps_l.data();
            sp.n_eps = (int)eps_l.size();
            // the previous level's final |J| serves as the reference of the
            // truncation rules for this level's warm start (the refined
            // potential), so its first evaluation need not run dense
            if (l > 0 && absJ_prev > 0.0) sp.absJ_start = absJ_prev;
            const bool last = (l == Lmax);
            if (!last && mp->level_tol > 0.0) sp.tol = mp->level_tol;
            rsot_solve_info si{};
            rsot_status s = rsot_solve(p, &sp, psi.data(), &si);
            inf.iterations[l] = si.iterations;
            inf.evaluations[l] = si.evaluations;
            inf.eval_ms[l] = si.eval_ms;
            inf.kept_frac[l] = si.kept_frac;
            inf.grad_l1 = si.grad_l1;
            absJ_prev = std::isfinite(si.J) ? std::fabs(si.J) : 0.0;   // 0: next level starts dense
            // a non-final step that stops short of level_tol (iteration cap or
            // a line search that cannot improve its iterate) still warm-starts
            // the next one; the final step's status is the solve's
            if (s == RSOT_ERR_LINESEARCH && !last) ++inf.stalled_levels;
            else if (s != RSOT_OK && !(s == RSOT_ERR_NOT_CONVERGED && !last)) status = s;
            eps_prev = eps_l.back();
        }
        inf.seconds[l] = secs(ts0, now());
        it_prev = it;
        is_prev = is;
    }
    (void)hipFree(d_a);
    (void)hipFree(d_b);
    inf.total_seconds = secs(t0, now());
    inf.status = status;
    if (info) *info = inf;
    if (!psi.empty() && psi.size() == (size_t)ml->nt.back())
        std::memcpy(psi_out, psi.data(), sizeof(double) * psi.size());
    return status;
}
