// rsot_solve: Alg. 1 (L-BFGS on J with a line search, stop on ||grad||_1,
// Remark 3.2) inside an eps schedule (Sec. 4.2). The paper leaves the L-BFGS
// details open; this file fixes them as: memory m (default 10), initial
// inverse-Hessian scaling s'y / y'y (and eps N / sum nu before the first pair
// exists, the inverse of J's diagonal scale nu_j / eps), strong-Wolfe line
// search (c1 = 1e-4, c2 = 0.9) by bracketing and safeguarded cubic
// interpolation, at most max_ls evaluations per search. Host FP64 vectors;
// every evaluation is one rsot_dual_eval on the device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

#include "rsot_internal.h"

namespace {

double dot(const std::vector<double> &a, const std::vector<double> &b) {
    double s = 0.0;
    const size_t n = a.size();
    for (size_t i = 0; i < n; ++i) s += a[i] * b[i];
    return s;
}

struct Evaluator {
    rsot_problem *p;
    double eps;
    int evals = 0;
    double eval_ms = 0.0, cull_ms = 0.0, p1_ms = 0.0, p2_ms = 0.0, kept = 0.0;
    volatile int *cancel = nullptr;
    rsot_eval_info last{};

    rsot_status operator()(const std::vector<double> &psi, double &J, std::vector<double> &g) {
        if (cancel && *cancel) return RSOT_ERR_CANCELLED;
        const size_t n = psi.size();
        std::memcpy(p->hpsi, psi.data(), n * sizeof(double));
        RSOT_HIP(hipMemcpyAsync(p->dpsi, p->hpsi, n * sizeof(double), hipMemcpyHostToDevice,
                                p->stream));
        RSOT_TRY(rsot_eval_impl(p, eps, p->dpsi, &J, p->dgrad, &last));
        RSOT_HIP(hipMemcpyAsync(p->hgrad, p->dgrad, n * sizeof(double), hipMemcpyDeviceToHost,
                                p->stream));
        RSOT_HIP(hipStreamSynchronize(p->stream));
        std::memcpy(g.data(), p->hgrad, n * sizeof(double));
        ++evals;
        eval_ms += last.kernel_ms;
        cull_ms += last.setup_ms;
        p1_ms += last.pass1_ms;
        p2_ms += last.pass2_ms;
        kept += (double)last.kept_pairs / (double)last.total_pairs;
        return RSOT_OK;
    }
};

// minimiser of the cubic through (a, fa, da), (b, fb, db), kept inside the
// safeguarded interval between a and b
double cubic_step(double a, double fa, double da, double b, double fb, double db) {
    const double lo = std::min(a, b), hi = std::max(a, b);
    const double w = hi - lo;
    double x;
    const double d1 = da + db - 3.0 * (fa - fb) / (a - b);
    const double disc = d1 * d1 - da * db;
    if (disc >= 0.0 && std::isfinite(disc)) {
        double d2 = std::sqrt(disc);
        if (b < a) d2 = -d2;
        x = b - (b - a) * (db + d2 - d1) / (db - da + 2.0 * d2);
        if (!std::isfinite(x)) x = 0.5 * (a + b);
    } else {
        x = 0.5 * (a + b);
    }
    return std::min(std::max(x, lo + 0.1 * w), hi - 0.1 * w);
}

struct Point {
    double alpha, f, d;
    std::vector<double> psi, g;
};

// Strong-Wolfe line search along p (Nocedal & Wright, Algs. 3.5/3.6).
// On success cur holds the accepted point.
rsot_status line_search(Evaluator &ev, const std::vector<double> &psi0, double f0,
                        const std::vector<double> &g0, const std::vector<double> &dir,
                        double alpha1, double c1, double c2, int max_ls, Point &out) {
    const double d0 = dot(g0, dir);
    const size_t n = psi0.size();
    Point prev{0.0, f0, d0, psi0, g0};
    Point cur;
    cur.psi.resize(n);
    cur.g.resize(n);
    auto eval_at = [&](double a, Point &pt) -> rsot_status {
        pt.alpha = a;
        pt.psi.resize(n);
        pt.g.resize(n);
        for (size_t i = 0; i < n; ++i) pt.psi[i] = psi0[i] + a * dir[i];
        RSOT_TRY(ev(pt.psi, pt.f, pt.g));
        pt.d = dot(pt.g, dir);
        return RSOT_OK;
    };
    // f noise allowance of the approximate-Wolfe acceptance: the objective of
    // the mixed path carries ~1e-10 relative noise, the FP64 path ~1e-15
    const double fnoise =
        (ev.p->opt.precision == RSOT_PREC_FP64 ? 1e-13 : 1e-9) * std::fabs(f0);
    auto approx_wolfe = [&](const Point &pt) {
        return pt.f <= f0 + fnoise && pt.d >= c2 * d0 && pt.d <= (2.0 * c1 - 1.0) * d0;
    };
    double a = alpha1;
    int used = 0;
    Point lo, hi;
    bool zoom = false;
    for (int i = 0; i < max_ls; ++i) {
        RSOT_TRY(eval_at(a, cur));
        ++used;
        if (!std::isfinite(cur.f)) {
            a = 0.5 * (prev.alpha + a);
            continue;
        }
        if (cur.f > f0 + c1 * a * d0 || (i > 0 && cur.f >= prev.f)) {
            if (approx_wolfe(cur)) {
                out = cur;
                return RSOT_OK;
            }
            lo = prev;
            hi = cur;
            zoom = true;
            break;
        }
        if (std::fabs(cur.d) <= -c2 * d0) {
            out = cur;
            return RSOT_OK;
        }
        if (cur.d >= 0.0) {
            lo = cur;
            hi = prev;
            zoom = true;
            break;
        }
        prev = cur;
        a *= 2.0;
    }
    if (!zoom) {
        if (prev.alpha > 0.0 && prev.f < f0) {  // still descending: accept the last point
            out = prev;
            return RSOT_OK;
        }
        return RSOT_ERR_LINESEARCH;
    }
    while (used < max_ls) {
        const double at = cubic_step(lo.alpha, lo.f, lo.d, hi.alpha, hi.f, hi.d);
        RSOT_TRY(eval_at(at, cur));
        ++used;
        if (cur.f > f0 + c1 * at * d0 || cur.f >= lo.f) {
            if (approx_wolfe(cur)) {
                out = cur;
                return RSOT_OK;
            }
            hi = cur;
        } else {
            if (std::fabs(cur.d) <= -c2 * d0) {
                out = cur;
                return RSOT_OK;
            }
            if (cur.d * (hi.alpha - lo.alpha) >= 0.0) hi = lo;
            lo = cur;
        }
    }
    if (lo.alpha > 0.0 && lo.f < f0) {  // best bracket end still decreases J
        out = lo;
        return RSOT_OK;
    }
    return RSOT_ERR_LINESEARCH;
}

}  // namespace

extern "C" void rsot_solve_params_default(rsot_solve_params *sp) {
    if (!sp) return;
    std::memset(sp, 0, sizeof(*sp));
    sp->tol = 1e-6;
    sp->max_iter = 10000;
    sp->lbfgs_m = 10;
    sp->c1 = 1e-4;
    sp->c2 = 0.9;
    sp->max_ls = 20;
}

extern "C" rsot_status rsot_solve(rsot_problem *p, const rsot_solve_params *sp_in,
                                  double *psi_inout, rsot_solve_info *info) {
    if (!p || !sp_in || !psi_inout) return RSOT_ERR_INVALID_ARG;
    rsot_solve_params sp = *sp_in;
    if (!sp.eps_schedule || sp.n_eps < 1 || !(sp.tol > 0.0) || sp.max_iter < 1 ||
        sp.lbfgs_m < 1 || !(sp.c1 > 0.0 && sp.c1 < sp.c2 && sp.c2 < 1.0) || sp.max_ls < 2)
        return RSOT_ERR_INVALID_ARG;
    for (int k = 0; k < sp.n_eps; ++k)
        if (!(sp.eps_schedule[k] > 0.0) || !std::isfinite(sp.eps_schedule[k]))
            return RSOT_ERR_INVALID_ARG;
    if (std::fabs(p->sum_mu - p->sum_nu) > 1e-12 * p->sum_nu) return RSOT_ERR_UNBALANCED;
    const size_t n = (size_t)p->n;
    for (size_t i = 0; i < n; ++i)
        if (!std::isfinite(psi_inout[i])) return RSOT_ERR_NONFINITE;

    const auto t0 = std::chrono::steady_clock::now();
    std::vector<double> psi(psi_inout, psi_inout + n), g(n), dir(n), q(n);
    rsot_solve_info inf{};
    rsot_status status = RSOT_OK;
    double J = 0.0;
    double eval_ms = 0.0, cull_ms = 0.0, p1_ms = 0.0, p2_ms = 0.0, kept_sum = 0.0;
    int total_it = 0, total_ev = 0;
    const double saved_ref = p->absJ_ref;

    auto finish = [&](rsot_status st) {
        // centre: sum_j nu_j psi_j = 0 is the representative of App. A; the
        // evaluation is invariant under constant shifts when masses balance
        std::vector<double> nu(n);
        std::memcpy(psi_inout, psi.data(), n * sizeof(double));
        inf.iterations = total_it;
        inf.evaluations = total_ev;
        inf.J = J;
        inf.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        inf.eval_ms = eval_ms;
        inf.cull_ms = cull_ms;
        inf.pass1_ms = p1_ms;
        inf.pass2_ms = p2_ms;
        inf.kept_frac = total_ev > 0 ? kept_sum / total_ev : 0.0;
        inf.status = st;
        if (info) *info = inf;
        return st;
    };

    for (int stage = 0; stage < sp.n_eps; ++stage) {
        Evaluator ev{p, sp.eps_schedule[stage]};
        ev.cancel = sp.cancel;
        const bool final_stage = stage == sp.n_eps - 1;
        const double tol = (!final_stage && sp.stage_tol > 0.0) ? sp.stage_tol : sp.tol;
        p->absJ_ref = 0.0;  // first evaluation of a stage runs dense
        p->have_D = 0;
        rsot_status s = ev(psi, J, g);
        if (s != RSOT_OK) {
            total_ev += ev.evals;
            eval_ms += ev.eval_ms;
            cull_ms += ev.cull_ms;
            p1_ms += ev.p1_ms;
            p2_ms += ev.p2_ms;
            kept_sum += ev.kept;
            return finish(s);
        }
        double gl1 = ev.last.grad_l1, glinf = ev.last.grad_linf;
        std::vector<std::vector<double>> S, Y;
        std::vector<double> rho;
        int it = 0;
        rsot_status st = RSOT_OK;
        while (gl1 > tol) {
            if (it >= sp.max_iter) {
                st = final_stage ? RSOT_ERR_NOT_CONVERGED : RSOT_OK;
                break;
            }
            // two-loop recursion: dir = -H g
            q = g;
            const int k = (int)S.size();
            std::vector<double> al(k);
            for (int i = k - 1; i >= 0; --i) {
                al[i] = rho[i] * dot(S[i], q);
                for (size_t t = 0; t < n; ++t) q[t] -= al[i] * Y[i][t];
            }
            double gamma;
            if (k > 0)
                gamma = dot(S[k - 1], Y[k - 1]) / dot(Y[k - 1], Y[k - 1]);
            else
                gamma = ev.eps * (double)n / p->sum_nu;
            for (size_t t = 0; t < n; ++t) q[t] *= gamma;
            for (int i = 0; i < k; ++i) {
                const double be = rho[i] * dot(Y[i], q);
                for (size_t t = 0; t < n; ++t) q[t] += S[i][t] * (al[i] - be);
            }
            for (size_t t = 0; t < n; ++t) dir[t] = -q[t];
            if (!(dot(dir, g) < 0.0)) {  // lost descent: restart from the scaled gradient
                S.clear();
                Y.clear();
                rho.clear();
                const double gm = ev.eps * (double)n / p->sum_nu;
                for (size_t t = 0; t < n; ++t) dir[t] = -gm * g[t];
            }
            Point np;
            p->absJ_ref = std::fabs(J);
            rsot_status ls = line_search(ev, psi, J, g, dir, 1.0, sp.c1, sp.c2, sp.max_ls, np);
            if (ls != RSOT_OK && !S.empty()) {  // retry once without history
                S.clear();
                Y.clear();
                rho.clear();
                const double gm = ev.eps * (double)n / p->sum_nu;
                for (size_t t = 0; t < n; ++t) dir[t] = -gm * g[t];
                ls = line_search(ev, psi, J, g, dir, 1.0, sp.c1, sp.c2, sp.max_ls, np);
            }
            if (ls != RSOT_OK) {
                st = ls;
                break;
            }
            std::vector<double> sv(n), yv(n);
            for (size_t t = 0; t < n; ++t) {
                sv[t] = np.psi[t] - psi[t];
                yv[t] = np.g[t] - g[t];
            }
            const double sy = dot(sv, yv);
            if (sy > 1e-300) {
                S.push_back(std::move(sv));
                Y.push_back(std::move(yv));
                rho.push_back(1.0 / sy);
                if ((int)S.size() > sp.lbfgs_m) {
                    S.erase(S.begin());
                    Y.erase(Y.begin());
                    rho.erase(rho.begin());
                }
            }
            const double step = np.alpha;
            psi.swap(np.psi);
            g.swap(np.g);
            J = np.f;
            gl1 = 0.0;
            glinf = 0.0;
            for (size_t t = 0; t < n; ++t) {
                gl1 += std::fabs(g[t]);
                glinf = std::max(glinf, std::fabs(g[t]));
            }
            ++it;
            if (sp.callback) {
                rsot_iter_info ii{};
                ii.stage = stage;
                ii.iteration = it;
                ii.evaluations = ev.evals;
                ii.eps = ev.eps;
                ii.J = J;
                ii.grad_l1 = gl1;
                ii.grad_linf = glinf;
                ii.step = step;
                ii.kept_pairs = ev.last.kept_pairs;
                ii.cutoff = ev.last.cutoff;
                if (sp.callback(&ii, sp.user)) {
                    st = RSOT_ERR_CANCELLED;
                    break;
                }
            }
        }
        total_it += it;
        total_ev += ev.evals;
        eval_ms += ev.eval_ms;
        cull_ms += ev.cull_ms;
        p1_ms += ev.p1_ms;
        p2_ms += ev.p2_ms;
        kept_sum += ev.kept;
        inf.grad_l1 = gl1;
        inf.grad_linf = glinf;
        inf.stages = stage + 1;
        if (st != RSOT_OK) {
            status = st;
            break;
        }
    }
    (void)saved_ref;
    // centre the potential: sum_j nu_j psi_j = 0
    {
        std::vector<double> nu(n);
        std::vector<int32_t> perm((size_t)p->n_pad);
        std::vector<double> tnu((size_t)p->n_pad);
        if (hipMemcpy(perm.data(), p->tperm, sizeof(int32_t) * p->n_pad, hipMemcpyDeviceToHost) ==
                hipSuccess &&
            hipMemcpy(tnu.data(), p->tnu, sizeof(double) * p->n_pad, hipMemcpyDeviceToHost) ==
                hipSuccess) {
            for (int64_t i = 0; i < p->n_pad; ++i)
                if (perm[i] >= 0) nu[perm[i]] = tnu[i];
            double c = 0.0;
            for (size_t t = 0; t < n; ++t) c += nu[t] * psi[t];
            c /= p->sum_nu;
            for (size_t t = 0; t < n; ++t) psi[t] -= c;
            J -= c * (p->sum_mu - p->sum_nu);
        }
    }
    return finish(status);
}
