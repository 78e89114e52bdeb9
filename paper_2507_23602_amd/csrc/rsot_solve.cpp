// rsot_solve: Alg. 1 (L-BFGS on J with a line search, stop on ||grad||_1,
// Remark 3.2) inside an eps schedule (Sec. 4.2). The paper leaves the L-BFGS
// details open; this file fixes them as: memory m (default 10), initial
// inverse-Hessian scaling s'y / y'y (and eps N / sum nu before the first pair
// exists, the inverse of J's diagonal scale nu_j / eps), strong-Wolfe line
// search (c1 = 1e-4, c2 = 0.9) by bracketing and safeguarded cubic
// interpolation, at most max_ls evaluations per search. Host FP64 vectors,
// their arithmetic spread over a small pool of threads; every evaluation is
// one rsot_dual_eval on the device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <functional>
#include <mutex>
#include <thread>
#include <vector>

#include "rsot_internal.h"

namespace {

// Vector arithmetic of the solver over NCH fixed chunks. Chunks are spread
// over up to 16 threads, and sums add the chunk partials in chunk order, so
// results do not depend on the machine's thread count. Short vectors run on
// the calling thread.
class Par {
  public:
    static constexpr int NCH = 16;
    static constexpr size_t MIN_PAR = 32768;

    explicit Par(size_t n) {
        if (n < MIN_PAR) return;
        unsigned hw = std::thread::hardware_concurrency();
        nt_ = (int)std::max(1u, std::min<unsigned>(hw ? hw : 1, NCH));
        for (int k = 1; k < nt_; ++k) th_.emplace_back([this, k] { worker(k); });
    }
    ~Par() {
        {
            std::lock_guard<std::mutex> l(m_);
            stop_ = true;
            ++gen_;
        }
        cv_.notify_all();
        for (auto &t : th_) t.join();
    }
    // f(i0, i1) over the chunks of [0, n)
    void chunks(size_t n, const std::function<void(size_t, size_t)> &f) {
        if (nt_ <= 1 || n < MIN_PAR) {
            f(0, n);
            return;
        }
        run([&](int k) {
            for (int c = k; c < NCH; c += nt_) f(n * c / NCH, n * (c + 1) / NCH);
        });
    }
    double dot(const double *a, const double *b, size_t n) {
        double part[NCH] = {0};
        if (nt_ <= 1 || n < MIN_PAR) {
            double s = 0.0;
            for (size_t i = 0; i < n; ++i) s += a[i] * b[i];
            return s;
        }
        run([&](int k) {
            for (int c = k; c < NCH; c += nt_) {
                double s = 0.0;
                for (size_t i = n * c / NCH; i < n * (c + 1) / NCH; ++i) s += a[i] * b[i];
                part[c] = s;
            }
        });
        double s = 0.0;
        for (int c = 0; c < NCH; ++c) s += part[c];
        return s;
    }
    double dot(const std::vector<double> &a, const std::vector<double> &b) {
        return dot(a.data(), b.data(), a.size());
    }

  private:
    // f(k) on thread k = 0..nt_-1 (k = 0 is the caller); returns when all end
    void run(const std::function<void(int)> &f) {
        {
            std::lock_guard<std::mutex> l(m_);
            job_ = &f;
            pending_ = nt_ - 1;
            ++gen_;
        }
        cv_.notify_all();
        f(0);
        std::unique_lock<std::mutex> l(m_);
        done_.wait(l, [this] { return pending_ == 0; });
        job_ = nullptr;
    }
    void worker(int k) {
        long seen = 0;
        for (;;) {
            const std::function<void(int)> *job = nullptr;
            {
                std::unique_lock<std::mutex> l(m_);
                cv_.wait(l, [&] { return gen_ != seen; });
                seen = gen_;
                if (stop_) return;
                job = job_;
            }
            (*job)(k);
            std::lock_guard<std::mutex> l(m_);
            if (--pending_ == 0) done_.notify_one();
        }
    }
    int nt_ = 1;
    std::vector<std::thread> th_;
    std::mutex m_;
    std::condition_variable cv_, done_;
    const std::function<void(int)> *job_ = nullptr;
    int pending_ = 0;
    long gen_ = 0;
    bool stop_ = false;
};

struct Evaluator {
    rsot_problem *p;
    Par *par;
    double eps;
    bool flip = false;           // test hook: hand the solver -grad
    int evals = 0;
    double eval_ms = 0.0, cull_ms = 0.0, p1_ms = 0.0, p2_ms = 0.0, kept = 0.0;
    volatile int *cancel = nullptr;
    rsot_eval_info last{};

    rsot_status operator()(const std::vector<double> &psi, double &J, std::vector<double> &g) {
        if (cancel && *cancel) return RSOT_ERR_CANCELLED;
        const size_t n = psi.size();
        par->chunks(n, [&](size_t a, size_t b) {
            std::memcpy(p->hpsi + a, psi.data() + a, (b - a) * sizeof(double));
        });
        RSOT_HIP(hipMemcpyAsync(p->dpsi, p->hpsi, n * sizeof(double), hipMemcpyHostToDevice,
                                p->stream));
        RSOT_TRY(rsot_eval_impl(p, eps, p->dpsi, &J, p->dgrad, &last));
        RSOT_HIP(hipMemcpyAsync(p->hgrad, p->dgrad, n * sizeof(double), hipMemcpyDeviceToHost,
                                p->stream));
        RSOT_HIP(hipStreamSynchronize(p->stream));
        par->chunks(n, [&](size_t a, size_t b) {
            std::memcpy(g.data() + a, p->hgrad + a, (b - a) * sizeof(double));
            if (flip)
                for (size_t i = a; i < b; ++i) g[i] = -g[i];
        });
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
    double gl1 = 0.0, glinf = 0.0;   // norms of g, from its evaluation
};

// Strong-Wolfe line search along p (Nocedal & Wright, Algs. 3.5/3.6).
// On success out holds the accepted point. Points trade their vectors by
// swap or move; the start point (alpha 0) carries none, since it is never
// returned.
rsot_status line_search(Evaluator &ev, const std::vector<double> &psi0, double f0,
                        const std::vector<double> &g0, const std::vector<double> &dir,
                        double alpha1, double c1, double c2, int max_ls, Point &out) {
    Par &par = *ev.par;
    const double d0 = par.dot(g0, dir);
    const size_t n = psi0.size();
    Point prev{0.0, f0, d0, {}, {}, 0.0, 0.0};
    Point cur;
    auto eval_at = [&](double a, Point &pt) -> rsot_status {
        pt.alpha = a;
        pt.psi.resize(n);
        pt.g.resize(n);
        par.chunks(n, [&](size_t i0, size_t i1) {
            for (size_t i = i0; i < i1; ++i) pt.psi[i] = psi0[i] + a * dir[i];
        });
        RSOT_TRY(ev(pt.psi, pt.f, pt.g));
        pt.d = par.dot(pt.g, dir);
        pt.gl1 = ev.last.grad_l1;
        pt.glinf = ev.last.grad_linf;
        return RSOT_OK;
    };
    // f noise allowance of the approximate-Wolfe acceptance: the objective of
    // the mixed path carries ~1e-10 relative noise, the FP64 path ~1e-15
    const double fnoise = (rsot_pairs_fp64(ev.p) ? 1e-13 : 1e-9) * std::fabs(f0);
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
                out = std::move(cur);
                return RSOT_OK;
            }
            lo = std::move(prev);
            std::swap(hi, cur);
            zoom = true;
            break;
        }
        if (std::fabs(cur.d) <= -c2 * d0) {
            out = std::move(cur);
            return RSOT_OK;
        }
        if (cur.d >= 0.0) {
            std::swap(lo, cur);
            hi = std::move(prev);
            zoom = true;
            break;
        }
        std::swap(prev, cur);
        a *= 2.0;
    }
    if (!zoom) {
        if (prev.alpha > 0.0 && prev.f < f0) {  // still descending: accept the last point
            out = std::move(prev);
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
                out = std::move(cur);
                return RSOT_OK;
            }
            std::swap(hi, cur);
        } else {
            if (std::fabs(cur.d) <= -c2 * d0) {
                out = std::move(cur);
                return RSOT_OK;
            }
            if (cur.d * (hi.alpha - lo.alpha) >= 0.0) std::swap(hi, lo);
            std::swap(lo, cur);
        }
    }
    if (lo.alpha > 0.0 && lo.f < f0) {  // best bracket end still decreases J
        out = std::move(lo);
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
        sp.lbfgs_m < 1 || !(sp.c1 > 0.0 && sp.c1 < sp.c2 && sp.c2 < 1.0) || sp.max_ls < 2 ||
        !(sp.absJ_start >= 0.0) || !std::isfinite(sp.absJ_start))
        return RSOT_ERR_INVALID_ARG;
    for (int k = 0; k < sp.n_eps; ++k)
        if (!(sp.eps_schedule[k] > 0.0) || !std::isfinite(sp.eps_schedule[k]))
            return RSOT_ERR_INVALID_ARG;
    if (std::fabs(p->sum_mu - p->sum_nu) > 1e-12 * p->sum_nu) return RSOT_ERR_UNBALANCED;
    const size_t n = (size_t)p->n;
    rsot_checkpoint *ck = sp.checkpoint;
    if (ck && (ck->n_target != (int64_t)n || ck->capacity < 0 ||
               (ck->capacity > 0 && (!ck->s || !ck->y))))
        return RSOT_ERR_INVALID_ARG;
    if (sp.resume && (!ck || !ck->valid || ck->stage < 0 || ck->stage >= sp.n_eps ||
                      ck->n_pairs < 0 || ck->n_pairs > ck->capacity || ck->iteration < 0 ||
                      !(ck->absJ_ref >= 0.0)))
        return RSOT_ERR_INVALID_ARG;
    for (size_t i = 0; i < n; ++i)
        if (!std::isfinite(psi_inout[i])) return RSOT_ERR_NONFINITE;

    const auto t0 = std::chrono::steady_clock::now();
    Par par(n);
    std::vector<double> psi(psi_inout, psi_inout + n), g(n), dir(n), q(n);
    rsot_solve_info inf{};
    rsot_status status = RSOT_OK;
    double J = 0.0;
    double eval_ms = 0.0, cull_ms = 0.0, p1_ms = 0.0, p2_ms = 0.0, kept_sum = 0.0;
    int total_it = 0, total_ev = 0;
    // L-BFGS memory of the current stage, and where the solve stands
    std::vector<std::vector<double>> S, Y;
    std::vector<double> rho;
    int cur_stage = sp.resume ? ck->stage : 0, cur_it = 0;

    auto finish = [&](rsot_status st) {
        if (ck) {
            const int keep = std::min<int>((int)S.size(), ck->capacity);
            const int first = (int)S.size() - keep;
            for (int i = 0; i < keep; ++i) {
                std::memcpy(ck->s + (size_t)i * n, S[first + i].data(), n * sizeof(double));
                std::memcpy(ck->y + (size_t)i * n, Y[first + i].data(), n * sizeof(double));
            }
            ck->n_pairs = keep;
            ck->stage = cur_stage;
            ck->iteration = cur_it;
            ck->absJ_ref = p->absJ_ref;
            ck->valid = 1;
        }
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

    for (int stage = cur_stage; stage < sp.n_eps; ++stage) {
        Evaluator ev{p, &par, sp.eps_schedule[stage]};
        ev.cancel = sp.cancel;
        ev.flip = sp.test_flip_gradient != 0;
        const bool resumed = sp.resume && stage == ck->stage;
        cur_stage = stage;
        S.clear();
        Y.clear();
        rho.clear();
        cur_it = 0;
        const bool final_stage = stage == sp.n_eps - 1;
        const double tol = (!final_stage && sp.stage_tol > 0.0) ? sp.stage_tol : sp.tol;
        // |J| reference of the truncation rules: for the first stage the
        // caller's (0: the warm start is evaluated densely to obtain it), for
        // later ones the last accepted iterate's, which the previous stage
        // left (the new stage's warm start is that iterate). D of the INT
        // rule depends on eps and is taken afresh.
        if (resumed) p->absJ_ref = ck->absJ_ref;
        else if (stage == 0) p->absJ_ref = sp.absJ_start;
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
        std::vector<double> sv, yv;
        int it = 0;
        if (resumed) {              // the stopped solve's history and count
            for (int i = 0; i < ck->n_pairs; ++i) {
                S.emplace_back(ck->s + (size_t)i * n, ck->s + (size_t)(i + 1) * n);
                Y.emplace_back(ck->y + (size_t)i * n, ck->y + (size_t)(i + 1) * n);
                const double sy = par.dot(S.back(), Y.back());
                if (!(sy > 1e-300)) return finish(RSOT_ERR_INVALID_ARG);
                rho.push_back(1.0 / sy);
            }
            while ((int)S.size() > sp.lbfgs_m) {
                S.erase(S.begin());
                Y.erase(Y.begin());
                rho.erase(rho.begin());
            }
            it = ck->iteration;
        }
        cur_it = it;
        rsot_status st = RSOT_OK;
        while (gl1 > tol) {
            if (it >= sp.max_iter) {
                st = final_stage ? RSOT_ERR_NOT_CONVERGED : RSOT_OK;
                break;
            }
            // two-loop recursion: dir = -H g
            auto axpy = [&](std::vector<double> &yv, double a, const std::vector<double> &xv) {
                par.chunks(n, [&](size_t i0, size_t i1) {
                    for (size_t t = i0; t < i1; ++t) yv[t] += a * xv[t];
                });
            };
            auto scaled = [&](std::vector<double> &yv, double a, const std::vector<double> &xv) {
                par.chunks(n, [&](size_t i0, size_t i1) {
                    for (size_t t = i0; t < i1; ++t) yv[t] = a * xv[t];
                });
            };
            scaled(q, 1.0, g);
            const int k = (int)S.size();
            std::vector<double> al(k);
            for (int i = k - 1; i >= 0; --i) {
                al[i] = rho[i] * par.dot(S[i], q);
                axpy(q, -al[i], Y[i]);
            }
            double gamma;
            if (k > 0)
                gamma = par.dot(S[k - 1], Y[k - 1]) / par.dot(Y[k - 1], Y[k - 1]);
            else
                gamma = ev.eps * (double)n / p->sum_nu;
            scaled(q, gamma, q);
            for (int i = 0; i < k; ++i) {
                const double be = rho[i] * par.dot(Y[i], q);
                axpy(q, al[i] - be, S[i]);
            }
            scaled(dir, -1.0, q);
            if (!(par.dot(dir, g) < 0.0)) {  // lost descent: restart from the scaled gradient
                S.clear();
                Y.clear();
                rho.clear();
                scaled(dir, -ev.eps * (double)n / p->sum_nu, g);
            }
            Point np;
            p->absJ_ref = std::fabs(J);
            rsot_status ls = line_search(ev, psi, J, g, dir, 1.0, sp.c1, sp.c2, sp.max_ls, np);
            if (ls != RSOT_OK && !S.empty()) {  // retry once without history
                S.clear();
                Y.clear();
                rho.clear();
                scaled(dir, -ev.eps * (double)n / p->sum_nu, g);
                ls = line_search(ev, psi, J, g, dir, 1.0, sp.c1, sp.c2, sp.max_ls, np);
            }
            if (ls != RSOT_OK) {
                // a non-final stage that cannot improve its iterate hands it
                // to the next eps; the final stage reports the failure
                if (ls == RSOT_ERR_LINESEARCH && !final_stage) ++inf.stalled_stages;
                else st = ls;
                break;
            }
            // history pair (sv, yv persist across iterations; the pair that
            // drops out of the memory lends its storage to the next one)
            sv.resize(n);
            yv.resize(n);
            par.chunks(n, [&](size_t i0, size_t i1) {
                for (size_t t = i0; t < i1; ++t) {
                    sv[t] = np.psi[t] - psi[t];
                    yv[t] = np.g[t] - g[t];
                }
            });
            const double sy = par.dot(sv, yv);
            if (sy > 1e-300) {
                std::vector<double> os, oy;
                if ((int)S.size() >= sp.lbfgs_m) {
                    os = std::move(S.front());
                    oy = std::move(Y.front());
                    S.erase(S.begin());
                    Y.erase(Y.begin());
                    rho.erase(rho.begin());
                }
                S.push_back(std::move(sv));
                Y.push_back(std::move(yv));
                rho.push_back(1.0 / sy);
                sv = std::move(os);
                yv = std::move(oy);
            }
            const double step = np.alpha;
            psi.swap(np.psi);
            g.swap(np.g);
            J = np.f;
            // norms of the accepted gradient (its evaluation's own, from the device)
            gl1 = np.gl1;
            glinf = np.glinf;
            ++it;
            cur_it = it;
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
    // centre the potential on success: sum_j nu_j psi_j = 0. Any other exit
    // returns the last accepted iterate as the solver holds it, so that a
    // resumed solve continues from exactly that point.
    if (status == RSOT_OK) {
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
