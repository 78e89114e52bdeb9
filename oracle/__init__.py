"""CPU oracle for the semi-discrete RSOT dual (TEST INFRASTRUCTURE ONLY).

Plain FP64 reference implementations of what the HIP library computes, used
by the tests, the smoke check and the benchmark's CPU-baseline leg and by
nothing else. It shares no code with the HIP library: the heavy loops live in
``rsot_oracle.c`` (plain C, libm exp/log, OpenMP over quadrature points),
the rest is numpy written from the paper's formulas.

Functions and the passage each follows:
  dual_eval         -- J^h and grad J^h, dense or cut at c < C
                       (Eqs. discretized_functional / discretized_gradient, Alg. 2)
  dual_eval_tile    -- same over tile/block pairs kept by the tile-local bound
                       derived from App. B (rule stated in rsot_oracle.c)
  covering_cost     -- C_0 = max_x min_j c(x, y_j) (Sec. 4.1, App. B)
  kept_counts       -- |I_q| = #{j : c_qj < C} per point (Sec. 4.1), brute force
  cutoff_geom/int/pw-- Eqs. truncation_cutoff_geom, truncation_cutoff_int,
                       cost_cutoff_delta
  softmax_refine    -- Eq. softmax_refinement_formula (log domain)
  plan_moments      -- nu~_j and sum_q mu_q p_qj x_q (Sec. 6.2, Eq. barycenter_fixed_point)
  transport_maps    -- barycentric and modal maps (Sec. 6.3, Eqs.
                       barycentric_map_registration / modal_map_registration)
  lbfgs_solve       -- Alg. 1 with a textbook L-BFGS (Sec. 3.4; memory 10,
                       strong-Wolfe or Armijo line search), stop on
                       ||grad||_1 (Remark 3.2)
  sinkhorn_psi      -- log-domain Sinkhorn on the discrete problem of
                       Remark 3.1 (independent route to psi*)
  power_cell_masses -- eps -> 0 limit (Remark 2.1): mass of each Laguerre
                       cell by brute-force argmax over the quadrature points
  laguerre_areas_2d -- exact Laguerre-cell areas in the unit square by
                       half-plane clipping (no quadrature)
  two_target_mass   -- closed form of int_0^1 sigma((a - b x)/eps) dx
  dual_eval_sphere, dual_eval_tile_sphere
                    -- the same with the squared geodesic cost on the unit
                       sphere, c = cost_scale d_g^2 (Sec. 6.4)
  sphere_karcher_step -- one Riemannian-barycentre step per target with the
                       plan's conditional measures held fixed (Alg. 5)

Parity pins for every function are in tests/test_oracle_pins.py and
tests/test_oracle_pins_cutoffs.py (two-sided cutoff windows, D); the sphere
functions in tests/test_oracle_pins_sphere.py.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rsot_oracle.c")
_LIB = os.path.join(_HERE, "librsot_oracle.so")
_lib = None

_D = ctypes.c_double
_I = ctypes.c_int
_I64 = ctypes.c_int64
_P = ctypes.c_void_p


def build(force: bool = False) -> str:
    """Compile rsot_oracle.c with gcc -O2 -fopenmp (no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        lib.oracle_dual_eval.restype = _I
        lib.oracle_dual_eval.argtypes = [_I, _I64, _P, _P, _I64, _P, _P, _P, _D, _D, _D, _I,
                                         _P, _P, _P, _P, _P]
        lib.oracle_kept_counts.restype = _I
        lib.oracle_kept_counts.argtypes = [_I, _I64, _P, _I64, _P, _D, _D, _D, _I, _P, _P]
        lib.oracle_covering_cost.restype = _D
        lib.oracle_covering_cost.argtypes = [_I, _I64, _P, _I64, _P, _D, _I]
        lib.oracle_cutoff_geom.restype = _D
        lib.oracle_cutoff_geom.argtypes = [_D] * 7
        lib.oracle_cutoff_int.restype = _D
        lib.oracle_cutoff_int.argtypes = [_D] * 6
        lib.oracle_cutoff_pw.restype = _D
        lib.oracle_cutoff_pw.argtypes = [_D] * 4
        lib.oracle_integral_D.restype = _D
        lib.oracle_integral_D.argtypes = [_I64, _P, _P]
        lib.oracle_softmax_refine.restype = _I
        lib.oracle_softmax_refine.argtypes = [_I, _I64, _P, _P, _P, _I64, _P, _D, _D, _I, _P]
        lib.oracle_plan_moments.restype = _I
        lib.oracle_plan_moments.argtypes = [_I, _I64, _P, _P, _I64, _P, _P, _P, _D, _D, _P, _P,
                                            _I64, _P, _D, _I, _P, _P]
        lib.oracle_transport_maps.restype = _I
        lib.oracle_transport_maps.argtypes = [_I, _I64, _P, _I64, _P, _P, _P, _D, _D, _P, _P,
                                              _I64, _P, _D, _I, _P, _P, _P]
        lib.oracle_dual_eval_sphere.restype = _I
        lib.oracle_dual_eval_sphere.argtypes = [_I64, _P, _P, _I64, _P, _P, _P, _D, _D, _I,
                                                _P, _P, _P]
        lib.oracle_dual_eval_tile_sphere.restype = _I
        lib.oracle_dual_eval_tile_sphere.argtypes = [_I64, _P, _P, _I64, _P, _P, _P, _D, _D,
                                                     _P, _I64, _P, _I64, _D, _D, _I,
                                                     _P, _P, _P, _P, _P]
        lib.oracle_sphere_karcher_step.restype = _I
        lib.oracle_sphere_karcher_step.argtypes = [_I64, _P, _P, _I64, _P, _P, _P, _D, _D, _P,
                                                   _D, _I, _P, _P, _P]
        lib.oracle_dual_eval_tile.restype = _I
        lib.oracle_dual_eval_tile.argtypes = [_I, _I64, _P, _P, _I64, _P, _P, _P, _D, _D,
                                              _P, _I64, _P, _I64, _D, _D, _I,
                                              _P, _P, _P, _P, _P]
        _lib = lib
    return _lib


def _c(a, dtype=np.float64):
    return np.ascontiguousarray(a, dtype=dtype)


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


class EvalResult:
    def __init__(self, J, grad, L, kept, nempty):
        self.J = J
        self.grad = grad
        self.L = L
        self.kept = kept
        self.nempty = nempty


def dual_eval(x, mu, y, nu, psi, eps, cost_scale=0.5, cutoff=math.inf,
              want_grad=True, want_L=False, threads=0) -> EvalResult:
    """J^h(psi), grad J^h(psi) (Eqs. discretized_functional/gradient, Alg. 2).

    ``cutoff`` = inf gives the dense sums; a finite C keeps j with c_qj < C.
    """
    lib = _load()
    x, mu, y, nu, psi = _c(x), _c(mu), _c(y), _c(nu), _c(psi)
    d = x.shape[1]
    nq, n = x.shape[0], y.shape[0]
    J = ctypes.c_double(0.0)
    kept = ctypes.c_int64(0)
    nempty = ctypes.c_int64(0)
    grad = np.empty(n) if want_grad else None
    L = np.empty(nq) if want_L else None
    rc = lib.oracle_dual_eval(d, nq, _ptr(x), _ptr(mu), n, _ptr(y), _ptr(nu), _ptr(psi),
                              float(eps), float(cost_scale), float(cutoff), int(threads),
                              ctypes.byref(J), _ptr(grad), _ptr(L),
                              ctypes.byref(kept), ctypes.byref(nempty))
    if rc != 0:
        raise ValueError("oracle_dual_eval: invalid arguments")
    return EvalResult(J.value, grad, L, kept.value, nempty.value)


def dual_eval_tile(x, mu, y, nu, psi, eps, tile_of, n_tiles, block_of, n_blocks,
                   tau, absJ_ref, cost_scale=0.5, want_L=False, want_keep=False,
                   threads=0):
    """Evaluation over the (tile, block) pairs kept by the tile-local bound."""
    lib = _load()
    x, mu, y, nu, psi = _c(x), _c(mu), _c(y), _c(nu), _c(psi)
    tile_of = _c(tile_of, np.int32)
    block_of = _c(block_of, np.int32)
    d = x.shape[1]
    nq, n = x.shape[0], y.shape[0]
    J = ctypes.c_double(0.0)
    kept = ctypes.c_int64(0)
    grad = np.empty(n)
    L = np.empty(nq) if want_L else None
    keep = np.empty((n_tiles, n_blocks), dtype=np.uint8) if want_keep else None
    rc = lib.oracle_dual_eval_tile(d, nq, _ptr(x), _ptr(mu), n, _ptr(y), _ptr(nu), _ptr(psi),
                                   float(eps), float(cost_scale), _ptr(tile_of), int(n_tiles),
                                   _ptr(block_of), int(n_blocks), float(tau), float(absJ_ref),
                                   int(threads), ctypes.byref(J), _ptr(grad), _ptr(L),
                                   ctypes.byref(kept), _ptr(keep))
    if rc != 0:
        raise ValueError("oracle_dual_eval_tile: invalid arguments")
    r = EvalResult(J.value, grad, L, kept.value, 0)
    r.keep = keep
    return r


def kept_counts(x, y, cutoff, cost_scale=0.5, rel_band=0.0, threads=0):
    """Per point |I_q| = #{j : c(x_q, y_j) < cutoff} (Sec. 4.1), and the
    number of targets whose cost is within rel_band * cutoff of the cutoff."""
    lib = _load()
    x, y = _c(x), _c(y)
    kept = np.empty(x.shape[0], dtype=np.int32)
    near = np.empty(x.shape[0], dtype=np.int32)
    rc = lib.oracle_kept_counts(x.shape[1], x.shape[0], _ptr(x), y.shape[0], _ptr(y),
                                float(cost_scale), float(cutoff), float(rel_band), int(threads),
                                _ptr(kept), _ptr(near))
    if rc != 0:
        raise ValueError("oracle_kept_counts: invalid arguments")
    return kept, near


def _keep_args(keep):
    """(tile_of, block_of, n_blocks, keep matrix) of a truncated plan, or Nones."""
    if keep is None:
        return None, None, 0, None
    tile_of, block_of, mat = keep
    mat = np.ascontiguousarray(mat, dtype=np.uint8)
    return _c(tile_of, np.int32), _c(block_of, np.int32), mat.shape[1], mat


def plan_moments(x, mu, y, nu, psi, eps, cost_scale=0.5, keep=None, cutoff=math.inf,
                 threads=0):
    """Target moments of the plan (Sec. 6.2): (nu~, first) with
    nu~_j = sum_q mu_q p_qj and first[j] = sum_q mu_q p_qj x_q. keep =
    (tile_of, block_of, keep matrix) restricts the plan to kept pairs, a
    finite cutoff to pairs with c < cutoff."""
    lib = _load()
    x, mu, y, nu, psi = _c(x), _c(mu), _c(y), _c(nu), _c(psi)
    d, nq, n = x.shape[1], x.shape[0], y.shape[0]
    mass = np.empty(n)
    first = np.empty((n, d))
    to, bo, nb, km = _keep_args(keep)
    rc = lib.oracle_plan_moments(d, nq, _ptr(x), _ptr(mu), n, _ptr(y), _ptr(nu), _ptr(psi),
                                 float(eps), float(cost_scale), _ptr(to), _ptr(bo), int(nb),
                                 _ptr(km), float(cutoff), int(threads), _ptr(mass),
                                 _ptr(first))
    if rc != 0:
        raise ValueError("oracle_plan_moments: invalid arguments")
    return mass, first


def transport_maps(x, y, nu, psi, eps, cost_scale=0.5, keep=None, cutoff=math.inf, threads=0):
    """Maps of the plan (Sec. 6.3): barycentric map (nq x d), modal target
    index (nq, lowest index on ties, -1 if a point has no kept pair) and the
    maximum of psi_j - c_qj + eps ln nu_j it attains."""
    lib = _load()
    x, y, nu, psi = _c(x), _c(y), _c(nu), _c(psi)
    d, nq, n = x.shape[1], x.shape[0], y.shape[0]
    bary = np.empty((nq, d))
    modal = np.empty(nq, dtype=np.int32)
    val = np.empty(nq)
    to, bo, nb, km = _keep_args(keep)
    rc = lib.oracle_transport_maps(d, nq, _ptr(x), n, _ptr(y), _ptr(nu), _ptr(psi), float(eps),
                                   float(cost_scale), _ptr(to), _ptr(bo), int(nb), _ptr(km),
                                   float(cutoff), int(threads), _ptr(bary), _ptr(modal),
                                   _ptr(val))
    if rc != 0:
        raise ValueError("oracle_transport_maps: invalid arguments")
    return bary, modal, val


def covering_cost(x, y, cost_scale=0.5, threads=0) -> float:
    """C_0 = max_q min_j c(x_q, y_j) (Sec. 4.1), brute force."""
    lib = _load()
    x, y = _c(x), _c(y)
    return lib.oracle_covering_cost(x.shape[1], x.shape[0], _ptr(x), y.shape[0], _ptr(y),
                                    float(cost_scale), int(threads))


def cutoff_geom(C0, psi, nu, tau, absJ, eps) -> float:
    """Eq. truncation_cutoff_geom, with C >= C_0 (App. B)."""
    psi = np.asarray(psi)
    return _load().oracle_cutoff_geom(C0, float(psi.max()), float(psi.min()),
                                      float(np.min(nu)), tau, absJ, eps)


def cutoff_int(C0, psi, D, tau, absJ, eps) -> float:
    """Eq. truncation_cutoff_int with D from the previous evaluation."""
    return _load().oracle_cutoff_int(C0, float(np.max(psi)), D, tau, absJ, eps)


def cutoff_pw(psi, nu, delta_thr, eps) -> float:
    """Eq. cost_cutoff_delta."""
    return _load().oracle_cutoff_pw(float(np.max(psi)), float(np.max(nu)), delta_thr, eps)


def integral_D(mu, L) -> float:
    """D = sum_q mu_q / S_trunc(x_q) from per-point L_q = ln S_trunc(x_q)."""
    mu, L = _c(mu), _c(L)
    return _load().oracle_integral_D(mu.shape[0], _ptr(mu), _ptr(L))


def softmax_refine(x, mu, L_coarse, y_fine, eps, cost_scale=0.5, threads=0):
    """Eq. softmax_refinement_formula: psi_k = -eps LSE_q(ln mu_q - L_q - c_qk/eps)."""
    lib = _load()
    x, mu, L, yf = _c(x), _c(mu), _c(L_coarse), _c(y_fine)
    out = np.empty(yf.shape[0])
    lib.oracle_softmax_refine(x.shape[1], x.shape[0], _ptr(x), _ptr(mu), _ptr(L),
                              yf.shape[0], _ptr(yf), float(eps), float(cost_scale),
                              int(threads), _ptr(out))
    return out


# ---------------------------------------------------------------------------
# solver side: L-BFGS (Alg. 1) and an independent Sinkhorn route to psi*
# ---------------------------------------------------------------------------
def _cubic_min(a, fa, da, b, fb, db):
    """Minimiser of the cubic interpolating f and f' at a and b, kept in the
    middle 80 % of [min(a, b), max(a, b)] (bisection if the cubic has none)."""
    lo, hi = min(a, b), max(a, b)
    d1 = da + db - 3.0 * (fa - fb) / (a - b)
    disc = d1 * d1 - da * db
    x = 0.5 * (a + b)
    if disc >= 0.0 and np.isfinite(disc):
        d2 = math.copysign(math.sqrt(disc), b - a)
        den = db - da + 2.0 * d2
        if den != 0.0:
            x = b - (b - a) * (db + d2 - d1) / den
    if not np.isfinite(x):
        x = 0.5 * (a + b)
    w = hi - lo
    return min(max(x, lo + 0.1 * w), hi - 0.1 * w)


def _wolfe_search(fun, psi, J, g, p, alpha1, c1, c2, max_ls, fnoise):
    """Strong-Wolfe line search (Nocedal & Wright, Algs. 3.5 and 3.6):
    bracket by doubling, then zoom by safeguarded cubic interpolation. Near
    the minimiser, where differences of J sink into its rounding noise, a
    point that meets Hager and Zhang's approximate Wolfe conditions
    (f <= J + fnoise, c2 d0 <= d <= (2 c1 - 1) d0) is accepted as well.
    Returns (alpha, J, g, evaluations), alpha = 0 when no step was found."""
    d0 = float(g.dot(p))
    ev = 0

    def approx(f, d):
        return f <= J + fnoise and c2 * d0 <= d <= (2.0 * c1 - 1.0) * d0

    a_prev, f_prev, d_prev = 0.0, J, d0
    a = alpha1
    lo = hi = None
    for i in range(max_ls):
        f, gn = fun(psi + a * p)
        ev += 1
        d = float(gn.dot(p))
        if f > J + c1 * a * d0 or (i > 0 and f >= f_prev):
            if approx(f, d):
                return a, f, gn, ev
            lo, hi = (a_prev, f_prev, d_prev), (a, f, d)
            break
        if abs(d) <= -c2 * d0:
            return a, f, gn, ev
        if d >= 0.0:
            lo, hi = (a, f, d), (a_prev, f_prev, d_prev)
            break
        a_prev, f_prev, d_prev, g_prev = a, f, d, gn
        a *= 2.0
    else:
        return (a_prev, f_prev, g_prev, ev) if a_prev > 0.0 else (0.0, J, g, ev)
    best = None
    while ev < max_ls:
        a = _cubic_min(lo[0], lo[1], lo[2], hi[0], hi[1], hi[2])
        f, gn = fun(psi + a * p)
        ev += 1
        d = float(gn.dot(p))
        if f > J + c1 * a * d0 or f >= lo[1]:
            if approx(f, d):
                return a, f, gn, ev
            hi = (a, f, d)
        else:
            if abs(d) <= -c2 * d0:
                return a, f, gn, ev
            if d * (hi[0] - lo[0]) >= 0.0:
                hi = lo
            lo = (a, f, d)
            best = (a, f, gn)
    if best is not None and best[1] < J:
        return best[0], best[1], best[2], ev
    return 0.0, J, g, ev


def lbfgs_solve(fun, psi0, tol=1e-6, max_iter=5000, m=10, c1=1e-4, c2=0.9, max_ls=20,
                h0=1.0, line_search="wolfe"):
    """Minimise J with textbook L-BFGS (two-loop recursion, H0 = s'y/y'y, and
    h0 I before the first pair), stopping when ||grad||_1 <= tol (Remark 3.2;
    Alg. 1 leaves the quasi-Newton details open).

    line_search: "wolfe" (strong Wolfe conditions, c1, c2, at most max_ls
    evaluations per search) or "armijo" (backtracking by halves).
    ``fun(psi) -> (J, grad)``. Returns (psi, J, grad, iterations, evaluations).
    """
    psi = np.array(psi0, dtype=np.float64)
    J, g = fun(psi)
    nev = 1
    S, Y = [], []
    it = 0
    while np.abs(g).sum() > tol and it < max_iter:
        q = g.copy()
        alphas = []
        for s, yv in reversed(list(zip(S, Y))):
            rho = 1.0 / yv.dot(s)
            a = rho * s.dot(q)
            alphas.append((rho, a))
            q -= a * yv
        q *= S[-1].dot(Y[-1]) / Y[-1].dot(Y[-1]) if S else h0
        for (s, yv), (rho, a) in zip(zip(S, Y), reversed(alphas)):
            b = rho * yv.dot(q)
            q += (a - b) * s
        p = -q
        slope = g.dot(p)
        if slope >= 0:                      # not a descent direction: reset
            S, Y = [], []
            p = -h0 * g
            slope = g.dot(p)
        if line_search == "wolfe":
            t, J_new, g_new, ne = _wolfe_search(fun, psi, J, g, p, 1.0, c1, c2, max_ls,
                                                1e-13 * abs(J))
            nev += ne
            if t == 0.0:
                if S:                       # restart from the scaled gradient once
                    S, Y = [], []
                    continue
                break
            psi_new = psi + t * p
        else:
            t = 1.0
            while True:
                psi_new = psi + t * p
                J_new, g_new = fun(psi_new)
                nev += 1
                if J_new <= J + c1 * t * slope or t < 1e-20:
                    break
                t *= 0.5
        s = psi_new - psi
        yv = g_new - g
        if s.dot(yv) > 1e-300:
            S.append(s)
            Y.append(yv)
            if len(S) > m:
                S.pop(0)
                Y.pop(0)
        psi, J, g = psi_new, J_new, g_new
        it += 1
    return psi, J, g, it, nev


def _lse(a, axis):
    m = np.max(a, axis=axis, keepdims=True)
    m = np.where(np.isfinite(m), m, 0.0)
    return (m + np.log(np.sum(np.exp(a - m), axis=axis, keepdims=True))).squeeze(axis)


def sinkhorn_psi(x, mu, y, nu, eps, cost_scale=0.5, iters=100000, tol=1e-13):
    """Log-domain Sinkhorn on the discrete problem (mu_q) -> (nu_j) of
    Remark 3.1 with plan pi_qj = mu_q nu_j exp((phi_q + psi_j - c_qj)/eps):
      phi_q = -eps ln sum_j nu_j exp((psi_j - c_qj)/eps)   (source marginal)
      psi_j = -eps ln sum_q mu_q exp((phi_q - c_qj)/eps)   (target marginal)
    Dense numpy, small problems only. Returns psi (unnormalised)."""
    x, y = np.asarray(x), np.asarray(y)
    C = cost_scale * ((x[:, None, :] - y[None, :, :]) ** 2).sum(-1)
    lmu = np.log(mu)
    lnu = np.log(nu)
    psi = np.zeros(y.shape[0])
    for _ in range(iters):
        phi = -eps * _lse((psi[None, :] - C) / eps + lnu[None, :], axis=1)
        psi_new = -eps * _lse((phi[:, None] - C) / eps + lmu[:, None], axis=0)
        if np.max(np.abs(psi_new - psi)) < tol:
            psi = psi_new
            break
        psi = psi_new
    return psi


def power_cell_masses(x, mu, y, psi, cost_scale=0.5):
    """eps -> 0 limit of nu~ (Remark 2.1): mu-mass of each Laguerre cell
    {x : j = argmax_k (psi_k - c(x, y_k))}, by brute-force argmax over the
    quadrature points. Also returns the smallest best-minus-second gap."""
    C = cost_scale * ((np.asarray(x)[:, None, :] - np.asarray(y)[None, :, :]) ** 2).sum(-1)
    v = psi[None, :] - C
    order = np.argsort(-v, axis=1)
    best = order[:, 0]
    gap = v[np.arange(v.shape[0]), order[:, 0]] - v[np.arange(v.shape[0]), order[:, 1]]
    masses = np.bincount(best, weights=mu, minlength=y.shape[0])
    return masses, gap


def _clip_polygon(poly, a, b):
    """Keep the part of a convex polygon with a . p <= b (Sutherland-Hodgman)."""
    out = []
    n = len(poly)
    for i in range(n):
        P, Q = poly[i], poly[(i + 1) % n]
        fp, fq = a.dot(P) - b, a.dot(Q) - b
        if fp <= 0:
            out.append(P)
        if (fp < 0 < fq) or (fq < 0 < fp):
            t = fp / (fp - fq)
            out.append(P + t * (Q - P))
    return out


def _area(poly):
    if len(poly) < 3:
        return 0.0
    p = np.asarray(poly)
    return 0.5 * abs(np.dot(p[:, 0], np.roll(p[:, 1], -1)) - np.dot(p[:, 1], np.roll(p[:, 0], -1)))


def laguerre_areas_2d(y, psi, cost_scale=0.5):
    """Exact areas of the Laguerre (power) cells in [0,1]^2 for cost
    cost_scale |x - y|^2: cell_j = {x : psi_j - c(x,y_j) >= psi_k - c(x,y_k)}.
    Each comparison is a half-plane 2 cs (y_k - y_j) . x <=
    psi_j - psi_k + cs (|y_k|^2 - |y_j|^2); the square is clipped by all."""
    y = np.asarray(y, dtype=np.float64)
    areas = np.zeros(y.shape[0])
    sq = [np.array([0.0, 0.0]), np.array([1.0, 0.0]), np.array([1.0, 1.0]), np.array([0.0, 1.0])]
    for j in range(y.shape[0]):
        poly = list(sq)
        for k in range(y.shape[0]):
            if k == j:
                continue
            a = 2.0 * cost_scale * (y[k] - y[j])
            b = psi[j] - psi[k] + cost_scale * (y[k].dot(y[k]) - y[j].dot(y[j]))
            poly = _clip_polygon(poly, a, b)
            if not poly:
                break
        areas[j] = _area(poly)
    return areas


def _softplus(t):
    return np.logaddexp(0.0, t)


def two_target_mass(a, b, eps):
    """int_0^1 sigma((a - b s)/eps) ds = (eps/b)[softplus(a/eps) - softplus((a-b)/eps)]."""
    return (eps / b) * (_softplus(a / eps) - _softplus((a - b) / eps))


# --------------------------------------------------------------------------
# squared geodesic cost on the unit sphere (Sec. 6.4, Algs. 4-5)
# --------------------------------------------------------------------------
def dual_eval_sphere(x, mu, y, nu, psi, eps, cost_scale=1.0, want_grad=True, want_L=False,
                     threads=0) -> EvalResult:
    """J^h and grad J^h with c(x, y) = cost_scale arccos(x . y)^2 for unit
    vectors x (nq x 3) and y (n x 3), dense."""
    lib = _load()
    x, mu, y, nu, psi = _c(x), _c(mu), _c(y), _c(nu), _c(psi)
    nq, n = x.shape[0], y.shape[0]
    J = ctypes.c_double(0.0)
    grad = np.empty(n) if want_grad else None
    L = np.empty(nq) if want_L else None
    rc = lib.oracle_dual_eval_sphere(nq, _ptr(x), _ptr(mu), n, _ptr(y), _ptr(nu), _ptr(psi),
                                     float(eps), float(cost_scale), int(threads),
                                     ctypes.byref(J), _ptr(grad), _ptr(L))
    if rc != 0:
        raise ValueError("oracle_dual_eval_sphere: invalid arguments")
    return EvalResult(J.value, grad, L, nq * n, 0)


def dual_eval_tile_sphere(x, mu, y, nu, psi, eps, tile_of, n_tiles, block_of, n_blocks, tau,
                          absJ_ref, cost_scale=1.0, want_L=False, want_keep=False,
                          threads=0) -> EvalResult:
    """The tile rule with the squared geodesic cost (geodesic bounds from the
    chord bounds of the boxes; rule stated in rsot_oracle.c)."""
    lib = _load()
    x, mu, y, nu, psi = _c(x), _c(mu), _c(y), _c(nu), _c(psi)
    tile_of = _c(tile_of, np.int32)
    block_of = _c(block_of, np.int32)
    nq, n = x.shape[0], y.shape[0]
    J = ctypes.c_double(0.0)
    kept = ctypes.c_int64(0)
    grad = np.empty(n)
    L = np.empty(nq) if want_L else None
    keep = np.empty((n_tiles, n_blocks), dtype=np.uint8) if want_keep else None
    rc = lib.oracle_dual_eval_tile_sphere(nq, _ptr(x), _ptr(mu), n, _ptr(y), _ptr(nu),
                                          _ptr(psi), float(eps), float(cost_scale),
                                          _ptr(tile_of), int(n_tiles), _ptr(block_of),
                                          int(n_blocks), float(tau), float(absJ_ref),
                                          int(threads), ctypes.byref(J), _ptr(grad), _ptr(L),
                                          ctypes.byref(kept), _ptr(keep))
    if rc != 0:
        raise ValueError("oracle_dual_eval_tile_sphere: invalid arguments")
    r = EvalResult(J.value, grad, L, kept.value, 0)
    r.keep = keep
    return r


def sphere_karcher_step(x, mu, y_plan, nu, psi, eps, y_cur, alpha=0.5, cost_scale=1.0,
                        threads=0):
    """Alg. 5, one step for every target: returns (y_next, step_norm, mass)
    with the conditional measures of the plan at (psi, y_plan) fixed and the
    log/exp maps taken at y_cur."""
    lib = _load()
    x, mu, y_plan, nu, psi, y_cur = (_c(a) for a in (x, mu, y_plan, nu, psi, y_cur))
    nq, n = x.shape[0], y_plan.shape[0]
    y_next = np.empty((n, 3))
    step = np.empty(n)
    mass = np.empty(n)
    rc = lib.oracle_sphere_karcher_step(nq, _ptr(x), _ptr(mu), n, _ptr(y_plan), _ptr(nu),
                                        _ptr(psi), float(eps), float(cost_scale), _ptr(y_cur),
                                        float(alpha), int(threads), _ptr(y_next), _ptr(step),
                                        _ptr(mass))
    if rc != 0:
        raise ValueError("oracle_sphere_karcher_step: invalid arguments")
    return y_next, step, mass
