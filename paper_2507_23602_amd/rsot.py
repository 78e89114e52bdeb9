"""Python binding of librsot (ctypes). Argument marshalling only: every step
of the evaluation and the solve runs inside the library; torch supplies
device buffers and the stream.

The library must be built (``python -m paper_2507_23602_amd.build``);
importing this module raises if it is missing, so no code path silently
falls back to anything else.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librsot.so")

OK = 0
ERR_INVALID_ARG = 1
ERR_NONFINITE = 2
ERR_UNBALANCED = 3
ERR_DEVICE = 4
ERR_OOM = 5
ERR_LINESEARCH = 6
ERR_NOT_CONVERGED = 7
ERR_CANCELLED = 8

PREC_MIXED = 0
PREC_FP64 = 1

TRUNC_DENSE = 0
TRUNC_GEOM = 1
TRUNC_INT = 2
TRUNC_PW = 3
TRUNC_TILE = 4

_TRUNC_NAMES = {"dense": TRUNC_DENSE, "geom": TRUNC_GEOM, "int": TRUNC_INT, "pw": TRUNC_PW,
                "tile": TRUNC_TILE}
_PREC_NAMES = {"mixed": PREC_MIXED, "fp64": PREC_FP64}
COST_SQEUCLID, COST_SPHERE = 0, 1
_COST_NAMES = {"sqeuclid": COST_SQEUCLID, "sphere": COST_SPHERE}


class RsotError(RuntimeError):
    """A library call returned an error status. Solves attach the best
    accepted iterate (``psi``) and the solve info (``info``), which the
    library writes on every outcome: they are the state to resume from."""

    def __init__(self, code: int, what: str, psi=None, info=None):
        self.code = code
        self.psi = psi
        self.info = info
        super().__init__(f"{what}: {status_string(code)} ({code})")


class Options(ctypes.Structure):
    _fields_ = [("cost_scale", ctypes.c_double), ("precision", ctypes.c_int),
                ("truncation", ctypes.c_int), ("tau", ctypes.c_double),
                ("delta_thr", ctypes.c_double), ("inputs_on_device", ctypes.c_int),
                ("seg_tiles", ctypes.c_int), ("seg_blocks", ctypes.c_int),
                ("mem_limit_bytes", ctypes.c_int64), ("fp64_below_points", ctypes.c_int64),
                ("tile_group", ctypes.c_int64), ("cost_kind", ctypes.c_int)]


class EvalInfo(ctypes.Structure):
    _fields_ = [("total_pairs", ctypes.c_int64), ("kept_pairs", ctypes.c_int64),
                ("n_empty_qp", ctypes.c_int64), ("cutoff", ctypes.c_double),
                ("absJ_ref", ctypes.c_double), ("log_D", ctypes.c_double),
                ("grad_l1", ctypes.c_double), ("grad_linf", ctypes.c_double),
                ("kernel_ms", ctypes.c_double), ("setup_ms", ctypes.c_double),
                ("passes_ms", ctypes.c_double), ("pass1_ms", ctypes.c_double),
                ("pass2_ms", ctypes.c_double), ("dense_fallback", ctypes.c_int),
                ("fp64_pairs", ctypes.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class IterInfo(ctypes.Structure):
    _fields_ = [("stage", ctypes.c_int), ("iteration", ctypes.c_int),
                ("evaluations", ctypes.c_int), ("eps", ctypes.c_double),
                ("J", ctypes.c_double), ("grad_l1", ctypes.c_double),
                ("grad_linf", ctypes.c_double), ("step", ctypes.c_double),
                ("kept_pairs", ctypes.c_int64), ("cutoff", ctypes.c_double)]


CALLBACK = ctypes.CFUNCTYPE(ctypes.c_int, ctypes.POINTER(IterInfo), ctypes.c_void_p)


class CheckpointStruct(ctypes.Structure):
    _fields_ = [("n_target", ctypes.c_int64), ("capacity", ctypes.c_int),
                ("s", ctypes.POINTER(ctypes.c_double)), ("y", ctypes.POINTER(ctypes.c_double)),
                ("n_pairs", ctypes.c_int), ("stage", ctypes.c_int), ("iteration", ctypes.c_int),
                ("absJ_ref", ctypes.c_double), ("valid", ctypes.c_int)]


class SolveParams(ctypes.Structure):
    _fields_ = [("eps_schedule", ctypes.POINTER(ctypes.c_double)), ("n_eps", ctypes.c_int),
                ("tol", ctypes.c_double), ("max_iter", ctypes.c_int),
                ("lbfgs_m", ctypes.c_int), ("c1", ctypes.c_double), ("c2", ctypes.c_double),
                ("max_ls", ctypes.c_int), ("stage_tol", ctypes.c_double),
                ("callback", CALLBACK), ("user", ctypes.c_void_p),
                ("cancel", ctypes.POINTER(ctypes.c_int)), ("absJ_start", ctypes.c_double),
                ("checkpoint", ctypes.POINTER(CheckpointStruct)), ("resume", ctypes.c_int),
                ("test_flip_gradient", ctypes.c_int)]


class Checkpoint:
    """Host buffers of an rsot_checkpoint: the solver state (eps stage,
    iterations in it, L-BFGS pairs, |J| reference) a stopped solve leaves,
    which a later solve resumes from together with the returned potential."""

    def __init__(self, n_target, capacity=10):
        self.s = np.zeros((capacity, n_target))
        self.y = np.zeros((capacity, n_target))
        self.c = CheckpointStruct()
        self.c.n_target = n_target
        self.c.capacity = capacity
        self.c.s = self.s.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        self.c.y = self.y.ctypes.data_as(ctypes.POINTER(ctypes.c_double))

    def as_dict(self):
        k = self.c.n_pairs
        return dict(valid=self.c.valid, stage=self.c.stage, iteration=self.c.iteration,
                    n_pairs=k, absJ_ref=self.c.absJ_ref, s=self.s[:k].copy(),
                    y=self.y[:k].copy())


class SolveInfo(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int), ("evaluations", ctypes.c_int),
                ("stages", ctypes.c_int), ("J", ctypes.c_double), ("grad_l1", ctypes.c_double),
                ("grad_linf", ctypes.c_double), ("seconds", ctypes.c_double),
                ("eval_ms", ctypes.c_double), ("cull_ms", ctypes.c_double),
                ("pass1_ms", ctypes.c_double), ("pass2_ms", ctypes.c_double),
                ("kept_frac", ctypes.c_double), ("status", ctypes.c_int),
                ("stalled_stages", ctypes.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


ML_MAX = 16


class MLParams(ctypes.Structure):
    _fields_ = [("eps", ctypes.POINTER(ctypes.c_double)), ("level", ctypes.POINTER(ctypes.c_int)),
                ("n_stages", ctypes.c_int), ("base", SolveParams), ("level_tol", ctypes.c_double),
                ("transfer", ctypes.c_int)]


class MLInfo(ctypes.Structure):
    _fields_ = [("n_steps", ctypes.c_int), ("source_level", ctypes.c_int * ML_MAX),
                ("target_level", ctypes.c_int * ML_MAX), ("iterations", ctypes.c_int * ML_MAX),
                ("evaluations", ctypes.c_int * ML_MAX), ("seconds", ctypes.c_double * ML_MAX),
                ("refine_seconds", ctypes.c_double * ML_MAX),
                ("refine_pairs", ctypes.c_int64 * ML_MAX), ("eval_ms", ctypes.c_double * ML_MAX),
                ("kept_frac", ctypes.c_double * ML_MAX), ("total_seconds", ctypes.c_double),
                ("grad_l1", ctypes.c_double), ("status", ctypes.c_int),
                ("stalled_levels", ctypes.c_int)]

    def as_dict(self):
        n = self.n_steps
        d = {k: list(getattr(self, k))[:n] for k in ["source_level", "target_level", "iterations",
                                                     "evaluations", "seconds", "refine_seconds",
                                                     "refine_pairs", "eval_ms", "kept_frac"]}
        d.update(n_steps=n, total_seconds=self.total_seconds, grad_l1=self.grad_l1,
                 status=self.status, stalled_levels=self.stalled_levels)
        return d


class LearnedInfo(ctypes.Structure):
    _fields_ = [("used_learned", ctypes.c_int), ("predict_ms", ctypes.c_double),
                ("J_pred", ctypes.c_double), ("J_zero", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_P = ctypes.c_void_p
_D = ctypes.c_double
_F = ctypes.c_float
_I = ctypes.c_int
_I64 = ctypes.c_int64

MLP_NPARAMS = 199425

# name -> (restype, argtypes); every symbol declared in include/rsot.h
SIGNATURES = {
    "rsot_options_default": (None, [ctypes.POINTER(Options)]),
    "rsot_status_string": (ctypes.c_char_p, [_I]),
    "rsot_problem_create": (_I, [_I, _I64, _P, _P, _I64, _P, _P, ctypes.POINTER(Options), _P,
                                 ctypes.POINTER(_P)]),
    "rsot_problem_destroy": (None, [_P]),
    "rsot_problem_sizes": (_I, [_P, ctypes.POINTER(_I), ctypes.POINTER(_I64),
                                ctypes.POINTER(_I64)]),
    "rsot_set_truncation": (_I, [_P, _I, _D, _D]),
    "rsot_set_precision": (_I, [_P, _I]),
    "rsot_set_reference": (_I, [_P, _D]),
    "rsot_dual_eval": (_I, [_P, _D, _P, ctypes.POINTER(_D), _P, ctypes.POINTER(EvalInfo)]),
    "rsot_dual_eval_noalloc": (_I, [_P, _D, _P, ctypes.POINTER(_D), _P,
                                    ctypes.POINTER(EvalInfo)]),
    "rsot_dual_eval_batched": (_I, [ctypes.POINTER(_P), _I, ctypes.POINTER(_D), ctypes.POINTER(_P),
                                    ctypes.POINTER(_D), ctypes.POINTER(_P),
                                    ctypes.POINTER(EvalInfo), ctypes.POINTER(_D)]),
    "rsot_autotune": (_I, [_P, _D, _P, _I, ctypes.POINTER(_I), ctypes.POINTER(_I),
                           ctypes.POINTER(_I), ctypes.POINTER(_D), ctypes.POINTER(_D)]),
    "rsot_set_tuning": (_I, [_P, _I, _I, _I]),
    "rsot_get_tile_chunk_keep": (_I, [_P, _P]),
    "rsot_sphere_karcher_step": (_I, [_P, _D, _P, _P, _D, _P, _P, _P, ctypes.POINTER(EvalInfo),
                                      ctypes.POINTER(_D)]),
    "rsot_get_target_slots": (_I, [_P, _P]),
    "rsot_get_lse": (_I, [_P, _P]),
    "rsot_get_kept_counts": (_I, [_P, _P]),
    "rsot_get_tile_keep": (_I, [_P, _P]),
    "rsot_covering_cost": (_I, [_P, ctypes.POINTER(_D)]),
    "rsot_get_partition": (_I, [_P, _P, _P, ctypes.POINTER(_I64), ctypes.POINTER(_I64)]),
    "rsot_softmax_refine": (_I, [_P, _D, _P, _I64, _P, _P]),
    "rsot_plan_moments": (_I, [_P, _D, _P, _P, _P, ctypes.POINTER(EvalInfo), ctypes.POINTER(_D)]),
    "rsot_transport_maps": (_I, [_P, _D, _P, _P, _P, ctypes.POINTER(EvalInfo),
                                 ctypes.POINTER(_D)]),
    "rsot_solve_params_default": (None, [ctypes.POINTER(SolveParams)]),
    "rsot_target_hierarchy": (_I, [_I, _I64, _P, _P, _I, ctypes.POINTER(_I64), _I, ctypes.c_uint64,
                                   _P, ctypes.POINTER(_P), ctypes.POINTER(_P), ctypes.POINTER(_P),
                                   ctypes.POINTER(_I64)]),
    "rsot_multilevel_create": (_I, [_I, _I, ctypes.POINTER(_I64), ctypes.POINTER(_P),
                                    ctypes.POINTER(_P), _I, ctypes.POINTER(_I64),
                                    ctypes.POINTER(_P), ctypes.POINTER(_P),
                                    ctypes.POINTER(Options), _P, ctypes.POINTER(_P)]),
    "rsot_multilevel_destroy": (None, [_P]),
    "rsot_multilevel_indices": (None, [_I, _I, _I, ctypes.POINTER(_I), ctypes.POINTER(_I)]),
    "rsot_solve_multilevel": (_I, [_P, ctypes.POINTER(MLParams), _P, ctypes.POINTER(MLInfo)]),
    "rsot_solve": (_I, [_P, ctypes.POINTER(SolveParams), _P, ctypes.POINTER(SolveInfo)]),
    # include/rsot_mlp.h
    "rsot_mlp_create": (_I, [_P, _P, ctypes.POINTER(_P)]),
    "rsot_mlp_destroy": (None, [_P]),
    "rsot_mlp_get_params": (_I, [_P, _I, _P]),
    "rsot_mlp_set_params": (_I, [_P, _P]),
    "rsot_mlp_set_normalization": (_I, [_P, _P, _P, _F, _F]),
    "rsot_mlp_get_normalization": (_I, [_P, _P, _P, ctypes.POINTER(_F), ctypes.POINTER(_F)]),
    "rsot_mlp_fit_normalization": (_I, [_P, _P, _P, _I64]),
    "rsot_mlp_features": (_I, [_I64, _P, _P, _P, _P]),
    "rsot_mlp_forward": (_I, [_P, _P, _I64, _P]),
    "rsot_mlp_backward": (_I, [_P, _P, _I64, _P, _P]),
    "rsot_mlp_adam_step": (_I, [_P, _P, _F, _F, _F, _F]),
    "rsot_mlp_train_step": (_I, [_P, _P, _P, _P, _I64, _F, _F, _F, _F, ctypes.POINTER(_D)]),
    "rsot_mlp_predict_psi": (_I, [_P, _I64, _P, _P, _P, _P]),
    "rsot_solve_learned": (_I, [_P, _P, _P, ctypes.POINTER(SolveParams), _P,
                                ctypes.POINTER(SolveInfo), ctypes.POINTER(LearnedInfo)]),
}

_lib = None


def load_library(path: str = LIB_PATH):
    """Loads librsot.so and binds every ABI symbol. Raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"librsot.so not built at {path}: run python -m paper_2507_23602_amd.build")
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def status_string(code: int) -> str:
    try:
        return load_library().rsot_status_string(code).decode()
    except Exception:
        return str(code)


def _check(code: int, what: str):
    if code != OK:
        raise RsotError(code, what)


def default_options(**kw) -> Options:
    o = Options()
    load_library().rsot_options_default(ctypes.byref(o))
    for k, v in kw.items():
        if k == "truncation" and isinstance(v, str):
            v = _TRUNC_NAMES[v]
        if k == "precision" and isinstance(v, str):
            v = _PREC_NAMES[v]
        setattr(o, k, v)
    return o


def _torch():
    import torch
    return torch


def _dev_f64(t, n=None):
    torch = _torch()
    if not isinstance(t, torch.Tensor):
        t = torch.as_tensor(np.ascontiguousarray(t, dtype=np.float64), device="cuda")
    if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous():
        t = t.to(device="cuda", dtype=torch.float64).contiguous()
    if n is not None and t.numel() != n:
        raise ValueError(f"expected {n} values, got {t.numel()}")
    return t


@dataclass
class EvalResult:
    J: float
    grad: object          # torch.Tensor (cuda, float64) or None
    info: dict


class Problem:
    """Owns an rsot_problem handle. Inputs are host numpy arrays or CUDA
    tensors (float64); the library copies them."""

    def __init__(self, x, mu, y, nu, *, cost_scale=0.5, precision="mixed", truncation="dense",
                 tau=1e-12, delta_thr=1e-12, seg_tiles=0, seg_blocks=0, mem_limit_bytes=0,
                 fp64_below_points=None, tile_group=0, cost="sqeuclid", stream=None):
        torch = _torch()
        lib = load_library()
        on_dev = isinstance(x, torch.Tensor) and x.is_cuda
        if on_dev:
            xs, mus, ys, nus = (t.to(torch.float64).contiguous() for t in (x, mu, y, nu))
            ptrs = [t.data_ptr() for t in (xs, mus, ys, nus)]
            self._keep = (xs, mus, ys, nus)
        else:
            xs, mus, ys, nus = (np.ascontiguousarray(a, dtype=np.float64) for a in (x, mu, y, nu))
            ptrs = [a.ctypes.data for a in (xs, mus, ys, nus)]
            self._keep = (xs, mus, ys, nus)
        dim = xs.shape[1]
        nq, n = xs.shape[0], ys.shape[0]
        extra = {} if fp64_below_points is None else {"fp64_below_points": fp64_below_points}
        opt = default_options(cost_scale=cost_scale, precision=precision, truncation=truncation,
                              tau=tau, delta_thr=delta_thr, inputs_on_device=int(on_dev),
                              seg_tiles=seg_tiles, seg_blocks=seg_blocks,
                              mem_limit_bytes=mem_limit_bytes, tile_group=tile_group,
                              cost_kind=_COST_NAMES[cost], **extra)
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        h = _P()
        _check(lib.rsot_problem_create(dim, nq, ptrs[0], ptrs[1], n, ptrs[2], ptrs[3],
                                       ctypes.byref(opt), _P(stream.cuda_stream), ctypes.byref(h)),
               "rsot_problem_create")
        self._h = h
        self._keep = None
        self.dim, self.nq, self.n = dim, nq, n

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load_library().rsot_problem_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    def set_truncation(self, truncation, tau=1e-12, delta_thr=1e-12):
        if isinstance(truncation, str):
            truncation = _TRUNC_NAMES[truncation]
        _check(load_library().rsot_set_truncation(self._h, truncation, tau, delta_thr),
               "rsot_set_truncation")

    def set_precision(self, precision):
        if isinstance(precision, str):
            precision = _PREC_NAMES[precision]
        _check(load_library().rsot_set_precision(self._h, precision), "rsot_set_precision")

    def set_reference(self, absJ):
        _check(load_library().rsot_set_reference(self._h, float(absJ)), "rsot_set_reference")

    def dual_eval(self, psi, eps, want_grad=True, out=None) -> EvalResult:
        """J(psi) and grad J(psi); psi (N,) float64 CUDA tensor or array."""
        torch = _torch()
        psi_t = _dev_f64(psi, self.n)
        grad = None
        if want_grad:
            grad = out if out is not None else torch.empty(self.n, dtype=torch.float64, device="cuda")
        J = _D(0.0)
        info = EvalInfo()
        _check(load_library().rsot_dual_eval(self._h, float(eps), psi_t.data_ptr(), ctypes.byref(J),
                                             grad.data_ptr() if grad is not None else None,
                                             ctypes.byref(info)), "rsot_dual_eval")
        return EvalResult(J.value, grad, info.as_dict())

    def dual_eval_noalloc(self, psi, eps, want_grad=True, out=None) -> EvalResult:
        """rsot_dual_eval_noalloc: the dense evaluation with no device
        allocation inside the call (psi and out must already be CUDA tensors)."""
        torch = _torch()
        psi_t = _dev_f64(psi, self.n)
        grad = None
        if want_grad:
            grad = out if out is not None else torch.empty(self.n, dtype=torch.float64, device="cuda")
        J = _D(0.0)
        info = EvalInfo()
        _check(load_library().rsot_dual_eval_noalloc(
            self._h, float(eps), psi_t.data_ptr(), ctypes.byref(J),
            grad.data_ptr() if grad is not None else None, ctypes.byref(info)),
            "rsot_dual_eval_noalloc")
        return EvalResult(J.value, grad, info.as_dict())

    def autotune(self, psi, eps, reps=2):
        """rsot_autotune: returns dict(seg_blocks, seg_tiles, tile_group,
        best_ms, default_ms)."""
        pt = _dev_f64(psi, self.n)
        sb, st, gr = _I(0), _I(0), _I(0)
        best, dflt = _D(0), _D(0)
        _check(load_library().rsot_autotune(self._h, float(eps), pt.data_ptr(), int(reps),
                                            ctypes.byref(sb), ctypes.byref(st), ctypes.byref(gr),
                                            ctypes.byref(best), ctypes.byref(dflt)),
               "rsot_autotune")
        return {"seg_blocks": sb.value, "seg_tiles": st.value, "tile_group": gr.value,
                "best_ms": best.value, "default_ms": dflt.value}

    def set_tuning(self, seg_blocks, seg_tiles, tile_group=0):
        _check(load_library().rsot_set_tuning(self._h, int(seg_blocks), int(seg_tiles),
                                              int(tile_group)), "rsot_set_tuning")

    def lse(self):
        torch = _torch()
        out = torch.empty(self.nq, dtype=torch.float64, device="cuda")
        _check(load_library().rsot_get_lse(self._h, out.data_ptr()), "rsot_get_lse")
        return out

    def kept_counts(self):
        """|I_q| of every point in the last evaluation (int32 CUDA tensor)."""
        torch = _torch()
        out = torch.empty(self.nq, dtype=torch.int32, device="cuda")
        _check(load_library().rsot_get_kept_counts(self._h, out.data_ptr()),
               "rsot_get_kept_counts")
        return out

    def tile_keep(self):
        """(tile, block) culling decisions of the last evaluation: uint8 CUDA
        tensor (n_tiles, n_blocks), 0 skipped, 1 tested per pair, 2 kept."""
        torch = _torch()
        nt, nb = _I64(0), _I64(0)
        _check(load_library().rsot_get_partition(self._h, None, None, ctypes.byref(nt),
                                                 ctypes.byref(nb)), "rsot_get_partition")
        out = torch.empty((nt.value, nb.value), dtype=torch.uint8, device="cuda")
        _check(load_library().rsot_get_tile_keep(self._h, out.data_ptr()), "rsot_get_tile_keep")
        return out

    def sphere_karcher_step(self, psi, eps, y_cur, alpha=0.5):
        """Alg. 5, one step for every target (squared geodesic cost on the
        sphere): the plan's conditional measures at (psi, the problem's
        targets) with the log and exp maps at y_cur (n x 3 unit vectors).
        Returns (y_next CUDA tensor n x 3, step norms |delta_j|, masses
        nu~_j, kernel ms)."""
        torch = _torch()
        psi_t = _dev_f64(psi, self.n)
        yc = _dev_f64(y_cur).reshape(self.n, 3).contiguous()
        yn = torch.empty((self.n, 3), dtype=torch.float64, device="cuda")
        st = torch.empty(self.n, dtype=torch.float64, device="cuda")
        ms = torch.empty(self.n, dtype=torch.float64, device="cuda")
        info, kms = EvalInfo(), _D(0.0)
        _check(load_library().rsot_sphere_karcher_step(self._h, float(eps), psi_t.data_ptr(),
                                                       yc.data_ptr(), float(alpha),
                                                       yn.data_ptr(), st.data_ptr(),
                                                       ms.data_ptr(), ctypes.byref(info),
                                                       ctypes.byref(kms)),
               "rsot_sphere_karcher_step")
        return yn, st, ms, kms.value

    def tile_chunk_keep(self):
        """Per (tile, block) of the last evaluation the bits of the block's
        8-target chunks whose pairs entered it: uint8 CUDA tensor
        (n_tiles, n_blocks)."""
        torch = _torch()
        nt, nb = _I64(0), _I64(0)
        _check(load_library().rsot_get_partition(self._h, None, None, ctypes.byref(nt),
                                                 ctypes.byref(nb)), "rsot_get_partition")
        out = torch.empty((nt.value, nb.value), dtype=torch.uint8, device="cuda")
        _check(load_library().rsot_get_tile_chunk_keep(self._h, out.data_ptr()),
               "rsot_get_tile_chunk_keep")
        return out

    def target_slots(self):
        """Each target's position in the sorted, padded order (int32 CUDA)."""
        torch = _torch()
        out = torch.empty(self.n, dtype=torch.int32, device="cuda")
        _check(load_library().rsot_get_target_slots(self._h, out.data_ptr()),
               "rsot_get_target_slots")
        return out

    def softmax_refine(self, psi_coarse, eps, y_fine):
        """Eq. softmax_refinement_formula: potentials of y_fine from this
        problem's (coarse) targets and psi_coarse at its points."""
        torch = _torch()
        pc = _dev_f64(psi_coarse, self.n)
        yf = _dev_f64(y_fine)
        nf = yf.numel() // self.dim
        out = torch.empty(nf, dtype=torch.float64, device="cuda")
        _check(load_library().rsot_softmax_refine(self._h, float(eps), pc.data_ptr(), nf,
                                                  yf.data_ptr(), out.data_ptr()),
               "rsot_softmax_refine")
        return out

    def plan_moments(self, psi, eps):
        """rsot_plan_moments: (nu~ (N,), first moments (N, dim), info, kernel ms)
        as CUDA float64 tensors."""
        torch = _torch()
        pt = _dev_f64(psi, self.n)
        mass = torch.empty(self.n, dtype=torch.float64, device="cuda")
        first = torch.empty((self.n, self.dim), dtype=torch.float64, device="cuda")
        info, ms = EvalInfo(), _D(0.0)
        _check(load_library().rsot_plan_moments(self._h, float(eps), pt.data_ptr(),
                                                mass.data_ptr(), first.data_ptr(),
                                                ctypes.byref(info), ctypes.byref(ms)),
               "rsot_plan_moments")
        return mass, first, info.as_dict(), ms.value

    def transport_maps(self, psi, eps):
        """rsot_transport_maps: (barycentric map (nq, dim), modal target index
        (nq,) int32, info, kernel ms) as CUDA tensors."""
        torch = _torch()
        pt = _dev_f64(psi, self.n)
        bary = torch.empty((self.nq, self.dim), dtype=torch.float64, device="cuda")
        modal = torch.empty(self.nq, dtype=torch.int32, device="cuda")
        info, ms = EvalInfo(), _D(0.0)
        _check(load_library().rsot_transport_maps(self._h, float(eps), pt.data_ptr(),
                                                  bary.data_ptr(), modal.data_ptr(),
                                                  ctypes.byref(info), ctypes.byref(ms)),
               "rsot_transport_maps")
        return bary, modal, info.as_dict(), ms.value

    def covering_cost(self) -> float:
        c = _D(0.0)
        _check(load_library().rsot_covering_cost(self._h, ctypes.byref(c)), "rsot_covering_cost")
        return c.value

    def partition(self):
        torch = _torch()
        t = torch.empty(self.nq, dtype=torch.int32, device="cuda")
        b = torch.empty(self.n, dtype=torch.int32, device="cuda")
        nt, nb = _I64(0), _I64(0)
        _check(load_library().rsot_get_partition(self._h, t.data_ptr(), b.data_ptr(),
                                                 ctypes.byref(nt), ctypes.byref(nb)),
               "rsot_get_partition")
        return t, b, nt.value, nb.value

    @staticmethod
    def _solve_params(eps_arr, tol, max_iter, lbfgs_m, stage_tol, callback, max_ls,
                      absJ_start=0.0):
        sp = SolveParams()
        load_library().rsot_solve_params_default(ctypes.byref(sp))
        sp.eps_schedule = eps_arr.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        sp.n_eps = eps_arr.shape[0]
        sp.tol = tol
        sp.max_iter = max_iter
        sp.lbfgs_m = lbfgs_m
        sp.stage_tol = stage_tol
        sp.max_ls = max_ls
        sp.absJ_start = absJ_start
        cb = None
        if callback is not None:
            def _cb(ptr, _user):
                return int(bool(callback(ptr.contents)))
            cb = CALLBACK(_cb)
            sp.callback = cb
        return sp, cb

    def solve(self, eps_schedule, psi0=None, tol=1e-6, max_iter=10000, lbfgs_m=10,
              stage_tol=0.0, callback=None, max_ls=20, absJ_start=0.0, checkpoint=None,
              resume=False, test_flip_gradient=False):
        """rsot_solve: returns (psi numpy array, info dict). Raises on error
        codes other than NOT_CONVERGED (reported in info['status']).
        ``absJ_start``: |J| reference of the truncation rules for the first
        evaluation (0: that evaluation runs dense to obtain it).
        ``checkpoint``: a Checkpoint the solver state is written to on exit;
        with ``resume`` the solve continues from it at ``psi0``.
        ``test_flip_gradient``: test hook, the solver is handed -grad."""
        eps_arr = np.ascontiguousarray(np.atleast_1d(eps_schedule), dtype=np.float64)
        psi = np.zeros(self.n) if psi0 is None else np.array(psi0, dtype=np.float64)
        sp, _keep = self._solve_params(eps_arr, tol, max_iter, lbfgs_m, stage_tol, callback,
                                       max_ls, absJ_start)
        if checkpoint is not None:
            sp.checkpoint = ctypes.pointer(checkpoint.c)
        sp.resume = int(bool(resume))
        sp.test_flip_gradient = int(bool(test_flip_gradient))
        info = SolveInfo()
        rc = load_library().rsot_solve(self._h, ctypes.byref(sp), psi.ctypes.data,
                                       ctypes.byref(info))
        if rc not in (OK, ERR_NOT_CONVERGED):
            raise RsotError(rc, "rsot_solve", psi=psi, info=info.as_dict())
        return psi, info.as_dict()

    def solve_learned(self, mlp, cond, eps_schedule, tol=1e-6, max_iter=10000, lbfgs_m=10,
                      stage_tol=0.0, max_ls=20):
        """rsot_solve_learned: returns (psi, solve info dict, learned info
        dict). cond = (c0, c1, s, eps) of the instance."""
        eps_arr = np.ascontiguousarray(np.atleast_1d(eps_schedule), dtype=np.float64)
        c = np.ascontiguousarray(cond, dtype=np.float64)
        psi = np.zeros(self.n)
        sp, _keep = self._solve_params(eps_arr, tol, max_iter, lbfgs_m, stage_tol, None, max_ls)
        info, linfo = SolveInfo(), LearnedInfo()
        rc = load_library().rsot_solve_learned(self._h, mlp.handle, c.ctypes.data,
                                               ctypes.byref(sp), psi.ctypes.data,
                                               ctypes.byref(info), ctypes.byref(linfo))
        if rc not in (OK, ERR_NOT_CONVERGED):
            raise RsotError(rc, "rsot_solve_learned")
        return psi, info.as_dict(), linfo.as_dict()


def multilevel_indices(n_source_levels: int, n_target_levels: int, l: int):
    a, b = _I(0), _I(0)
    load_library().rsot_multilevel_indices(n_source_levels, n_target_levels, l, ctypes.byref(a),
                                           ctypes.byref(b))
    return a.value, b.value


def target_hierarchy(y, nu, n_per_level, lloyd_iters=20, seed=6, with_parents=False):
    """k-means coarsening (Sec. 5.2); returns [(y_l, nu_l)] coarsest first, as
    CUDA float64 tensors (and the parent maps when asked)."""
    torch = _torch()
    y_t = _dev_f64(y)
    dim = y_t.shape[1] if y_t.dim() == 2 else int(np.asarray(y).shape[1])
    nu_t = _dev_f64(nu)
    n = nu_t.numel()
    L = len(n_per_level)
    ys = [torch.empty((int(k), dim), dtype=torch.float64, device="cuda") for k in n_per_level]
    ns = [torch.empty(int(k), dtype=torch.float64, device="cuda") for k in n_per_level]
    npl = (_I64 * L)(*[int(k) for k in n_per_level])
    nout = (_I64 * L)()
    par = [torch.full((int(k),), -1, dtype=torch.int32, device="cuda") for k in n_per_level]
    yp = (_P * L)(*[t.data_ptr() for t in ys])
    npp = (_P * L)(*[t.data_ptr() for t in ns])
    pp = (_P * L)(*[t.data_ptr() for t in par])
    stream = torch.cuda.current_stream().cuda_stream
    _check(load_library().rsot_target_hierarchy(dim, n, y_t.data_ptr(), nu_t.data_ptr(), L, npl,
                                                int(lloyd_iters), int(seed), _P(stream), yp, npp,
                                                pp, nout), "rsot_target_hierarchy")
    levels = [(ys[l][:nout[l]], ns[l][:nout[l]]) for l in range(L)]
    if with_parents:
        return levels, [par[l][:nout[l]] for l in range(L)]
    return levels


class Multilevel:
    """Combined source/target multilevel solver (Sec. 5.3)."""

    def __init__(self, sources, targets, *, cost_scale=0.5, precision="mixed",
                 truncation="tile", tau=1e-12, tile_group=0, fp64_below_points=None):
        torch = _torch()
        lib = load_library()
        self._src = [(_dev_f64(x).reshape(len(m) if not isinstance(m, torch.Tensor) else m.numel(), -1),
                      _dev_f64(m)) for x, m in sources]
        self._tgt = [(_dev_f64(y).reshape(len(v) if not isinstance(v, torch.Tensor) else v.numel(), -1),
                      _dev_f64(v)) for y, v in targets]
        dim = self._src[0][0].shape[1]
        ns, nt = len(self._src), len(self._tgt)
        nq = (_I64 * ns)(*[m.numel() for _, m in self._src])
        ntg = (_I64 * nt)(*[v.numel() for _, v in self._tgt])
        xp = (_P * ns)(*[x.data_ptr() for x, _ in self._src])
        mp = (_P * ns)(*[m.data_ptr() for _, m in self._src])
        yp = (_P * nt)(*[y.data_ptr() for y, _ in self._tgt])
        vp = (_P * nt)(*[v.data_ptr() for _, v in self._tgt])
        extra = {} if fp64_below_points is None else {"fp64_below_points": fp64_below_points}
        opt = default_options(cost_scale=cost_scale, precision=precision, truncation=truncation,
                              tau=tau, inputs_on_device=1, tile_group=tile_group, **extra)
        h = _P()
        _check(lib.rsot_multilevel_create(dim, ns, nq, xp, mp, nt, ntg, yp, vp, ctypes.byref(opt),
                                          _P(torch.cuda.current_stream().cuda_stream),
                                          ctypes.byref(h)), "rsot_multilevel_create")
        self._h = h
        self.n_final = self._tgt[-1][1].numel()

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load_library().rsot_multilevel_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def solve(self, eps, level, tol=1e-6, level_tol=0.0, max_iter=10000, callback=None,
              stage_tol=0.0, lbfgs_m=10, test_flip_gradient=False):
        """rsot_solve_multilevel. ``callback(iter_info)`` is called after every
        accepted iteration of every level; a true return value cancels.
        ``level_tol`` / ``stage_tol``: ||grad||_1 targets of non-final levels
        and of non-final eps stages within a level (0 = tol)."""
        lib = load_library()
        e = np.ascontiguousarray(eps, dtype=np.float64)
        lv = np.ascontiguousarray(level, dtype=np.int32)
        mp = MLParams()
        lib.rsot_solve_params_default(ctypes.byref(mp.base))
        mp.base.tol = tol
        mp.base.max_iter = max_iter
        mp.base.stage_tol = stage_tol
        mp.base.lbfgs_m = lbfgs_m
        mp.base.test_flip_gradient = int(bool(test_flip_gradient))
        cb = None
        if callback is not None:
            def _cb(ptr, _user):
                return int(bool(callback(ptr.contents)))
            cb = CALLBACK(_cb)
            mp.base.callback = cb
        mp.eps = e.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        mp.level = lv.ctypes.data_as(ctypes.POINTER(ctypes.c_int))
        mp.n_stages = len(e)
        mp.level_tol = level_tol
        mp.transfer = 0
        psi = np.zeros(self.n_final)
        info = MLInfo()
        rc = lib.rsot_solve_multilevel(self._h, ctypes.byref(mp), psi.ctypes.data,
                                       ctypes.byref(info))
        if rc not in (OK, ERR_NOT_CONVERGED):
            raise RsotError(rc, "rsot_solve_multilevel", psi=psi, info=info.as_dict())
        return psi, info.as_dict()


def dual_eval_batched(problems, eps, psis, want_grad=True):
    """rsot_dual_eval_batched over Problem objects; returns (J list, grads,
    infos, batch_ms)."""
    torch = _torch()
    n = len(problems)
    hs = (_P * n)(*[pr.handle for pr in problems])
    e = (_D * n)(*[float(v) for v in eps])
    ps = [_dev_f64(v, pr.n) for v, pr in zip(psis, problems)]
    pp = (_P * n)(*[t.data_ptr() for t in ps])
    J = (_D * n)()
    grads = [torch.empty(pr.n, dtype=torch.float64, device="cuda") for pr in problems] \
        if want_grad else None
    gp = (_P * n)(*[g.data_ptr() for g in grads]) if want_grad else None
    infos = (EvalInfo * n)()
    ms = _D(0.0)
    _check(load_library().rsot_dual_eval_batched(hs, n, e, pp, J, gp, infos, ctypes.byref(ms)),
           "rsot_dual_eval_batched")
    return list(J), grads, [i.as_dict() for i in infos], ms.value


def shape_class(dim, nq, n, eps, truncation):
    """Key of the autotuner cache: dimension, log2 sizes, decade of eps, rule."""
    import math
    return f"d{dim}_q{int(round(math.log2(nq)))}_n{int(round(math.log2(n)))}" \
           f"_e{int(math.floor(math.log10(eps)))}_{truncation}"


def tuned(problem, psi, eps, truncation, cache_path, reps=2):
    """Applies cached tuning for the problem's shape class, or runs the
    autotuner and stores the result in the JSON cache."""
    import json
    key = shape_class(problem.dim, problem.nq, problem.n, eps, truncation)
    cache = {}
    if cache_path and os.path.exists(cache_path):
        with open(cache_path) as f:
            cache = json.load(f)
    if key in cache:
        problem.set_tuning(cache[key]["seg_blocks"], cache[key]["seg_tiles"],
                           cache[key].get("tile_group", 0))
        return dict(cache[key], cached=True)
    res = problem.autotune(psi, eps, reps=reps)
    cache[key] = res
    if cache_path:
        with open(cache_path, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
    return dict(res, cached=False)


def _dev_f32(t, n=None):
    torch = _torch()
    if not isinstance(t, torch.Tensor):
        t = torch.as_tensor(np.ascontiguousarray(t, dtype=np.float32), device="cuda")
    if t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous():
        t = t.to(device="cuda", dtype=torch.float32).contiguous()
    if n is not None and t.numel() != n:
        raise ValueError(f"expected {n} values, got {t.numel()}")
    return t


class MLP:
    """Owns an rsot_mlp handle (include/rsot_mlp.h): the warm-start network,
    its training kernels and its prediction. Device arrays are CUDA tensors."""

    def __init__(self, params, stream=0):
        p = np.ascontiguousarray(params, dtype=np.float32)
        if p.shape != (MLP_NPARAMS,):
            raise ValueError(f"expected {MLP_NPARAMS} parameters")
        h = _P()
        _check(load_library().rsot_mlp_create(p.ctypes.data, stream, ctypes.byref(h)),
               "rsot_mlp_create")
        self._h = h

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None):
            load_library().rsot_mlp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def params(self, which=0):
        out = np.empty(MLP_NPARAMS, dtype=np.float32)
        _check(load_library().rsot_mlp_get_params(self._h, int(which), out.ctypes.data),
               "rsot_mlp_get_params")
        return out

    def set_params(self, params):
        p = np.ascontiguousarray(params, dtype=np.float32)
        _check(load_library().rsot_mlp_set_params(self._h, p.ctypes.data), "rsot_mlp_set_params")

    def set_normalization(self, feat_mean, feat_std, out_mean, out_std):
        fm = np.ascontiguousarray(feat_mean, dtype=np.float32)
        fs = np.ascontiguousarray(feat_std, dtype=np.float32)
        _check(load_library().rsot_mlp_set_normalization(self._h, fm.ctypes.data, fs.ctypes.data,
                                                         float(out_mean), float(out_std)),
               "rsot_mlp_set_normalization")

    def normalization(self):
        fm, fs = np.empty(6, dtype=np.float32), np.empty(6, dtype=np.float32)
        om, osd = _F(), _F()
        _check(load_library().rsot_mlp_get_normalization(self._h, fm.ctypes.data, fs.ctypes.data,
                                                         ctypes.byref(om), ctypes.byref(osd)),
               "rsot_mlp_get_normalization")
        return fm, fs, om.value, osd.value

    def fit_normalization(self, feats, target):
        f = _dev_f32(feats)
        t = _dev_f32(target)
        rows = t.numel()
        if f.numel() != 6 * rows:
            raise ValueError("feature rows and targets differ in count")
        _check(load_library().rsot_mlp_fit_normalization(self._h, f.data_ptr(), t.data_ptr(),
                                                         rows), "rsot_mlp_fit_normalization")

    def forward(self, feats):
        torch = _torch()
        f = _dev_f32(feats)
        rows = f.numel() // 6
        out = torch.empty(rows, dtype=torch.float32, device="cuda")
        _check(load_library().rsot_mlp_forward(self._h, f.data_ptr(), rows, out.data_ptr()),
               "rsot_mlp_forward")
        return out

    def backward(self, feats, dout):
        torch = _torch()
        f = _dev_f32(feats)
        rows = f.numel() // 6
        d = _dev_f32(dout, rows)
        g = torch.empty(MLP_NPARAMS, dtype=torch.float32, device="cuda")
        _check(load_library().rsot_mlp_backward(self._h, f.data_ptr(), rows, d.data_ptr(),
                                                g.data_ptr()), "rsot_mlp_backward")
        return g

    def adam_step(self, grad, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        g = _dev_f32(grad, MLP_NPARAMS)
        _check(load_library().rsot_mlp_adam_step(self._h, g.data_ptr(), lr, b1, b2, eps),
               "rsot_mlp_adam_step")

    def train_step(self, feats, target, idx=None, rows=None, lr=1e-3, b1=0.9, b2=0.999,
                   eps=1e-8, want_loss=True):
        """One fused step on the device tables feats (N x 6) / target (N); idx
        (int64 CUDA tensor of row numbers) selects the batch."""
        if rows is None:
            rows = idx.numel() if idx is not None else target.numel()
        loss = _D(0.0)
        _check(load_library().rsot_mlp_train_step(
            self._h, feats.data_ptr(), target.data_ptr(),
            idx.data_ptr() if idx is not None else None, int(rows), lr, b1, b2, eps,
            ctypes.byref(loss) if want_loss else None), "rsot_mlp_train_step")
        return loss.value if want_loss else None

    def predict_psi(self, y, nu, cond):
        torch = _torch()
        yt = _dev_f64(y)
        n = yt.numel() // 2
        nt = _dev_f64(nu, n)
        c = np.ascontiguousarray(cond, dtype=np.float64)
        out = torch.empty(n, dtype=torch.float64, device="cuda")
        _check(load_library().rsot_mlp_predict_psi(self._h, n, yt.data_ptr(), nt.data_ptr(),
                                                   c.ctypes.data, out.data_ptr()),
               "rsot_mlp_predict_psi")
        return out


def mlp_features(y, cond):
    """rsot_mlp_features: (y0, y1, c0, c1, s, log eps) rows on the device."""
    torch = _torch()
    yt = _dev_f64(y)
    n = yt.numel() // 2
    c = np.ascontiguousarray(cond, dtype=np.float64)
    out = torch.empty((n, 6), dtype=torch.float32, device="cuda")
    _check(load_library().rsot_mlp_features(n, yt.data_ptr(), c.ctypes.data, out.data_ptr(),
                                            None), "rsot_mlp_features")
    return out
