"""Benchmark of the RSOT dual evaluation on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

A step is one rsot_dual_eval (objective + gradient, dense, mixed precision)
on the 3D workload: unit cube, 64^3 cells x 6 Kuhn tetrahedra x 4 points =
6,291,456 quadrature points, 3-Gaussian-mixture source, 65,536 mixture
targets, eps = 1e-3, psi a seeded N(0, eps^2) perturbation. Inputs are
resident in device memory before the timed region. The JSON line (stdout)
reports dense pairs/s as ``value``, the roofline of the dominant kernel and
the CPU oracle on a bounded sample, and under "extras" every other workload:
the truncated rules and the FP64 path on this workload; time to
||grad||_1 < 1e-6 on the 2D square (FP64), on this workload from psi = 0 and
from the multilevel start; the multilevel disk workload; 64 uneven batched
instances against single calls; the learned warm start against the zero and
multilevel starts on held-out instances; the network kernels. Each solve's
returned potential is re-checked independently (the oracle where it finishes
in seconds, else the FP64 path). --quick skips the disk, batched and learned
legs. Progress goes to stderr.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X figures used by the roofline (256 CUs at 2.4 GHz):
#   FP32 vector 157.3 TFLOP/s -> 7.86e13 lane-ops/s (128 lanes/clk/CU, an FMA
#   counted as one op); a rate microbenchmark reached 6.26e13/s with
#   non-packed v_fma_f32.
#   v_exp_f32 at 32 lanes/clk/CU = 1.966e13/s: a quarter of the 128-lane FP32
#   rate (the microbenchmark measured 1.905e13/s). The per-pair op counts are
#   the algorithm's, not the kernel's.
PEAK_VALU_OPS = 256 * 2.4e9 * 128          # 7.86e13 FP32 lane-ops/s
PEAK_EXP = 256 * 2.4e9 * 32                # 1.966e13 exp/s


def log(*a):
    print(*a, file=sys.stderr, flush=True)


TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "dense_eval_cube64_n65536_hbm_traffic.md")
# the evaluation passes' source: the kernels and the pair helpers they include
EVAL_SOURCES = [os.path.join(ROOT, "paper_2507_23602_amd", "csrc", f)
                for f in ("rsot_eval.hip", "rsot_pairs.h", "rsot_device.h")]


def eval_source_sha():
    """sha256 of the evaluation sources, concatenated in order"""
    h = hashlib.sha256()
    for f in EVAL_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def counter_traffic(kernel: str):
    """HBM bytes per launch of `kernel` from the committed FETCH_SIZE /
    WRITE_SIZE summary (scaled by the plain-copy calibration it records), or
    None when that summary was taken on another version of the kernel source."""
    if not os.path.exists(TRAFFIC_SUMMARY):
        return None
    txt = open(TRAFFIC_SUMMARY).read()
    m = re.search(r"kernel source sha256: ([0-9a-f]{64})", txt)
    if not m or m.group(1) != eval_source_sha():
        return None
    m = re.search(re.escape(kernel) + r" HBM bytes per launch: ([0-9.eE+]+)", txt)
    return float(m.group(1)) if m else None


def pair_roofline(d: int, n_exp: int, n_ops: int) -> float:
    """pairs/s at the ALU roofline for n_exp exponentials and n_ops FP32 ops per pair"""
    return 1.0 / (n_exp / PEAK_EXP + n_ops / PEAK_VALU_OPS)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--no-extras", action="store_true", help="dense mixed only")
    ap.add_argument("--main-extras", type=int, default=1,
                    help="0: skip the extras on the benchmark workload itself (rules, FP64, "
                         "moments, solves) and run only the legs; 2: only its GEOM and "
                         "tile-rule rows")
    ap.add_argument("--quick", action="store_true",
                    help="skip the disk multilevel, batched and learned legs")
    ap.add_argument("--ml-spread", action="store_true",
                    help="multilevel leg with the eps stages spread over all four levels")
    ap.add_argument("--no-multilevel", action="store_true",
                    help="skip the combined multilevel solve of the 2D disk workload")
    ap.add_argument("--batched", type=int, default=64,
                    help="N uneven 3D instances: one batched call vs single calls (0: skip)")
    ap.add_argument("--copy-calib", action="store_true",
                    help="run one plain 256 MiB device copy first (scale for HBM counters)")
    ap.add_argument("--mlp", type=str, default="65536,20",
                    help="time the warm-start network kernels: 'ROWS,STEPS' training steps "
                         "and forward passes on synthetic rows ('' to skip)")
    ap.add_argument("--tile-group", type=int, default=0,
                    help="targets per culling group of the tile rule in the multilevel leg "
                         "(0: library default)")
    ap.add_argument("--trunc-study", type=int, default=1,
                    help="truncation-strategy study on both densities (0: skip)")
    ap.add_argument("--sphere", type=int, default=1,
                    help="blue-noise sampling and evaluation rate on the sphere (0: skip)")
    ap.add_argument("--barycenter", type=int, default=1,
                    help="damped-Lloyd Wasserstein barycentre of two 2D sources (0: skip)")
    ap.add_argument("--trunc-tol", type=str, default="1e-3",
                    help="stopping tolerances of the truncation study, comma separated")
    ap.add_argument("--gpu-size", type=str, default="2-5x1-3",
                    help="App. C sizes 'R0-R1xG0-G1' (refinements x Gauss orders; '' to skip)")
    ap.add_argument("--learned", type=str, default="448,64,30",
                    help="learned warm start on the blob family: 'TRAIN,TEST,EPOCHS': dataset "
                         "from the solver, training, comparison ('' to skip)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported "
              "(the multi-GPU path is a design note only)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2507_23602_amd import rsot, workloads as W

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.copy_calib:
        a = torch.ones(32 << 20, dtype=torch.float64, device=dev)     # 256 MiB
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        log("[bench] copy calibration: 268435456 bytes read, 268435456 bytes written")
        del a, b
    t0 = time.time()
    p = W.config2()
    log(f"[bench] workload {p.name}: nq={p.nq} n={p.n} eps={p.eps} (gen {time.time()-t0:.1f}s)")
    x_d = torch.as_tensor(p.x, device=dev)
    mu_d = torch.as_tensor(p.mu, device=dev)
    y_d = torch.as_tensor(p.y, device=dev)
    nu_d = torch.as_tensor(p.nu, device=dev)
    torch.cuda.synchronize()
    t1 = time.time()
    prob = rsot.Problem(x_d, mu_d, y_d, nu_d, precision="mixed")
    torch.cuda.synchronize()
    setup_s = time.time() - t1
    log(f"[bench] setup (sort, tiles, boxes) {setup_s:.3f}s")
    psi = torch.as_tensor(W.random_psi(11, p.n, p.eps), device=dev)
    grad = torch.empty(p.n, dtype=torch.float64, device=dev)

    def run(k):
        infos = []
        r = None
        for _ in range(k):
            r = prob.dual_eval(psi, p.eps, out=grad)
            infos.append(r.info)
        return r, infos

    run(args.warmup)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    r, infos = run(args.steps)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t2) / args.steps
    pairs = p.nq * p.n
    value = pairs / dt
    p1 = float(np.mean([i["pass1_ms"] for i in infos]))
    p2 = float(np.mean([i["pass2_ms"] for i in infos]))
    log(f"[bench] dense mixed: {dt*1e3:.2f} ms/eval, {value:.3e} pairs/s, "
        f"pass1 {p1:.2f} ms, pass2 {p2:.2f} ms, J={r.J:.12e}")

    d = 3
    roof_p1 = pair_roofline(d, 1, 2 * d + 4)
    roof_p2 = pair_roofline(d, 1, 2 * d + 3)
    roof_all = pair_roofline(d, 2, 4 * d + 7)
    if p1 >= p2:
        name, key, ms, peak = "objective pass (k_pass1, dense)", "k_pass1", p1, roof_p1
    else:
        name, key, ms, peak = "gradient pass (k_pass2, dense)", "k_pass2", p2, roof_p2
    achieved = pairs / (ms * 1e-3)
    roofline = {"bound": "alu", "kernel": name, "achieved": achieved / 1e9,
                "peak": peak / 1e9, "unit": "Gpair/s", "frac": achieved / peak,
                "traffic": counter_traffic(key),
                "eval_frac": value / roof_all, "eval_peak_Gpair_s": roof_all / 1e9}

    out = {"metric": "quad-target pairs/s for dual obj+grad (dense, truncated); "
                     "time-to-||g||1<1e-6",
           "value": value, "unit": "pairs/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": dt * 1e3, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64-arg/f32-exp/f64-acc",
           "data": "synthetic",
           "config": {"workload": p.name, "n_quad": p.nq, "n_target": p.n, "dim": 3,
                      "eps": p.eps, "precision": "mixed", "truncation": "dense",
                      "psi": "N(0, eps^2) seed 11"},
           "roofline": roofline,
           "setup_s": setup_s,
           "J": r.J, "grad_l1": r.info["grad_l1"]}

    psi1 = None
    if not args.no_extras and args.main_extras:
        extras = {}
        absJ = abs(r.J)
        for rule in ["geom", "tile"]:
            prob.set_truncation(rule, tau=1e-12)
            prob.set_reference(absJ)
            rr = prob.dual_eval(psi, p.eps, out=grad)           # warm
            torch.cuda.synchronize()
            ts = time.perf_counter()
            k = max(2, args.steps)
            for _ in range(k):
                rr = prob.dual_eval(psi, p.eps, out=grad)
            torch.cuda.synchronize()
            tt = (time.perf_counter() - ts) / k
            kept = rr.info["kept_pairs"]
            extras[rule] = {"ms_per_eval": tt * 1e3, "effective_pairs_s": pairs / tt,
                            "kept_pairs": kept, "kept_frac": kept / pairs,
                            "kept_pairs_s": kept / tt, "J": rr.J,
                            "J_minus_dense_rel": (r.J - rr.J) / absJ,
                            "cutoff": rr.info["cutoff"], "setup_ms": rr.info["setup_ms"],
                            "pass1_ms": rr.info["pass1_ms"], "pass2_ms": rr.info["pass2_ms"]}
            log(f"[bench] {rule}: {tt*1e3:.2f} ms/eval, kept {kept/pairs:.4f}, "
                f"effective {pairs/tt:.3e} pairs/s, kept {kept/tt:.3e} pairs/s")
        if args.main_extras != 2:
            # the tile rule at each culling granularity (targets per group)
            extras["tile_groups"] = {}
            prob.set_truncation("tile", tau=1e-12)
            for g in (64, 32, 16, 8):
                prob.set_tuning(0, 0, g)
                rr = prob.dual_eval(psi, p.eps, out=grad)
                torch.cuda.synchronize()
                ts = time.perf_counter()
                k = max(2, args.steps)
                for _ in range(k):
                    rr = prob.dual_eval(psi, p.eps, out=grad)
                torch.cuda.synchronize()
                tt = (time.perf_counter() - ts) / k
                kept = rr.info["kept_pairs"]
                extras["tile_groups"][str(g)] = {
                    "ms_per_eval": tt * 1e3, "kept_frac": kept / pairs, "kept_pairs_s": kept / tt,
                    "setup_ms": rr.info["setup_ms"], "pass1_ms": rr.info["pass1_ms"],
                    "pass2_ms": rr.info["pass2_ms"], "J_minus_dense_rel": (r.J - rr.J) / absJ}
                log(f"[bench] tile rule, groups of {g}: {tt*1e3:.2f} ms/eval, kept {kept/pairs:.4f}, "
                    f"culling {rr.info['setup_ms']:.2f} ms, pass1 {rr.info['pass1_ms']:.2f} ms, "
                    f"pass2 {rr.info['pass2_ms']:.2f} ms")
            # the autotuner's choice for this problem (culling group, then the
            # work segments of both passes), timed like the rows above
            prob.set_tuning(0, 0, 0)
            tune = prob.autotune(psi, p.eps, reps=2)
            rr = prob.dual_eval(psi, p.eps, out=grad)
            torch.cuda.synchronize()
            ts = time.perf_counter()
            k = max(2, args.steps)
            for _ in range(k):
                rr = prob.dual_eval(psi, p.eps, out=grad)
            torch.cuda.synchronize()
            tt = (time.perf_counter() - ts) / k
            extras["tile_tuned"] = dict(tune, ms_per_eval=tt * 1e3,
                                        kept_frac=rr.info["kept_pairs"] / pairs,
                                        J_minus_dense_rel=(r.J - rr.J) / absJ)
            log(f"[bench] tile rule, autotuned {tune}: {tt*1e3:.2f} ms/eval, "
                f"kept {rr.info['kept_pairs']/pairs:.4f}")
            prob.set_tuning(0, 0, 0)
            prob.set_truncation("dense")
            prob.set_precision("fp64")
            rr = prob.dual_eval(psi, p.eps, out=grad)
            ts = time.perf_counter()
            rr = prob.dual_eval(psi, p.eps, out=grad)
            torch.cuda.synchronize()
            tf = time.perf_counter() - ts
            extras["fp64_dense"] = {"ms_per_eval": tf * 1e3, "pairs_s": pairs / tf, "J": rr.J,
                                    "J_mixed_minus_fp64_rel": (r.J - rr.J) / abs(rr.J)}
            g64 = grad.clone()
            prob.set_precision("mixed")
            rm = prob.dual_eval(psi, p.eps, out=grad)
            # plan moments and transport maps (Secs. 6.2, 6.3), dense, at the same
            # psi: device time of the moment / map kernels after the evaluation
            prob.plan_moments(psi, p.eps)
            prob.transport_maps(psi, p.eps)
            mom_ms = min(prob.plan_moments(psi, p.eps)[3] for _ in range(3))
            map_ms = min(prob.transport_maps(psi, p.eps)[3] for _ in range(3))
            extras["plan_moments"] = {"moments_ms": mom_ms, "moments_pairs_s": pairs / (mom_ms * 1e-3),
                                      "maps_ms": map_ms, "maps_pairs_s": pairs / (map_ms * 1e-3),
                                      "note": "kernels after the evaluation that gives L_q; "
                                              "dense, mixed precision"}
            log(f"[bench] plan moments {mom_ms:.1f} ms ({pairs / (mom_ms * 1e-3):.3e} pairs/s), "
                f"maps {map_ms:.1f} ms ({pairs / (map_ms * 1e-3):.3e} pairs/s)")
            nu_t = torch.as_tensor(p.nu, device=dev)
            eg = torch.max(torch.abs(grad - g64) / (nu_t + g64 + nu_t)).item()
            extras["fp64_dense"]["grad_err_mixed_vs_fp64"] = eg
            log(f"[bench] fp64 dense: {tf*1e3:.1f} ms/eval; mixed vs fp64: "
                f"J rel {(rm.J - rr.J)/abs(rr.J):.2e}, grad err {eg:.2e}")
            prob.close()

            # time to ||grad||_1 < 1e-6 on the 2D workload (FP64 path)
            c1 = W.config1()
            pr1 = rsot.Problem(c1.x, c1.mu, c1.y, c1.nu, precision="fp64")
            pr1.solve([c1.eps], tol=1e-6)                     # warm (kernels loaded)
            ts = time.perf_counter()
            psi1, info1 = pr1.solve([c1.eps], tol=1e-6)
            tsol = time.perf_counter() - ts
            extras["time_to_tol_config1"] = {"workload": c1.name, "seconds": tsol,
                                             "iterations": info1["iterations"],
                                             "evaluations": info1["evaluations"],
                                             "grad_l1": info1["grad_l1"],
                                             "status": info1["status"]}
            log(f"[bench] config1 solve: {tsol*1e3:.1f} ms, {info1['iterations']} it, "
                f"{info1['evaluations']} evals, |g|_1={info1['grad_l1']:.2e}")
            pr1.close()

            # time to ||grad||_1 < 1e-6 on the 3D workload from psi = 0: mixed
            # precision, tile rule, eps schedule eps*2^K .. eps (Sec. 4.2), stages
            # before the last to 1e-5
            K = int(math.floor(math.log2(0.1 / p.eps)))
            sched = [p.eps * 2.0 ** k for k in range(K, 0, -1)] + [p.eps]
            pr2 = rsot.Problem(p.x, p.mu, p.y, p.nu, truncation="tile", tau=1e-12)
            ts = time.perf_counter()
            psi2, info2 = pr2.solve(sched, tol=1e-6, stage_tol=1e-5)
            t2 = time.perf_counter() - ts
            extras["time_to_tol_config2"] = {"workload": p.name, "seconds": t2, "eps_schedule": sched,
                                             "truncation": "tile", "tau": 1e-12,
                                             "iterations": info2["iterations"],
                                             "evaluations": info2["evaluations"],
                                             "grad_l1": info2["grad_l1"],
                                             "kept_frac": info2["kept_frac"],
                                             "status": info2["status"],
                                             "recheck": fp64_recheck(p, psi2)}
            log(f"[bench] config2 solve: {t2:.2f} s, {info2['iterations']} it, "
                f"{info2['evaluations']} evals, |g|_1={info2['grad_l1']:.2e}")
            pr2.close()

            # the same from the combined multilevel start (Sec. 5.3): source cubes
            # of 16^3 / 32^3 / 64^3 cells (same mixture density), k-means targets
            # 4,096 / 16,384 / 65,536; the schedule on the coarsest level, the final
            # eps on the finer ones; every level to 1e-6
            srcs = [(q.x, q.mu) for q in (W.cube_mixture(16, p.n, p.eps),
                                          W.cube_mixture(32, p.n, p.eps))] + [(p.x, p.mu)]
            ts = time.perf_counter()
            hier = rsot.target_hierarchy(torch.as_tensor(p.y, device=dev),
                                         torch.as_tensor(p.nu, device=dev),
                                         [4096, 16384, p.n], lloyd_iters=20, seed=6)
            ml2 = rsot.Multilevel(srcs, hier, precision="mixed", truncation="tile", tau=1e-12)
            psi3, info3 = ml2.solve(sched + [p.eps] * 2, [0] * len(sched) + [1, 2], tol=1e-6,
                                    stage_tol=1e-5)
            torch.cuda.synchronize()
            t3 = time.perf_counter() - ts
            ml2.close()
            extras["time_to_tol_config2_multilevel"] = {
                "workload": p.name, "seconds": t3, "source_cells": [16, 32, 64],
                "targets": [int(h[1].numel()) for h in hier], "iterations": info3["iterations"],
                "seconds_per_level": info3["seconds"], "grad_l1": info3["grad_l1"],
                "status": info3["status"], "recheck": fp64_recheck(p, psi3)}
            log(f"[bench] config2 multilevel solve: {t3:.2f} s (hierarchy included), iterations "
                f"{info3['iterations']}, |g|_1={info3['grad_l1']:.2e}")
        out["extras"] = extras

    legs = []
    if not args.no_extras:
        if not (args.quick or args.no_multilevel):
            legs.append(("multilevel", lambda: multilevel_leg(spread=args.ml_spread,
                                                              tile_group=args.tile_group)))
        if args.batched and not args.quick:
            legs.append(("batched", lambda: batched_leg(args.batched)))
        if args.trunc_study and not args.quick:
            tols = tuple(float(v) for v in args.trunc_tol.split(","))
            legs.append(("trunc_study", lambda: trunc_study_leg(tols=tols)))
        if args.sphere and not args.quick:
            legs.append(("sphere", sphere_leg))
        if args.barycenter and not args.quick:
            legs.append(("barycenter", barycenter_leg))
        if args.gpu_size and not args.quick:
            rr, gg = args.gpu_size.split("x")
            r0, r1 = (int(v) for v in rr.split("-"))
            g0, g1 = (int(v) for v in gg.split("-"))
            spec = [(r, g) for r in range(r0, r1 + 1) for g in range(g0, g1 + 1)]
            legs.append(("gpu_size", lambda: {"rows": gpu_size_leg(spec)}))
        if args.mlp:
            rows, steps = (int(v) for v in args.mlp.split(","))
            legs.append(("mlp", lambda: mlp_leg(rows, steps)))
        if args.learned and not args.quick:
            n_train, n_test, epochs = (int(v) for v in args.learned.split(","))
            legs.append(("learned", lambda: learned_leg(n_train, n_test, epochs)))
    for name, leg in legs:
        ts = time.perf_counter()
        try:
            res = leg()
        except Exception as e:          # a failing leg is reported, the line still printed
            log(f"[bench] {name} leg failed: {e!r}")
            res = {"error": repr(e)}
        res["leg_seconds"] = time.perf_counter() - ts
        out.setdefault("extras", {})[name] = res

    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(p, psi.cpu().numpy(), psi1)
    print(json.dumps(out, default=json_value), flush=True)


def json_value(v):
    """numpy scalars and arrays in the result line as plain numbers and lists"""
    if isinstance(v, np.ndarray):
        return v.tolist()
    if isinstance(v, np.generic):
        return v.item()
    raise TypeError(f"{type(v).__name__} in the result line")


def fp64_recheck(p, psi, n_sample=256, seed=0):
    """Independent check of a solve's returned potential: ||grad||_1 and J by
    the library's FP64 dense path (which the oracle pins in the tests; a dense
    oracle pass at these sizes would take minutes to hours), and the largest
    difference of that path's per-point L_q from the oracle's at n_sample
    seeded points. p: x, mu, y, nu, eps."""
    import torch
    import oracle
    from paper_2507_23602_amd import rsot
    pr = rsot.Problem(*[torch.as_tensor(a, device="cuda") for a in (p.x, p.mu, p.y, p.nu)],
                      precision="fp64")
    r = pr.dual_eval(torch.as_tensor(psi, device="cuda"), p.eps)
    L = pr.lse().cpu().numpy()
    pr.close()
    idx = np.random.default_rng(seed).choice(p.x.shape[0], n_sample, replace=False)
    ref = oracle.dual_eval(p.x[idx], p.mu[idx], p.y, p.nu, psi, p.eps, want_grad=False,
                           want_L=True)
    el = float(np.max(np.abs(L[idx] - ref.L) / np.maximum(1.0, np.abs(ref.L))))
    log(f"[bench] re-check: FP64 ||g||_1 {r.info['grad_l1']:.3e}, sampled L vs oracle {el:.1e}")
    return {"fp64_grad_l1": r.info["grad_l1"], "fp64_J": r.J, "fp64_ms": r.info["kernel_ms"],
            "sampled_L_err_vs_oracle": el, "n_sample": n_sample}


MLP_FWD_FLOP_PER_ROW = 2 * (6 * 256 + 3 * 256 * 256 + 256)      # multiply-adds x 2
MLP_TRAIN_FLOP_PER_ROW = 3 * MLP_FWD_FLOP_PER_ROW                # forward + data and weight grads


def mlp_leg(rows, steps):
    """Warm-start network kernels on synthetic rows: fused training steps
    (forward, MSE, backward, Adam) and forward passes, device time per call
    with HIP events on the library's stream, against the dense bf16 MFMA peak."""
    import torch
    from paper_2507_23602_amd import rsot, workloads as W
    rng = np.random.default_rng(3)
    f = np.empty((rows, 6), dtype=np.float32)
    f[:, :2] = rng.uniform(0, 1, (rows, 2))
    f[:, 2:4] = rng.uniform(0.2, 0.8, (rows, 2))
    f[:, 4] = rng.uniform(0.05, 0.2, rows)
    f[:, 5] = np.log(rng.uniform(1e-3, 1e-1, rows))
    t = (0.05 * np.sin(4 * f[:, 0]) * np.cos(3 * f[:, 1])).astype(np.float32)
    ft, tt = torch.as_tensor(f, device="cuda"), torch.as_tensor(t, device="cuda")
    m = rsot.MLP(W.mlp_init_params(0))
    m.fit_normalization(ft, tt)
    for _ in range(2):
        m.train_step(ft, tt, None, want_loss=False)
        m.forward(ft)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        m.train_step(ft, tt, None, want_loss=False)
    e1.record()
    torch.cuda.synchronize()
    t_train = e0.elapsed_time(e1) / steps
    e0.record()
    for _ in range(steps):
        m.forward(ft)
    e1.record()
    torch.cuda.synchronize()
    t_fwd = e0.elapsed_time(e1) / steps
    peak = 2.5e15
    tr = MLP_TRAIN_FLOP_PER_ROW * rows / (t_train * 1e-3)
    fw = MLP_FWD_FLOP_PER_ROW * rows / (t_fwd * 1e-3)
    log(f"[bench] mlp: {rows} rows, train step {t_train:.3f} ms ({tr / 1e12:.1f} TFLOP/s), "
        f"forward {t_fwd:.3f} ms ({fw / 1e12:.1f} TFLOP/s); bf16 dense peak 2500 TFLOP/s")
    return {"rows": rows, "steps": steps, "train_step_ms": t_train, "forward_ms": t_fwd,
            "train_tflops": tr / 1e12, "forward_tflops": fw / 1e12, "peak_tflops": peak / 1e12,
            "train_frac": tr / peak, "forward_frac": fw / peak}


def learned_leg(n_train, n_test, epochs):
    """Learned warm start (blob family: 128x128 mesh x 3 points = 98,304
    quadrature points, 65,536 fixed uniform targets, eps logU[1e-3,1e-1]):
    instances 0..n_train-1 are solved from zero to make the dataset, the
    network is trained on it with the library's kernels, and the next n_test
    instances are solved from zero, from the learned start and from the
    multilevel start, to ||grad||_1 < 1e-6."""
    import torch
    from paper_2507_23602_amd import warmstart as WS
    from paper_2507_23602_amd import workloads as W4
    t0 = time.perf_counter()
    train_ids = list(range(n_train))
    test_ids = list(range(n_train, n_train + n_test))
    feats, target, drecs = WS.build_dataset(train_ids)
    t_data = time.perf_counter() - t0
    tf, tt, _ = WS.build_dataset(test_ids[:min(8, n_test)], every=8)   # held-out loss only
    t1 = time.perf_counter()
    m, tlog = WS.train(feats, target, epochs=epochs, test=(tf, tt))
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t1
    rows = target.numel()
    del feats, target
    recs = WS.compare(m, test_ids, keep_psi=2)
    summ = WS.summarize(recs)
    # the oracle re-checks ||grad||_1 at the learned-start solutions of the
    # first two held-out instances
    import oracle
    rechecks = []
    for r in recs[:2]:
        q = W4.config4_instance(r["id"])
        psi = r["learned"].pop("psi")
        ev = oracle.dual_eval(q.x, q.mu, q.y, q.nu, psi, q.eps,
                              threads=int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1)))
        rechecks.append({"id": r["id"], "oracle_grad_l1": float(np.abs(ev.grad).sum())})
    for r in recs[2:]:
        r["learned"].pop("psi", None)
    log(f"[bench] learned: oracle re-check of ||g||_1 {[round(c['oracle_grad_l1'], 9) for c in rechecks]}")
    log(f"[bench] learned: dataset {t_data:.1f}s ({n_train} solves), training {t_train:.1f}s "
        f"({epochs} epochs x {rows} rows); test {summ}")
    return {"workload": "blob_square128_tri3_nq98304_n65536", "train_instances": n_train,
            "test_instances": n_test, "dataset_seconds": t_data, "train_seconds": t_train,
            "train_rows": rows, "epochs": epochs, "train_log": tlog, "summary": summ,
            "dataset_mean_iterations": float(np.mean([r["iterations"] for r in drecs])),
            "dataset_mean_seconds": float(np.mean([r["seconds"] for r in drecs])),
            "learned_vs_multilevel_seconds": [summ["learned"]["total_seconds"],
                                              summ.get("multilevel", {}).get("total_seconds")],
            "oracle_recheck": rechecks, "per_instance": recs}


def batched_leg(k):
    """k uneven 3D instances (points logU[1e5,4e6], targets logU[4096,262144],
    eps logU[1e-4,1e-2], mixture sources/targets), tile rule tau = 1e-12,
    mixed precision: one batched call against k single calls, with
    the library defaults and with autotuned work granularity."""
    import torch
    from paper_2507_23602_amd import rsot, workloads as W
    t0 = time.perf_counter()
    insts = [W.config5_instance(i) for i in range(k)]
    log(f"[bench] batched: generated {k} instances in {time.perf_counter()-t0:.1f}s, "
        f"points {sum(p.nq for p in insts)}, targets {sum(p.n for p in insts)}")
    probs, psis = [], []
    for i, p in enumerate(insts):
        pr = rsot.Problem(torch.as_tensor(p.x, device="cuda"), torch.as_tensor(p.mu, device="cuda"),
                          torch.as_tensor(p.y, device="cuda"), torch.as_tensor(p.nu, device="cuda"),
                          truncation="tile", tau=1e-12)
        ps = torch.as_tensor(W.random_psi(100 + i, p.n, p.eps), device="cuda")
        pr.dual_eval(ps, p.eps)                       # dense: |J_ref| for the tile rule
        probs.append(pr)
        psis.append(ps)
    eps = [p.eps for p in insts]
    dense_pairs = sum(p.nq * p.n for p in insts)

    def singles():
        torch.cuda.synchronize()
        t = time.perf_counter()
        kept = 0
        for pr, ps, e in zip(probs, psis, eps):
            kept += pr.dual_eval(ps, e).info["kept_pairs"]
        torch.cuda.synchronize()
        return time.perf_counter() - t, kept

    def batch():
        torch.cuda.synchronize()
        t = time.perf_counter()
        J, g, infos, ms = rsot.dual_eval_batched(probs, eps, psis)
        torch.cuda.synchronize()
        return time.perf_counter() - t, sum(i["kept_pairs"] for i in infos), ms

    singles()
    batch()
    res = {}
    ts, kept = singles()
    tb, kept_b, ms = batch()
    assert kept == kept_b
    res["untuned"] = {"singles_s": ts, "batched_s": tb, "batched_device_ms": ms,
                      "kept_pairs": kept, "kept_pairs_s_batched": kept / tb,
                      "kept_pairs_s_singles": kept / ts}
    t0 = time.perf_counter()
    groups = []
    for pr, ps, e in zip(probs, psis, eps):
        groups.append(pr.autotune(ps, e, reps=1)["tile_group"] or 64)
    t_tune = time.perf_counter() - t0
    singles()
    ts, kept = singles()
    tb, kept_b, ms = batch()
    res["tuned"] = {"singles_s": ts, "batched_s": tb, "batched_device_ms": ms,
                    "kept_pairs_s_batched": kept / tb, "kept_pairs_s_singles": kept / ts,
                    "tune_seconds": t_tune}
    res["tuned"]["tile_groups"] = {str(g): groups.count(g) for g in sorted(set(groups))}
    res.update(instances=k, dense_pairs=dense_pairs, kept_frac=kept / dense_pairs,
               effective_pairs_s_batched=dense_pairs / tb)
    # the oracle on the four smallest members, against the batched call's
    # results (tile rule: the oracle applies the same rule to the same
    # partition, cut into the member's tuned culling groups, and |J_ref|)
    import oracle
    J, grads, infos, _ = rsot.dual_eval_batched(probs, eps, psis)
    order = sorted(range(k), key=lambda i: insts[i].nq * insts[i].n)[:4]
    checks = []
    for i in order:
        q = insts[i]
        tile_of, _, nt, nb = probs[i].partition()
        g = groups[i]
        group_of = (probs[i].target_slots().cpu().numpy() // g).astype(np.int32)
        ref = oracle.dual_eval_tile(q.x, q.mu, q.y, q.nu, psis[i].cpu().numpy(), q.eps,
                                    tile_of.cpu().numpy(), nt, group_of, nb * 64 // g,
                                    1e-12, infos[i]["absJ_ref"],
                                    threads=int(os.environ.get("OMP_NUM_THREADS",
                                                               os.cpu_count() or 1)))
        gi = grads[i].cpu().numpy()
        checks.append({"instance": i, "nq": q.nq, "n": q.n, "tile_group": g,
                       "J_rel_err": abs(J[i] - ref.J) / abs(ref.J),
                       "grad_err": float(np.max(np.abs(gi - ref.grad) / (q.nu + ref.grad + q.nu))),
                       "kept_equal": infos[i]["kept_pairs"] == ref.kept})
    res["oracle_check"] = checks
    worst_j = max(c["J_rel_err"] for c in checks)
    worst_g = max(c["grad_err"] for c in checks)
    log(f"[bench] batched: oracle on the 4 smallest members: J rel err <= {worst_j:.1e}, "
        f"e_g <= {worst_g:.1e}, kept sets equal: {all(c['kept_equal'] for c in checks)}")
    log(f"[bench] batched {k}: kept {kept/dense_pairs:.4f} of {dense_pairs:.3e}; untuned singles "
        f"{res['untuned']['singles_s']*1e3:.1f} ms, batched {res['untuned']['batched_s']*1e3:.1f} ms; "
        f"tuned singles {ts*1e3:.1f} ms, batched {tb*1e3:.1f} ms (tuning {t_tune:.1f}s)")
    for pr in probs:
        pr.close()
    res["small"] = small_batch(256)
    res["small_fp32"] = small_batch(256, fp64_below_points=0)
    return res


def small_batch(k, fp64_below_points=None):
    """k uneven small 2D instances (6,144 to 98,304 points, 256 to 65,536
    targets), dense, mixed precision: one batched call against k single calls,
    wall clock on the host (where per-call launch and synchronisation costs
    show), and the device time of the batch. With the library's routing the
    members with few effective points run the FP64 pair loop, one problem at a
    time inside the batched call too; fp64_below_points=0 keeps every member
    on the batched FP32 loop."""
    import torch
    from paper_2507_23602_amd import rsot, workloads as W
    insts = [W.small_square_instance(i) for i in range(k)]
    probs = [rsot.Problem(p.x, p.mu, p.y, p.nu, fp64_below_points=fp64_below_points)
             for p in insts]
    psis = [torch.as_tensor(W.random_psi(500 + i, p.n, p.eps), device="cuda")
            for i, p in enumerate(insts)]
    eps = [p.eps for p in insts]
    pairs = sum(p.nq * p.n for p in insts)

    def singles():
        torch.cuda.synchronize()
        t = time.perf_counter()
        for pr, ps, e in zip(probs, psis, eps):
            pr.dual_eval(ps, e)
        torch.cuda.synchronize()
        return time.perf_counter() - t

    def batch():
        torch.cuda.synchronize()
        t = time.perf_counter()
        _, _, _, ms = rsot.dual_eval_batched(probs, eps, psis)
        torch.cuda.synchronize()
        return time.perf_counter() - t, ms

    singles()
    batch()
    ts = min(singles() for _ in range(3))
    tb, ms = min(batch() for _ in range(3))
    for pr in probs:
        pr.close()
    log(f"[bench] small batch {k} (fp64_below_points {fp64_below_points}): {pairs:.3e} pairs; "
        f"singles {ts*1e3:.1f} ms, batched {tb*1e3:.1f} ms (device {ms:.1f} ms): {ts/tb:.2f}x")
    return {"instances": k, "pairs": pairs, "singles_s": ts, "batched_s": tb,
            "fp64_below_points": fp64_below_points,
            "batched_device_ms": ms, "speedup": ts / tb,
            "points": [min(p.nq for p in insts), max(p.nq for p in insts)],
            "targets": [min(p.n for p in insts), max(p.n for p in insts)]}


def multilevel_leg(spread=False, tile_group=0):
    """Time to ||grad||_1 < 1e-6 of the combined multilevel solve (Sec. 5.3)
    with the eps schedule, on the 2D disk workload; per-level breakdown.
    Default: the schedule on the two coarsest levels and the final eps on the
    finer ones; spread=True: the final eps first on the finest level."""
    import torch
    from paper_2507_23602_amd import rsot, workloads as W
    c3 = W.config3()
    log(f"[bench] multilevel workload {c3['name']}")
    t0 = time.perf_counter()
    levels = rsot.target_hierarchy(torch.as_tensor(c3["y"], device="cuda"),
                                   torch.as_tensor(c3["nu"], device="cuda"),
                                   c3["target_levels"], lloyd_iters=20, seed=6)
    torch.cuda.synchronize()
    t_h = time.perf_counter() - t0
    ml = rsot.Multilevel(c3["sources"], levels, precision="mixed", truncation="tile", tau=1e-12,
                         tile_group=tile_group)
    t0 = time.perf_counter()
    def progress(it):
        if it.iteration % 25 == 0:
            log(f"[bench] multilevel: stage eps {it.eps:.2e}, iteration {it.iteration}, "
                f"|g|_1 {it.grad_l1:.2e}, kept {it.kept_pairs:.3e}")
        return 0
    key = "_spread" if spread else ""
    # every level to the final tolerance (a looser one on the coarser levels
    # costs more finest-level iterations than it saves); non-final eps
    # stages to 1e-5
    psi, info = ml.solve(c3["eps" + key], c3["level" + key], tol=1e-6,
                         level_tol=1e-5 if spread else 0.0, stage_tol=1e-5, callback=progress)
    t_s = time.perf_counter() - t0
    ml.close()
    from types import SimpleNamespace
    fin = SimpleNamespace(x=c3["sources"][-1][0], mu=c3["sources"][-1][1], y=c3["y"],
                          nu=c3["nu"], eps=c3["eps" + key][-1])
    recheck = fp64_recheck(fin, psi)
    log(f"[bench] multilevel: hierarchy {t_h:.2f}s, solve {t_s:.2f}s, status {info['status']}, "
        f"|g|_1 {info['grad_l1']:.2e}, iterations {info['iterations']}, "
        f"seconds {[round(v, 3) for v in info['seconds']]}, "
        f"refine {[round(v, 3) for v in info['refine_seconds']]}")
    return {"workload": c3["name"], "schedule": "spread" if spread else "coarse",
            "tile_group": tile_group,
            "hierarchy_seconds": t_h, "solve_seconds": t_s,
            "time_to_tol_seconds": t_h + t_s, "recheck": recheck,
            "target_sizes": [int(l[1].numel()) for l in levels], **info}


TRUNC_STUDY = [("dense", None), ("pw", 1e-12), ("pw", 1e-10), ("pw", 1e-7),
               ("int", 1e-6), ("int", 1e-5), ("int", 1e-4),
               ("geom", 1e-6), ("geom", 1e-5), ("geom", 1e-4),
               ("tile", 1e-6), ("tile", 1e-5), ("tile", 1e-4)]


def trunc_study_leg(densities=("custom", "uniform"), tols=(1e-3,), max_iter=2000):
    """The truncation-strategy study (Sec. 6.1, Table of strategies) on the
    synthetic stand-in of its inputs (375,000 points x 14,761 targets, eps
    1e-2): one solve from psi = 0 per (density, rule, parameter) to
    ||grad||_1 <= tol (the study's 1e-3 by default), mixed precision;
    iterations, seconds, converged (status OK) and E_rel = |J_trunc -
    J_dense| / |J_dense| of the final values (Eq. relative_error_definition).
    With a loose tol that figure also holds the two solves' different
    stopping points, so E_rel_same_psi adds |J_trunc(psi) - J_dense(psi)| /
    |J_dense(psi)| at the truncated solve's own potential (the truncation's
    share alone). Each returned potential is re-evaluated without truncation
    (FP64) for its true ||grad||_1; the baseline's potential is re-checked by
    the oracle's dense pass."""
    import torch
    import oracle
    from paper_2507_23602_amd import rsot, workloads as W
    res = {}
    for dens, tol in ((d, t) for d in densities for t in tols):
        p = W.trunc_study(dens)
        dev = [torch.as_tensor(a, device="cuda") for a in (p.x, p.mu, p.y, p.nu)]
        chk = rsot.Problem(*dev, precision="fp64")
        rows = []
        base_J = None
        for rule, par in TRUNC_STUDY:
            kw = {} if rule == "dense" else (
                {"truncation": rule, "delta_thr": par} if rule == "pw" else
                {"truncation": rule, "tau": par})
            pr = rsot.Problem(*dev, precision="mixed", **kw)
            try:                                             # kernels loaded, lists sized
                pr.solve([p.eps], tol=tol, max_iter=2)
            except rsot.RsotError:
                pass
            torch.cuda.synchronize()
            ts = time.perf_counter()
            try:
                psi, info = pr.solve([p.eps], tol=tol, max_iter=max_iter)
                status = info["status"]
            except rsot.RsotError as e:
                psi, info, status = e.psi, e.info, e.code
            sec = time.perf_counter() - ts
            pr.close()
            rd = chk.dual_eval(torch.as_tensor(psi, device="cuda"), p.eps)
            if rule == "dense":
                base_J = info["J"]
                ref = oracle.dual_eval(p.x, p.mu, p.y, p.nu, psi, p.eps)
                orc = {"oracle_grad_l1": float(np.abs(ref.grad).sum()),
                       "oracle_J_rel": abs(ref.J - info["J"]) / abs(ref.J)}
            row = {"rule": rule, "param": par, "iterations": info["iterations"],
                   "evaluations": info["evaluations"], "seconds": sec, "status": status,
                   "converged": status == rsot.OK, "J": info["J"],
                   "E_rel": abs(info["J"] - base_J) / abs(base_J),
                   "E_rel_same_psi": abs(info["J"] - rd.J) / abs(rd.J),
                   "kept_frac": info["kept_frac"], "grad_l1": info["grad_l1"],
                   "dense_grad_l1": rd.info["grad_l1"]}
            if rule == "dense":
                row.update(orc)
            rows.append(row)
            log(f"[bench] trunc study {dens} tol {tol:g}: {rule:5s} {str(par):6s} "
                f"{info['iterations']:4d} it {sec:6.2f} s  status {status}  E_rel "
                f"{row['E_rel']:.1e} (same psi {row['E_rel_same_psi']:.1e})  kept "
                f"{info['kept_frac']:.3f}  dense |g|_1 {rd.info['grad_l1']:.2e}")
        chk.close()
        res[f"{dens}_tol{tol:g}"] = {"workload": p.name, "tol": tol, "rows": rows}
    return res


def gpu_size_leg(spec, tol=1e-3, solve_below=2.5e11, solve_also=((5, 3),)):
    """The workload at the problem sizes of App. C (uniform [-1, 1]^3 hex
    meshes, Gauss 1-3, targets uniform in the unit ball, eps 1e-2, no
    truncation): per (refinement, order) the device time of one dense mixed
    evaluation at psi = 0 and, where N_q N <= solve_below or for the cases in
    solve_also (default: the finest, 7,077,888 x 232,609), a dense solve from
    psi = 0 to ||grad||_1 <= 1e-3 (seconds, iterations, mean seconds per
    iteration), its potential re-checked (FP64 ||grad||_1 and oracle L_q)."""
    import torch
    from paper_2507_23602_amd import rsot, workloads as W
    out = []
    for r, order in spec:
        p = W.gpu_size(r, order)
        dev = [torch.as_tensor(a, device="cuda") for a in (p.x, p.mu, p.y, p.nu)]
        pr = rsot.Problem(*dev, precision="mixed")
        z = torch.zeros(p.n, dtype=torch.float64, device="cuda")
        pr.dual_eval(z, p.eps)
        ms = min(pr.dual_eval(z, p.eps).info["kernel_ms"] for _ in range(3))
        row = {"workload": p.name, "refinement": r, "gauss": order, "n_quad": p.nq,
               "n_target": p.n, "eval_ms": ms, "pairs_s": p.nq * p.n / (ms * 1e-3)}
        if p.nq * p.n <= solve_below or (r, order) in solve_also:
            torch.cuda.synchronize()
            ts = time.perf_counter()
            psi, info = pr.solve([p.eps], tol=tol)
            sec = time.perf_counter() - ts
            row.update(solve_seconds=sec, iterations=info["iterations"],
                       evaluations=info["evaluations"], status=info["status"],
                       seconds_per_iteration=sec / max(1, info["iterations"]),
                       recheck=fp64_recheck(p, psi, n_sample=64))
            log(f"[bench] gpu-size {p.name}: eval {ms:.2f} ms, solve {sec:.2f} s, "
                f"{info['iterations']} it, status {info['status']}")
        else:
            log(f"[bench] gpu-size {p.name}: eval {ms:.2f} ms")
        pr.close()
        out.append(row)
    return out


def sphere_leg(eval_k=7, eval_n=65536):
    """Sec. 6.4 on the unit sphere (squared geodesic cost, density 1 + 0.9 P2):
    blue-noise sampling by Lloyd's algorithm with Riemannian barycentres
    (Algs. 4-5) for N = 4..9 at eps = 1e-2 and tol 1e-3, as in the paper's
    figure; then the evaluation rate of the sphere pair loop on icosphere(7)
    (983,040 points) against 65,536 targets, dense, mixed and FP64 (the
    mixed gradient re-checked against the FP64 one), one barycentre step in
    each, and the geodesic tile rule at tau 1e-12 against the dense J."""
    import torch
    from paper_2507_23602_amd import rsot, sphere, workloads as W
    x, mu = W.sphere_quadrature(4, "harmonic")
    runs = []
    for n in range(4, 10):
        y0 = W.sphere_points(200 + n, n)
        y, lg = sphere.lloyd(x, mu, y0, 1e-2, tol=1e-3)
        runs.append({"n": n, "iterations": len(lg), "seconds": lg[-1]["seconds"],
                     "W_start": -lg[0]["J"], "W_end": -lg[-1]["J"],
                     "min_angle": float(sphere.pairwise_angles(y)[0])})
        log(f"[bench] sphere blue noise N={n}: {len(lg)} Lloyd iterations, "
            f"{lg[-1]['seconds']:.2f} s, W {-lg[0]['J']:.5f} -> {-lg[-1]['J']:.5f}")
    p = W.sphere_problem(eval_k, eval_n, 1e-2, seed=40)
    dev = [torch.as_tensor(a, device="cuda") for a in (p.x, p.mu, p.y, p.nu)]
    psi = torch.as_tensor(W.random_psi(48, p.n, p.eps), device="cuda")
    rates = {}
    grads = {}
    for prec in ("mixed", "fp64"):
        pr = rsot.Problem(*dev, cost="sphere", cost_scale=1.0, precision=prec)
        pr.dual_eval(psi, p.eps)
        best = min(pr.dual_eval(psi, p.eps).info["kernel_ms"] for _ in range(3))
        grads[prec] = pr.dual_eval(psi, p.eps).grad.clone()
        # one Alg. 5 step from the targets themselves (its kernels only; the
        # step's own evaluation is timed above)
        kms = min(pr.sphere_karcher_step(psi, p.eps, dev[2], alpha=0.5)[3] for _ in range(2))
        # dense-equivalent rate: the passes skip pairs, blocks and tiles whose
        # exponentials provably underflow, so fewer pairs are formed
        rates[prec] = {"ms": best, "effective_pairs_s": p.nq * p.n / (best * 1e-3),
                       "karcher_ms": kms}
        pr.close()
    # the geodesic tile rule (tau 1e-12, |J| reference from the dense FP64
    # evaluation) on the same problem
    pr = rsot.Problem(*dev, cost="sphere", cost_scale=1.0, precision="mixed", truncation="tile",
                      tau=1e-12)
    dense_J = rsot.Problem(*dev, cost="sphere", cost_scale=1.0, precision="fp64")
    Jref = dense_J.dual_eval(psi, p.eps).J
    dense_J.close()
    pr.set_reference(abs(Jref))
    pr.dual_eval(psi, p.eps)
    rt = min((pr.dual_eval(psi, p.eps) for _ in range(3)), key=lambda r: r.info["kernel_ms"])
    rates["tile"] = {"ms": rt.info["kernel_ms"], "kept_frac": rt.info["kept_pairs"] / (p.nq * p.n),
                     "effective_pairs_s": p.nq * p.n / (rt.info["kernel_ms"] * 1e-3),
                     "J_rel_vs_fp64_dense": abs(rt.J - Jref) / abs(Jref), "tau": 1e-12}
    # the same rule over culling groups of 32, 16 and 8 targets
    groups = {}
    for g in (32, 16, 8):
        pr.set_tuning(0, 0, g)
        pr.dual_eval(psi, p.eps)
        rg = min((pr.dual_eval(psi, p.eps) for _ in range(3)), key=lambda r: r.info["kernel_ms"])
        groups[str(g)] = {"ms": rg.info["kernel_ms"],
                          "kept_frac": rg.info["kept_pairs"] / (p.nq * p.n),
                          "J_rel_vs_fp64_dense": abs(rg.J - Jref) / abs(Jref)}
    rates["tile"]["groups"] = groups
    pr.close()
    nu_t = torch.as_tensor(p.nu, device="cuda")
    eg = torch.max(torch.abs(grads["mixed"] - grads["fp64"]) /
                   (nu_t + grads["fp64"] + nu_t)).item()
    log(f"[bench] sphere evaluation {p.name}: mixed {rates['mixed']['ms']:.1f} ms "
        f"({rates['mixed']['effective_pairs_s']:.3e} dense-equivalent pairs/s), fp64 "
        f"{rates['fp64']['ms']:.1f} ms; "
        f"mixed vs fp64 e_g {eg:.1e}; barycentre step {rates['mixed']['karcher_ms']:.1f} / "
        f"{rates['fp64']['karcher_ms']:.1f} ms; tile rule {rates['tile']['ms']:.1f} ms, kept "
        f"{rates['tile']['kept_frac']:.4f}, J vs FP64 dense {rates['tile']['J_rel_vs_fp64_dense']:.1e}; "
        + ", ".join(f"groups of {g} {v['ms']:.1f} ms kept {v['kept_frac']:.4f}"
                    for g, v in groups.items()))
    return {"blue_noise": runs, "eval_workload": p.name, "eval": rates,
            "grad_err_mixed_vs_fp64": eg}


def barycenter_leg(n_cells=128, n_points=4096, eps=5e-3, tol=1e-4):
    """Sec. 6.2: the damped Lloyd barycentre (theta = 1/2, lambda = 1/2 each)
    of two Gaussian-blob densities on 128 x 128 squares (98,304 points each)
    with 4,096 support points from uniform starts, eps 5e-3, FP64 pair loop,
    to ||dy|| <= 1e-4 ||y||; the points' mean against the sources' weighted
    mean (an invariant of the iteration)."""
    import numpy as np
    from paper_2507_23602_amd import barycenter, workloads as W
    y = np.zeros((1, 2))
    a = W.gaussian_blob_square(n_cells, (0.3, 0.35), 0.10, y, eps)
    b = W.gaussian_blob_square(n_cells, (0.7, 0.6), 0.12, y, eps)
    src = [(a.x, a.mu), (b.x, b.mu)]
    y0 = W.uniform_targets(33, n_points, 2) * 0.6 + 0.2
    yb, lg = barycenter.damped_lloyd(src, y0, eps, tol=tol, max_outer=300, solve_tol=1e-8)
    M = 0.5 * ((a.mu[:, None] * a.x).sum(0) + (b.mu[:, None] * b.x).sum(0))
    merr = float(np.max(np.abs(yb.mean(0) - M)))
    solves = sum(sum(r["solve_iterations"]) for r in lg)
    log(f"[bench] barycenter: {len(lg)} Lloyd iterations, {lg[-1]['seconds']:.2f} s, "
        f"{solves} solver iterations, rel dy {lg[-1]['rel_dy']:.1e}, mean vs sources {merr:.1e}")
    return {"workload": f"blob2_square{n_cells}_nb{n_points}_eps{eps:g}", "iterations": len(lg),
            "seconds": lg[-1]["seconds"], "solver_iterations": solves,
            "rel_dy": lg[-1]["rel_dy"], "mean_err": merr, "J_first": lg[0]["J"],
            "J_last": lg[-1]["J"]}


def cpu_model():
    """The host CPU's model name (first entry of /proc/cpuinfo)."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(p, psi, psi_c1):
    """The oracle (plain FP64 C, OpenMP) on a bounded sample of the same
    workload: a seeded subset of quadrature points against all targets,
    sized to take ~15 s on all threads and ~4 s on one. value is the rate on
    that sample; the time of a full evaluation is extrapolated from it (and
    labelled so). The config-1 solve runs the oracle's strong-Wolfe L-BFGS,
    the line search the GPU solver uses."""
    import oracle
    from paper_2507_23602_amd import workloads as W
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    rng = np.random.default_rng(0)

    def rate(seconds, nth):
        probe = rng.choice(p.nq, size=512 if nth == 1 else 2048, replace=False)
        ts = time.perf_counter()
        oracle.dual_eval(p.x[probe], p.mu[probe], p.y, p.nu, psi, p.eps, threads=nth)
        tp = time.perf_counter() - ts
        m = int(min(p.nq, max(probe.size, probe.size * seconds / max(tp, 1e-3))))
        idx = rng.choice(p.nq, size=m, replace=False)
        ts = time.perf_counter()
        oracle.dual_eval(p.x[idx], p.mu[idx], p.y, p.nu, psi, p.eps, threads=nth)
        return m, time.perf_counter() - ts

    m, t = rate(15.0, threads)
    m1, t1 = rate(4.0, 1)
    value = m * p.n / t
    res = {"value": value, "unit": "pairs/s", "cores": threads, "kind": "oracle",
           "sample": f"{m} random quadrature points of the workload x all {p.n} targets "
                     f"(dense objective + gradient) in {t:.1f} s on {threads} threads; "
                     f"pairs/s measured on that sample",
           "extrapolated": True,
           "full_eval_seconds_extrapolated": p.nq * p.n / value,
           "cpu_model": cpu_model(), "nproc": os.cpu_count(),
           "single_thread_pairs_s": m1 * p.n / t1,
           "single_thread_sample": f"{m1} points x {p.n} targets in {t1:.1f} s"}
    log(f"[bench] cpu oracle ({res['cpu_model']}): {value:.3e} pairs/s on {threads} threads "
        f"({t:.1f}s), {res['single_thread_pairs_s']:.3e} on one; a full evaluation would take "
        f"{res['full_eval_seconds_extrapolated']:.0f} s (extrapolated)")
    if psi_c1 is not None:
        c1 = W.config1()

        def fun(v):
            e = oracle.dual_eval(c1.x, c1.mu, c1.y, c1.nu, v, c1.eps, threads=threads)
            return e.J, e.grad
        ts = time.perf_counter()
        _, _, g, it, nev = oracle.lbfgs_solve(fun, np.zeros(c1.n), tol=1e-6,
                                              h0=c1.eps * c1.n / c1.nu.sum(),
                                              line_search="wolfe")
        res["config1_solve_seconds"] = time.perf_counter() - ts
        res["config1_solve_iterations"] = it
        res["config1_solve_evaluations"] = nev
        res["config1_solve_line_search"] = "strong Wolfe (c1 1e-4, c2 0.9, <= 20 evaluations)"
        recheck = oracle.dual_eval(c1.x, c1.mu, c1.y, c1.nu, psi_c1, c1.eps, threads=threads)
        res["config1_gpu_psi_grad_l1_recheck"] = float(np.abs(recheck.grad).sum())
        log(f"[bench] cpu oracle config1 solve {res['config1_solve_seconds']:.2f}s ({it} it, "
            f"{nev} evaluations); recheck of GPU psi: |g|_1 = "
            f"{res['config1_gpu_psi_grad_l1_recheck']:.2e}")
    return res


if __name__ == "__main__":
    main()
