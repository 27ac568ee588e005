"""Throughput of the LDG implicit Euler step on one MI355X.

One "step" is one implicit Euler step of the whole hot path: sampling the
coefficient data at the quadrature points, L2 projection, block assembly,
block-Jacobi setup, the learned preconditioner's setup (network inference and
factor blocks), the Krylov solve to the relative residual of the full 3KN
system, recovery of Z.  Metric: DOF*steps/s with DOF = 3KN (C, Z1, Z2).

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--config combined-p4-1024]
                  [--precision fp64|fp32|bf16] [--precond bj|learned] [--weights F]
                  [--no-baseline] [--no-cpu-baseline]

Two further workloads are not time-step benchmarks of the five sizes: the
stationary verification problem of Table 2 (`--config table2-p4-96`, one
"step" is one solve of A Y = V) and the problem of the paper's main script
(`--config main-p2-8`, h = 1/8, p = 2, steps of pi/20).

The default run times the mixed-precision (BF16 contractions, FP64
refinement) solver with the learned factored preconditioner on the combined
workload, then the plain FP64 block-Jacobi solver on the same workload for
comparison.  Prints one JSON line (rank 0).  Progress goes to stderr.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from inputs.fields import (LOGNORMAL, LOGNORMAL_T, MAIN, SMOOTH1, SMOOTH2, TABLE2,  # noqa: E402
                           Workload, lognormal_blocks, triangle_values)
from inputs.meshes import NORTH, SOUTH, square_mesh  # noqa: E402

HBM_PEAK_GBS = 8000.0
MFMA_PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3}   # dense matrix-core peaks of the MI355X

# The five workloads: mesh of n x n cells (2 n^2 triangles), order p, data.
CONFIGS = {
    "plain-p1-8": dict(n=8, p=1, jitter=None, kind=SMOOTH1, dt=1e-2),
    "plain-p2-64": dict(n=64, p=2, jitter=1002, kind=SMOOTH2, dt=1e-3),
    "mixed-p4-512": dict(n=512, p=4, jitter=1003, kind=SMOOTH2, dt=1e-4),
    "learned-p3-256": dict(n=256, p=3, jitter=1004, kind=LOGNORMAL, sigma=1.5, field_seed=4100,
                           dt=1e-4),
    "combined-p4-1024": dict(n=1024, p=4, jitter=1005, kind=LOGNORMAL_T, sigma=1.0,
                             field_seed=5000, dt=1e-4),
    # stationary solves of the Table 2 problem (h = 1/96), and the main script's problem
    "table2-p4-96": dict(n=96, p=4, jitter=None, kind=TABLE2, neumann=(SOUTH, NORTH),
                         stationary=True, dt=0.0, restart=150, max_iters=200000, cpu_cells=16),
    "main-p2-8": dict(n=8, p=2, jitter=None, kind=MAIN, neumann=(SOUTH, NORTH), dt=np.pi / 20),
}
DEFAULT = "combined-p4-1024"
# trained weights of the factored preconditioner per order (learned.py)
WEIGHTS = {4: os.path.join(ROOT, "paper_1408_3877_amd", "weights", "factor_p4.npy"),
           3: os.path.join(ROOT, "paper_1408_3877_amd", "weights", "factor_p3.npy")}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_inputs(cfg):
    coordV, V0T, kind = square_mesh(cfg["n"], seed=cfg["jitter"],
                                    neumann_sides=cfg.get("neumann", ()))
    dT = None
    if cfg["kind"] in (LOGNORMAL, LOGNORMAL_T):
        blocks = lognormal_blocks(cfg["n"], cfg["field_seed"], cfg["sigma"], block=8)
        dT = triangle_values(blocks, cfg["n"], block=8)
    return coordV, V0T, kind, dT


def triangle_area2(coordV, V0T):
    """2|T_k| from the vertex coordinates."""
    a, b, c = (coordV[V0T[:, i]] for i in range(3))
    return np.abs((b[:, 0] - a[:, 0]) * (c[:, 1] - a[:, 1]) - (b[:, 1] - a[:, 1]) * (c[:, 0] - a[:, 0]))


def dt_of(cfg):
    return cfg["dt"]


def kernel_table(stats):
    return {k: {"launches": v["launches"], "ms": round(v["total_ms"], 3),
                "GB/s": round(v["bytes"] / (v["total_ms"] * 1e-3) / 1e9, 1)
                if v["total_ms"] > 0 else None} for k, v in stats.items()}


def timed_run(Solver, torch, cfg, coordV, V0T, kind, dT, prec, learned, weights, args, label):
    """Warmup steps, then args.steps timed steps of one solver configuration."""
    t0 = time.perf_counter()
    s = Solver(coordV, V0T, kind, cfg["p"], rtol=args.rtol, restart=args.restart,
               max_iters=cfg.get("max_iters", 20000), precision=prec, inner_rtol=args.inner_rtol,
               precond=1 if learned else 0, keep_direction=not args.fresh_cg_sweeps,
               edge_traces=not args.stored_blocks)
    if learned:
        s.gnn_set_mode("factor")
        s.gnn_factor_storage(args.fac_storage)
        s.gnn_set_params(weights)
    s.set_time_scheme(args.time_scheme)
    if args.matrix_free:
        s.set_matrix_free(True)
    log("[bench] %s: context K=%d N=%d (%.1f s)" % (label, s.K, s.N, time.perf_counter() - t0))
    gk = cfg["kind"]
    s.set_initial_samples(s.sample_workload(gk, 0.0, dT=dT, want=("c0",))["c0"])
    state = {"t": 0.0}
    dt = cfg["dt"]

    def one_step():
        if cfg.get("stationary"):
            smp = s.sample_workload(gk, 0.0, dT=dT)
            return s.solve_stationary_sampled(smp["d"], smp["f"], smp["cD"], smp["gN"])
        state["t"] += dt
        smp = s.sample_workload(gk, state["t"], dT=dT)
        return s.step_sampled(dt, smp["d"], smp["f"], smp["cD"], smp["gN"])

    for i in range(args.warmup):
        info = one_step()
        log("[bench] %s warmup %d: iters=%d learned=%d rel_res=%.2e" %
            (label, i, info["iters"], info["learned_iters"], info["rel_residual"]))
    if args.copy_calibration:
        a = torch.empty(1 << 27, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        a.fill_(1.0)
        b.copy_(a)
        torch.cuda.synchronize()
    torch.cuda.synchronize()
    s.set_timing(not args.no_kernel_timing)
    torch.cuda.synchronize()
    infos = []
    t0 = time.perf_counter()
    for i in range(args.steps):
        info = one_step()
        infos.append(info)
        log("[bench] %s step %d: iters=%d learned=%d sweeps=%d fallbacks=%d krylov=%d rel_res=%.2e"
            % (label, i, info["iters"], info["learned_iters"], info["restarts"], info["fallbacks"],
               info["krylov"], info["rel_residual"]))
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    stats = s.kernel_stats()
    s.set_timing(False)
    return {"solver": s, "elapsed": el, "infos": infos, "stats": stats}


def kernel_source_hash():
    h = hashlib.sha256()
    for f in sorted(os.listdir(os.path.join(ROOT, "paper_1408_3877_amd", "csrc"))):
        with open(os.path.join(ROOT, "paper_1408_3877_amd", "csrc", f), "rb") as fh:
            h.update(f.encode() + fh.read())
    return h.hexdigest()[:16]


def measured_traffic(config, kernel, precision, precond, matrix_free=False):
    """HBM bytes per launch of the dominant kernel from the committed counter
    summaries, or None when absent, for another run, or the kernels changed
    since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "traffic_%s.json" % config)
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    for r in rec.get("records", [rec]):
        if r.get("kernel_source_hash") != kernel_source_hash():
            continue
        if (r.get("kernel"), r.get("precision"), r.get("precond"),
                bool(r.get("matrix_free", False))) == (kernel, precision, precond, matrix_free):
            return r.get("bytes_per_launch")
    return None


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_extrapolated(cfg, K_target, iters_target, n=48):
    """The oracle's iterative step (block-Jacobi CG on its explicitly formed
    eliminated matrix, the solver the FP64 block-Jacobi GPU baseline runs) on
    an n x n-cell sample of the same family, with one thread, extrapolated to
    the benchmarked mesh.  The step runs twice, to relative residuals 1e-4 and
    1e-10: the difference gives the cost of one CG iteration, the rest is the
    per-step work (assembly of the blocks and the eliminated matrix, the
    block-Jacobi inverses, the recovery of Z).  Both grow linearly with K
    (sparse products, blockwise work); the iteration count is the GPU
    baseline's on the benchmarked mesh.  A model, not a measurement of the
    whole mesh (one such step would take hours), and labelled as such."""
    from threadpoolctl import threadpool_limits

    from oracle.ldg import Problem, step_schur_cg
    coordV, V0T, kind = square_mesh(n, seed=cfg["jitter"], neumann_sides=cfg.get("neumann", ()))
    w = Workload(cfg["kind"], n_cells=n,
                 blocks=lognormal_blocks(n, cfg["field_seed"], cfg["sigma"], block=8), block=8)
    runs = {}
    with threadpool_limits(1):
        pr = Problem(coordV, V0T, kind, cfg["p"])
        C = pr.initial(w)
        data = pr.data(w, cfg["dt"])
        for rtol in (1e-4, 1e-10):
            t0 = time.perf_counter()
            _, _, _, info = step_schur_cg(pr, C, cfg["dt"], cfg["dt"], w, rtol=rtol, data=data)
            runs[rtol] = (time.perf_counter() - t0, info["iters"])
    (t4, i4), (t8, i8) = runs[1e-4], runs[1e-10]
    t_iter = max(t8 - t4, 0.0) / max(i8 - i4, 1)
    t_fixed = max(t8 - i8 * t_iter, 0.0)
    K_s = pr.grid.numT
    t_target = (t_fixed + t_iter * iters_target) * K_target / K_s
    dof = 3 * K_target * pr.N
    return {"value": dof / t_target, "unit": "DOF*steps/s", "cores": 1,
            "kind": "oracle, extrapolated per-step",
            "seconds_per_step": t_target,
            "sample": "%dx%d cells (K=%d), one step by the oracle's block-Jacobi CG: %.2f s for %d "
                      "iterations to 1e-4, %.2f s for %d to 1e-10, i.e. %.4f s per iteration and "
                      "%.2f s per-step work; scaled by K=%d/%d with %d iterations (the FP64 "
                      "block-Jacobi GPU baseline's on this mesh)" % (
                          n, n, K_s, t4, i4, t8, i8, t_iter, t_fixed, K_target, K_s,
                          round(iters_target))}


def cpu_baseline(cfg):
    """The oracle (direct sparse solve of the full 3KN system, Sec. 2.5) on a
    bounded sample of the same workload family: 24 x 24 cells (16 x 16 for the
    stationary workload), same p, same fields, 2 steps.  Timed with one BLAS
    thread and with every host thread the process may use; the faster run is
    the reported value.  The oracle's sparse assembly and SuperLU dominate;
    its direct solve's fill-in grows faster than K, and its iterative step
    (block-Jacobi CG on the explicitly formed eliminated matrix) is slower
    still at these sizes, so no larger sample fits in the seconds this
    measurement may take."""
    from threadpoolctl import threadpool_limits

    from oracle.ldg import Problem
    n = cfg.get("cpu_cells", 24)
    coordV, V0T, kind = square_mesh(n, seed=cfg["jitter"], neumann_sides=cfg.get("neumann", ()))
    if cfg["kind"] in (LOGNORMAL, LOGNORMAL_T):
        w = Workload(cfg["kind"], n_cells=n,
                     blocks=lognormal_blocks(n, cfg["field_seed"], cfg["sigma"], block=8), block=8)
    else:
        w = Workload(cfg["kind"])
    steps = 2
    nthreads = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    runs = []
    for threads in sorted({1, nthreads}):
        with threadpool_limits(threads):
            pr = Problem(coordV, V0T, kind, cfg["p"])
            t0 = time.perf_counter()
            if cfg.get("stationary"):
                for _ in range(steps):
                    pr.solve_stationary(w)
            else:
                C = pr.initial(w)
                t = 0.0
                for _ in range(steps):
                    t += cfg["dt"]
                    C, _, _, _ = pr.step(C, t, cfg["dt"], w)
            runs.append((time.perf_counter() - t0, threads))
    el, cores = min(runs)
    dof = 3 * pr.grid.numT * pr.N
    what = "solves" if cfg.get("stationary") else "steps"
    return {"value": dof * steps / el, "unit": "DOF*%s/s" % what, "cores": cores, "kind": "oracle",
            "cpu": cpu_model(),
            "runs": [{"threads": th, "seconds": round(e, 2), "value": dof * steps / e}
                     for e, th in runs],
            "sample": "%dx%d-cell mesh of the same family (K=%d, p=%d, DOF=%d), %d %s, "
                      "sparse direct solve of the full system; %s" % (
                          n, n, pr.grid.numT, cfg["p"], dof, steps, what,
                          ", ".join("%.1f s with %d thread%s" % (e, th, "s" if th > 1 else "")
                                    for e, th in runs))}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default=DEFAULT, choices=sorted(CONFIGS))
    ap.add_argument("--restart", type=int, default=None,
                    help="GMRES restart length (default 30; 150 for the stationary workload)")
    ap.add_argument("--rtol", type=float, default=1e-8)
    ap.add_argument("--precision", default="bf16", choices=["fp64", "fp32", "bf16"],
                    help="inner-solve precision (fp32/bf16: mixed with FP64 refinement)")
    ap.add_argument("--precond", default=None, choices=["bj", "learned"],
                    help="block-Jacobi, or the learned factored preconditioner (CG on symmetric "
                         "steps, GMRES on the symmetric part's factor otherwise; default: learned "
                         "where trained weights exist for the order and the workload steps in "
                         "time, else block-Jacobi)")
    ap.add_argument("--weights", default=None, help="network weights (.npy); default per order")
    ap.add_argument("--fac-storage", default="fp8", choices=["f32", "bf16", "fp8", "fp8w"],
                    help="storage of the learned preconditioner's factor blocks")
    ap.add_argument("--time-scheme", default="euler", choices=["euler", "bdf2"],
                    help="implicit Euler (the paper's) or two-step backward differentiation")
    ap.add_argument("--matrix-free", action="store_true",
                    help="apply the operator without streaming stored blocks (both runs)")
    ap.add_argument("--no-kernel-timing", action="store_true",
                    help="time the steps without per-kernel HIP events (no roofline)")
    ap.add_argument("--no-baseline", action="store_true",
                    help="skip timing the plain FP64 block-Jacobi solver for comparison")
    ap.add_argument("--inner-rtol", type=float, default=1e-2,
                    help="relative tolerance of each inner solve of the mixed modes (1e-2: fewest "
                         "CG iterations on the combined workload in a sweep over 1e-4 .. 1e-1)")
    ap.add_argument("--stored-blocks", action="store_true",
                    help="mixed modes: inner solves apply the stored FP32/BF16 blocks instead of "
                         "the FP32 quadrature form")
    ap.add_argument("--fresh-cg-sweeps", action="store_true",
                    help="start CG afresh in every refinement sweep instead of continuing "
                         "from the previous sweep's search direction")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB device copy (for counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path; "
              "use --gpus 1", file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_1408_3877_amd import Solver
    cfg = CONFIGS[args.config]
    if args.restart is None:
        args.restart = cfg.get("restart", 30)
    log("[bench] config %s: building inputs" % args.config)
    coordV, V0T, kind, dT = make_inputs(cfg)
    torch.cuda.set_device(0)
    if args.precond is None:
        args.precond = "learned" if cfg["p"] in WEIGHTS and not cfg.get("stationary") else "bj"
    learned = args.precond == "learned"
    weights = None
    if learned:
        path = args.weights or WEIGHTS.get(cfg["p"])
        if not path or not os.path.exists(path):
            log("[bench] no trained weights for p=%d (%s)" % (cfg["p"], path))
            sys.exit(2)
        weights = np.load(path).astype(np.float32)
    prec = {"fp64": 0, "fp32": 1, "bf16": 2}[args.precision]
    run = timed_run(Solver, torch, cfg, coordV, V0T, kind, dT, prec, learned, weights, args,
                    "headline")
    base = None
    if not args.no_baseline and (prec != 0 or learned):
        base = timed_run(Solver, torch, cfg, coordV, V0T, kind, dT, 0, False, None, args,
                         "fp64 block-Jacobi")
    s, el, infos, stats = run["solver"], run["elapsed"], run["infos"], run["stats"]
    dof = 3 * s.K * s.N
    value = dof * args.steps / el
    # roofline of the kernel that takes the most time in the timed steps
    if args.no_kernel_timing:
        log("[bench] no kernel timing: %.4g DOF*steps/s, %.1f ms per step" %
            (dof * args.steps / el, el * 1e3 / args.steps))
        return
    name = max(("div", "factor", "bj_apply", "grad", "mf"), key=lambda k: stats[k]["total_ms"])
    kv = stats[name]
    per_launch = kv["bytes"] / max(kv["launches"], 1)
    avg_ms = kv["total_ms"] / max(kv["launches"], 1)
    kernel_desc = {"div": "k_div (operator apply, divergence half)",
                   "factor": "k_fac_w + k_fac_f (learned factored preconditioner apply)",
                   "bj_apply": "k_bj_apply (block-Jacobi apply)",
                   "grad": "k_grad (operator gradient half)",
                   "mf": "k_mf_blocks (matrix-free block terms on the matrix cores)"}[name]
    traffic = None if args.stored_blocks else measured_traffic(
        args.config, name, args.precision, args.precond + ("-" + args.fac_storage if learned else ""),
        args.matrix_free)
    if name == "mf":
        # bound by the matrix cores: useful flops of the contraction per launch
        flops = kv["flops"] / max(kv["launches"], 1)
        peak = MFMA_PEAK_TFLOPS["fp64" if prec == 0 else "fp32"]
        ach = flops / (avg_ms * 1e-3) / 1e12 if avg_ms > 0 else 0.0
        roof = {"bound": "mfma", "kernel": kernel_desc, "achieved": ach, "peak": peak,
                "unit": "TFLOP/s", "frac": ach / peak, "algorithmic_flops_per_launch": flops,
                "algorithmic_bytes_per_launch": per_launch, "avg_launch_ms": avg_ms,
                "traffic": traffic}
    else:
        ach = kv["bytes"] / (kv["total_ms"] * 1e-3) / 1e9 if kv["total_ms"] > 0 else 0.0
        roof = {"bound": "hbm", "kernel": kernel_desc, "achieved": ach, "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": ach / HBM_PEAK_GBS,
                "algorithmic_bytes_per_launch": per_launch, "avg_launch_ms": avg_ms,
                "traffic": traffic}
    solver_desc = "%s %s %s%s" % (
        args.precision,
        "learned factored (%s factor blocks)" % args.fac_storage if learned else "block-Jacobi",
        "CG" if infos[-1]["krylov"] == 2 else "GMRES(%d)" % args.restart,
        "" if prec == 0 else " + FP64 refinement (inner rtol %g, %s%s)" % (
            args.inner_rtol,
            "matrix-free operator" if args.matrix_free else
            "stored %s operator blocks" % args.precision if args.stored_blocks
            else "operator in FP32 quadrature form",
            "" if infos[-1]["krylov"] != 2 else
            ", fresh CG per sweep" if args.fresh_cg_sweeps else ", CG direction kept across sweeps"))
    stationary = bool(cfg.get("stationary"))
    res = {
        "metric": ("DOF·solves/s of the stationary Table 2 problem to 1e-8 rel res" if stationary
                   else "DOF·steps/s (p=4, 2M tris) to 1e-8 rel res: plain FP64 vs mixed+learned "
                        "precond"),
        "value": value,
        "unit": "DOF*solves/s" if stationary else "DOF*steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": el * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32+f64", "bf16": "bf16+f32+f64"}[args.precision],
        "data": "synthetic",
        "config": {"workload": args.config, "K": s.K, "N": s.N, "p": cfg["p"], "DOF": dof,
                   "dt": dt_of(cfg), "rtol": args.rtol,
                   "time_scheme": "stationary" if stationary else args.time_scheme,
                   "matrix_free": args.matrix_free,
                   "solver": solver_desc,
                   "weights": os.path.relpath(args.weights or WEIGHTS.get(cfg["p"]), ROOT)
                   if learned else None,
                   "iters_per_step": sum(i["iters"] for i in infos) / len(infos),
                   "learned_iters_per_step": sum(i["learned_iters"] for i in infos) / len(infos),
                   "refinement_sweeps_per_step": sum(i["ir_steps"] for i in infos) / len(infos),
                   "fallbacks": sum(i["fallbacks"] for i in infos),
                   "max_rel_residual": max(i["rel_residual"] for i in infos)},
        "roofline": roof,
        "kernels": kernel_table(stats),
    }
    if base is not None:
        bs = base["solver"]
        bv = dof * args.steps / base["elapsed"]
        bk = base["stats"]["div"]
        res["baseline_fp64_bj"] = {
            "value": bv, "ms_per_step": base["elapsed"] * 1e3 / args.steps,
            "iters_per_step": sum(i["iters"] for i in base["infos"]) / len(base["infos"]),
            "k_div_GBs": bk["bytes"] / (bk["total_ms"] * 1e-3) / 1e9 if bk["total_ms"] > 0 else None,
            "kernels": kernel_table(base["stats"])}
        res["speedup_vs_fp64_bj"] = value / bv
        # relative L2 difference of c_h (orthonormal basis: ||c_h||^2 = sum_k 2|T_k| |C_k|^2)
        c1 = s.get_solution()[0].double().cpu().numpy()
        c0 = bs.get_solution()[0].double().cpu().numpy()
        a2 = triangle_area2(coordV, V0T)
        res["rel_l2_diff_vs_fp64_bj"] = float(np.sqrt(np.sum(a2[:, None] * (c1 - c0) ** 2) /
                                                      np.sum(a2[:, None] * c0 ** 2)))
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle) ...")
        res["cpu_baseline"] = cpu_baseline(cfg)
        if base is not None and cfg["kind"] in (LOGNORMAL, LOGNORMAL_T) and not cfg.get("stationary"):
            log("[bench] cpu baseline, extrapolated (oracle block-Jacobi CG) ...")
            res["cpu_baseline"]["extrapolated"] = cpu_extrapolated(
                cfg, s.K, res["baseline_fp64_bj"]["iters_per_step"])
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
