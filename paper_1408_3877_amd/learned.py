"""Training and evaluation of the learned preconditioner on the method's own systems.

    python -m paper_1408_3877_amd.learned --p 3 --n 256 --sigma 1.5 \
        --train-seeds 4000-4019 --eval-seeds 4100,4101 --out weights.npy

1. Data: for every training field seed, run implicit Euler steps with plain
   block-Jacobi CG and keep (BJ^{-1} r / rho, (e - BJ^{-1} r) / rho) pairs from
   CG iterates (ldg_gnn_collect): the systems and solutions the method itself
   generates.  Later rounds add pairs from the iterates of flexible CG with
   the network trained so far, whose residuals differ from plain CG's.
2. Training: Adam, one system sample per step, on the device
   (ldg_gnn_train_step), on the energy-norm error of the preconditioned step
   relative to that of the block-Jacobi step (default) or, for the
   residual-correction network, on the mean squared error of the correction.
   --mode factor (default) trains the factored preconditioner (a linear SPD
   operator built once per system), by default on the Frobenius objective
   ||G S G^T - I||_F^2 estimated with Gaussian probe vectors on the systems
   of the method's steps; --mode correction the per-iteration
   residual-correction network.
3. Evaluation: the same steps on held-out fields with block-Jacobi CG and
   with the learned preconditioner (flexible CG, block-Jacobi fallback);
   iterations and time per step for both.
4. Calibration (--calibrate, factored network): the Frobenius objective
   fixes where omega is larger or smaller, but its optimum level lies below
   the one with the fewest CG iterations.  The head's output bias b_o (omega =
   OMEGA_MAX sigmoid(... + b_o)) is shifted by the listed value that gives
   the fewest iterations over one step on each calibration field (training
   fields by default), with the solver configuration that is deployed:
   BF16 inner solves at inner tolerance 1e-2 with FP64 refinement.

Only argument marshalling and the loop live here; every kernel runs in the
library.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from inputs.fields import LOGNORMAL, LOGNORMAL_T, lognormal_blocks, triangle_values  # noqa: E402
from inputs.meshes import square_mesh  # noqa: E402

SNAPS = [0, 1, 2, 3, 5, 8, 12, 18, 27, 40, 60, 90, 135, 200, 300, 450, 675, 1000, 1500, 2250]
# the optimal-step loss learns from the smooth late errors, which decide CG's iteration count
SNAPS_LATE = [90, 135, 200, 300, 450, 675, 1000, 1500]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def glorot(N, seed, width=32, e_in=13, layers=3):
    """Initial parameters in the library's flat layout (Glorot-uniform, zero biases)."""
    rng = np.random.default_rng(seed)
    parts = []

    def mat(r, c):
        lim = np.sqrt(6.0 / (r + c))
        parts.append(rng.uniform(-lim, lim, r * c))

    mat(2 * N + 3, width)
    parts.append(np.zeros(width))
    for _ in range(layers):
        mat(width, width)
        mat(e_in, width)
        parts.append(np.zeros(width))
        mat(2 * width, width)
        parts.append(np.zeros(width))
    mat(width, N)
    parts.append(np.zeros(N))
    return np.concatenate(parts).astype(np.float32)


def factor_init(N, seed, width=32, e_in=13, layers=3, omega0=0.6, omega_max=0.95):
    """Initial parameters of the factored network: Glorot-uniform trunk on the
    N + 3 node features, a small edge head whose bias gives omega = omega0."""
    rng = np.random.default_rng(seed)
    parts = []

    def mat(r, c):
        lim = np.sqrt(6.0 / (r + c))
        parts.append(rng.uniform(-lim, lim, r * c))

    mat(N + 3, width)
    parts.append(np.zeros(width))
    for _ in range(layers):
        mat(width, width)
        mat(e_in, width)
        parts.append(np.zeros(width))
        mat(2 * width, width)
        parts.append(np.zeros(width))
    for r in (width, width, e_in):
        lim = np.sqrt(6.0 / (r + 1))
        parts.append(0.1 * rng.uniform(-lim, lim, r))
    q = omega0 / omega_max
    parts.append(np.array([0.0, np.log(q / (1.0 - q))]))
    return np.concatenate(parts).astype(np.float32)


KIND = LOGNORMAL   # field family: LOGNORMAL, or LOGNORMAL_T (times 1 + 0.1 sin t)


def field(n, seed, sigma):
    return triangle_values(lognormal_blocks(n, seed, sigma, block=8), n, block=8)


def collect(solver, n, seeds, sigma, steps, dt, snaps=SNAPS, per_step=None):
    """(rhat, target, D) triples on the device, from BJ-CG steps of every seed."""
    torch = solver.torch
    data = []
    for sd in seeds:
        dT = field(n, sd, sigma)
        solver.set_initial_samples(solver.sample_workload(KIND, 0.0, dT=dT, want=("c0",))["c0"])
        D = solver.project(solver.sample_workload(KIND, dt, dT=dT, want=("d",))["d"]).clone()
        t = 0.0
        for _ in range(steps):
            t += dt
            r, tg = solver.gnn_collect(snaps if per_step is None else snaps[:per_step])
            smp = solver.sample_workload(KIND, t, dT=dT)
            info = solver.step_sampled(dt, smp["d"], smp["f"], smp["cD"], smp["gN"])
            m = solver.gnn_collected()
            for q in range(m):
                data.append((r[q].clone(), tg[q].clone(), D))
            log("[collect] seed %d t=%.1e iters=%d pairs=%d total=%d" % (sd, t, info["iters"], m, len(data)))
        torch.cuda.synchronize()
    return data


def train(solver, data, epochs, lr, dt, seed):
    rng = np.random.default_rng(seed)
    losses = []
    step = 0
    total = epochs * len(data)
    for ep in range(epochs):
        order = rng.permutation(len(data))
        acc = 0.0
        for i in order:
            r, tg, D = data[i]
            solver.gnn_set_context(D, dt)
            lr_t = lr * 0.5 * (1 + np.cos(np.pi * step / total))   # cosine decay
            acc += solver.gnn_train_step(r, tg, lr_t)
            step += 1
        losses.append(acc / len(data))
        log("[train] epoch %d mean loss %.5f" % (ep, losses[-1]))
    return losses


def systems(solver, n, seeds, sigma, steps, dt):
    """The projected coefficients of the method's steps (one system per step)."""
    out = []
    for sd in seeds:
        dT = field(n, sd, sigma)
        t = 0.0
        for _ in range(steps):
            t += dt
            out.append(solver.project(solver.sample_workload(KIND, t, dT=dT, want=("d",))["d"]).clone())
    return out


def train_probes(solver, sys_list, epochs, probes, lr, dt, seed):
    """Adam on the Frobenius loss: every system, `probes` Gaussian probe vectors
    per visit (drawn here, seeded, and passed in)."""
    rng = np.random.default_rng(seed)
    K, N = solver.K, solver.N
    losses = []
    step, total = 0, epochs * len(sys_list) * probes
    for ep in range(epochs):
        acc = 0.0
        for i in rng.permutation(len(sys_list)):
            solver.gnn_set_context(sys_list[i], dt)
            for _ in range(probes):
                w = rng.standard_normal((K, N)).astype(np.float32)
                lr_t = lr * 0.5 * (1 + np.cos(np.pi * step / total))
                acc += solver.gnn_train_step(w, w, lr_t)
                step += 1
        losses.append(acc / (len(sys_list) * probes))
        log("[train] epoch %d mean loss %.5f" % (ep, losses[-1]))
    return losses


def evaluate(solver, n, seeds, sigma, steps, dt, use_gnn):
    """Mean iterations and seconds per step (block-Jacobi or learned)."""
    torch = solver.torch
    its, secs, fbs, lits, why = [], [], 0, 0, []
    for sd in seeds:
        dT = field(n, sd, sigma)
        solver.set_initial_samples(solver.sample_workload(KIND, 0.0, dT=dT, want=("c0",))["c0"])
        t = 0.0
        for _ in range(steps):
            t += dt
            smp = solver.sample_workload(KIND, t, dT=dT)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            info = solver.step_sampled(dt, smp["d"], smp["f"], smp["cD"], smp["gN"])
            torch.cuda.synchronize()
            secs.append(time.perf_counter() - t0)
            its.append(info["iters"])
            fbs += info["fallbacks"]
            lits += info["learned_iters"]
            if info["fallbacks"]:
                why.append(info["fallback_reason"])
            log("[eval] %s seed %d t=%.1e %s" % ("learned" if use_gnn else "bj", sd, t, info))
    return {"iters_per_step": float(np.mean(its)), "s_per_step": float(np.mean(secs)),
            "fallbacks": fbs, "fallback_reasons": why, "learned_iters": lits, "steps": len(its)}


def calibrate(solver, w, shifts, n, seeds, sigma, dt):
    """The shift of the output bias b_o (the last parameter of the factored
    network) from `shifts` with the fewest CG iterations per step on `seeds`;
    returns (shifted weights, [(shift, iterations per step)])."""
    table = []
    for d in shifts:
        wd = w.copy()
        wd[-1] += np.float32(d)
        solver.gnn_set_params(wd)
        r = evaluate(solver, n, seeds, sigma, 1, dt, True)
        table.append((float(d), r["iters_per_step"]))
        log("[calibrate] b_o shift %+.2f: %.1f iterations per step" % (d, r["iters_per_step"]))
    best = min(table, key=lambda x: (x[1], abs(x[0])))
    w = w.copy()
    w[-1] += np.float32(best[0])
    return w, table


HEAD = 2 * 32 + 13 + 2   # head parameters at the end of the factored network's vector


def cg_cases(solver, n, seeds, sigma, dt):
    """First-step systems of the training fields: device samples of c0 and of
    the data at t = dt, for repeated solves."""
    out = []
    for sd in seeds:
        dT = field(n, sd, sigma)
        c0 = solver.sample_workload(KIND, 0.0, dT=dT, want=("c0",))["c0"].clone()
        smp = solver.sample_workload(KIND, dt, dT=dT)
        out.append((c0, {k: v.clone() for k, v in smp.items() if v is not None}))
    return out


def cg_objective(solver, w, cases, dt):
    """Mean log10 of the relative residual of the full system after the
    solver's max_iters preconditioned CG iterations (FP64), over the cases:
    how far CG gets with the preconditioner these weights build."""
    from .ldg import LdgError
    solver.gnn_set_params(w)
    vals = []
    for c0, smp in cases:
        solver.set_initial_samples(c0, 0.0)
        try:
            info = solver.step_sampled(dt, smp["d"], smp["f"], smp.get("cD"), smp.get("gN"))
        except LdgError as e:
            if e.code != -5:
                raise
            info = e.info
        if info["fallbacks"]:
            return np.inf                     # a curvature breakdown: the weights are unusable
        vals.append(np.log10(max(info["rel_residual"], 1e-300)))
    return float(np.mean(vals))


def with_head(w, head):
    out = w.copy()
    out[-HEAD:] = head.astype(np.float32)
    return out


def constant_head(omega, omega_max=0.95):
    """Head parameters giving omega on every edge: zero weights, the bias alone."""
    h = np.zeros(HEAD)
    q = omega / omega_max
    h[-1] = np.log(q / (1.0 - q))
    return h


def train_head_cg(solver, w, cases, dt, omegas, iters, c, a, seed, from_start=False):
    """Fit the head (the last HEAD parameters; the trunk stays) to the CG
    objective: the best constant omega on the grid `omegas` first, then
    simultaneous-perturbation stochastic approximation (SPSA) from there, with
    Rademacher perturbations of size c_k = c / (k+1)^0.101 and steps
    a_k = a / (k+11)^0.602.  Every evaluated head is a candidate; the best
    one is returned with the history."""
    rng = np.random.default_rng(seed)
    hist = {"constant": [], "spsa": []}
    best_h, best_v = None, np.inf
    for om in omegas:
        h = constant_head(om)
        v = cg_objective(solver, with_head(w, h), cases, dt)
        hist["constant"].append((float(om), v))
        log("[cg-head] constant omega %.2f: %.4f" % (om, v))
        if v < best_v:
            best_h, best_v = h, v
    hist["best_constant"] = min(hist["constant"], key=lambda x: x[1])
    if from_start:
        best_h = w[-HEAD:].astype(np.float64).copy()
        best_v = cg_objective(solver, w, cases, dt)
        hist["start"] = best_v
        hist.pop("best_at", None)
        log("[cg-head] start weights: %.4f" % best_v)
    # the head's inputs differ in scale by orders of magnitude: measure how far
    # each parameter moves omega (RMS over the interior edges of the first
    # case's system) and search in coordinates u where a unit step of any one
    # parameter moves omega by 1 / sqrt(HEAD) in RMS
    c0, smp = cases[0]
    solver.gnn_set_context(solver.project(smp["d"]), dt)
    solver.gnn_set_params(with_head(w, best_h))
    om0 = solver.gnn_factor_omega().double().cpu().numpy()
    inner = om0 != 0.0
    sens = np.zeros(HEAD)
    eps = 1e-2
    for i in range(HEAD):
        h = best_h.copy()
        h[i] += eps
        solver.gnn_set_params(with_head(w, h))
        om = solver.gnn_factor_omega().double().cpu().numpy()
        sens[i] = np.sqrt(np.mean((om - om0)[inner] ** 2)) / eps
    # a parameter that does not move omega on the training systems (an edge
    # feature that never occurs there, such as an (n, n+) pair the training
    # meshes lack) stays where it is: the objective cannot see it, and an
    # unconstrained value would set omega arbitrarily on meshes that have it
    seen = sens > 1e-9 * sens.max()
    scale = np.where(seen, 1.0 / (np.maximum(sens, 1e-300) * np.sqrt(HEAD)), 0.0)
    hist["frozen"] = np.flatnonzero(~seen).tolist()
    hist["sensitivity"] = sens.tolist()
    u = np.zeros(HEAD)
    for k in range(iters):
        ck = c / (k + 1) ** 0.101
        ak = a / (k + 11) ** 0.602
        delta = rng.choice([-1.0, 1.0], HEAD)
        hp, hm = best_h + scale * (u + ck * delta), best_h + scale * (u - ck * delta)
        vp = cg_objective(solver, with_head(w, hp), cases, dt)
        vm = cg_objective(solver, with_head(w, hm), cases, dt)
        for v, h in ((vp, hp), (vm, hm)):
            if v < best_v:
                best_v, best_new = v, h.copy()
                hist["best_at"] = k
        if np.isfinite(vp) and np.isfinite(vm):
            g = (vp - vm) / (2 * ck) * delta
            u = u - np.clip(ak * g, -0.05, 0.05)
        hist["spsa"].append((vp, vm, best_v))
        log("[cg-head] spsa %d: %.4f %.4f best %.4f" % (k, vp, vm, best_v))
    if "best_at" in hist:
        best_h = best_new
    return with_head(w, best_h), best_v, hist


def seeds_arg(s):
    if "-" in s:
        a, b = s.split("-")
        return list(range(int(a), int(b) + 1))
    return [int(x) for x in s.split(",")]


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--p", type=int, default=3)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--jitter", type=int, default=1004)
    ap.add_argument("--sigma", type=float, default=1.5)
    ap.add_argument("--kind", type=int, default=LOGNORMAL, choices=(LOGNORMAL, LOGNORMAL_T),
                    help="3: block log-normal field, 4: the same times (1 + 0.1 sin t)")
    ap.add_argument("--dt", type=float, default=1e-4)
    ap.add_argument("--train-seeds", default="4000-4019")
    ap.add_argument("--eval-seeds", default="4100,4101")
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--eval-steps", type=int, default=3)
    ap.add_argument("--epochs", type=int, default=4, help="epochs per round")
    ap.add_argument("--rounds", type=int, default=2,
                    help="collection rounds (1: block-Jacobi solves only)")
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--init-seed", type=int, default=7)
    ap.add_argument("--loss", choices=("frobenius", "energy", "mse", "optstep", "cg"), default=None,
                    help="default: frobenius (factor mode), energy (correction mode); cg: fit the "
                         "factored head to CG convergence (after a Frobenius training, or on "
                         "--start-weights)")
    ap.add_argument("--start-weights", default=None,
                    help="cg loss: trunk to keep (\"init\": the untrained initialisation; default: "
                         "train it on the Frobenius objective)")
    ap.add_argument("--spsa-from", choices=("constant", "start"), default="constant",
                    help="cg loss: start the SPSA search at the best constant omega, or at the "
                         "head of the start weights")
    ap.add_argument("--cg-iters", type=int, default=150,
                    help="cg loss: CG iterations after which the residual is scored")
    ap.add_argument("--cg-omegas", default="0.5,0.6,0.7,0.75,0.8,0.85,0.9",
                    help="cg loss: constant omegas tried before the SPSA search")
    ap.add_argument("--spsa-iters", type=int, default=120)
    ap.add_argument("--spsa-c", type=float, default=0.03,
                    help="RMS change of omega of a perturbation")
    ap.add_argument("--spsa-a", type=float, default=0.5)
    ap.add_argument("--cg-seeds", default=None,
                    help="cg loss: training fields for the head fit (default: the first six "
                         "training seeds)")
    ap.add_argument("--compare", default=None,
                    help="comma list of extra weight files evaluated on the held-out fields "
                         "(\"init\": the untrained initialisation)")
    ap.add_argument("--probes", type=int, default=8, help="probe vectors per system visit")
    ap.add_argument("--mode", choices=("correction", "factor"), default="factor",
                    help="per-iteration residual correction, or factored preconditioner")
    ap.add_argument("--out", default=None)
    ap.add_argument("--weights", default=None, help="skip collection and training, evaluate these")
    ap.add_argument("--report", default=None)
    ap.add_argument("--calibrate", default=None,
                    help="comma list of shifts of the factored head's output bias b_o; the one with "
                         "the fewest CG iterations is applied before saving")
    ap.add_argument("--calib-seeds", default=None,
                    help="fields for the calibration (default: the first two training seeds)")
    ap.add_argument("--snaps", default=None,
                    help="CG iterations whose errors are collected (comma list; default: every "
                         "stage, late ones only for the optimal-step loss)")
    a = ap.parse_args(argv)
    global KIND
    KIND = a.kind
    if a.loss is None:
        a.loss = "frobenius" if a.mode == "factor" else "energy"
    if a.loss in ("frobenius", "optstep", "cg") and a.mode != "factor":
        ap.error("the %s loss belongs to the factored preconditioner" % a.loss)
    snaps = ([int(x) for x in a.snaps.split(",")] if a.snaps else
             (SNAPS_LATE if a.loss == "optstep" else SNAPS))
    import torch

    from . import Solver
    coordV, V0T, kind = square_mesh(a.n, seed=a.jitter)
    torch.cuda.set_device(0)
    sv = Solver(coordV, V0T, kind, a.p, rtol=1e-8, max_iters=20000)
    sv.gnn_set_mode(a.mode)
    init = factor_init if a.mode == "factor" else glorot

    def learned_solver():
        s_ = Solver(coordV, V0T, kind, a.p, rtol=1e-8, max_iters=20000, precond=1)
        s_.gnn_set_mode(a.mode)
        return s_

    if a.weights:
        w = np.load(a.weights).astype(np.float32)
        data, losses, t_collect, t_train = [], [], 0.0, 0.0
    else:
        # round 0 learns from block-Jacobi CG solves; later rounds add the
        # residuals that flexible CG with the current network produces
        w = init(sv.N, a.init_seed)
        data, losses, t_collect, t_train = [], [], 0.0, 0.0
        sl = None
        if a.loss == "cg" and a.start_weights:
            w = (init(sv.N, a.init_seed) if a.start_weights == "init" else
                 np.load(a.start_weights).astype(np.float32))
        elif a.loss in ("frobenius", "cg"):
            t0 = time.perf_counter()
            data = systems(sv, a.n, seeds_arg(a.train_seeds), a.sigma, a.steps, a.dt)
            t_collect = time.perf_counter() - t0
            sv.gnn_set_params(w)
            sv.gnn_set_loss("frobenius")
            t0 = time.perf_counter()
            losses = train_probes(sv, data, a.epochs, a.probes, a.lr, a.dt, a.init_seed)
            t_train = time.perf_counter() - t0
            w = sv.gnn_get_params()
        for rd in range(a.rounds if a.loss not in ("frobenius", "cg") else 0):
            src = sv
            if rd > 0:
                if sl is None:
                    sl = learned_solver()
                sl.gnn_set_params(w)
                src = sl
            t0 = time.perf_counter()
            data += collect(src, a.n, seeds_arg(a.train_seeds), a.sigma, a.steps, a.dt, snaps=snaps)
            t_collect += time.perf_counter() - t0
            sv.gnn_set_params(w)
            sv.gnn_set_loss(a.loss)
            t0 = time.perf_counter()
            losses += train(sv, data, a.epochs, a.lr, a.dt, a.init_seed + rd)
            t_train += time.perf_counter() - t0
            w = sv.gnn_get_params()
        del sl
    n_samples = len(data)
    del data[:]
    cg_fit = None
    if a.loss == "cg" and not a.weights:
        scg = Solver(coordV, V0T, kind, a.p, rtol=1e-14, max_iters=a.cg_iters, precond=1)
        scg.gnn_set_mode("factor")
        cseeds = seeds_arg(a.cg_seeds) if a.cg_seeds else seeds_arg(a.train_seeds)[:6]
        cases = cg_cases(scg, a.n, cseeds, a.sigma, a.dt)
        t0 = time.perf_counter()
        w, best, hist = train_head_cg(scg, w, cases, a.dt,
                                      [float(x) for x in a.cg_omegas.split(",")], a.spsa_iters,
                                      a.spsa_c, a.spsa_a, a.init_seed,
                                      from_start=a.spsa_from == "start")
        cg_fit = {"objective": best, "seconds": time.perf_counter() - t0, "seeds": cseeds,
                  "cg_iters": a.cg_iters, **hist}
        t_train += cg_fit["seconds"]
        del cases, scg
    calib = None
    if a.calibrate:
        if a.mode != "factor":
            ap.error("--calibrate shifts the factored network's output bias")
        from .ldg import LDG_MIXED_BF16
        sc = Solver(coordV, V0T, kind, a.p, rtol=1e-8, max_iters=20000, precision=LDG_MIXED_BF16,
                    inner_rtol=1e-2, precond=1)
        sc.gnn_set_mode("factor")
        cseeds = seeds_arg(a.calib_seeds) if a.calib_seeds else seeds_arg(a.train_seeds)[:2]
        w, calib = calibrate(sc, w, [float(x) for x in a.calibrate.split(",")], a.n, cseeds,
                             a.sigma, a.dt)
        del sc
    if a.out:
        np.save(a.out, w)
    # the training loss on held-out systems (one step per evaluation field)
    sv.gnn_set_params(w)
    sv.gnn_set_loss("frobenius" if a.loss == "cg" else a.loss)
    hl = []
    if a.loss in ("frobenius", "cg"):
        rng = np.random.default_rng(a.init_seed + 1000)
        for D in systems(sv, a.n, seeds_arg(a.eval_seeds), a.sigma, 1, a.dt):
            sv.gnn_set_context(D, a.dt)
            for _ in range(4):
                pw = rng.standard_normal((sv.K, sv.N)).astype(np.float32)
                hl.append(sv.gnn_loss_grad(pw, pw)[0])
    else:
        held = collect(sv, a.n, seeds_arg(a.eval_seeds), a.sigma, 1, a.dt, snaps=snaps)
        for r, tg, D in held:
            sv.gnn_set_context(D, a.dt)
            hl.append(sv.gnn_loss_grad(r, tg)[0])
        del held[:]
    ev = evaluate(sv, a.n, seeds_arg(a.eval_seeds), a.sigma, a.eval_steps, a.dt, False)
    sg = learned_solver()
    sg.gnn_set_params(w)
    eg = evaluate(sg, a.n, seeds_arg(a.eval_seeds), a.sigma, a.eval_steps, a.dt, True)
    extra = {}
    if a.compare:
        for f in a.compare.split(","):
            wc = init(sv.N, a.init_seed) if f == "init" else np.load(f).astype(np.float32)
            sg.gnn_set_params(wc)
            extra[f] = evaluate(sg, a.n, seeds_arg(a.eval_seeds), a.sigma, a.eval_steps, a.dt, True)
    if cg_fit is not None:
        # the best constant omega of the fit, on the held-out fields
        sg.gnn_set_params(with_head(w, constant_head(cg_fit["best_constant"][0])))
        extra["constant omega %.2f" % cg_fit["best_constant"][0]] = evaluate(
            sg, a.n, seeds_arg(a.eval_seeds), a.sigma, a.eval_steps, a.dt, True)
    rep = {"p": a.p, "n": a.n, "kind": a.kind, "sigma": a.sigma, "dt": a.dt, "K": sv.K, "samples": n_samples, "collect_s": t_collect, "train_s": t_train,
           "epochs": a.epochs, "rounds": a.rounds, "mode": a.mode, "loss": a.loss, "probes": a.probes, "loss_per_epoch": losses,
           "heldout_loss": float(np.mean(hl)), "block_jacobi": ev, "learned": eg,
           "iteration_ratio": eg["iters_per_step"] / ev["iters_per_step"],
           "time_ratio": eg["s_per_step"] / ev["s_per_step"], "calibration": calib,
           "cg_fit": cg_fit, "compare": extra}
    print(json.dumps(rep), flush=True)
    if a.report:
        with open(a.report, "w") as fh:
            json.dump(rep, fh, indent=1)
    return rep


if __name__ == "__main__":
    main()
