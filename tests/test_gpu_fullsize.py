"""Parity at the full benchmark sizes, on sampled outputs.

For each large workload the GPU runs in the launch configuration bench.py
times (same mesh, order, solver options).  The oracle cannot solve systems
of this size, so it recomputes sampled triangles one by one from the same
seeded inputs: projections, stored blocks, rows of the eliminated operator,
block-Jacobi inverses, and, for a full-size implicit Euler step computed on
the GPU, the rows of the full system's residual and of the Z recovery.
Sampled triangles are at least three edges apart, so a unit vector on all
of them at once exposes each one's diagonal block of the operator.
"""
import numpy as np
import pytest

from bench import CONFIGS
from inputs.fields import LOGNORMAL, LOGNORMAL_T, Workload, lognormal_blocks
from inputs.meshes import square_mesh
from oracle import gnn, gnn_factor as gf
from oracle.ldg import Blocks, boundary_vectors, project, schur_apply_rows
from oracle.mesh import Grid
from oracle.refelem import RefTensors
from tests.gpu_common import to_np

pytestmark = pytest.mark.gpu


def _sample(grid, rng, n=40):
    """Triangles pairwise >= 3 edges apart, including the first and last."""
    K = grid.numT
    cand = np.concatenate([[0, K - 1], rng.choice(K, 4 * n, replace=False)])
    banned = np.zeros(K, dtype=bool)
    out = []
    for k in cand:
        if banned[k]:
            continue
        out.append(k)
        ring = {int(k)}
        for _ in range(4):
            nb = grid.kp[list(ring)].reshape(-1)
            ring |= set(int(x) for x in nb[nb >= 0])
        banned[list(ring)] = True
        if len(out) >= n:
            break
    return np.sort(np.array(out))


def _workload(cfg):
    if cfg["kind"] in (LOGNORMAL, LOGNORMAL_T):
        blk = lognormal_blocks(cfg["n"], cfg["field_seed"], cfg["sigma"], block=8)
        return Workload(cfg["kind"], n_cells=cfg["n"], blocks=blk, block=8)
    return Workload(cfg["kind"])


@pytest.mark.parametrize("name,precision", [
    ("combined-p4-1024", 0),
    ("combined-p4-1024", 2),
    ("mixed-p4-512", 1),
    ("mixed-p4-512", 2),
    ("learned-p3-256", 0),
])
def test_fullsize_sampled(name, precision):
    import torch

    from paper_1408_3877_amd import Solver
    assert torch.cuda.is_available()
    cfg = CONFIGS[name]
    p, dt, eta = cfg["p"], cfg["dt"], 1.0
    coordV, V0T, kind = square_mesh(cfg["n"], seed=cfg["jitter"])
    w = _workload(cfg)
    grid = Grid(coordV, V0T, kind)
    refs = RefTensors(p)
    K, N = grid.numT, refs.N
    rng = np.random.default_rng(4242)
    el = _sample(grid, rng)
    print("[fullsize] %s precision=%d K=%d sampled=%d" % (name, precision, K, len(el)), flush=True)
    s = Solver(coordV, V0T, kind, p, rtol=1e-8, restart=30, max_iters=20000, precision=precision)
    dT = w.dT
    # (1) projection of d at t = dt on the sampled triangles
    smp = s.sample_workload(cfg["kind"], dt, dT=dT)
    Dg = to_np(s.project(smp["d"]))[el]
    Do = project(grid, p, lambda x, y: w.restrict(el).d(dt, x, y), refs.hatM, elems=el)
    assert np.abs(Dg - Do).max() <= 1e-13 * np.abs(Do).max()
    # (2) stored blocks from a seeded coefficient
    Dr = 1.0 + 0.3 * rng.standard_normal((K, N))
    s.assemble(Dr)
    blk = to_np(s.get_blocks_rows(el))
    b = Blocks(grid, refs, Dr, elems=el)
    for r, k in enumerate(el):
        sl = slice(r * N, (r + 1) * N)
        for m in range(2):
            want = (-b.G[m] + b.R[m] + b.RD[m])[sl, k * N:(k + 1) * N].toarray()
            assert np.abs(blk[r, m] - want).max() <= 1e-12 * max(np.abs(want).max(), 1e-30)
        for n in range(3):
            kp = grid.kp[k, n]
            if kp < 0:
                continue
            want = sum(grid.nuE0T[k, n, m] * (-b.G[m] + b.R[m] + b.RD[m])[sl, kp * N:(kp + 1) * N].toarray()
                       for m in range(2))
            assert np.abs(blk[r, 2 + n] - want).max() <= 1e-12 * np.abs(want).max()
    # (3) rows of the eliminated operator for a seeded vector
    Cr = rng.standard_normal((K, N))
    yg = to_np(s.apply_schur(dt, Cr))[el]
    yo, _ = schur_apply_rows(grid, refs, Dr, Cr, dt, eta, el)
    assert np.abs(yg - yo).max() <= 1e-12 * np.abs(yo).max()
    # (4) block-Jacobi inverses: columns of the diagonal blocks via unit vectors
    s.bj_setup(dt)
    bjg = to_np(s.get_bj_rows(el))
    cols = []
    for j in range(N):
        E = np.zeros((K, N))
        E[el, j] = 1.0
        cols.append(schur_apply_rows(grid, refs, Dr, E, dt, eta, el)[0])
    diag = np.stack(cols, axis=-1)                       # [len(el)][i][j]
    inv = np.linalg.inv(diag)
    assert np.abs(bjg - inv).max() <= 1e-9 * np.abs(inv).max()
    # (5) one full-size implicit Euler step on the GPU; residual rows by the oracle
    _step_residual_rows(s, cfg, w, grid, refs, el, dt, eta)


def _step_residual_rows(s, cfg, w, grid, refs, el, dt, eta):
    """One implicit Euler step on the GPU from the projected initial state; the
    oracle recomputes the full system's residual rows and Z on the sample."""
    p = cfg["p"]
    dT = w.dT
    c0 = s.sample_workload(cfg["kind"], 0.0, dT=dT, want=("c0",))["c0"]
    s.set_initial_samples(c0, 0.0)
    C0g = to_np(s.get_solution()[0])
    smp = s.sample_workload(cfg["kind"], dt, dT=dT)
    info = s.step_sampled(dt, smp["d"], smp["f"], smp["cD"], smp["gN"])
    print("[fullsize] step: %s" % info, flush=True)
    assert info["rel_residual"] <= 1e-8
    C1, Z1, Z2 = (to_np(x) for x in s.get_solution())
    # oracle data at t = dt: all triangles (for ||b||), neighbours of the sample for the rows
    C0 = project(grid, p, lambda x, y: w.c0(x, y), refs.hatM)
    assert np.abs(C0g[el] - C0[el]).max() <= 1e-13 * np.abs(C0).max()
    F = project(grid, p, lambda x, y: w.f(dt, x, y), refs.hatM)
    D = project(grid, p, lambda x, y: w.d(dt, x, y), refs.hatM)
    J1, J2, KD, KN = boundary_vectors(grid, p, lambda x, y: w.c_D(dt, x, y),
                                      lambda x, y, a, bb: w.g_N(dt, x, y, a, bb), D)
    a2 = (2 * grid.areaT)[:, None]
    b3 = a2 * C0 + dt * (eta * KD - KN + a2 * F)
    bnorm = np.sqrt(np.sum(b3 ** 2) + dt ** 2 * (np.sum(J1 ** 2) + np.sum(J2 ** 2)))
    y, Zo = schur_apply_rows(grid, refs, D, C1, dt, eta, el, J=(J1, J2))
    # each sampled residual row against its own scale: the row of b3, or the
    # triangle-RMS of the whole right-hand side where that row is small.  A
    # stopping test ||r|| <= rtol ||b|| spread over K triangles leaves about
    # rtol * rms per row; 20 x that allows for an uneven spread, while a local
    # error of 1e-6 relative on a sampled triangle exceeds it.
    rms = bnorm / np.sqrt(grid.numT)
    scale = np.maximum(np.linalg.norm(b3[el], axis=1), rms)
    ratio = np.linalg.norm(b3[el] - y, axis=1) / (1e-8 * scale)
    print("[fullsize] residual rows / (rtol x own scale): max %.2f median %.2f"
          % (ratio.max(), np.median(ratio)), flush=True)
    assert ratio.max() <= 20.0, ratio.max()
    for m, Zg in enumerate((Z1, Z2)):
        assert np.abs(Zg[el] - Zo[m]).max() <= 1e-9 * np.abs(Zo[m]).max()


def test_fullsize_matrix_free_apply_and_step():
    # the matrix-free apply at the benchmark's size (combined workload, FP64):
    # every row against the stored-block apply, sampled rows against the oracle,
    # and a full-size step whose residual rows the oracle recomputes
    from paper_1408_3877_amd import Solver
    cfg = CONFIGS["combined-p4-1024"]
    p, dt, eta = cfg["p"], cfg["dt"], 1.0
    coordV, V0T, kind = square_mesh(cfg["n"], seed=cfg["jitter"])
    w = _workload(cfg)
    grid = Grid(coordV, V0T, kind)
    refs = RefTensors(p)
    K, N = grid.numT, refs.N
    rng = np.random.default_rng(4343)
    el = _sample(grid, rng)
    print("[fullsize-mf] K=%d sampled=%d" % (K, len(el)), flush=True)
    s = Solver(coordV, V0T, kind, p, rtol=1e-8, restart=30, max_iters=20000)
    Dr = 1.0 + 0.3 * rng.standard_normal((K, N))
    s.assemble(Dr)
    Cr = rng.standard_normal((K, N))
    ys = to_np(s.apply_schur(dt, Cr))
    s.set_matrix_free(True)
    ym = to_np(s.apply_schur(dt, Cr))
    a = grid.areaT[:, None]
    assert np.sqrt(np.sum(a * (ym - ys) ** 2) / np.sum(a * ys ** 2)) < 1e-13
    yo, _ = schur_apply_rows(grid, refs, Dr, Cr, dt, eta, el)
    assert np.abs(ym[el] - yo).max() <= 1e-12 * np.abs(yo).max()
    _step_residual_rows(s, cfg, w, grid, refs, el, dt, eta)


def test_fullsize_learned_factor_blocks_and_omega():
    """The combined workload in bench.py's launch configuration (BF16 inner solves,
    learned factored preconditioner with the trained weights, W in BF16 and O in
    FP8):
    one step, then the factor blocks and omega of sampled triangles against the
    oracle, which takes the blocks S_kk, S_kj, S_jj of the eliminated operator
    from row-restricted applies to unit vectors."""
    import os

    import torch

    from bench import WEIGHTS
    from paper_1408_3877_amd import Solver
    cfg = CONFIGS["combined-p4-1024"]
    p, dt, eta = cfg["p"], cfg["dt"], 1.0
    coordV, V0T, kind = square_mesh(cfg["n"], seed=cfg["jitter"])
    w = _workload(cfg)
    grid = Grid(coordV, V0T, kind)
    refs = RefTensors(p)
    K, N = grid.numT, refs.N
    el = _sample(grid, np.random.default_rng(4343), n=24)
    el = el[np.all(grid.kp[el] >= 0, axis=1)]           # interior triangles
    print("[fullsize-factor] K=%d sampled=%d" % (K, len(el)), flush=True)
    theta = np.load(WEIGHTS[p]).astype(np.float32)
    s = Solver(coordV, V0T, kind, p, rtol=1e-8, max_iters=20000, precision=2, precond=1)
    s.gnn_set_mode("factor")
    s.gnn_set_params(theta)
    c0 = s.sample_workload(cfg["kind"], 0.0, dT=w.dT, want=("c0",))["c0"]
    s.set_initial_samples(c0, 0.0)
    smp = s.sample_workload(cfg["kind"], dt, dT=w.dT)
    info = s.step_sampled(dt, smp["d"], smp["f"], smp["cD"], smp["gN"])
    print("[fullsize-factor] step: %s" % info, flush=True)
    assert info["rel_residual"] <= 1e-8 and info["fallbacks"] == 0
    assert info["learned_iters"] == info["iters"] > 0
    blk, ln = (to_np(x) for x in s.gnn_factor_export_rows(el))
    om = to_np(s.gnn_factor_omega())[el]
    # oracle blocks of S around the sample: unit vectors on the sample (self) or on
    # its n-th neighbours; the sample is >= 5 edges apart, so no two overlap
    D = project(grid, p, lambda x, y: w.d(dt, x, y), refs.hatM)
    nb = grid.kp[el]
    rows = np.unique(np.concatenate([el, nb.reshape(-1)]))
    pos = {int(k): i for i, k in enumerate(rows)}
    cols = {}
    for src in ["self", 0, 1, 2]:
        tgt = el if src == "self" else nb[:, src]
        out = np.zeros((len(rows), N, N))
        for c in range(N):
            E = np.zeros((K, N))
            E[tgt, c] = 1.0
            out[:, :, c] = schur_apply_rows(grid, refs, D, E, dt, eta, rows)[0]
        cols[src] = out
    inv = np.linalg.inv
    Wof = lambda Skk: np.linalg.cholesky(inv(0.5 * (Skk + Skk.T))).T
    node, edge = gnn.features(grid, D, dt, eta)
    P = gnn.unpack(theta.astype(np.float64), N, gf.param_shapes(N))
    h, _ = gnn.trunk_forward(P, grid, node, edge)
    worst = 0.0
    for r, k in enumerate(el):
        Wk = Wof(cols["self"][pos[int(k)]])
        bound = 2.0 ** -8 * (1 + 2.0 ** -16) * np.abs(Wk) + 1e-10 * np.abs(Wk).max()
        assert np.all(np.abs(blk[r, 0] - Wk) <= bound)
        for n in range(3):
            j = int(nb[r, n])
            Skj = cols[n][pos[int(k)]]
            Wj = Wof(cols[n][pos[j]])
            O = Wk @ Skj @ Wj.T
            # E4M3: relative 2^-4 for normal values, absolute 2^-10 below 2^-6
            bound = np.maximum(2.0 ** -4 * (1 + 2.0 ** -20) * np.abs(O), 2.0 ** -10) + 1e-9
            worst = max(worst, np.max(np.abs(blk[r, 1 + n] - O) / bound))
            lno = np.log(np.linalg.norm(O))
            assert abs(ln[r, n] - lno) <= 1e-5 * max(1.0, abs(lno))
            a = gf.head_preactivation(P, h[k], h[j], edge[k, n], lno)
            assert abs(om[r, n] - gf.OMEGA_MAX / (1.0 + np.exp(-a))) <= 1e-4
    print("[fullsize-factor] worst O error / FP8 bound = %.3f" % worst, flush=True)
    assert worst <= 1.0
