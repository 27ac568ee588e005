"""The factored learned preconditioner on the GPU against the FP64 oracle.

The factor blocks (W_k and the scaled neighbour blocks O_kn, stored in FP32),
log ||O_kn||, the network's omega, and the energy loss with its gradient
match oracle/gnn_factor.py; steps with the preconditioner reach the FP64
tolerance and the oracle's solution in fewer CG iterations than
block-Jacobi; non-finite weights and nonsymmetric steps fall back.
"""
import numpy as np
import pytest

from inputs.fields import LOGNORMAL, SMOOTH1, Workload, lognormal_blocks, triangle_values
from inputs.meshes import NORTH, square_mesh
from oracle import gnn, gnn_factor as gf
from oracle.ldg import Blocks, Problem, schur_matrix
from oracle.mesh import Grid
from oracle.refelem import RefTensors
from tests.gpu_common import rel_l2, to_np

pytestmark = pytest.mark.gpu


def _setup(n, p, seed, ratio=6.5, storage="f32"):
    from paper_1408_3877_amd import Solver
    cV, V0T, kind = square_mesh(n, seed=seed, neumann_sides=(NORTH,))
    g = Grid(cV, V0T, kind)
    refs = RefTensors(p)
    blk = max(1, n // 4)
    dT = triangle_values(lognormal_blocks(n, seed + 1, 1.5, block=blk), n, block=blk)
    D = np.zeros((g.numT, refs.N))
    D[:, 0] = dT / np.sqrt(2.0)
    dt = ratio / n ** 2
    sy = gf.System(g, schur_matrix(Blocks(g, refs, D), g, refs, 1.0, dt))
    s = Solver(cV, V0T, kind, p)
    s.gnn_set_mode("factor")
    s.gnn_factor_storage(storage)
    return g, D, dt, sy, s


def _theta(N, seed):
    rng = np.random.default_rng(seed)
    return (gf.init_params(N, seed) + 0.05 * rng.standard_normal(gf.n_params(N))).astype(np.float32)


@pytest.mark.parametrize("n,p,seed", [(8, 2, 701), (5, 4, 702), (6, 1, 703)])
def test_factor_blocks_and_omega_match_the_oracle(n, p, seed):
    g, D, dt, sy, s = _setup(n, p, seed)
    N = sy.N
    print("[factor] blocks n=%d p=%d K=%d" % (n, p, sy.K), flush=True)
    assert s.gnn_num_params() == gf.n_params(N)
    th = _theta(N, seed)
    s.gnn_set_params(th)
    s.gnn_set_context(D, dt)
    blk, ln = (to_np(x) for x in s.gnn_factor_export())
    assert np.abs(blk[:, 0] - sy.Wk).max() <= 1e-6 * np.abs(sy.Wk).max()
    m = sy.mask
    Og = blk[:, 1:][m]
    assert np.abs(Og - sy.O[m]).max() <= 2e-6 * np.abs(sy.O).max()
    assert np.abs(ln[m] - sy.lognorm[m]).max() <= 1e-5
    node, edge = gnn.features(g, D, dt, 1.0)
    want = gf.omega(th.astype(np.float64), g, node, edge, sy)
    got = to_np(s.gnn_factor_omega())
    assert np.abs(got - want).max() <= 1e-5
    assert np.all(got[~m] == 0.0)


def test_factor_bf16_storage_rounds_the_fp32_blocks():
    g, D, dt, sy, s = _setup(8, 3, 705, storage="bf16")
    s.gnn_set_params(_theta(sy.N, 705))
    s.gnn_set_context(D, dt)
    blk = to_np(s.gnn_factor_export()[0])
    m = sy.mask
    # BF16 carries 8 bits of precision (7 stored): round to nearest (FP64 -> FP32
    # -> BF16) has relative error <= 2^-8 (1 + 2^-16) per entry, plus the FP64
    # difference of the two computations for entries that vanish up to rounding
    for got, want in ((blk[:, 0], sy.Wk), (blk[:, 1:][m], sy.O[m])):
        bound = 2.0 ** -8 * (1 + 2.0 ** -16) * np.abs(want) + 1e-12 * np.abs(want).max()
        assert np.all(np.abs(got - want) <= bound), np.max(np.abs(got - want) / bound)


def test_factor_fp8_storage_rounds_the_blocks():
    g, D, dt, sy, s = _setup(8, 3, 706, storage="fp8")
    s.gnn_set_params(_theta(sy.N, 706))
    s.gnn_set_context(D, dt)
    blk = to_np(s.gnn_factor_export()[0])
    m = sy.mask
    Wk, O = sy.Wk, sy.O[m]
    bw = 2.0 ** -8 * (1 + 2.0 ** -16) * np.abs(Wk) + 1e-12 * np.abs(Wk).max()
    assert np.all(np.abs(blk[:, 0] - Wk) <= bw)
    # E4M3: 4 bits of precision for normal values (>= 2^-6), subnormal spacing 2^-9
    assert np.abs(O).max() <= 1.0 + 1e-12
    bo = np.maximum(2.0 ** -4 * (1 + 2.0 ** -20) * np.abs(O), 2.0 ** -10) + 1e-12
    got = blk[:, 1:][m]
    assert np.all(np.abs(got - O) <= bo), np.max(np.abs(got - O) / bo)


def test_factor_fp8w_storage_rounds_the_scaled_blocks():
    g, D, dt, sy, s = _setup(8, 4, 707, storage="fp8w")
    s.gnn_set_params(_theta(sy.N, 707))
    s.gnn_set_context(D, dt)
    blk = to_np(s.gnn_factor_export()[0])
    m = sy.mask
    Wk, O = sy.Wk, sy.O[m]
    # W_k = s_k W8_k, s_k = 2^round(log2(max |W_k| / 256)): E4M3 keeps 4 bits for
    # |W8| >= 2^-6 and spacing 2^-9 below, i.e. |error| <= max(2^-4 |W|, 2^-10 s_k);
    # s_k is taken one binade up to cover a rounding tie of the exponent
    sk = 2.0 ** (np.round(np.log2(np.abs(Wk).max(axis=(1, 2)) / 256.0)) + 1)
    bw = np.maximum(2.0 ** -4 * (1 + 2.0 ** -20) * np.abs(Wk), 2.0 ** -10 * sk[:, None, None]) + 1e-300
    assert np.all(np.abs(blk[:, 0] - Wk) <= bw), np.max(np.abs(blk[:, 0] - Wk) / bw)
    # the largest entry of each block is within 2^-4 of itself (normal range)
    big = np.abs(Wk).reshape(len(Wk), -1).argmax(axis=1)
    wb = Wk.reshape(len(Wk), -1)[np.arange(len(Wk)), big]
    gb = blk[:, 0].reshape(len(Wk), -1)[np.arange(len(Wk)), big]
    assert np.all(np.abs(gb - wb) <= 2.0 ** -4 * np.abs(wb))
    bo = np.maximum(2.0 ** -4 * (1 + 2.0 ** -20) * np.abs(O), 2.0 ** -10) + 1e-12
    assert np.all(np.abs(blk[:, 1:][m] - O) <= bo)


@pytest.mark.parametrize("n,p,seed", [(7, 2, 711), (4, 3, 712)])
def test_factor_energy_loss_and_gradient(n, p, seed):
    g, D, dt, sy, s = _setup(n, p, seed)
    N = sy.N
    th = _theta(N, seed)
    s.gnn_set_params(th)
    s.gnn_set_context(D, dt)
    rng = np.random.default_rng(seed)
    rhat = rng.standard_normal((sy.K, N)).astype(np.float32)
    tgt = rng.standard_normal((sy.K, N)).astype(np.float32)
    node, edge = gnn.features(g, D, dt, 1.0)
    L, G = gf.energy_loss_grad(th.astype(np.float64), g, node, edge, sy, rhat.astype(np.float64),
                               tgt.astype(np.float64))
    Lg, Gg = s.gnn_loss_grad(rhat, tgt)
    Gg = to_np(Gg)
    print("[factor] loss gpu %.8f oracle %.8f" % (Lg, L), flush=True)
    assert abs(Lg - L) <= 1e-4 * L
    assert np.linalg.norm(Gg - G) <= 2e-3 * np.linalg.norm(G)


@pytest.mark.parametrize("n,p,seed", [(7, 2, 751), (5, 4, 752)])
def test_factor_optstep_loss_and_gradient(n, p, seed):
    g, D, dt, sy, s = _setup(n, p, seed)
    N = sy.N
    th = _theta(N, seed)
    s.gnn_set_params(th)
    s.gnn_set_loss("optstep")
    s.gnn_set_context(D, dt)
    rng = np.random.default_rng(seed)
    rhat = rng.standard_normal((sy.K, N)).astype(np.float32)
    tgt = rng.standard_normal((sy.K, N)).astype(np.float32)
    node, edge = gnn.features(g, D, dt, 1.0)
    L, G = gf.optstep_loss_grad(th.astype(np.float64), g, node, edge, sy, rhat.astype(np.float64),
                                tgt.astype(np.float64))
    Lg, Gg = s.gnn_loss_grad(rhat, tgt)
    Gg = to_np(Gg)
    print("[factor] optstep gpu %.8f oracle %.8f" % (Lg, L), flush=True)
    assert abs(Lg - L) <= 1e-4 * L
    assert np.linalg.norm(Gg - G) <= 2e-3 * np.linalg.norm(G)


@pytest.mark.parametrize("n,p,seed", [(7, 2, 741), (4, 4, 742)])
def test_factor_frobenius_loss_and_gradient(n, p, seed):
    g, D, dt, sy, s = _setup(n, p, seed)
    N = sy.N
    th = _theta(N, seed)
    s.gnn_set_params(th)
    s.gnn_set_loss("frobenius")
    s.gnn_set_context(D, dt)
    rng = np.random.default_rng(seed)
    w = rng.standard_normal((sy.K, N)).astype(np.float32)
    node, edge = gnn.features(g, D, dt, 1.0)
    L, G = gf.frobenius_loss_grad(th.astype(np.float64), g, node, edge, sy, w.astype(np.float64))
    Lg, Gg = s.gnn_loss_grad(w, w)
    Gg = to_np(Gg)
    print("[factor] frobenius gpu %.8f oracle %.8f" % (Lg, L), flush=True)
    assert abs(Lg - L) <= 1e-4 * L
    assert np.linalg.norm(Gg - G) <= 2e-3 * np.linalg.norm(G)


def _steps(s, w, pr, C, dt, nsteps):
    t, out = 0.0, []
    for _ in range(nsteps):
        t += dt
        smp = s.sample_workload(w.kind, t, dT=w.dT)
        info = s.step_sampled(dt, smp["d"], smp["f"], smp["cD"], smp["gN"])
        C, _, _, _ = pr.step(C, t, dt, w)
        out.append((info, rel_l2(pr.grid.areaT, to_np(s.get_solution()[0]), C)))
    return out


@pytest.mark.parametrize("weights", ["init", "nan", "init-bf16", "init-fp8", "init-fp8w"])
def test_factor_preconditioner_steps(weights):
    from paper_1408_3877_amd import Solver
    n, p, dt = 12, 2, 0.02
    cV, V0T, kind = square_mesh(n, seed=721)
    w = Workload(LOGNORMAL, n_cells=n, blocks=lognormal_blocks(n, 722, 1.5, block=3), block=3)
    pr = Problem(cV, V0T, kind, p)
    runs = {}
    for name, pc in (("bj", 0), ("learned", 1)):
        s = Solver(cV, V0T, kind, p, rtol=1e-13, max_iters=20000, precond=pc)
        if pc:
            s.gnn_set_mode("factor")
            s.gnn_factor_storage(weights.split("-")[1] if "-" in weights else "f32")
            th = _theta(s.N, 723)
            if weights == "nan":
                th = np.full_like(th, np.nan)
            s.gnn_set_params(th)
        s.set_initial_samples(s.sample_workload(LOGNORMAL, 0.0, dT=w.dT, want=("c0",))["c0"])
        runs[name] = _steps(s, w, pr, pr.initial(w), dt, 2)
        for info, err in runs[name]:
            print("[factor-steps] %s %s %s err=%.2e" % (weights, name, info, err), flush=True)
            assert info["rel_residual"] <= 1e-13 and info["krylov"] == 2
            assert err < 1e-10
    for (ib, _), (il, _) in zip(runs["bj"], runs["learned"]):
        if weights.startswith("init"):
            assert il["fallbacks"] == 0 and il["learned_iters"] == il["iters"]
            assert il["iters"] < ib["iters"]
        else:
            assert il["fallbacks"] == 1 and il["fallback_reason"] == 1
            assert il["learned_iters"] == 0


@pytest.mark.parametrize("storage,precision", [("f32", 0), ("fp8", 0), ("fp8", 2)])
def test_factor_nonsymmetric_steps_use_the_symmetric_part(storage, precision):
    # d varies inside the triangles, so the steps are nonsymmetric and run
    # GMRES; the factored preconditioner is built from the operator's symmetric
    # part (W_k from the symmetric part of BJ_k^{-1}, O_kn from (S_kj + S_jk^T)/2)
    # and applied as a fixed right preconditioner.  Blocks against the oracle's
    # symmetric-part construction; steps against the oracle's direct solve, in
    # fewer iterations than block-Jacobi GMRES
    from paper_1408_3877_amd import Solver
    n, p, dt = 8, 3, 0.01
    cV, V0T, kind = square_mesh(n, seed=741, neumann_sides=(NORTH,))
    w = Workload(SMOOTH1)
    pr = Problem(cV, V0T, kind, p)
    th = _theta(pr.N, 741)
    runs = {}
    for name, pc in (("bj", 0), ("learned", 1)):
        s = Solver(cV, V0T, kind, p, rtol=1e-12, max_iters=20000, precond=pc, precision=precision,
                   restart=30)
        if pc:
            s.gnn_set_mode("factor")
            s.gnn_factor_storage(storage)
            s.gnn_set_params(th)
        s.set_initial_samples(s.sample_workload(SMOOTH1, 0.0, want=("c0",))["c0"])
        runs[name] = _steps(s, w, pr, pr.initial(w), dt, 2)
        for info, err in runs[name]:
            print("[factor-gmres] %s %s %d %s err=%.2e" % (storage, name, precision, info, err),
                  flush=True)
            assert info["krylov"] == 1 and info["rel_residual"] <= 1e-12
            assert err < 1e-9
        if pc and storage == "f32" and precision == 0:
            # the blocks of the last step (t = 2 dt) against the oracle
            D = pr.data(w, 2 * dt)["D"]
            refs = RefTensors(p)
            sy = gf.System(pr.grid, schur_matrix(Blocks(pr.grid, refs, D), pr.grid, refs, 1.0, dt),
                           symmetric_part=True)
            blk = to_np(s.gnn_factor_export()[0])
            m = sy.mask
            assert np.abs(blk[:, 0] - sy.Wk).max() <= 1e-6 * np.abs(sy.Wk).max()
            assert np.abs(blk[:, 1:][m] - sy.O[m]).max() <= 2e-6 * np.abs(sy.O).max()
    for (ib, _), (il, _) in zip(runs["bj"], runs["learned"]):
        assert il["fallbacks"] == 0 and il["learned_iters"] == il["iters"] > 0
        assert ib["learned_iters"] == 0
        assert il["iters"] < ib["iters"], (il["iters"], ib["iters"])


def test_factor_blocks_at_degree_three_vertices():
    # The neighbour blocks S_kj of the eliminated operator gain a path through a
    # third triangle l adjacent to both k and j: B_kl M_l^{-1} A_lj.  On a mesh
    # that exists only around interior vertices of degree three, and the
    # factor kernel leaves it out.  Here such vertices are made by splitting
    # triangles at their centroids: away from them O_kn matches the oracle's
    # W_k S_kj W_j^T to FP32 rounding; on the edges that meet them it deviates
    # by the left-out path (measured and bounded below), and the preconditioner
    # stays exactly SPD, so steps still reach the oracle's solution.
    from inputs.meshes import edge_kinds, split_at_centroids
    from paper_1408_3877_amd import Solver
    n, p = 6, 3
    cV0, V00, _ = square_mesh(n, seed=731)
    rng = np.random.default_rng(731)
    interior = [k for k in range(V00.shape[0])
                if np.all((cV0[V00[k]] > 1e-9) & (cV0[V00[k]] < 1 - 1e-9))]
    cV, V0T = split_at_centroids(cV0, V00, rng.choice(interior, 8, replace=False))
    kind = edge_kinds(cV, V0T, (NORTH,))
    g = Grid(cV, V0T, kind)
    refs = RefTensors(p)
    dT = 10.0 ** rng.uniform(-1.0, 1.0, g.numT)
    D = np.zeros((g.numT, refs.N))
    D[:, 0] = dT / np.sqrt(2.0)
    dt = 6.5 / n ** 2
    sy = gf.System(g, schur_matrix(Blocks(g, refs, D), g, refs, 1.0, dt))
    s = Solver(cV, V0T, kind, p)
    s.gnn_set_mode("factor")
    s.gnn_factor_storage("f32")
    s.gnn_set_params(_theta(sy.N, 731))
    s.gnn_set_context(D, dt)
    blk = to_np(s.gnn_factor_export()[0])
    assert np.abs(blk[:, 0] - sy.Wk).max() <= 1e-6 * np.abs(sy.Wk).max()
    # edges (k, n) whose two triangles have a common neighbour
    nb = [set(int(j) for j in g.kp[k] if j >= 0) for k in range(g.numT)]
    third = np.zeros((g.numT, 3), dtype=bool)
    for k in range(g.numT):
        for e in range(3):
            j = g.kp[k, e]
            third[k, e] = j >= 0 and len(nb[k] & nb[int(j)]) > 0
    m = sy.mask
    assert third.sum() >= 8 * 6
    plain = m & ~third
    assert np.abs(blk[:, 1:][plain] - sy.O[plain]).max() <= 2e-6 * np.abs(sy.O).max()
    dev = (np.linalg.norm(blk[:, 1:][third] - sy.O[third], axis=(1, 2)) /
           np.linalg.norm(sy.O[third], axis=(1, 2)))
    print("[factor-degree-3] %d edges: relative Frobenius deviation of O_kn max %.3f median %.3f"
          % (third.sum(), dev.max(), np.median(dev)), flush=True)
    assert 1e-6 < dev.max() < 1.0
    # steps with the learned preconditioner on this mesh match the oracle (d
    # constant on every triangle, so the steps are SPD and run learned CG)
    smooth = Workload(SMOOTH1)

    class TriangleD(Workload):
        # d constant per triangle (oracle point arrays are [K x R]); the
        # forcing and boundary data are those of the smooth workload
        def d(self, t, x, y):
            return np.broadcast_to(dT[:, None], np.shape(x)) + 0.0 * t

        def f(self, t, x, y):
            return smooth.f(t, x, y)

    w = TriangleD(SMOOTH1)
    pr = Problem(cV, V0T, kind, p)
    sl = Solver(cV, V0T, kind, p, rtol=1e-13, max_iters=20000, precond=1)
    sl.gnn_set_mode("factor")
    sl.gnn_set_params(_theta(sy.N, 731))
    C = pr.initial(w)
    sl.set_state(C, 0.0)
    x, y = (to_np(v) for v in sl.quad_points(0))
    xb, yb = (to_np(v) for v in sl.quad_points(1))
    n1, n2 = (to_np(v) for v in sl.quad_points(2))
    dv = np.tile(dT, len(x) // g.numT)
    t = 0.0
    for _ in range(2):
        t += 0.01
        info = sl.step_sampled(0.01, dv, w.f(t, x, y), w.c_D(t, xb, yb), w.g_N(t, xb, yb, n1, n2))
        C, Z1, Z2, _ = pr.step(C, t, 0.01, w)
        assert info["rel_residual"] <= 1e-13 and info["krylov"] == 2
        assert info["learned_iters"] == info["iters"] > 0 and info["fallbacks"] == 0
        assert rel_l2(pr.grid.areaT, to_np(sl.get_solution()[0]), C) < 1e-10


@pytest.mark.parametrize("p,precision", [(3, 0), (4, 2)])
def test_shipped_weights_on_a_delaunay_mesh(p, precision):
    # An unstructured mesh with its local numbering rotated at random has every
    # local edge pair (n, n+), including n = n+,
    # which the training meshes lack: the shipped networks keep the initial
    # weights on those features, give omega inside (0, 0.95) on every interior
    # edge, and their preconditioner (of the symmetric part: d varies inside the
    # triangles) takes GMRES steps to the oracle's solution in fewer iterations
    # than block-Jacobi
    import os

    from inputs.meshes import SOUTH, delaunay_square, edge_kinds, rotate_local_numbering
    from paper_1408_3877_amd import Solver
    cV, V0T = delaunay_square(10, 761)
    V0T, kind = rotate_local_numbering(V0T, edge_kinds(cV, V0T, (SOUTH,)), 762)
    pr = Problem(cV, V0T, kind, p)
    kp = pr.grid.kp
    pairs = set()
    for k in range(pr.grid.numT):
        for n in range(3):
            j = kp[k, n]
            if j >= 0:
                pairs.add((n, int(np.flatnonzero(kp[j] == k)[0])))
    assert {(0, 0), (1, 1), (2, 2)} <= pairs
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    th = np.load(os.path.join(root, "paper_1408_3877_amd", "weights", "factor_p%d.npy" % p))
    w = Workload(SMOOTH1)
    dt = 0.01
    runs = {}
    for name, pc in (("bj", 0), ("learned", 1)):
        s = Solver(cV, V0T, kind, p, rtol=1e-12, max_iters=20000, precond=pc, precision=precision,
                   restart=30)
        if pc:
            s.gnn_set_mode("factor")
            s.gnn_factor_storage("fp8")
            s.gnn_set_params(th)
        s.set_initial_samples(s.sample_workload(SMOOTH1, 0.0, want=("c0",))["c0"])
        runs[name] = _steps(s, w, pr, pr.initial(w), dt, 2)
        for info, err in runs[name]:
            print("[delaunay-learned] p=%d %s %s err=%.2e" % (p, name, info, err), flush=True)
            assert info["krylov"] == 1 and info["rel_residual"] <= 1e-12
            assert err < 1e-9
        if pc:
            om = to_np(s.gnn_factor_omega())
            inner = kp >= 0
            assert np.all(om[inner] > 0.0) and np.all(om[inner] < 0.95)
    for (ib, _), (il, _) in zip(runs["bj"], runs["learned"]):
        assert il["fallbacks"] == 0 and il["learned_iters"] == il["iters"] > 0
        assert il["iters"] < ib["iters"], (il["iters"], ib["iters"])
