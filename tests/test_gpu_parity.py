"""Parity of the HIP path (through the C ABI) with the CPU FP64 oracle.

Inputs are seeded: meshes and fields from the `inputs` package, random
coefficient vectors from numpy generators; nothing the oracle consumes is
produced by the GPU.  Sizes span one partial tile (K < 64), several tiles
with a ragged tail, every order p = 0..4, all edge kinds.
"""
import numpy as np
import pytest

from inputs.fields import LOGNORMAL, LOGNORMAL_T, SMOOTH1, SMOOTH2, TABLE2
from inputs.meshes import EAST, NORTH, SOUTH, WEST, rotate_local_numbering, square_mesh
from oracle.ldg import Blocks, Problem, minv_blocks, schur_matrix, system, mass_W
from tests.gpu_common import rel_l2, to_np, workload

pytestmark = pytest.mark.gpu

CASES = [  # (n cells, jitter seed, Neumann sides, p)
    (5, 101, (SOUTH,), 0),
    (5, 102, (), 1),
    (9, 103, (SOUTH, NORTH), 2),
    (9, 104, (EAST,), 3),
    (5, 105, (WEST, NORTH), 4),
    (9, 106, (), 4),
]


@pytest.fixture(scope="module")
def torch_mod():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    return torch


def _solver(coordV, V0T, kind, p, **kw):
    from paper_1408_3877_amd import Solver
    return Solver(coordV, V0T, kind, p, **kw)


@pytest.mark.parametrize("n,seed,neu,p", CASES)
def test_projection_and_quad_points(torch_mod, n, seed, neu, p):
    cV, V0T, kind = square_mesh(n, seed=seed, neumann_sides=neu)
    pr = Problem(cV, V0T, kind, p)
    s = _solver(cV, V0T, kind, p)
    w = workload(SMOOTH2, n)
    t = 0.37
    smp = s.sample_workload(2, t)
    D = to_np(s.project(smp["d"]))
    F = to_np(s.project(smp["f"]))
    data = pr.data(w, t)
    assert rel_l2(pr.grid.areaT, D, data["D"]) < 1e-13
    assert rel_l2(pr.grid.areaT, F, data["F"]) < 1e-13
    x, y = s.quad_points(0)
    assert x.numel() == s.R * s.K


def _oracle_blocks(pr, D):
    """[K][5][N][N] oracle blocks: B^1_kk, B^2_kk, U_kn = sum_m nu^m_kn R^m_{k k+}."""
    b = Blocks(pr.grid, pr.refs, D)
    g, N = pr.grid, pr.N
    Bm = [(-b.G[m] + b.R[m] + b.RD[m]).tocsr() for m in range(2)]
    out = np.zeros((g.numT, 5, N, N))
    for k in range(g.numT):
        sl = slice(k * N, (k + 1) * N)
        for m in range(2):
            out[k, m] = Bm[m][sl, sl].toarray()
        for nn in range(3):
            kp = g.kp[k, nn]
            if kp >= 0:
                slp = slice(kp * N, (kp + 1) * N)
                out[k, 2 + nn] = sum(g.nuE0T[k, nn, m] * Bm[m][sl, slp].toarray() for m in range(2))
    return out


@pytest.mark.parametrize("precision,tol", [(1, 3e-6), (2, 3e-2)])
@pytest.mark.parametrize("n,seed,p,rotate", [(5, 501, 4, False), (9, 502, 3, True), (6, 503, 2, True)])
def test_blocks_low_precision_contraction(torch_mod, precision, tol, n, seed, p, rotate):
    # FP32 / BF16-operand MFMA contractions against the FP64 oracle blocks
    cV, V0T, kind = square_mesh(n, seed=seed, neumann_sides=(SOUTH,))
    if rotate:
        V0T, kind = rotate_local_numbering(V0T, kind, seed)
    pr = Problem(cV, V0T, kind, p)
    rng = np.random.default_rng(seed)
    D = 1.0 + 0.5 * rng.standard_normal((pr.grid.numT, pr.N))
    s = _solver(cV, V0T, kind, p, precision=precision)
    s.assemble(D)
    want = _oracle_blocks(pr, D)
    got = to_np(s.get_blocks_lowp())
    scale = np.abs(want).max()
    assert np.abs(got - want).max() <= tol * scale, (np.abs(got - want).max() / scale)
    assert np.abs(to_np(s.get_blocks()) - want).max() <= 1e-12 * scale


@pytest.mark.parametrize("n,seed,p", [(9, 511, 4), (7, 512, 1), (9, 513, 2)])
def test_rotated_local_numbering_steps(torch_mod, n, seed, p):
    # local edge numbers vary per triangle (mixed n+ inside a wave): blocks and steps
    cV, V0T, kind = square_mesh(n, seed=seed, neumann_sides=(NORTH,))
    V0T, kind = rotate_local_numbering(V0T, kind, seed)
    pr = Problem(cV, V0T, kind, p)
    rng = np.random.default_rng(seed)
    D = rng.standard_normal((pr.grid.numT, pr.N))
    s = _solver(cV, V0T, kind, p, rtol=1e-13, restart=40, max_iters=20000)
    s.assemble(D)
    want = _oracle_blocks(pr, D)
    assert np.abs(to_np(s.get_blocks()) - want).max() <= 1e-12 * np.abs(want).max()
    w = workload(TABLE2, n)
    smp0 = s.sample_workload(5, 0.0, want=("c0",))
    s.set_initial_samples(smp0["c0"], 0.0)
    C = pr.initial(w)
    smp = s.sample_workload(5, 0.03)
    info = s.step_sampled(0.03, smp["d"], smp["f"], smp["cD"], smp["gN"])
    C, Z1, Z2, _ = pr.step(C, 0.03, 0.03, w)
    assert rel_l2(pr.grid.areaT, to_np(s.get_solution()[0]), C) < 1e-10


@pytest.mark.parametrize("n,seed,neu,p", CASES)
def test_blocks(torch_mod, n, seed, neu, p):
    cV, V0T, kind = square_mesh(n, seed=seed, neumann_sides=neu)
    pr = Problem(cV, V0T, kind, p)
    rng = np.random.default_rng(seed)
    D = rng.standard_normal((pr.grid.numT, pr.N))
    s = _solver(cV, V0T, kind, p)
    s.assemble(D)
    blk = to_np(s.get_blocks())
    b = Blocks(pr.grid, pr.refs, D)
    g = pr.grid
    N = pr.N
    Bm = [(-b.G[m] + b.R[m] + b.RD[m]).tocsr() for m in range(2)]
    err, ref = 0.0, 0.0
    for k in range(g.numT):
        sl = slice(k * N, (k + 1) * N)
        for m in range(2):
            want = Bm[m][sl, sl].toarray()
            err = max(err, np.abs(blk[k, m] - want).max())
            ref = max(ref, np.abs(want).max())
        for nn in range(3):
            kp = g.kp[k, nn]
            if kp < 0:
                assert np.all(blk[k, 2 + nn] == 0)
                continue
            slp = slice(kp * N, (kp + 1) * N)
            # sum_m nu^m R^m_{k k+} = U_kn
            want = sum(g.nuE0T[k, nn, m] * Bm[m][sl, slp].toarray() for m in range(2))
            err = max(err, np.abs(blk[k, 2 + nn] - want).max())
    assert err <= 1e-12 * max(ref, 1.0), (err, ref)


@pytest.mark.parametrize("n,seed,neu,p", CASES)
def test_apply_and_preconditioner(torch_mod, n, seed, neu, p):
    cV, V0T, kind = square_mesh(n, seed=seed, neumann_sides=neu)
    pr = Problem(cV, V0T, kind, p)
    rng = np.random.default_rng(seed + 7)
    K, N = pr.grid.numT, pr.N
    D = 1.0 + 0.3 * rng.standard_normal((K, N))
    Cv = rng.standard_normal((K, N))
    dt = 0.013
    s = _solver(cV, V0T, kind, p)
    s.assemble(D)
    b = Blocks(pr.grid, pr.refs, D)
    S = schur_matrix(b, pr.grid, pr.refs, 1.0, dt)
    want = (S @ Cv.reshape(-1)).reshape(K, N)
    got = to_np(s.apply_schur(dt, Cv))
    assert rel_l2(pr.grid.areaT, got, want) < 1e-12
    # full 3KN operator (W + dt A) Y
    Y = rng.standard_normal(3 * K * N)
    full = (mass_W(b) + dt * system(b, 1.0)) @ Y
    gotf = to_np(s.apply_full(dt, Y))
    assert np.linalg.norm(gotf - full) <= 1e-12 * np.linalg.norm(full)
    # block-Jacobi: inverses of the diagonal blocks of S
    s.bj_setup(dt)
    bj = to_np(s.get_bj())
    Sd = S.toarray() if K * N < 3000 else None
    for k in range(K):
        sl = slice(k * N, (k + 1) * N)
        blkS = Sd[sl, sl] if Sd is not None else S[sl, sl].toarray()
        inv = np.linalg.inv(blkS)
        assert np.abs(bj[k] - inv).max() <= 1e-10 * np.abs(inv).max(), k


def _run_steps(p, n, seed, neu, wkind, steps, dt, sigma=1.0, block=4, t0=0.0, krylov=0,
               expect_krylov=None, precision=0, rtol=1e-13, infos=None, **kw):
    cV, V0T, kind = square_mesh(n, seed=seed, neumann_sides=neu)
    pr = Problem(cV, V0T, kind, p)
    w = workload(wkind, n, seed=seed, sigma=sigma, block=block)
    s = _solver(cV, V0T, kind, p, rtol=rtol, restart=40, max_iters=20000, krylov=krylov,
                precision=precision, **kw)
    gk = {SMOOTH1: 1, SMOOTH2: 2, LOGNORMAL: 3, LOGNORMAL_T: 4, TABLE2: 5}[wkind]
    dT = getattr(w, "dT", None)
    smp0 = s.sample_workload(gk, t0, dT=dT, want=("c0",))
    s.set_initial_samples(smp0["c0"], t0)
    C = pr.initial(w)
    assert rel_l2(pr.grid.areaT, to_np(s.get_solution()[0]), C) < 1e-13
    t = t0
    worst = 0.0
    for _ in range(steps):
        t += dt
        smp = s.sample_workload(gk, t, dT=dT)
        info = s.step_sampled(dt, smp["d"], smp["f"], smp["cD"], smp["gN"])
        assert info["rel_residual"] <= rtol
        if infos is not None:
            infos.append(info)
        if expect_krylov is not None:
            assert info["krylov"] == expect_krylov and info["fallbacks"] == 0, info
        C, Z1, Z2, oi = pr.step(C, t, dt, w)
        Cg, Z1g, Z2g = (to_np(x) for x in s.get_solution())
        worst = max(worst, rel_l2(pr.grid.areaT, Cg, C))
        zerr = rel_l2(pr.grid.areaT, np.stack([Z1g, Z2g]), np.stack([Z1, Z2]))
        assert zerr < 1e-9, zerr
    return worst


def test_steps_config1(torch_mod):
    # 8 x 8 cells, p = 1, smooth d, manufactured c, Dirichlet, 10 steps of 0.01
    assert _run_steps(1, 8, None, (), SMOOTH1, 10, 0.01) < 1e-10


@pytest.mark.parametrize("p,n,seed,neu,wk", [
    (2, 6, 201, (SOUTH, NORTH), TABLE2),
    (3, 5, 202, (), SMOOTH2),
    (4, 5, 203, (EAST,), LOGNORMAL_T),
    (0, 7, 204, (), SMOOTH1),
])
def test_steps_small(torch_mod, p, n, seed, neu, wk):
    assert _run_steps(p, n, seed, neu, wk, 3, 0.02, block=2) < 1e-10


@pytest.mark.parametrize("p,n,seed,neu,wk,krylov,expect", [
    (4, 6, 301, (), LOGNORMAL_T, 0, 2),         # auto picks CG for an element-wise constant d
    (3, 9, 302, (SOUTH,), LOGNORMAL, 1, 1),     # GMRES forced on the same kind of data
    (2, 9, 303, (), SMOOTH2, 0, 1),             # auto picks GMRES when d varies inside triangles
    (1, 10, 304, (EAST, WEST), LOGNORMAL, 2, 2),
])
def test_krylov_selection(torch_mod, p, n, seed, neu, wk, krylov, expect):
    assert _run_steps(p, n, seed, neu, wk, 2, 0.05, block=3, krylov=krylov,
                      expect_krylov=expect) < 1e-10


@pytest.mark.parametrize("precision", [1, 2])
@pytest.mark.parametrize("p,n,seed,neu,wk", [
    (4, 6, 401, (), LOGNORMAL_T),        # CG inner solves
    (3, 7, 402, (SOUTH,), SMOOTH2),      # GMRES inner solves
])
def test_mixed_precision_refinement(torch_mod, precision, p, n, seed, neu, wk):
    # FP32 / BF16 inner solves, FP64 residual and correction: the FP64 result
    infos = []
    err = _run_steps(p, n, seed, neu, wk, 2, 0.02, block=3, precision=precision, rtol=1e-12,
                     infos=infos)
    assert err < 1e-9, err
    assert all(i["ir_steps"] >= 1 for i in infos)


@pytest.mark.parametrize("precision", [1, 2])
def test_mixed_cg_sweeps_with_and_without_the_kept_direction(torch_mod, precision):
    # CG refinement sweeps either continue from the last search direction (the
    # FP64 residual replacing the iterated one) or start afresh: both reach the
    # oracle's solution, over several sweeps per step
    res = {}
    for keep in (True, False):
        infos = []
        err = _run_steps(4, 12, 403, (), LOGNORMAL_T, 2, 0.02, block=3, precision=precision,
                         rtol=1e-12, infos=infos, keep_direction=keep)
        assert err < 1e-9, (keep, err)
        assert all(i["krylov"] == 2 and i["ir_steps"] >= 2 for i in infos), infos
        res[keep] = [i["iters"] for i in infos]
    print("[keep-direction] precision %d iterations kept %s fresh %s"
          % (precision, res[True], res[False]), flush=True)


@pytest.mark.parametrize("p,n,seed,neu,wk", [
    (2, 6, 801, (NORTH,), SMOOTH1),
    (3, 6, 802, (), LOGNORMAL),
])
def test_bdf2_steps_match_the_oracle(torch_mod, p, n, seed, neu, wk):
    # first step implicit Euler (no history yet), then two-step BDF; a change of
    # dt falls back to implicit Euler
    cV, V0T, kind = square_mesh(n, seed=seed, neumann_sides=neu)
    pr = Problem(cV, V0T, kind, p)
    w = workload(wk, n, seed=seed, sigma=1.5, block=2)
    s = _solver(cV, V0T, kind, p, rtol=1e-13, restart=40, max_iters=20000)
    s.set_time_scheme("bdf2")
    gk = {SMOOTH1: 1, LOGNORMAL: 3}[wk]
    dT = getattr(w, "dT", None)
    s.set_initial_samples(s.sample_workload(gk, 0.0, dT=dT, want=("c0",))["c0"], 0.0)
    C = pr.initial(w)
    Cm = None
    t = 0.0
    for i, dt in enumerate([0.02, 0.02, 0.02, 0.01]):
        t += dt
        smp = s.sample_workload(gk, t, dT=dT)
        info = s.step_sampled(dt, smp["d"], smp["f"], smp["cD"], smp["gN"])
        order = 2 if i in (1, 2) else 1
        assert info["bdf_order"] == order and info["rel_residual"] <= 1e-13, info
        if order == 2:
            Cn, _, _, _ = pr.step_bdf2(C, Cm, t, dt, w)
        else:
            Cn, _, _, _ = pr.step(C, t, dt, w)
        Cm, C = C, Cn
        assert rel_l2(pr.grid.areaT, to_np(s.get_solution()[0]), C) < 1e-10


@pytest.mark.parametrize("p", [1, 3])
def test_bdf2_exact_for_quadratic_in_time(torch_mod, p):
    # c = P(x)(1 + a t + b t^2) with linear d, data sampled on the host at the
    # library's own points: from exact C^0, C^1 every BDF2 step reproduces the
    # projection of c to rounding
    from tests.test_oracle_solver import PolyWorkload
    from oracle.ldg import project
    cV, V0T, kind = square_mesh(3, seed=35, neumann_sides=(NORTH, WEST))
    pr = Problem(cV, V0T, kind, p)
    w = PolyWorkload(p, a=1.5, seed=40 + p, b=-2.0)
    s = _solver(cV, V0T, kind, p, rtol=1e-13, restart=40, max_iters=20000, krylov=1)
    xv, yv = (to_np(a) for a in s.quad_points(0))
    xb, yb = (to_np(a) for a in s.quad_points(1))
    n1, n2 = (to_np(a) for a in s.quad_points(2))
    dev = lambda a: torch_mod.as_tensor(np.ascontiguousarray(a), device="cuda")
    dt = 0.05
    s.set_state(to_np(s.project(dev(w.c(dt, xv, yv)))), dt)
    s.set_history(to_np(s.project(dev(w.c(0.0, xv, yv)))), dt)
    s.set_time_scheme("bdf2")
    t = dt
    for _ in range(3):
        t += dt
        info = s.step_sampled(dt, dev(w.d(t, xv, yv)), dev(w.f(t, xv, yv)),
                              dev(w.c_D(t, xb, yb)), dev(w.g_N(t, xb, yb, n1, n2)))
        assert info["bdf_order"] == 2
        want = project(pr.grid, p, lambda x, y: w.c(t, x, y), pr.refs.hatM, order=2 * p + 2)
        got = to_np(s.get_solution()[0])
        assert np.abs(got - want).max() <= 1e-10 * np.abs(want).max()


def _numbered_mesh(mesh, n, seed):
    from inputs.meshes import delaunay_square, edge_kinds, pair_numbering
    if mesh == "delaunay":
        cV, V0T = delaunay_square(n, seed)
        kind = edge_kinds(cV, V0T, (SOUTH,))
    else:
        cV, V0T, kind = square_mesh(n, seed=seed, neumann_sides=(SOUTH,))
    if mesh in ("pairs", "pairs-rotated", "delaunay"):
        V0T, kind, _ = pair_numbering(V0T, kind)
    if mesh == "pairs-rotated":
        V0T, kind = rotate_local_numbering(V0T, kind, seed)
    return cV, V0T, kind


@pytest.mark.parametrize("edge_traces", [True, False])
@pytest.mark.parametrize("precision,tol", [(1, 2e-5), (2, 1e-2)])
@pytest.mark.parametrize("mesh,p", [("paper", 3), ("pairs", 3), ("pairs", 4), ("pairs-rotated", 2),
                                    ("delaunay", 4)])
def test_inner_precision_apply(torch_mod, precision, tol, mesh, p, edge_traces):
    # the operator as the mixed-precision inner solves evaluate it (FP32 vectors,
    # FP32 / BF16 blocks; the off-diagonal edge terms from the neighbours' flux
    # traces, or from the stored blocks) against the oracle's FP64 eliminated
    # matrix.  With the triangles numbered in neighbour pairs, the neighbours
    # beside a triangle in its tile are read from the lanes beside it (the edges
    # of 64-triangle tiles and the ragged last tile included: K = 288 or more)
    cV, V0T, kind = _numbered_mesh(mesh, 12, 611 + p)
    pr = Problem(cV, V0T, kind, p)
    rng = np.random.default_rng(612 + p)
    K, N = pr.grid.numT, pr.N
    D = 1.0 + 0.3 * rng.standard_normal((K, N))
    Cv = rng.standard_normal((K, N))
    dt = 0.011
    s = _solver(cV, V0T, kind, p, precision=precision, edge_traces=edge_traces)
    s.assemble(D)
    want = (schur_matrix(Blocks(pr.grid, pr.refs, D), pr.grid, pr.refs, 1.0, dt)
            @ Cv.reshape(-1)).reshape(K, N)
    got = to_np(s.apply_schur_lowp(dt, Cv))
    err = rel_l2(pr.grid.areaT, got, want)
    print("inner-precision apply %s p=%d precision=%d traces=%d: rel L2 %.2e"
          % (mesh, p, precision, edge_traces, err))
    assert err < tol, err


@pytest.mark.parametrize("p", [0, 1, 2, 3, 4])
def test_edge_trace_form_of_the_neighbour_blocks(torch_mod, p):
    # the FP32 apply with the off-diagonal edge terms from the neighbours' flux
    # traces (ceil((3p+1)/2) Gauss points per edge, exact for the degree-3p
    # integrands) agrees with the one reading all five stored FP32 blocks to
    # FP32 rounding, on a mesh whose local edge numbering is rotated at random
    # (every neighbour edge n+ inside a wave) with Dirichlet and Neumann sides;
    # d varies inside the triangles, so the traces carry every mode of d_h
    cV, V0T, kind = _numbered_mesh("pairs-rotated", 11, 631 + p)
    pr = Problem(cV, V0T, kind, p)
    rng = np.random.default_rng(632 + p)
    K, N = pr.grid.numT, pr.N
    D = 1.0 + 0.3 * rng.standard_normal((K, N))
    Cv = rng.standard_normal((K, N))
    ys = []
    for tr in (True, False):
        s = _solver(cV, V0T, kind, p, precision=1, edge_traces=tr)
        s.assemble(D)
        ys.append(to_np(s.apply_schur_lowp(0.013, Cv)))
    want = (schur_matrix(Blocks(pr.grid, pr.refs, D), pr.grid, pr.refs, 1.0, 0.013)
            @ Cv.reshape(-1)).reshape(K, N)
    e_tr, e_st = (rel_l2(pr.grid.areaT, y, want) for y in ys)
    d = rel_l2(pr.grid.areaT, ys[0], ys[1])
    print("edge traces p=%d: vs oracle %.2e (stored blocks %.2e), between %.2e" % (p, e_tr, e_st, d))
    assert e_tr < 2e-5 and d < 2e-5, (e_tr, d)


def test_inner_precision_apply_is_independent_of_the_numbering(torch_mod):
    # the same mesh in the paper's numbering and in neighbour pairs: the FP32
    # apply agrees to FP32 rounding once rows are matched
    from inputs.meshes import pair_numbering
    p = 4
    cV, V0T, kind = square_mesh(10, seed=621, neumann_sides=(NORTH,))
    V2, k2, order = pair_numbering(V0T, kind)
    rng = np.random.default_rng(622)
    K, N = V0T.shape[0], (p + 1) * (p + 2) // 2
    D = 1.0 + 0.3 * rng.standard_normal((K, N))
    Cv = rng.standard_normal((K, N))
    ys = []
    for (V, k_, perm) in ((V0T, kind, np.arange(K)), (V2, k2, order)):
        s = _solver(cV, V, k_, p, precision=1)
        s.assemble(D[perm])
        ys.append(to_np(s.apply_schur_lowp(0.007, Cv[perm]))[np.argsort(perm)])
    area = Problem(cV, V0T, kind, p).grid.areaT
    assert rel_l2(area, ys[1], ys[0]) < 1e-6
