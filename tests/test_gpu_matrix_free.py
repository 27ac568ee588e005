"""The matrix-free apply against the oracle's assembled operator and steps.

The eliminated operator applied with the block terms contracted on the fly
(no stored blocks streamed) equals the oracle's Schur matrix times C, for
every order, Dirichlet/Neumann mixes, and local numberings that vary inside a
wave (the neighbour edge index n+ then differs between the triangles of a
matrix-core tile).  Steps with it (FP64 CG and GMRES, FP32 inner solves with
FP64 refinement, the learned preconditioner) match the oracle's steps.
"""
import numpy as np
import pytest

from inputs.fields import LOGNORMAL, SMOOTH2, Workload, lognormal_blocks
from inputs.meshes import EAST, NORTH, SOUTH, WEST, rotate_local_numbering, square_mesh
from oracle import gnn_factor as gf
from oracle.ldg import Blocks, Problem, schur_matrix
from tests.gpu_common import rel_l2, to_np

pytestmark = pytest.mark.gpu

CASES = [  # (n cells, jitter seed, Neumann sides, p, rotate local numbering)
    (5, 801, (SOUTH,), 0, False),
    (9, 802, (), 1, True),
    (9, 803, (SOUTH, NORTH), 2, False),
    (7, 804, (EAST,), 3, True),
    (9, 805, (WEST, NORTH), 4, False),
    (6, 806, (), 4, True),
]


def _solver(cV, V0T, kind, p, **kw):
    from paper_1408_3877_amd import Solver
    return Solver(cV, V0T, kind, p, **kw)


@pytest.mark.parametrize("n,seed,neu,p,rot", CASES)
def test_matrix_free_apply_matches_the_oracle(n, seed, neu, p, rot):
    cV, V0T, kind = square_mesh(n, seed=seed, neumann_sides=neu)
    if rot:
        V0T, kind = rotate_local_numbering(V0T, kind, seed)
    pr = Problem(cV, V0T, kind, p)
    rng = np.random.default_rng(seed)
    K, N = pr.grid.numT, pr.N
    D = 1.0 + 0.3 * rng.standard_normal((K, N))
    Cv = rng.standard_normal((K, N))
    dt = 0.017
    s = _solver(cV, V0T, kind, p)
    s.assemble(D)
    stored = to_np(s.apply_schur(dt, Cv))
    s.set_matrix_free(True)
    got = to_np(s.apply_schur(dt, Cv))
    want = (schur_matrix(Blocks(pr.grid, pr.refs, D), pr.grid, pr.refs, 1.0, dt)
            @ Cv.reshape(-1)).reshape(K, N)
    print("[mf] n=%d p=%d rot=%s: vs oracle %.2e, vs stored %.2e"
          % (n, p, rot, rel_l2(pr.grid.areaT, got, want), rel_l2(pr.grid.areaT, got, stored)),
          flush=True)
    assert rel_l2(pr.grid.areaT, got, want) < 1e-12
    assert rel_l2(pr.grid.areaT, got, stored) < 1e-13


def _steps(n, seed, p, kind_w, precision, precond=0, nsteps=2, rot=False):
    cV, V0T, kind = square_mesh(n, seed=seed, neumann_sides=(NORTH,))
    if rot:
        V0T, kind = rotate_local_numbering(V0T, kind, seed)
    blk = max(1, n // 4)
    w = (Workload(LOGNORMAL, n_cells=n, blocks=lognormal_blocks(n, seed + 1, 1.0, block=blk),
                  block=blk) if kind_w == LOGNORMAL else Workload(kind_w))
    pr = Problem(cV, V0T, kind, p)
    s = _solver(cV, V0T, kind, p, rtol=1e-13, restart=40, max_iters=20000, precision=precision,
                precond=precond)
    if precond:
        s.gnn_set_mode("factor")
        s.gnn_set_params(gf.init_params(s.N, seed).astype(np.float32))
    s.set_matrix_free(True)
    dT = w.dT
    s.set_initial_samples(s.sample_workload(kind_w, 0.0, dT=dT, want=("c0",))["c0"], 0.0)
    C = pr.initial(w)
    dt, t = 0.01, 0.0
    for _ in range(nsteps):
        t += dt
        smp = s.sample_workload(kind_w, t, dT=dT)
        info = s.step_sampled(dt, smp["d"], smp["f"], smp["cD"], smp["gN"])
        C, Z1, Z2, _ = pr.step(C, t, dt, w)
        Cg, Z1g, Z2g = (to_np(x) for x in s.get_solution())
        a = pr.grid.areaT
        errs = (rel_l2(a, Cg, C), rel_l2(a, Z1g, Z1), rel_l2(a, Z2g, Z2))
        print("[mf-steps] p=%d prec=%d pc=%d %s errs %s" % (p, precision, precond, info, errs),
              flush=True)
        assert info["rel_residual"] <= 1e-13 and max(errs) < 1e-10
        yield info


@pytest.mark.parametrize("n,seed,p,kind_w,precision,rot", [
    (12, 811, 2, LOGNORMAL, 0, False),    # FP64 CG
    (10, 812, 3, SMOOTH2, 0, True),       # FP64 GMRES, varying n+
    (12, 813, 4, LOGNORMAL, 1, False),    # FP32 inner CG + FP64 refinement
    (10, 814, 2, SMOOTH2, 1, False),      # FP32 inner GMRES + FP64 refinement
])
def test_matrix_free_steps_match_the_oracle(n, seed, p, kind_w, precision, rot):
    for info in _steps(n, seed, p, kind_w, precision, rot=rot):
        assert info["krylov"] == (2 if kind_w == LOGNORMAL else 1)


def test_matrix_free_steps_with_the_learned_preconditioner():
    for info in _steps(12, 821, 3, LOGNORMAL, 2, precond=1):
        assert info["learned_iters"] == info["iters"] and info["fallbacks"] == 0
