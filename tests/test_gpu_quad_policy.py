"""The paper's quadrature policy for the reference tensors (LDG_QUAD_PAPER).

The blocks assembled with the paper's rules (order max(2p, 1) on triangles,
2p + 1 on edges) match the oracle's blocks under its "paper" policy, and steps
match the oracle's steps under that policy; for p <= 1 the two policies agree,
for p >= 2 they differ by O(1) (the three-factor integrands are under-
integrated).
"""
import numpy as np
import pytest

from inputs.fields import LOGNORMAL, SMOOTH1, Workload, lognormal_blocks
from inputs.meshes import NORTH, SOUTH, square_mesh
from oracle.ldg import Problem
from tests.gpu_common import rel_l2, to_np
from tests.test_gpu_parity import _oracle_blocks

pytestmark = pytest.mark.gpu


def _solver(cV, V0T, kind, p, quad, **kw):
    from paper_1408_3877_amd import Solver
    return Solver(cV, V0T, kind, p, rtol=1e-13, restart=40, max_iters=20000, quad=quad, **kw)


@pytest.mark.parametrize("n,seed,p", [(5, 981, 1), (7, 982, 2), (6, 983, 3), (5, 984, 4)])
def test_paper_policy_blocks_match_the_oracle(n, seed, p):
    cV, V0T, kind = square_mesh(n, seed=seed, neumann_sides=(SOUTH,))
    rng = np.random.default_rng(seed)
    pr = Problem(cV, V0T, kind, p, policy="paper")
    D = 1.0 + 0.3 * rng.standard_normal((pr.grid.numT, pr.N))
    s = _solver(cV, V0T, kind, p, "paper")
    s.assemble(D)
    got = to_np(s.get_blocks())
    want = _oracle_blocks(pr, D)
    assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max()
    e = _solver(cV, V0T, kind, p, "exact")
    e.assemble(D)
    diff = np.abs(to_np(e.get_blocks()) - got).max() / np.abs(want).max()
    print("[quad] p=%d exact vs paper blocks: %.2e" % (p, diff), flush=True)
    assert diff < 1e-12 if p <= 1 else diff > 1e-3


@pytest.mark.parametrize("p,wk", [(2, LOGNORMAL), (4, SMOOTH1)])
def test_paper_policy_steps_match_the_oracle(p, wk):
    n, dt = 8, 0.01
    cV, V0T, kind = square_mesh(n, seed=990 + p, neumann_sides=(NORTH,))
    w = (Workload(LOGNORMAL, n_cells=n, blocks=lognormal_blocks(n, 991, 1.0, block=2), block=2)
         if wk == LOGNORMAL else Workload(wk))
    pr = Problem(cV, V0T, kind, p, policy="paper")
    s = _solver(cV, V0T, kind, p, "paper")
    s.set_initial_samples(s.sample_workload(wk, 0.0, dT=w.dT, want=("c0",))["c0"], 0.0)
    C, t = pr.initial(w), 0.0
    for _ in range(2):
        t += dt
        smp = s.sample_workload(wk, t, dT=w.dT)
        info = s.step_sampled(dt, smp["d"], smp["f"], smp["cD"], smp["gN"])
        C = pr.step(C, t, dt, w)[0]
        print("[quad] p=%d step %s" % (p, info), flush=True)
        assert info["rel_residual"] <= 1e-13
        assert rel_l2(pr.grid.areaT, to_np(s.get_solution()[0]), C) < 1e-10
