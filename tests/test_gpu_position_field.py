"""The log-normal block field sampled by position on a jittered mesh.

Each quadrature point takes the value of the block of cells of the unjittered
grid that contains it, so triangles straddle block boundaries: the projected
coefficient jumps inside triangles, over- and undershoots (below zero for
p >= 2), and the step's operator is nonsymmetric with an indefinite symmetric
part.  The library solves such steps with GMRES (its restart grows where
cycles stagnate), with block-Jacobi or with the learned factored
preconditioner of the symmetric part (block-Jacobi where that part's
diagonal blocks have no Cholesky factor), and reaches the oracle's direct
solution.
"""
import numpy as np
import pytest

from inputs.fields import LOGNORMAL, Workload, lognormal_blocks, position_values
from inputs.meshes import NORTH, square_mesh
from oracle import gnn_factor as gf
from oracle.ldg import Problem
from tests.gpu_common import rel_l2, to_np

pytestmark = pytest.mark.gpu


class PositionField(Workload):
    """Block field sampled by position; forcing and boundary data of the
    manufactured solution with d taken as 1 (a forcing only, for parity)."""

    def __init__(self, n_cells, blocks, block):
        super().__init__(LOGNORMAL, n_cells=n_cells, blocks=blocks, block=block)

    def d(self, t, x, y):
        return position_values(self.blocks, self.n_cells, x, y, self.block)

    def f(self, t, x, y):
        c = self.c(t, x, y)
        return -c + 98.0 * c


@pytest.mark.parametrize("precond", [0, 1])
def test_position_sampled_field_steps_match_the_oracle(precond):
    from paper_1408_3877_amd import Solver
    n, p, dt = 16, 3, 1e-3
    cV, V0T, kind = square_mesh(n, seed=1004, neumann_sides=(NORTH,))
    w = PositionField(n, lognormal_blocks(n, 4100, 1.5, block=2), 2)
    pr = Problem(cV, V0T, kind, p)
    s = Solver(cV, V0T, kind, p, rtol=1e-13, restart=30, max_iters=50000, precond=precond)
    if precond:
        s.gnn_set_mode("factor")
        s.gnn_set_params(gf.init_params(s.N, 7).astype(np.float32))
    x, y = (to_np(v) for v in s.quad_points(0))
    xb, yb = (to_np(v) for v in s.quad_points(1))
    n1, n2 = (to_np(v) for v in s.quad_points(2))
    C = pr.initial(w)
    s.set_state(C, 0.0)
    t = 0.0
    for _ in range(2):
        t += dt
        info = s.step_sampled(dt, w.d(t, x, y), w.f(t, x, y), w.c_D(t, xb, yb),
                              w.g_N(t, xb, yb, n1, n2))
        C, Z1, Z2, _ = pr.step(C, t, dt, w)
        err = rel_l2(pr.grid.areaT, to_np(s.get_solution()[0]), C)
        print("[position-field] precond=%d %s err=%.2e" % (precond, info, err), flush=True)
        assert info["krylov"] == 1 and info["rel_residual"] <= 1e-13
        if precond:
            # where the projected d is negative the symmetric part's diagonal
            # blocks are indefinite and have no Cholesky factor: the step then
            # runs block-Jacobi GMRES and reports that fallback
            learned = info["learned_iters"] == info["iters"] and info["fallbacks"] == 0
            fell_back = info["fallback_reason"] == 5 and info["learned_iters"] == 0
            assert learned or fell_back, info
        assert err < 1e-10
