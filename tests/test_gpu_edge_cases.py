"""Degenerate and boundary cases of the HIP path against the oracle.

A mesh of one triangle (a single partial tile, no interior edge), the two
triangles of the paper's Fig. 6 grid with a Neumann side, a step whose data
are all zero (zero right-hand side: the zero solution in no iterations), and
meshes the library must refuse before any device work.
"""
import numpy as np
import pytest

from inputs.fields import SMOOTH1, Workload
from oracle.ldg import Problem
from tests.gpu_common import rel_l2, to_np

pytestmark = pytest.mark.gpu


def _steps(cV, V0T, kind, p, wkind, nsteps, dt, **kw):
    from paper_1408_3877_amd import Solver
    pr = Problem(cV, V0T, kind, p)
    w = Workload(wkind)
    s = Solver(cV, V0T, kind, p, rtol=1e-13, max_iters=20000, **kw)
    s.set_initial_samples(s.sample_workload(wkind, 0.0, want=("c0",))["c0"])
    C = pr.initial(w)
    a = pr.grid.areaT
    assert rel_l2(a, to_np(s.get_solution()[0]), C) < 1e-13
    t = 0.0
    for _ in range(nsteps):
        t += dt
        smp = s.sample_workload(wkind, t)
        info = s.step_sampled(dt, smp["d"], smp["f"], smp["cD"], smp["gN"])
        C, Z1, Z2, _ = pr.step(C, t, dt, w)
        Cg, Z1g, Z2g = (to_np(x) for x in s.get_solution())
        errs = (rel_l2(a, Cg, C), rel_l2(a, np.stack([Z1g, Z2g]), np.stack([Z1, Z2])))
        print("[edge-case] K=%d p=%d %s errs %s" % (pr.grid.numT, p, info, errs), flush=True)
        assert info["rel_residual"] <= 1e-13
        assert max(errs) < 1e-10, errs


@pytest.mark.parametrize("p,precision", [(0, 0), (1, 0), (2, 0), (3, 0), (4, 0), (5, 0), (0, 2), (3, 2)])
def test_one_triangle(p, precision):
    # K = 1: one lane of one tile, three Dirichlet edges, no neighbour (the
    # mixed mode's quadrature form then has only the triangle's own traces;
    # at p = 0 no volume points)
    cV = np.array([[0.0, 0.0], [1.0, 0.0], [0.2, 0.9]])
    V0T = np.array([[0, 1, 2]], dtype=np.int32)
    kind = np.array([[1, 1, 1]], dtype=np.int8)
    _steps(cV, V0T, kind, p, SMOOTH1, 2, 0.05, precision=precision)


@pytest.mark.parametrize("p,precision", [(0, 2), (1, 0), (2, 0), (2, 1), (4, 0), (4, 2)])
def test_two_triangles_with_a_neumann_side(p, precision):
    # the grid of Fig. 6: two triangles sharing the diagonal of the unit square,
    # one Neumann side (local edge 0 of the first triangle, on x = 1)
    cV = np.array([[0.0, 0.0], [1.0, 0.0], [1.0, 1.0], [0.0, 1.0]])
    V0T = np.array([[0, 1, 2], [0, 2, 3]], dtype=np.int32)
    kind = np.array([[2, 0, 1], [1, 1, 0]], dtype=np.int8)
    _steps(cV, V0T, kind, p, SMOOTH1, 3, 0.02, precision=precision)


@pytest.mark.parametrize("precision", [0, 2])
def test_zero_data_give_the_zero_solution(precision):
    # d = 1, f = 0, c_D = 0, g_N = 0 from c0 = 0: the right-hand side is zero,
    # so the step returns the zero solution without a Krylov iteration
    import torch

    from inputs.meshes import SOUTH, square_mesh
    from paper_1408_3877_amd import Solver
    cV, V0T, kind = square_mesh(6, seed=871, neumann_sides=(SOUTH,))
    s = Solver(cV, V0T, kind, 3, rtol=1e-10, precision=precision)
    dev = torch.device("cuda")
    s.set_initial_samples(torch.zeros(s.R * s.K, dtype=torch.float64, device=dev))
    zb = torch.zeros(s.R1 * s.n_bnd, dtype=torch.float64, device=dev)
    info = s.step_sampled(0.01, torch.ones(s.R * s.K, dtype=torch.float64, device=dev),
                          torch.zeros(s.R * s.K, dtype=torch.float64, device=dev), zb, zb)
    assert info["iters"] == 0 and info["rel_residual"] == 0.0
    for x in s.get_solution():
        assert torch.count_nonzero(x).item() == 0


def test_invalid_meshes_are_refused():
    # refused at create, before any kernel runs: bad arguments with LDG_EINVAL,
    # an inconsistent triangulation with LDG_EMESH, each with its message
    from paper_1408_3877_amd import Solver
    from paper_1408_3877_amd.ldg import LdgError
    cV = np.array([[0.0, 0.0], [1.0, 0.0], [1.0, 1.0], [0.0, 1.0]])
    good = np.array([[0, 1, 2], [0, 2, 3]], dtype=np.int32)
    kind = np.array([[1, 0, 1], [1, 1, 0]], dtype=np.int8)
    cases = {
        "empty mesh": (good[:0], kind[:0], -1),
        "vertex index out of range": (np.array([[0, 1, 7], [0, 2, 3]], np.int32), kind, -1),
        "edge kind out of range": (good, np.array([[1, 0, 5], [1, 1, 0]], np.int8), -1),
        "not counter-clockwise": (np.array([[0, 2, 1], [0, 2, 3]], np.int32), kind, -2),
        "disagrees with the topology": (good, np.array([[1, 1, 1], [1, 1, 0]], np.int8), -2),
    }
    for msg, (V0T, kd, code) in cases.items():
        with pytest.raises(LdgError, match=msg) as e:
            Solver(cV, V0T, kd, 2)
        assert e.value.code == code, (msg, e.value.code)
