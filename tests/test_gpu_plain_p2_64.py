"""The 64 x 64-cell, p = 2 workload over all 100 steps against the oracle's
trajectory (sparse direct solves, tests/golden/make_plain_p2_64.py).

Jittered Friedrichs-Keller mesh (seed 1002), smooth d = exp(sin 2 pi x sin 2 pi y / 2)
(1 + t/10), Dirichlet data of c = cos 7x cos 7y e^-t, 100 implicit Euler steps
of 1e-3 (eq:fullSystem, Sec. 2.5).  The coefficient varies inside each
triangle, so every step is nonsymmetric and runs block-Jacobi GMRES.

Bars (relative L2 with M_k = 2|T_k| I, as in the design notes):
  FP64 solves at rtol 1e-13:                  <= 1e-10 for C, Z1, Z2;
  BF16 inner solves + FP64 refinement, 1e-12: <= 1e-9.
Checked at every step on 128 stored triangles and through the L2 norms of
c_h and z_h over the whole mesh, and in full at steps 1 and 100.
"""
import os

import numpy as np
import pytest

from inputs.meshes import square_mesh
from oracle.mesh import Grid
from tests.gpu_common import rel_l2, to_np

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "plain_p2_64.npz")


@pytest.fixture(scope="module")
def torch_mod():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    return torch


@pytest.mark.timeout(600)
@pytest.mark.parametrize("precision,rtol,tol", [(0, 1e-13, 1e-10), (2, 1e-12, 1e-9)])
def test_plain_p2_64_all_steps_match_the_oracle(torch_mod, precision, rtol, tol):
    from paper_1408_3877_amd import Solver
    g = np.load(GOLDEN)
    sample = g["sample"]
    cV, V0T, kind = square_mesh(64, seed=1002)
    area = Grid(cV, V0T, kind).areaT
    s = Solver(cV, V0T, kind, 2, rtol=rtol, restart=40, max_iters=20000, precision=precision)
    s.set_initial_samples(s.sample_workload(2, 0.0, want=("c0",))["c0"], 0.0)
    dt = float(g["dt"])
    t = 0.0
    worst = 0.0
    for n in g["steps"]:
        t += dt
        smp = s.sample_workload(2, t)
        info = s.step_sampled(dt, smp["d"], smp["f"], smp["cD"], smp["gN"])
        assert info["rel_residual"] <= rtol and info["krylov"] == 1, (n, info)
        C, Z1, Z2 = (to_np(x) for x in s.get_solution())
        i = n - 1
        errs = [rel_l2(area[sample], C[sample], g["C_s"][i]),
                rel_l2(area[sample], np.stack([Z1[sample], Z2[sample]]),
                       np.stack([g["Z1_s"][i], g["Z2_s"][i]]))]
        nc = np.sqrt(np.sum(2 * area[:, None] * C ** 2))
        nz = np.sqrt(np.sum(2 * area[:, None] * (Z1 ** 2 + Z2 ** 2)))
        errs += [abs(nc - g["norm_c"][i]) / g["norm_c"][i], abs(nz - g["norm_z"][i]) / g["norm_z"][i]]
        if "C_%d" % n in g:
            errs += [rel_l2(area, C, g["C_%d" % n]), rel_l2(area, Z1, g["Z1_%d" % n]),
                     rel_l2(area, Z2, g["Z2_%d" % n])]
        worst = max(worst, max(errs))
        assert max(errs) <= tol, (n, errs)
    print("plain-p2-64 precision %d: worst relative L2 over 100 steps %.2e" % (precision, worst))
