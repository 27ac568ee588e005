"""Fields as host callbacks (ldg_step, ldg_set_initial) and the alias entry points.

Steps whose data the library samples through Python callbacks of the
workload's own formulas match the oracle's steps and the steps driven by the
device sampler; a failing or non-finite callback returns ECALLBACK and leaves
the state unchanged.
"""
import ctypes as C

import numpy as np
import pytest

from inputs.fields import SMOOTH2, Workload
from inputs.meshes import NORTH, SOUTH, square_mesh
from oracle import gnn_factor as gf
from oracle.ldg import Problem
from tests.gpu_common import rel_l2, to_np

pytestmark = pytest.mark.gpu


def _solver(cV, V0T, kind, p, **kw):
    from paper_1408_3877_amd import Solver
    return Solver(cV, V0T, kind, p, rtol=1e-13, restart=40, max_iters=20000, **kw)


@pytest.mark.parametrize("p", [1, 3])
def test_callback_steps_match_the_oracle_and_the_sampled_steps(p):
    cV, V0T, kind = square_mesh(9, seed=950 + p, neumann_sides=(SOUTH, NORTH))
    w = Workload(SMOOTH2)
    pr = Problem(cV, V0T, kind, p)
    s = _solver(cV, V0T, kind, p)
    ref = _solver(cV, V0T, kind, p)
    s.set_initial(lambda t, x, y: w.c0(x, y))
    ref.set_initial_samples(ref.sample_workload(SMOOTH2, 0.0, want=("c0",))["c0"], 0.0)
    C0 = pr.initial(w)
    a = pr.grid.areaT
    assert rel_l2(a, to_np(s.get_solution()[0]), C0) < 1e-13
    C, t, dt = C0, 0.0, 0.02
    for _ in range(2):
        t += dt
        info = s.step(dt, w.d, w.f, w.c_D, w.g_N)
        smp = ref.sample_workload(SMOOTH2, t)
        ref.step_sampled(dt, smp["d"], smp["f"], smp["cD"], smp["gN"])
        C = pr.step(C, t, dt, w)[0]
        Cg = to_np(s.get_solution()[0])
        print("[callbacks] p=%d t=%.2f %s" % (p, t, info), flush=True)
        assert abs(info["t"] - t) < 1e-15 and info["rel_residual"] <= 1e-13
        assert rel_l2(a, Cg, C) < 1e-10
        assert rel_l2(a, Cg, to_np(ref.get_solution()[0])) < 1e-12


def test_failing_callbacks_return_ecallback_and_keep_the_state():
    from paper_1408_3877_amd.ldg import LdgError
    cV, V0T, kind = square_mesh(5, seed=961, neumann_sides=(NORTH,))
    w = Workload(SMOOTH2)
    s = _solver(cV, V0T, kind, 2)
    s.set_initial(lambda t, x, y: w.c0(x, y))
    C0 = to_np(s.get_solution()[0]).copy()

    def boom(t, x, y):
        raise RuntimeError("no coefficient here")

    for d, f in ((boom, w.f), (w.d, lambda t, x, y: np.full_like(x, np.nan))):
        with pytest.raises(LdgError) as e:
            s.step(0.01, d, f, w.c_D, w.g_N)
        assert e.value.code == -8
        assert np.array_equal(to_np(s.get_solution()[0]), C0)
    with pytest.raises(LdgError) as e:      # Neumann edges but no g_N
        s.step(0.01, w.d, w.f, w.c_D, None)
    assert e.value.code == -1
    info = s.step(0.01, w.d, w.f, w.c_D, w.g_N)      # and the context still steps
    assert info["rel_residual"] <= 1e-13


def test_alias_entry_points():
    cV, V0T, kind = square_mesh(4, seed=971)
    s = _solver(cV, V0T, kind, 2)
    C0 = np.random.default_rng(971).standard_normal((s.K, s.N))
    Cd = s._dev(C0)
    s._check(s.lib.ldg_set_initial_dofs(s.h, C.c_void_p(Cd.data_ptr()), 1))
    assert np.array_equal(to_np(s.get_solution()[0]), C0)
    s.gnn_set_mode("factor")
    th = gf.init_params(s.N, 971).astype(np.float32)
    s._check(s.lib.ldg_gnn_load(s.h, th.ctypes.data, th.size))
    back = np.zeros_like(th)
    s._check(s.lib.ldg_gnn_save(s.h, back.ctypes.data, back.size))
    assert np.array_equal(back, th)
