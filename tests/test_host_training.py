"""Host logic of the training CLI that needs no GPU: the choice the output-bias
calibration makes from the iteration counts it measures."""
import numpy as np


def test_calibration_applies_the_shift_with_the_fewest_iterations(monkeypatch):
    # iteration counts as a function of the shift of b_o, with a tie between
    # +0.5 and -0.5: the fewest iterations win, ties go to the smaller |shift|
    # and then to the earlier entry, and only b_o (the last parameter) changes
    from paper_1408_3877_amd import learned
    w0 = learned.factor_init(6, 3)
    b0 = float(w0[-1])
    cost = {-1.0: 120.0, 0.0: 110.0, 0.5: 100.0, -0.5: 100.0, 2.0: 130.0}
    seen = []

    class FakeSolver:
        def gnn_set_params(self, w):
            assert np.array_equal(w[:-1], w0[:-1])
            self.b = float(w[-1])

    def fake_evaluate(solver, n, seeds, sigma, steps, dt, use_gnn):
        assert use_gnn and steps == 1 and seeds == [4000, 4001]
        d = round(solver.b - b0, 4)
        seen.append(d)
        return {"iters_per_step": cost[d]}

    monkeypatch.setattr(learned, "evaluate", fake_evaluate)
    shifts = [-1.0, 0.5, 0.0, -0.5, 2.0]
    w, table = learned.calibrate(FakeSolver(), w0, shifts, 16, [4000, 4001], 1.0, 1e-3)
    assert seen == shifts
    assert table == [(d, cost[d]) for d in shifts]
    assert np.array_equal(w[:-1], w0[:-1])
    assert w[-1] == np.float32(w0[-1] + np.float32(0.5))
    assert w0[-1] == np.float32(b0)     # the input is left unchanged


def test_calibration_prefers_no_shift_on_a_flat_curve(monkeypatch):
    from paper_1408_3877_amd import learned
    w0 = learned.factor_init(3, 5)

    class FakeSolver:
        def gnn_set_params(self, w):
            pass

    monkeypatch.setattr(learned, "evaluate", lambda *a: {"iters_per_step": 50.0})
    w, table = learned.calibrate(FakeSolver(), w0, [1.0, -1.0, 0.0], 8, [1], 1.0, 1e-3)
    assert [it for _, it in table] == [50.0, 50.0, 50.0]
    assert np.array_equal(w, w0)


def test_constant_head_gives_the_requested_omega():
    # the head with zero weights and bias logit(omega / 0.95) gives omega on
    # every edge; with_head replaces only the head (the last 79 parameters)
    import numpy as np

    from paper_1408_3877_amd import learned
    h = learned.constant_head(0.6)
    assert h.shape == (learned.HEAD,) and np.all(h[:-1] == 0)
    assert abs(0.95 / (1 + np.exp(-h[-1])) - 0.6) < 1e-12
    w = learned.factor_init(10, 7)
    w2 = learned.with_head(w, h)
    assert np.array_equal(w2[:-learned.HEAD], w[:-learned.HEAD])
    assert np.allclose(w2[-learned.HEAD:], h)
