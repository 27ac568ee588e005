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


def test_head_fit_freezes_parameters_that_do_not_move_omega(monkeypatch):
    # SPSA on the CG objective (stubbed here): head parameters whose change does
    # not move omega on the training systems (edge features absent there) stay
    # at their starting values; the others move
    from paper_1408_3877_amd import learned
    H = learned.HEAD
    unseen = [67, 71, 75]

    class Arr:
        def __init__(self, a):
            self.a = a

        def double(self):
            return self

        def cpu(self):
            return self

        def numpy(self):
            return self.a

    class FakeSolver:
        def project(self, d):
            return d

        def gnn_set_context(self, D, dt):
            pass

        def gnn_set_params(self, w):
            self.h = np.asarray(w[-H:], dtype=np.float64)

        def gnn_factor_omega(self):
            h = self.h.copy()
            h[unseen] = 0.0                   # these features are zero on every edge
            x = np.linspace(-1.0, 1.0, 40)
            return Arr(0.95 / (1.0 + np.exp(-(h[:-1].sum() * 0.01 * x + h[-1]))))

    def fake_objective(solver, w, cases, dt):
        solver.gnn_set_params(w)
        om = solver.gnn_factor_omega().numpy()
        return float(np.mean((om - 0.7) ** 2))

    monkeypatch.setattr(learned, "cg_objective", fake_objective)
    w0 = learned.factor_init(6, 3)
    cases = [(None, {"d": None})]
    w, best, hist = learned.train_head_cg(FakeSolver(), w0, cases, 1e-3, [0.6], 30, 0.03, 0.5, 11,
                                         from_start=True)
    assert hist["frozen"] == unseen
    assert np.array_equal(w[-H:][unseen], w0[-H:][unseen])
    assert not np.array_equal(w[-H:], w0[-H:])
    assert best <= hist["start"]


def test_shipped_heads_stay_near_their_initialisation():
    # the shipped weights keep the seeded trunk and move the head by less than
    # two units per parameter (no parameter drifted where the fit could not see it)
    import os

    from paper_1408_3877_amd import learned
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    for p, N in ((3, 10), (4, 15)):
        w = np.load(os.path.join(root, "paper_1408_3877_amd", "weights", "factor_p%d.npy" % p))
        init = learned.factor_init(N, 7)
        assert w.shape == init.shape
        assert np.array_equal(w[:-learned.HEAD], init[:-learned.HEAD])
        assert np.abs(w[-learned.HEAD:].astype(np.float64) - init[-learned.HEAD:]).max() < 2.0
