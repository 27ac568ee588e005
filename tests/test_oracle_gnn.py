"""Pins of the FP64 network oracle: its backward pass against central finite
differences of its forward pass, shapes, and one Adam step against the
closed form of the first update."""
import numpy as np
import pytest

from inputs.meshes import NORTH, square_mesh
from oracle import gnn
from oracle.mesh import Grid


def _setup(p, n=3, seed=0):
    cV, V0T, kind = square_mesh(n, seed=11 + seed, neumann_sides=(NORTH,))
    g = Grid(cV, V0T, kind)
    N = (p + 1) * (p + 2) // 2
    rng = np.random.default_rng(seed)
    D = np.zeros((g.numT, N))
    D[:, 0] = np.exp(rng.standard_normal(g.numT)) / np.sqrt(2)
    D[:, 1:] = 0.05 * rng.standard_normal((g.numT, N - 1))
    node, edge = gnn.features(g, D, 1e-3, 1.0)
    rhat = rng.standard_normal((g.numT, N))
    target = rng.standard_normal((g.numT, N))
    theta = gnn.init_params(N, seed)
    # non-zero biases so every parameter is exercised
    theta = theta + 0.05 * rng.standard_normal(theta.size)
    return g, node, edge, rhat, target, theta


def test_param_count_and_feature_shapes():
    g, node, edge, rhat, target, theta = _setup(2)
    N = 6
    assert theta.size == gnn.n_params(N)
    assert node.shape == (g.numT, N + 3) and edge.shape == (g.numT, 3, gnn.E_IN)
    # one-hot of (n, n+) on interior edges only
    hot = edge[:, :, 3:12].sum(-1)
    np.testing.assert_array_equal(hot, (g.kp >= 0).astype(float))


@pytest.mark.parametrize("p", [1, 2])
def test_backward_matches_finite_differences(p):
    g, node, edge, rhat, target, theta = _setup(p, seed=p)
    L, G = gnn.loss_grad(theta, g, node, edge, rhat, target)
    assert abs(L - gnn.loss(theta, g, node, edge, rhat, target)) < 1e-14
    rng = np.random.default_rng(100 + p)
    idx = np.unique(np.concatenate([rng.choice(theta.size, 250, replace=False),
                                    np.arange(theta.size - 40, theta.size)]))
    eps = 1e-6
    worst = 0.0
    for i in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += eps
        tm[i] -= eps
        fd = (gnn.loss(tp, g, node, edge, rhat, target) - gnn.loss(tm, g, node, edge, rhat, target)) / (2 * eps)
        worst = max(worst, abs(fd - G[i]) / max(1e-3, abs(G[i])))
    assert worst < 1e-5, worst


def test_adam_first_step_closed_form():
    # after one step from zero moments, the update is lr * g / (|g| + eps) elementwise
    theta = np.array([1.0, -2.0, 0.5])
    grad = np.array([0.3, -4.0, 1e-9])
    t2, m, v = gnn.adam_step(theta, grad, np.zeros(3), np.zeros(3), 1, 0.01)
    np.testing.assert_allclose(t2, theta - 0.01 * grad / (np.abs(grad) + 1e-8), rtol=1e-12)


def test_energy_loss_gradient_matches_finite_differences():
    from oracle.ldg import Blocks, schur_matrix
    from oracle.refelem import RefTensors
    g, node, edge, rhat, target, theta = _setup(1, seed=5)
    refs = RefTensors(1)
    D = np.zeros((g.numT, refs.N))
    D[:, 0] = 1.0
    S = schur_matrix(Blocks(g, refs, D), g, refs, 1.0, 0.01).toarray()
    L, G = gnn.energy_loss_grad(theta, g, node, edge, rhat, target, S)
    assert abs(L - gnn.energy_loss(theta, g, node, edge, rhat, target, S)) < 1e-13 * L
    rng = np.random.default_rng(9)
    eps = 1e-6
    worst = 0.0
    for i in rng.choice(theta.size, 200, replace=False):
        tp, tm = theta.copy(), theta.copy()
        tp[i] += eps
        tm[i] -= eps
        fd = (gnn.energy_loss(tp, g, node, edge, rhat, target, S)
              - gnn.energy_loss(tm, g, node, edge, rhat, target, S)) / (2 * eps)
        worst = max(worst, abs(fd - G[i]) / max(1e-4, abs(G[i])))
    assert worst < 1e-5, worst
    # predicting the target exactly gives zero, predicting zero gives one
    assert gnn.energy_loss(theta, g, node, edge, rhat, target, S) > 0
