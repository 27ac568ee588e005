"""Pins of the learned factored preconditioner's oracle (oracle/gnn_factor.py).

The scaled operator has identity diagonal blocks and symmetric neighbour
blocks; omega = 0 gives block-Jacobi exactly; P is symmetric positive
definite; the gradient of the energy loss matches central differences; and a
constant omega of the right sign cuts preconditioned-CG iterations while the
wrong sign raises them (a sign or index slip in F fails one of these).
"""
import numpy as np
import pytest

from inputs.fields import lognormal_blocks, triangle_values
from inputs.meshes import NORTH, square_mesh
from oracle import gnn, gnn_factor as gf
from oracle.ldg import Blocks, schur_matrix
from oracle.mesh import Grid
from oracle.refelem import RefTensors


def _system(n, p, seed, ratio=6.5, sigma=1.5, neumann=(NORTH,)):
    cV, V0T, kind = square_mesh(n, seed=seed, neumann_sides=neumann)
    g = Grid(cV, V0T, kind)
    refs = RefTensors(p)
    blk = max(1, n // 4)
    dT = triangle_values(lognormal_blocks(n, seed + 1, sigma, block=blk), n, block=blk)
    D = np.zeros((g.numT, refs.N))
    D[:, 0] = dT / np.sqrt(2.0)              # d = dT on every triangle (phi_1 = sqrt 2)
    dt = ratio / n ** 2
    S = schur_matrix(Blocks(g, refs, D), g, refs, 1.0, dt)
    return g, D, dt, gf.System(g, S)


def _pcg(S, b, P, tol=1e-8, maxit=5000):
    x = np.zeros_like(b)
    r = b.copy()
    z = P @ r
    d = z.copy()
    rz = r @ z
    nb = np.linalg.norm(b)
    for it in range(1, maxit + 1):
        q = S @ d
        a = rz / (d @ q)
        x += a * d
        r -= a * q
        if np.linalg.norm(r) <= tol * nb:
            return it
        z = P @ r
        rzn = r @ z
        d = z + (rzn / rz) * d
        rz = rzn
    return maxit


def test_scaled_operator_blocks():
    g, D, dt, sy = _system(6, 2, 11)
    N = sy.N
    Sd = sy.S.toarray()
    Wd = sy.Wg.toarray()
    Sh = Wd @ Sd @ Wd.T
    for k in range(sy.K):
        assert np.abs(sy.Wk[k].T @ sy.Wk[k] - sy.BJinv[k]).max() <= 1e-12 * np.abs(sy.BJinv[k]).max()
        assert np.abs(np.tril(sy.Wk[k], -1)).max() == 0.0          # W_k upper triangular
        assert np.abs(Sh[k * N:(k + 1) * N, k * N:(k + 1) * N] - np.eye(N)).max() < 1e-12
        for n in range(3):
            j = g.kp[k, n]
            if j < 0:
                continue
            assert np.abs(sy.O[k, n] - Sh[k * N:(k + 1) * N, j * N:(j + 1) * N]).max() < 1e-12
            assert np.abs(sy.O[k, n] - sy.O[j, g.np_[k, n]].T).max() < 1e-12


def test_zero_omega_is_block_jacobi_and_P_is_spd():
    g, D, dt, sy = _system(6, 2, 12)
    P0 = sy.P(np.zeros((sy.K, 3))).toarray()
    assert np.abs(P0 - sy.BJg.toarray()).max() <= 1e-13 * np.abs(P0).max()
    rng = np.random.default_rng(3)
    om = np.where(sy.mask, rng.uniform(0.0, gf.OMEGA_MAX, (sy.K, 3)), 0.0)
    Pm = sy.P(om).toarray()
    assert np.abs(Pm - Pm.T).max() <= 1e-13 * np.abs(Pm).max()
    assert np.linalg.eigvalsh(Pm).min() > 0.0


def test_constant_omega_cuts_cg_iterations_and_the_wrong_sign_does_not():
    g, D, dt, sy = _system(16, 2, 13)
    rng = np.random.default_rng(4)
    b = sy.S @ rng.standard_normal(sy.K * sy.N)
    it_bj = _pcg(sy.S, b, sy.BJg)
    om = np.where(sy.mask, 0.6, 0.0)
    it_good = _pcg(sy.S, b, sy.P(om))
    it_bad = _pcg(sy.S, b, sy.P(-om))
    assert it_good < 0.75 * it_bj, (it_good, it_bj)
    assert it_bad > it_bj, (it_bad, it_bj)


@pytest.mark.parametrize("p", [1, 2])
def test_energy_loss_gradient_matches_finite_differences(p):
    g, D, dt, sy = _system(4, p, 20 + p)
    N = sy.N
    node, edge = gnn.features(g, D, dt, 1.0)
    rng = np.random.default_rng(5 + p)
    theta = gf.init_params(N, 7) + 0.05 * rng.standard_normal(gf.n_params(N))
    rhat = rng.standard_normal((sy.K, N))
    target = rng.standard_normal((sy.K, N))
    L, G = gf.energy_loss_grad(theta, g, node, edge, sy, rhat, target)
    assert abs(L - gf.energy_loss(theta, g, node, edge, sy, rhat, target)) <= 1e-12 * L
    n_head = sum(int(np.prod(s)) for _, s in gf.HEAD)
    idx = np.concatenate([np.arange(gf.n_params(N) - n_head, gf.n_params(N)),
                          rng.choice(gf.n_params(N) - n_head, 150, replace=False)])
    eps = 1e-6
    worst = 0.0
    floor = 1e-3 * np.abs(G).max()              # central differences resolve no less
    for i in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += eps
        tm[i] -= eps
        fd = (gf.energy_loss(tp, g, node, edge, sy, rhat, target)
              - gf.energy_loss(tm, g, node, edge, sy, rhat, target)) / (2 * eps)
        worst = max(worst, abs(fd - G[i]) / max(floor, abs(G[i])))
    assert worst < 1e-5, worst
    assert np.abs(G).max() > 0.0


def test_loss_is_one_at_zero_omega():
    g, D, dt, sy = _system(4, 1, 30)
    N = sy.N
    node, edge = gnn.features(g, D, dt, 1.0)
    theta = gf.init_params(N, 1)
    P = gnn.unpack(theta, N, gf.param_shapes(N))
    P["b_o"][...] = -200.0                        # sigmoid underflows: omega = 0
    rng = np.random.default_rng(8)
    L = gf.energy_loss(gnn.pack(P, N, gf.param_shapes(N)), g, node, edge, sy,
                       rng.standard_normal((sy.K, N)), rng.standard_normal((sy.K, N)))
    assert abs(L - 1.0) < 1e-12


@pytest.mark.parametrize("p", [1, 2])
def test_frobenius_loss_gradient_matches_finite_differences(p):
    g, D, dt, sy = _system(4, p, 40 + p)
    N = sy.N
    node, edge = gnn.features(g, D, dt, 1.0)
    rng = np.random.default_rng(15 + p)
    theta = gf.init_params(N, 9) + 0.05 * rng.standard_normal(gf.n_params(N))
    w = rng.standard_normal((sy.K, N))
    L, G = gf.frobenius_loss_grad(theta, g, node, edge, sy, w)
    assert abs(L - gf.frobenius_loss(theta, g, node, edge, sy, w)) <= 1e-12 * L
    n_head = sum(int(np.prod(s_)) for _, s_ in gf.HEAD)
    idx = np.concatenate([np.arange(gf.n_params(N) - n_head, gf.n_params(N)),
                          rng.choice(gf.n_params(N) - n_head, 150, replace=False)])
    eps = 1e-6
    floor = 1e-3 * np.abs(G).max()
    worst = 0.0
    for i in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += eps
        tm[i] -= eps
        fd = (gf.frobenius_loss(tp, g, node, edge, sy, w)
              - gf.frobenius_loss(tm, g, node, edge, sy, w)) / (2 * eps)
        worst = max(worst, abs(fd - G[i]) / max(floor, abs(G[i])))
    assert worst < 1e-5, worst


def test_frobenius_loss_is_the_fsai_functional_in_expectation():
    # E_w ||(G S G^T - I) w||^2 = ||G S G^T - I||_F^2 for w ~ N(0, I): average
    # over many probes against the exact Frobenius norms (ratio of the two)
    g, D, dt, sy = _system(4, 1, 50)
    N, K = sy.N, sy.K
    node, edge = gnn.features(g, D, dt, 1.0)
    theta = gf.init_params(N, 2)
    om = gf.omega(theta, g, node, edge, sy)
    Gm = ((np.eye(K * N) + sy.F(om).toarray()) @ sy.Wg.toarray())
    Sd = sy.S.toarray()
    num = np.linalg.norm(Gm @ Sd @ Gm.T - np.eye(K * N)) ** 2
    W = sy.Wg.toarray()
    den = np.linalg.norm(W @ Sd @ W.T - np.eye(K * N)) ** 2
    rng = np.random.default_rng(0)
    nums, dens = [], []
    for _ in range(400):
        w = rng.standard_normal(K * N)
        nums.append(np.sum((Gm @ (Sd @ (Gm.T @ w)) - w) ** 2))
        dens.append(np.sum((W @ (Sd @ (W.T @ w)) - w) ** 2))
    assert abs(np.mean(nums) / num - 1) < 0.1
    assert abs(np.mean(dens) / den - 1) < 0.1
    # one probe's loss is the ratio the device computes
    w = rng.standard_normal((K, N))
    r = Gm @ (Sd @ (Gm.T @ w.reshape(-1))) - w.reshape(-1)
    r0 = W @ (Sd @ (W.T @ w.reshape(-1))) - w.reshape(-1)
    assert abs(gf.frobenius_loss(theta, g, node, edge, sy, w) - (r @ r) / (r0 @ r0)) < 1e-12


@pytest.mark.parametrize("p", [1, 2])
def test_optstep_loss_gradient_matches_finite_differences(p):
    g, D, dt, sy = _system(4, p, 40 + p)
    N = sy.N
    node, edge = gnn.features(g, D, dt, 1.0)
    rng = np.random.default_rng(15 + p)
    theta = gf.init_params(N, 7) + 0.05 * rng.standard_normal(gf.n_params(N))
    rhat = rng.standard_normal((sy.K, N))
    target = rng.standard_normal((sy.K, N))
    L, G = gf.optstep_loss_grad(theta, g, node, edge, sy, rhat, target)
    assert abs(L - gf.optstep_loss(theta, g, node, edge, sy, rhat, target)) <= 1e-12
    n_head = sum(int(np.prod(s)) for _, s in gf.HEAD)
    idx = np.concatenate([np.arange(gf.n_params(N) - n_head, gf.n_params(N)),
                          rng.choice(gf.n_params(N) - n_head, 150, replace=False)])
    eps = 1e-6
    worst = 0.0
    floor = 1e-3 * np.abs(G).max()
    for i in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += eps
        tm[i] -= eps
        fd = (gf.optstep_loss(tp, g, node, edge, sy, rhat, target)
              - gf.optstep_loss(tm, g, node, edge, sy, rhat, target)) / (2 * eps)
        worst = max(worst, abs(fd - G[i]) / max(floor, abs(G[i])))
    assert worst < 1e-5, worst
    assert np.abs(G).max() > 0.0


def test_optstep_loss_is_the_steepest_descent_energy_and_scale_free():
    # brute force over the step length, invariance under scaling e, the range
    # [0, 1], and zero where the preconditioner is the exact inverse
    g, D, dt, sy = _system(4, 2, 51)
    N = sy.N
    node, edge = gnn.features(g, D, dt, 1.0)
    rng = np.random.default_rng(51)
    theta = gf.init_params(N, 7) + 0.05 * rng.standard_normal(gf.n_params(N))
    rhat, target = rng.standard_normal((2, sy.K, N))
    L = gf.optstep_loss(theta, g, node, edge, sy, rhat, target)
    e = (target + rhat).reshape(-1)
    z = sy.P(gf.omega(theta, g, node, edge, sy)) @ (sy.S @ e)
    ts = np.linspace(0.0, 4.0, 40001)
    en = [(e - t * z) @ (sy.S @ (e - t * z)) for t in ts]
    assert abs(min(en) / (e @ (sy.S @ e)) - L) < 1e-6
    assert 0.0 <= L <= 1.0
    assert abs(gf.optstep_loss(theta, g, node, edge, sy, 3.7 * rhat, 3.7 * target) - L) < 1e-12
    # a single triangle: no neighbours, P = BJ^{-1} = S^{-1} exactly
    cV = np.array([[0.0, 0.0], [1.0, 0.0], [0.0, 1.0]])
    V0T = np.array([[0, 1, 2]], dtype=np.int32)
    kind = np.ones((1, 3), dtype=np.int8)
    g1 = Grid(cV, V0T, kind)
    refs = RefTensors(2)
    D1 = np.zeros((1, refs.N))
    D1[0, 0] = 1.3 / np.sqrt(2.0)
    s1 = gf.System(g1, schur_matrix(Blocks(g1, refs, D1), g1, refs, 1.0, 0.1))
    node1, edge1 = gnn.features(g1, D1, 0.1, 1.0)
    th1 = gf.init_params(refs.N, 3)
    r1, t1 = rng.standard_normal((2, 1, refs.N))
    assert gf.optstep_loss(th1, g1, node1, edge1, s1, r1, t1) < 1e-12


def _nonsymmetric_system(n, p, seed, ratio=6.5):
    # d varying inside the triangles (a random P_p coefficient around 1):
    # B^m != -(A^m)^T diag(d), the eliminated operator is nonsymmetric
    cV, V0T, kind = square_mesh(n, seed=seed, neumann_sides=(NORTH,))
    g = Grid(cV, V0T, kind)
    refs = RefTensors(p)
    rng = np.random.default_rng(seed)
    D = 0.3 * rng.standard_normal((g.numT, refs.N)) / np.sqrt(refs.N)
    D[:, 0] = 1.0 / np.sqrt(2.0) * (1.0 + 0.5 * rng.random(g.numT))
    dt = ratio / n ** 2
    return g, D, dt, schur_matrix(Blocks(g, refs, D), g, refs, 1.0, dt)


def _gmres_iters(S, b, M, tol=1e-8, restart=30):
    import scipy.sparse.linalg as spla
    its = [0]
    Mop = spla.LinearOperator(S.shape, matvec=lambda v: M @ v)
    spla.gmres(S, b, rtol=tol, atol=0.0, restart=restart, maxiter=200, M=Mop,
               callback=lambda _: its.__setitem__(0, its[0] + 1), callback_type="pr_norm")
    return its[0]


def test_symmetric_part_construction():
    # on an SPD operator the symmetric-part construction is the plain one;
    # on a nonsymmetric one W_k^T W_k is the symmetric part of BJ_k^{-1}, the
    # neighbour blocks are those of (S + S^T) / 2 (so O_{k+ n+} = O_kn^T), P is
    # SPD, and as a right preconditioner of GMRES a constant omega of the
    # right sign beats block-Jacobi while the wrong sign does not
    g, D, dt, sy = _system(5, 2, 31)
    sy2 = gf.System(g, sy.S, symmetric_part=True)
    assert np.abs(sy2.Wk - sy.Wk).max() <= 1e-12 * np.abs(sy.Wk).max()
    assert np.abs(sy2.O - sy.O).max() <= 1e-12 * np.abs(sy.O).max()
    g, D, dt, S = _nonsymmetric_system(6, 2, 32)
    Sd = S.toarray()
    assert np.abs(Sd - Sd.T).max() > 1e-3 * np.abs(Sd).max()
    sy = gf.System(g, S, symmetric_part=True)
    N = sy.N
    for k in range(sy.K):
        sl = slice(k * N, (k + 1) * N)
        B = np.linalg.inv(Sd[sl, sl])
        np.testing.assert_allclose(sy.Wk[k].T @ sy.Wk[k], 0.5 * (B + B.T), atol=1e-12 * np.abs(B).max())
        for n in range(3):
            j = g.kp[k, n]
            if j < 0:
                continue
            sj = slice(j * N, (j + 1) * N)
            want = sy.Wk[k] @ (0.5 * (Sd[sl, sj] + Sd[sj, sl].T)) @ sy.Wk[j].T
            np.testing.assert_allclose(sy.O[k, n], want, atol=1e-12 * np.abs(want).max())
            np.testing.assert_allclose(sy.O[j, g.np_[k, n]], sy.O[k, n].T, atol=1e-13)
    om = np.where(sy.mask, 0.6, 0.0)
    P = sy.P(om).toarray() if hasattr(sy.P(om), "toarray") else sy.P(om)
    assert np.abs(P - P.T).max() <= 1e-12 * np.abs(P).max()
    assert np.linalg.eigvalsh(0.5 * (P + P.T)).min() > 0
    b = np.random.default_rng(33).standard_normal(S.shape[0])
    it_bj = _gmres_iters(S, b, sy.P(np.zeros_like(om)))
    it_p = _gmres_iters(S, b, sy.P(om))
    it_neg = _gmres_iters(S, b, sy.P(-om))
    assert it_p < 0.8 * it_bj and it_neg > it_p, (it_bj, it_p, it_neg)
