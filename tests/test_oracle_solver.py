"""Solver-level pins of the oracle: exactness, convergence, the paper's examples."""
import json
import os

import numpy as np
import pytest

from inputs.fields import SMOOTH1, TABLE2, Workload
from inputs.meshes import EAST, NORTH, SOUTH, WEST, square_mesh, two_triangle_mesh
from oracle import basis
from oracle.ldg import (Blocks, Problem, full_residual, l2_error, project, schur_matrix,
                        step_schur)
from oracle.mesh import Grid
from oracle.refelem import RefTensors

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


class PolyWorkload:
    """c = P(x, y) (1 + a t), d linear; f, c_D, g_N consistent with eq:diffusion:nonmixed."""

    def __init__(self, p, a=1.0, seed=0, b=0.0):
        rng = np.random.default_rng(seed)
        self.terms = [(rng.uniform(-1, 1), i, j) for i in range(p + 1) for j in range(p + 1 - i)]
        self.a, self.b = a, b          # time factor s(t) = 1 + a t + b t^2
        self.d0, self.d1, self.d2 = 1.3, 0.4, -0.3

    def s(self, t):
        return 1 + self.a * t + self.b * t * t

    def P(self, x, y, dx=0, dy=0):
        out = 0 * x
        for c, i, j in self.terms:
            if i < dx or j < dy:
                continue
            fi = np.prod(range(i - dx + 1, i + 1)) if dx else 1
            fj = np.prod(range(j - dy + 1, j + 1)) if dy else 1
            out = out + c * fi * fj * x ** (i - dx) * y ** (j - dy)
        return out

    def c(self, t, x, y):
        return self.P(x, y) * self.s(t)

    def d(self, t, x, y):
        return self.d0 + self.d1 * x + self.d2 * y

    def f(self, t, x, y):
        s = self.s(t)
        lap = self.P(x, y, 2, 0) + self.P(x, y, 0, 2)
        dgc = self.d1 * self.P(x, y, 1, 0) + self.d2 * self.P(x, y, 0, 1)
        return (self.a + 2 * self.b * t) * self.P(x, y) - s * (dgc + self.d(t, x, y) * lap)

    def c_D(self, t, x, y):
        return self.c(t, x, y)

    def g_N(self, t, x, y, n1, n2):
        s = self.s(t)
        return -s * (self.P(x, y, 1, 0) * n1 + self.P(x, y, 0, 1) * n2)

    def c0(self, x, y):
        return self.c(0.0, x, y)


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5, 6])
def test_stationary_patch_exact(p):
    # c in P_p, linear d, consistent data: the LDG solution is c itself
    cV, V0T, kind = square_mesh(3, seed=21, neumann_sides=(SOUTH, EAST))
    pr = Problem(cV, V0T, kind, p)
    w = PolyWorkload(p, a=0.0, seed=p)
    C, Z1, Z2 = pr.solve_stationary(w)
    Cex = project(pr.grid, p, lambda x, y: w.c(0, x, y), pr.refs.hatM, order=2 * p + 2)
    np.testing.assert_allclose(C, Cex, atol=1e-11)
    Zex = project(pr.grid, p, lambda x, y: -w.P(x, y, 1, 0), pr.refs.hatM, order=2 * p + 2)
    np.testing.assert_allclose(Z1, Zex, atol=1e-10)


@pytest.mark.parametrize("p", [1, 2, 3, 5])
def test_implicit_euler_exact_for_linear_in_time(p):
    # c = P(x)(1+t): implicit Euler reproduces c at every step (eq:fullSystem)
    cV, V0T, kind = square_mesh(3, seed=31, neumann_sides=(NORTH,))
    pr = Problem(cV, V0T, kind, p)
    w = PolyWorkload(p, a=2.0, seed=10 + p)
    C = pr.initial(w)
    t, tau = 0.0, 0.05
    for _ in range(3):
        t += tau
        C, Z1, Z2, info = pr.step(C, t, tau, w)
        assert info["rel_residual"] < 1e-12
        Cex = project(pr.grid, p, lambda x, y: w.c(t, x, y), pr.refs.hatM, order=2 * p + 2)
        np.testing.assert_allclose(C, Cex, atol=1e-10)


@pytest.mark.parametrize("p", [1, 3])
def test_bdf2_exact_for_quadratic_in_time_and_euler_is_not(p):
    # c = P(x)(1 + a t + b t^2): the two-step formula differentiates quadratics
    # exactly, so from exact C^0, C^1 every BDF2 step reproduces c; implicit
    # Euler does not (its error is dt b P per step)
    cV, V0T, kind = square_mesh(3, seed=35, neumann_sides=(NORTH, WEST))
    pr = Problem(cV, V0T, kind, p)
    w = PolyWorkload(p, a=1.5, seed=40 + p, b=-2.0)
    dt = 0.05
    proj = lambda t: project(pr.grid, p, lambda x, y: w.c(t, x, y), pr.refs.hatM, order=2 * p + 2)
    Cm, C = proj(0.0), proj(dt)
    t = dt
    for _ in range(3):
        t += dt
        Cn, _, _, info = pr.step_bdf2(C, Cm, t, dt, w)
        assert info["rel_residual"] < 1e-12
        np.testing.assert_allclose(Cn, proj(t), atol=1e-10)
        Cm, C = C, Cn
    Ce, _, _, _ = pr.step(proj(dt), 2 * dt, dt, w)
    assert np.abs(Ce - proj(2 * dt)).max() > 1e-4


def test_bdf2_converges_at_second_order_in_time():
    # smooth manufactured data, end time 0.4, dt = 0.4/8 ... 0.4/64 with the same
    # space discretisation: differences of successive solutions shrink by ~4
    # under BDF2 (implicit Euler first step) and by ~2 under implicit Euler
    cV, V0T, kind = square_mesh(4, seed=36)
    p = 3
    pr = Problem(cV, V0T, kind, p)
    w = Workload(SMOOTH1)
    T = 0.4
    area = pr.grid.areaT[:, None]
    norm = lambda X: np.sqrt(np.sum(area * X ** 2))
    sol2, sol1 = [], []
    for nsteps in (8, 16, 32, 64):
        dt = T / nsteps
        C0 = pr.initial(w)
        C1, _, _, _ = pr.step(C0, dt, dt, w)
        Cm, C, Ce, t = C0, C1, C1, dt
        for _ in range(nsteps - 1):
            t += dt
            Cn, _, _, _ = pr.step_bdf2(C, Cm, t, dt, w)
            Cm, C = C, Cn
            Ce, _, _, _ = pr.step(Ce, t, dt, w)
        sol2.append(C)
        sol1.append(Ce)
    d2 = [norm(sol2[i] - sol2[i + 1]) for i in range(3)]
    d1 = [norm(sol1[i] - sol1[i + 1]) for i in range(3)]
    r2 = [d2[i] / d2[i + 1] for i in range(2)]
    r1 = [d1[i] / d1[i + 1] for i in range(2)]
    assert all(3.4 < r < 4.6 for r in r2), (d2, r2)
    assert all(1.7 < r < 2.3 for r in r1), (d1, r1)


def test_z_history_does_not_enter_the_step():
    # W has zero Z rows, so Y^{n+1} depends on C^n only
    cV, V0T, kind = square_mesh(2, seed=3)
    pr = Problem(cV, V0T, kind, 2)
    w = PolyWorkload(2, a=1.0)
    C0 = pr.initial(w)
    C1, Z1, Z2, info = pr.step(C0, 0.1, 0.1, w)
    from oracle.ldg import mass_W
    W = mass_W(info["blocks"])
    KN = C0.size
    Ya = np.concatenate([np.zeros(2 * KN), C0.reshape(-1)])
    Yb = np.concatenate([np.random.default_rng(1).standard_normal(2 * KN), C0.reshape(-1)])
    np.testing.assert_array_equal(W @ Ya, W @ Yb)


@pytest.mark.parametrize("neumann", [(), (SOUTH, NORTH), (EAST, WEST, SOUTH)])
def test_constant_d_adjointness(neumann):
    # constant d, exact tensors: B^m = -d (A^m)^T, so the Schur complement is SPD
    cV, V0T, kind = square_mesh(3, seed=41, neumann_sides=neumann)
    g = Grid(cV, V0T, kind)
    refs = RefTensors(2)
    D = np.zeros((g.numT, refs.N))
    D[:, 0] = 2.5 / np.sqrt(2)
    b = Blocks(g, refs, D)
    for m in range(2):
        A = (-b.H[m] + b.Q[m] + b.QN[m]).toarray()
        B = (-b.G[m] + b.R[m] + b.RD[m]).toarray()
        np.testing.assert_allclose(B, -2.5 * A.T, atol=1e-12)
    S = schur_matrix(b, g, refs, 1.0, 0.01).toarray()
    np.testing.assert_allclose(S, S.T, atol=1e-12)
    assert np.linalg.eigvalsh(S).min() > 0


@pytest.mark.parametrize("p", [1, 2, 4])
def test_elementwise_constant_d_gives_spd_operator(p):
    # d constant on every triangle: B^m = -(A^m)^T diag(d), so the eliminated
    # operator M + tau(eta S' + sum_m A^mT diag(d) M^-1 A^m) is SPD (CG applies)
    cV, V0T, kind = square_mesh(4, seed=61, neumann_sides=(NORTH,))
    g = Grid(cV, V0T, kind)
    refs = RefTensors(p)
    rng = np.random.default_rng(p)
    d = np.exp(2.0 * rng.standard_normal(g.numT))
    D = np.zeros((g.numT, refs.N))
    D[:, 0] = d / np.sqrt(2)
    b = Blocks(g, refs, D)
    N = refs.N
    for m in range(2):
        A = (-b.H[m] + b.Q[m] + b.QN[m]).toarray()
        B = (-b.G[m] + b.R[m] + b.RD[m]).toarray()
        np.testing.assert_allclose(B, -A.T * np.repeat(d, N)[None, :], atol=1e-11 * d.max())
    S = schur_matrix(b, g, refs, 1.0, 0.05).toarray()
    np.testing.assert_allclose(S, S.T, atol=1e-13 * np.abs(S).max())
    assert np.linalg.eigvalsh(0.5 * (S + S.T)).min() > 0
    # a coefficient varying inside the triangles breaks the symmetry
    D[:, 1] = 0.1
    S2 = schur_matrix(Blocks(g, refs, D), g, refs, 1.0, 0.05).toarray()
    assert np.abs(S2 - S2.T).max() > 1e-6 * np.abs(S2).max()


def test_row_restricted_schur_apply_matches_global_matrix():
    # the sampled-rows form used at full size equals rows of the global Schur matrix
    from oracle.ldg import schur_apply_rows
    cV, V0T, kind = square_mesh(6, seed=71, neumann_sides=(EAST,))
    g = Grid(cV, V0T, kind)
    refs = RefTensors(3)
    rng = np.random.default_rng(5)
    D = rng.standard_normal((g.numT, refs.N))
    C = rng.standard_normal((g.numT, refs.N))
    S = schur_matrix(Blocks(g, refs, D), g, refs, 1.3, 0.02)
    elems = np.array([0, 7, 19, 40, g.numT - 1])
    y, Z = schur_apply_rows(g, refs, D, C, 0.02, 1.3, elems)
    full = (S @ C.reshape(-1)).reshape(g.numT, refs.N)
    np.testing.assert_allclose(y, full[elems], atol=1e-12 * np.abs(full).max())


def test_schur_elimination_equals_full_solve():
    cV, V0T, kind = square_mesh(4, seed=51, neumann_sides=(SOUTH,))
    pr = Problem(cV, V0T, kind, 2)
    w = Workload(TABLE2)
    w.stationary = False                      # time dependent use of the same fields
    C0 = pr.initial(w)
    Ca, Z1a, Z2a, _ = pr.step(C0, 0.01, 0.01, w)
    Cb, Z1b, Z2b, info = step_schur(pr, C0, 0.01, 0.01, w)
    np.testing.assert_allclose(Cb, Ca, atol=1e-12)
    np.testing.assert_allclose(Z1b, Z1a, atol=1e-10)
    np.testing.assert_allclose(Z2b, Z2a, atol=1e-10)
    assert full_residual(pr, info["blocks"], info["data"], 0.01, C0, Cb, Z1b, Z2b) < 1e-12


def _table2_errors(p, levels):
    w = Workload(TABLE2)
    errs = []
    for j in levels:
        n = 3 * 2 ** j
        cV, V0T, kind = square_mesh(n, neumann_sides=(SOUTH, NORTH))
        pr = Problem(cV, V0T, kind, p)
        C, _, _ = pr.solve_stationary(w)
        errs.append(l2_error(pr.grid, C, lambda x, y: w.c(0, x, y)))
    return errs


@pytest.mark.parametrize("p,levels", [(1, [1, 2, 3]), (2, [1, 2, 3]), (3, [0, 1, 2]), (4, [0, 1, 2])])
def test_table2_convergence_rates(p, levels):
    # Table 2: order p+1 for p >= 1 (the paper's asymptotic rates: 2.00, 3.04, 4.01, 4.94)
    with open(os.path.join(GOLDEN, "table2.json")) as fh:
        tab = json.load(fh)
    errs = _table2_errors(p, levels)
    rate = np.log(errs[-2] / errs[-1]) / np.log(2)
    assert abs(rate - tab["final_rate"][str(p)]) < 0.35, (errs, rate)


def test_order_five_converges_at_order_six():
    # beyond the paper's orders: the Table 2 problem at p = 5 (basis functions
    # of degree 5 by recursion) converges at the LDG order p + 1 = 6
    errs = _table2_errors(5, [0, 1, 2])
    rate = np.log(errs[-2] / errs[-1]) / np.log(2)
    assert abs(rate - 6.0) < 0.35, (errs, rate)


def test_table2_p0_stagnates():
    # Table 2, p = 0: the error does not decay (stays near 0.1)
    errs = _table2_errors(0, [2, 3, 4])
    assert min(errs) > 0.08
    rate = np.log(errs[-2] / errs[-1]) / np.log(2)
    assert rate < 0.5


def test_fig7_projection_ranges():
    # Sec. 3.8 / Fig. 7: ranges of the projected function at the Lagrange nodes
    from oracle.io import lagrange_values
    with open(os.path.join(GOLDEN, "fig7_ranges.json")) as fh:
        ranges = json.load(fh)["ranges"]
    cV, V0T, kind = two_triangle_mesh()
    g = Grid(cV, V0T, kind)
    fAlg = lambda x, y: np.where(x < 0, x ** 2 - y ** 2 - 1, -x ** 2 - y ** 2 + 1)
    for N, (lo, hi) in zip((1, 3, 6), ranges):
        p = basis.order_of(N)
        D = project(g, p, fAlg, RefTensors(p).hatM, order=6)
        vals = lagrange_values(D)
        assert abs(vals.min() - lo) < 1e-12 and abs(vals.max() - hi) < 1e-12, (N, vals)


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5])
def test_discrete_functions_do_not_depend_on_the_basis(p):
    # the same method in a Gram-Schmidt basis of the monomials (Sec. 2.4.1):
    # every tensor, projection and block changes, the functions c_h, z_h do not
    from oracle.quadrature import triangle_rule
    cV, V0T, kind = square_mesh(4, seed=61, neumann_sides=(SOUTH,))
    w = Workload(SMOOTH1)
    q1, q2, _ = triangle_rule(2 * p + 2)
    out = {}
    for b in ("paper", "gram-schmidt"):
        with basis.use(b):
            pr = Problem(cV, V0T, kind, p)
            C0 = pr.initial(w)
            C1, Z1, Z2, _ = pr.step(C0, 0.05, 0.05, w)
            N = pr.N
            Phi = basis.phi_all(N, q1, q2)
            out[b] = [X @ Phi.T for X in (C0, C1, Z1, Z2)]
    for a, g in zip(out["paper"], out["gram-schmidt"]):
        assert np.abs(a - g).max() <= 1e-9 * np.abs(a).max()


def test_step_ignores_the_previous_flux():
    # W has zero Z rows (eq:fullSystem): perturbing Z^n leaves Y^{n+1} unchanged
    import scipy.sparse.linalg as spla

    from oracle.ldg import mass_W
    cV, V0T, kind = square_mesh(3, seed=62, neumann_sides=(NORTH,))
    pr = Problem(cV, V0T, kind, 2)
    w = Workload(SMOOTH1)
    data = pr.data(w, 0.02)
    b, A, V = pr.assemble(data)
    W = mass_W(b)
    KN = pr.grid.numT * pr.N
    rng = np.random.default_rng(62)
    C0 = pr.initial(w).reshape(-1)
    Ys = []
    for zn in (np.zeros(2 * KN), rng.standard_normal(2 * KN)):
        Yn = np.concatenate([zn, C0])
        Ys.append(spla.spsolve((W + 0.02 * A).tocsc(), W @ Yn + 0.02 * V))
    assert np.abs(Ys[0] - Ys[1]).max() == 0.0


def test_l2_error_absolute_scale():
    # Sec. 3.5: ||c_h - c||_{L2(Omega)} on the unit square.  With c_h = 0 and
    # c = x y the error is (int x^2 y^2)^(1/2) = 1/3; with c = 0 and only the
    # constant coefficient a set, c_h = a sqrt(2) and the error is a sqrt(2)
    # (|Omega| = 1).  A constant factor in the rule's weights or the 2|T_k|
    # scaling fails this, which the convergence orders alone do not see.
    coordV, V0T, kind = square_mesh(5, seed=3)
    grid = Grid(coordV, V0T, kind)
    for p in (0, 2, 4):
        N = basis.num_basis(p)
        C = np.zeros((grid.numT, N))
        assert abs(l2_error(grid, C, lambda x, y: x * y) - 1 / 3) < 1e-13
        C[:, 0] = 0.7
        assert abs(l2_error(grid, C, lambda x, y: 0 * x) - 0.7 * np.sqrt(2)) < 1e-13


def test_cg_step_matches_the_direct_step_on_spd_systems():
    # the iterative oracle used at large sizes reaches the direct solve's result
    # (element-wise constant d: SPD eliminated system)
    from inputs.fields import LOGNORMAL, lognormal_blocks
    from oracle.ldg import step_schur_cg
    n, p = 8, 3
    coordV, V0T, kind = square_mesh(n, seed=9, neumann_sides=(NORTH,))
    pr = Problem(coordV, V0T, kind, p)
    w = Workload(LOGNORMAL, n_cells=n, blocks=lognormal_blocks(n, 17, 1.5, block=2), block=2)
    C0 = pr.initial(w)
    Cd, Z1d, Z2d, _ = step_schur(pr, C0, 1e-3, 1e-3, w)
    Cc, Z1c, Z2c, info = step_schur_cg(pr, C0, 1e-3, 1e-3, w, rtol=1e-14)
    assert info["flag"] == 0 and info["rel_residual"] <= 1e-14 and info["iters"] > 10
    for a, b in ((Cc, Cd), (Z1c, Z1d), (Z2c, Z2d)):
        assert np.abs(a - b).max() <= 1e-11 * np.abs(b).max()
