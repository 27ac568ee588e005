"""Exactness of the quadrature rules behind the FP32 apply in quadrature form.

The mixed modes evaluate the block terms of B^m (the tensors of Sec. 3.6,
eq:hatG, eq:hatRdiag, eq:hatRoffdiag) and the penalty from point values.  That
equals the stored-block apply only if each rule integrates its integrand
exactly:
  - volume: dphi_i/dx_m d_h Z_h, degree 3p - 1, on the unit square collapsed
    onto the reference triangle (x1 = u, x2 = (1 - u) v), Gauss-Jacobi points
    for the weight 1 - u in u and Gauss-Legendre points in v, ceil(3p / 2) each;
  - edges: phi_i d_h phi_j, degree 3p, ceil((3p + 1) / 2) Gauss-Legendre points;
  - penalty: phi_i phi_j, degree 2p, p + 1 Gauss-Legendre points.
The neighbour's traces are read at the reversed points, which needs the
Gauss-Legendre nodes to be symmetric about 1/2.  These checks use SciPy's
nodes and the closed-form monomial integrals, independent of the library.
"""
from math import factorial

import numpy as np
import pytest
from scipy.special import roots_jacobi, roots_legendre


def _vol_points(p):
    # the counts the library uses (ceil(3p / 2) per direction, none at p = 0)
    return 0 if p == 0 else (3 * p + 1) // 2


def _edge_points(p):
    return (3 * p + 2) // 2


def _collapsed_rule(nu, nv):
    xj, wj = roots_jacobi(nu, 1.0, 0.0)   # weight (1 - x) on (-1, 1)
    u, wu = 0.5 * (xj + 1.0), 0.25 * wj   # weight (1 - u) on (0, 1)
    xl, wl = roots_legendre(nv)
    v, wv = 0.5 * (xl + 1.0), 0.5 * wl
    U, V = np.meshgrid(u, v, indexing="ij")
    W = np.outer(wu, wv)
    return U.ravel(), ((1.0 - U) * V).ravel(), W.ravel()


def _monomial_errors(rule, degree):
    x1, x2, w = rule
    worst = 0.0
    for a in range(degree + 1):
        for b in range(degree + 1 - a):
            exact = factorial(a) * factorial(b) / factorial(a + b + 2)
            worst = max(worst, abs(np.sum(w * x1**a * x2**b) - exact) / exact)
    return worst


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5, 6])
def test_volume_rule_is_exact_for_degree_3p_minus_1(p):
    n = _vol_points(p)
    assert n * n == {1: 4, 2: 9, 3: 25, 4: 36, 5: 64, 6: 81}[p]
    assert _monomial_errors(_collapsed_rule(n, n), 3 * p - 1) < 1e-13
    # one point fewer in u no longer integrates the degree-(3p - 1) monomials
    if n > 1:
        assert _monomial_errors(_collapsed_rule(n - 1, n), 3 * p - 1) > 1e-6


@pytest.mark.parametrize("p", [0, 1, 2, 3, 4, 5, 6])
def test_edge_rules_are_exact_and_symmetric(p):
    for q, degree in ((_edge_points(p), 3 * p), (p + 1, 2 * p)):
        x, w = roots_legendre(q)
        s, ws = 0.5 * (x + 1.0), 0.5 * w
        for d in range(degree + 1):
            assert abs(np.sum(ws * s**d) - 1.0 / (d + 1)) < 1e-14
        # the neighbour's parameter runs the other way: its point Q-1-q is 1 - s_q
        assert np.allclose(s[::-1], 1.0 - s, atol=1e-15, rtol=0)
        assert np.allclose(ws[::-1], ws, atol=1e-15, rtol=0)
    # 2Q - 1 >= 3p, and one point fewer would not integrate degree 3p
    assert 2 * _edge_points(p) - 1 >= 3 * p > 2 * (_edge_points(p) - 1) - 1
