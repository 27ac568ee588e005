"""Pins of the oracle's basis and quadrature against the paper and closed forms."""
from math import factorial

import numpy as np
import pytest

from oracle import basis
from oracle.quadrature import collapsed_rule, gauss_legendre_01, rule_1d, triangle_rule

RNG = np.random.default_rng(7)


def _tri_points(n):
    u = RNG.random((n, 2))
    flip = u.sum(1) > 1
    u[flip] = 1 - u[flip]
    return u[:, 0], u[:, 1]


def test_closed_forms_up_to_order_two():
    # Sec. 2.4.1 prints phi_1..phi_6 in closed form
    x, y = _tri_points(50)
    s2, s3, s5, s6 = np.sqrt([2.0, 3.0, 5.0, 6.0])
    printed = [
        np.full_like(x, s2),
        2 - 6 * x,
        2 * s3 * (1 - x - 2 * y),
        s6 * ((10 * x - 8) * x + 1),
        s3 * ((5 * x - 4) * x + (-15 * y + 12) * y - 1),
        3 * s5 * ((3 * x + 8 * y - 4) * x + (3 * y - 4) * y + 1),
    ]
    for i, ref in enumerate(printed):
        np.testing.assert_allclose(basis.phi(i, x, y), ref, rtol=0, atol=1e-13)


def test_closed_forms_orders_three_and_four():
    # Sec. 2.4.1: phi_7..phi_15 as the paper's basis routine prints them (nested
    # Horner form in x1 = x, x2 = y); a sign, scale or within-degree permutation
    # slip in the oracle's coefficient table fails here
    x, y = _tri_points(60)
    s2, s6, s10, s14, s30, s70 = np.sqrt([2.0, 6.0, 10.0, 14.0, 30.0, 70.0])
    printed = [
        2 * s2 * (-1 + (15 + (-45 + 35 * x) * x) * x),
        2 * s6 * (-1 + (13 + (-33 + 21 * x) * x) * x + (2 + (-24 + 42 * x) * x) * y),
        2 * s10 * (-1 + (9 + (-15 + 7 * x) * x) * x
                   + (6 + (-48 + 42 * x) * x + (-6 + 42 * x) * y) * y),
        2 * s14 * (-1 + (3 + (-3 + x) * x) * x
                   + (12 + (-24 + 12 * x) * x + (-30 + 30 * x + 20 * y) * y) * y),
        s10 * (1 + (-24 + (126 + (-224 + 126 * x) * x) * x) * x),
        s30 * (1 + (-22 + (105 + (-168 + 84 * x) * x) * x) * x
               + (-2 + (42 + (-168 + 168 * x) * x) * x) * y),
        5 * s2 * (1 + (-18 + (69 + (-88 + 36 * x) * x) * x) * x
                  + (-6 + (102 + (-312 + 216 * x) * x) * x + (6 + (-96 + 216 * x) * x) * y) * y),
        s70 * (1 + (-12 + (30 + (-28 + 9 * x) * x) * x) * x
               + (-12 + (132 + (-228 + 108 * x) * x) * x
                  + (30 + (-300 + 270 * x) * x + (-20 + 180 * x) * y) * y) * y),
        3 * s10 * (1 + (-4 + (6 + (-4 + x) * x) * x) * x
                   + (-20 + (60 + (-60 + 20 * x) * x) * x
                      + (90 + (-180 + 90 * x) * x + (-140 + 140 * x + 70 * y) * y) * y) * y),
    ]
    for j, ref in enumerate(printed):
        i = 6 + j
        np.testing.assert_allclose(basis.phi(i, x, y), ref, rtol=0, atol=1e-12 * max(1.0, np.abs(ref).max()))


def test_orthonormal_exact_mass():
    # M_hat = identity (eq:hatM, Sec. 2.4.1) with a rule exact for degree 8
    x1, x2, w = collapsed_rule(6)
    P = basis.phi_all(15, x1, x2)
    np.testing.assert_allclose(P.T @ (w[:, None] * P), np.eye(15), atol=1e-13)


def test_degrees_hierarchical():
    degs = [basis.degree(i) for i in range(15)]
    assert degs == [0, 1, 1, 2, 2, 2, 3, 3, 3, 3, 4, 4, 4, 4, 4]
    for p in range(5):
        assert basis.num_basis(p) == (p + 1) * (p + 2) // 2
        assert basis.order_of(basis.num_basis(p)) == p


def test_gradient_is_derivative_of_phi():
    x, y = _tri_points(40)
    h = 1e-6
    for i in range(15):
        fd1 = (basis.phi(i, x + h, y) - basis.phi(i, x - h, y)) / (2 * h)
        fd2 = (basis.phi(i, x, y + h) - basis.phi(i, x, y - h)) / (2 * h)
        np.testing.assert_allclose(basis.grad_phi(i, 0, x, y), fd1, atol=2e-6)
        np.testing.assert_allclose(basis.grad_phi(i, 1, x, y), fd2, atol=2e-6)


def test_gradient_matches_printed_gradients():
    # a few of the paper's printed gradient formulas (routine gradPhi)
    x, y = _tri_points(30)
    s3, s5, s10 = np.sqrt([3.0, 5.0, 10.0])
    np.testing.assert_allclose(basis.grad_phi(5, 0, x, y), 6 * s5 * (3 * x + 4 * y - 2), atol=1e-12)
    np.testing.assert_allclose(basis.grad_phi(4, 1, x, y), 2 * s3 * (-15 * y + 6), atol=1e-12)
    np.testing.assert_allclose(
        basis.grad_phi(14, 1, x, y),
        3 * s10 * (-20 + (60 + (-60 + 20 * x) * x) * x + (180 + (-360 + 180 * x) * x
                   + (-420 + 420 * x + 280 * y) * y) * y), atol=1e-10)


def test_quad1d_example():
    # quadRule1D example: int_0^1 s^2 ds = 1/3
    s, w = rule_1d(2)
    assert abs(np.dot(w, s ** 2) - 1 / 3) < 1e-15
    for R in range(1, 10):
        s, w = gauss_legendre_01(R)
        for a in range(2 * R):
            assert abs(np.dot(w, s ** a) - 1 / (a + 1)) < 1e-14


def test_quad2d_example_mass_is_identity():
    # quadRule2D example: order-2 rule gives M = eye(3) for N = 3
    x1, x2, w = triangle_rule(2)
    P = basis.phi_all(3, x1, x2)
    np.testing.assert_allclose(P.T @ (w[:, None] * P), np.eye(3), atol=1e-14)


@pytest.mark.parametrize("order,tol", [(1, 1e-15), (2, 1e-15), (3, 2e-10), (4, 1e-14),
                                       (5, 1e-15), (6, 1e-14), (8, 1e-14), (10, 1e-14)])
def test_triangle_rules_exact(order, tol):
    # int_T x^a y^b = a! b! / (a+b+2)!
    x1, x2, w = triangle_rule(order)
    for a in range(order + 1):
        for b in range(order + 1 - a):
            exact = factorial(a) * factorial(b) / factorial(a + b + 2)
            assert abs(np.dot(w, x1 ** a * x2 ** b) - exact) < tol, (a, b)
    assert np.all(w > 0)
    assert np.all((x1 > 0) & (x2 > 0) & (x1 + x2 < 1))


def test_order3_rule_has_nine_digits_only():
    # the printed order-3 rule is accurate to ~1e-10 only: never used for p >= 1 projections
    x1, x2, w = triangle_rule(3)
    err = abs(np.dot(w, x1 ** 3) - 1 / 20)
    assert 1e-12 < err < 1e-9
