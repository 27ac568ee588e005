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
    # M_hat = identity (eq:hatM, Sec. 2.4.1) with a rule exact for degree 8, and
    # for the order-5/6 functions (against each other and against the paper's
    # fifteen) with one exact for degree 12
    x1, x2, w = collapsed_rule(6)
    P = basis.phi_all(15, x1, x2)
    np.testing.assert_allclose(P.T @ (w[:, None] * P), np.eye(15), atol=1e-13)
    x1, x2, w = collapsed_rule(8)
    P = basis.phi_all(28, x1, x2)
    np.testing.assert_allclose(P.T @ (w[:, None] * P), np.eye(28), atol=1e-13)


def test_degrees_hierarchical():
    degs = [basis.degree(i) for i in range(28)]
    assert degs == [0, 1, 1, 2, 2, 2, 3, 3, 3, 3, 4, 4, 4, 4, 4] + [5] * 6 + [6] * 7
    for p in range(7):
        assert basis.num_basis(p) == (p + 1) * (p + 2) // 2
        assert basis.order_of(basis.num_basis(p)) == p


def test_orders_five_and_six_span_the_polynomials():
    # the 28 functions span P_6 and the first 21 span P_5: least-squares fits of
    # every monomial of degree <= 6 (<= 5) on many points are exact, and no
    # degree-6 monomial lies in the span of the first 21
    x, y = _tri_points(200)
    P6 = basis.phi_all(28, x, y)
    P5 = P6[:, :21]
    for d in range(7):
        for b in range(d + 1):
            m = x ** (d - b) * y ** b
            r6 = m - P6 @ np.linalg.lstsq(P6, m, rcond=None)[0]
            r5 = m - P5 @ np.linalg.lstsq(P5, m, rcond=None)[0]
            assert np.abs(r6).max() < 1e-11
            if d <= 5:
                assert np.abs(r5).max() < 1e-11
            else:
                assert np.abs(r5).max() > 1e-4


def test_orders_five_and_six_match_a_symbolic_construction():
    # the collapsed-coordinate functions built symbolically (sympy's Legendre
    # and Jacobi polynomials, exact normalisation by symbolic integration over
    # the triangle, gradients by symbolic differentiation) against the
    # oracle's numerical evaluation, at interior points and the vertex (0, 1)
    import sympy as sp
    X, Y = sp.symbols("x y")
    x, y = _tri_points(12)
    x = np.append(x, 0.0)
    y = np.append(y, 1.0)
    i = 15
    for d in (5, 6):
        for q in range(d + 1):
            a = d - q
            s = 2 * X - (1 - Y)                      # (1 - y) xi
            A = sp.expand(sp.expand_func(sp.legendre(a, sp.Symbol("t"))).subs(
                sp.Symbol("t"), s / (1 - Y)) * (1 - Y) ** a)
            A = sp.cancel(A)
            B = sp.expand_func(sp.jacobi(q, 2 * a + 1, 0, 2 * Y - 1))
            f = sp.expand(A * B)
            nrm = sp.integrate(sp.integrate(f ** 2, (X, 0, 1 - Y)), (Y, 0, 1))
            f = f / sp.sqrt(nrm)
            fx, fy = sp.diff(f, X), sp.diff(f, Y)
            for k in range(len(x)):
                sub = {X: sp.Rational(x[k]), Y: sp.Rational(y[k])}
                v = float(f.evalf(30, subs=sub))
                assert abs(basis.phi(i, x[k], y[k]) - v) <= 1e-12 * max(1.0, abs(v)), (i, k)
                if k < len(x) - 1:
                    for m, g in enumerate((fx, fy)):
                        gv = float(g.evalf(30, subs=sub))
                        assert abs(basis.grad_phi(i, m, x[k], y[k]) - gv) <= 1e-11 * max(1.0, abs(gv))
            i += 1


def test_gradient_is_derivative_of_phi():
    x, y = _tri_points(40)
    h = 1e-6
    for i in range(28):
        fd1 = (basis.phi(i, x + h, y) - basis.phi(i, x - h, y)) / (2 * h)
        fd2 = (basis.phi(i, x, y + h) - basis.phi(i, x, y - h)) / (2 * h)
        np.testing.assert_allclose(basis.grad_phi(i, 0, x, y), fd1, atol=2e-6 * max(1, np.abs(fd1).max()))
        np.testing.assert_allclose(basis.grad_phi(i, 1, x, y), fd2, atol=2e-6 * max(1, np.abs(fd2).max()))


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
