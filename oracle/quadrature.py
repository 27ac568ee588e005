"""Quadrature rules (Sec. 3.3, eq:quadrature, routines quadRule1D / quadRule2D).

* Gauss-Legendre rules on (0,1); an R-point rule is exact to degree 2R-1,
  so a rule "of order q" has R = ceil((q+1)/2) points.  Nodes and weights are
  those of numpy's Gauss-Legendre routine, mapped from (-1,1) to (0,1).
* Triangle rules on the reference triangle with the area 1/2 folded into
  the weights: the printed rules of orders 1, 2, 4, 5, 6 (the order-3 rule
  is printed with only nine digits and is kept for completeness only), and
  for orders above 6 Gauss points on the unit square collapsed onto the
  triangle (Duffy map x1 = u, x2 = (1-u) v, Jacobian 1-u) with q points per
  direction, the reading of the paper's collapsed-square rule.
"""
import numpy as np


def gauss_legendre_01(R):
    """R-point Gauss-Legendre nodes/weights on (0,1), weights summing to 1."""
    t, w = np.polynomial.legendre.leggauss(R)
    return (t + 1) / 2, w / 2


def rule_1d(order):
    """Gauss rule on (0,1) exact for polynomials of degree <= order."""
    R = max(1, int(np.ceil((order + 1) / 2)))
    return gauss_legendre_01(R)


def collapsed_rule(n):
    """n*n-point collapsed Gauss rule on the reference triangle.

    Exact for total degree <= 2n-2 (GL in both directions, the Jacobian 1-u
    costing one degree)."""
    u, wu = gauss_legendre_01(n)
    v, wv = gauss_legendre_01(n)
    U, V = np.meshgrid(u, v, indexing="ij")
    WU, WV = np.meshgrid(wu, wv, indexing="ij")
    x1 = U.reshape(-1)
    x2 = ((1 - U) * V).reshape(-1)
    w = (WU * WV * (1 - U)).reshape(-1)
    return x1, x2, w


def triangle_rule(order):
    """(x1, x2, w) of the triangle rule of the given order (area 1/2 in w)."""
    if order <= 1:
        return np.array([1 / 3]), np.array([1 / 3]), np.array([0.5])
    if order == 2:
        return (np.array([1 / 6, 2 / 3, 1 / 6]), np.array([1 / 6, 1 / 6, 2 / 3]),
                np.full(3, 1 / 6))
    if order == 3:  # printed with nine digits only (Hillion)
        x1 = np.array([0.666390246, 0.178558728, 0.280019915, 0.075031109])
        x2 = np.array([0.178558728, 0.666390246, 0.075031109, 0.280019915])
        w = np.array([0.159020691, 0.159020691, 0.090979309, 0.090979309])
        return x1, x2, w
    if order == 4:  # Cowper, 6 points: two orbits of three
        a, a2 = 0.445948490915965, 0.108103018168070
        b, b2 = 0.091576213509771, 0.816847572980458
        wa, wb = 0.111690794839005, 0.054975871827661
        x1 = np.array([a, a2, a, b, b2, b])
        x2 = np.array([a2, a, a, b2, b, b])
        return x1, x2, np.array([wa, wa, wa, wb, wb, wb])
    if order == 5:  # Stroud, 7 points, closed form
        r = np.sqrt(15.0)
        a1, a2 = (6 - r) / 21, (6 + r) / 21
        w1, w2 = (155 - r) / 2400, (155 + r) / 2400
        x1 = np.array([1 / 3, a1, 1 - 2 * a1, a1, a2, 1 - 2 * a2, a2])
        x2 = np.array([1 / 3, 1 - 2 * a1, a1, a1, 1 - 2 * a2, a2, a2])
        return x1, x2, np.array([9 / 80, w1, w1, w1, w2, w2, w2])
    if order == 6:  # Cowper, 12 points
        a, b = 0.063089014491502, 0.249286745170910
        c, d = 0.310352451033785, 0.053145049844816
        a2, b2, cd = 0.873821971016996, 0.501426509658179, 0.636502499121399
        x1 = np.array([a, a2, a, b, b2, b, c, d, cd, d, cd, c])
        x2 = np.array([a, a, a2, b, b, b2, d, c, d, cd, c, cd])
        wa, wb, wc = 0.025422453185103, 0.058393137863189, 0.041425537809187
        return x1, x2, np.array([wa] * 3 + [wb] * 3 + [wc] * 6)
    return collapsed_rule(order)


def projection_order(p):
    """Order of the volume rule used for L2 projections: max(2p, 1) (main script)."""
    return max(2 * p, 1)


def boundary_order(p):
    """Order of the edge rule used for the boundary data integrals: 2p+1."""
    return 2 * p + 1
