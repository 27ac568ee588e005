"""Orthonormal modal basis on the reference triangle (Sec. 2.4.1).

The paper gives the functions up to order two in closed form and up to order
four in its basis routine.  Here every function is stored as a normalisation
constant times a polynomial with integer coefficients, expanded by hand from
the paper's formulas; the gradients are obtained by differentiating those
polynomials term by term (they are pinned against the paper's printed
gradient formulas in the tests).

Basis index i is 0-based here (the paper's phi_{i+1}).

Orders five and six (N = 21, 28) go beyond the paper's routine, which stops
at four; Sec. 2.4.1 names Gram-Schmidt orthonormalisation or recursion for
higher orders.  Here the functions of total degree d = 5, 6 are the
orthonormal collapsed-coordinate polynomials of the reference triangle,
    psi_{a,q}(x1, x2) = c_{a,q} P_a(xi) (1 - x2)^a P_q^{(2a+1,0)}(2 x2 - 1),
    xi = 2 x1 / (1 - x2) - 1,   c_{a,q} = sqrt(2 (2a+1) (a+q+1)),
with a + q = d and q = 0..d in that order (P_a Legendre, P_q^{(2a+1,0)}
Jacobi).  Each is orthogonal to every polynomial of lower degree, so they
are exactly what Gram-Schmidt gives when the paper's fifteen functions are
followed by these, and unlike a Gram-Schmidt of monomials they evaluate
without cancellation.  (1 - x2)^a P_a(xi) is a polynomial; at the vertex
x2 = 1 it equals 1 for a = 0 and 0 otherwise.
"""
import contextlib
from math import factorial

import numpy as np

# (normalisation, [(coefficient, power of x1, power of x2), ...])
_TABLE = [
    (np.sqrt(2.0), [(1, 0, 0)]),
    (1.0, [(2, 0, 0), (-6, 1, 0)]),
    (2 * np.sqrt(3.0), [(1, 0, 0), (-1, 1, 0), (-2, 0, 1)]),
    (np.sqrt(6.0), [(1, 0, 0), (-8, 1, 0), (10, 2, 0)]),
    (np.sqrt(3.0), [(-1, 0, 0), (-4, 1, 0), (12, 0, 1), (5, 2, 0), (-15, 0, 2)]),
    (3 * np.sqrt(5.0), [(1, 0, 0), (-4, 1, 0), (-4, 0, 1), (3, 2, 0), (8, 1, 1), (3, 0, 2)]),
    (2 * np.sqrt(2.0), [(-1, 0, 0), (15, 1, 0), (-45, 2, 0), (35, 3, 0)]),
    (2 * np.sqrt(6.0), [(-1, 0, 0), (13, 1, 0), (2, 0, 1), (-33, 2, 0), (-24, 1, 1),
                        (21, 3, 0), (42, 2, 1)]),
    (2 * np.sqrt(10.0), [(-1, 0, 0), (9, 1, 0), (6, 0, 1), (-15, 2, 0), (-48, 1, 1),
                         (-6, 0, 2), (7, 3, 0), (42, 2, 1), (42, 1, 2)]),
    (2 * np.sqrt(14.0), [(-1, 0, 0), (3, 1, 0), (12, 0, 1), (-3, 2, 0), (-24, 1, 1),
                         (-30, 0, 2), (1, 3, 0), (12, 2, 1), (30, 1, 2), (20, 0, 3)]),
    (np.sqrt(10.0), [(1, 0, 0), (-24, 1, 0), (126, 2, 0), (-224, 3, 0), (126, 4, 0)]),
    (np.sqrt(30.0), [(1, 0, 0), (-22, 1, 0), (-2, 0, 1), (105, 2, 0), (42, 1, 1),
                     (-168, 3, 0), (-168, 2, 1), (84, 4, 0), (168, 3, 1)]),
    (5 * np.sqrt(2.0), [(1, 0, 0), (-18, 1, 0), (-6, 0, 1), (69, 2, 0), (102, 1, 1),
                        (6, 0, 2), (-88, 3, 0), (-312, 2, 1), (-96, 1, 2), (36, 4, 0),
                        (216, 3, 1), (216, 2, 2)]),
    (np.sqrt(70.0), [(1, 0, 0), (-12, 1, 0), (-12, 0, 1), (30, 2, 0), (132, 1, 1),
                     (30, 0, 2), (-28, 3, 0), (-228, 2, 1), (-300, 1, 2), (-20, 0, 3),
                     (9, 4, 0), (108, 3, 1), (270, 2, 2), (180, 1, 3)]),
    (3 * np.sqrt(10.0), [(1, 0, 0), (-4, 1, 0), (-20, 0, 1), (6, 2, 0), (60, 1, 1),
                         (90, 0, 2), (-4, 3, 0), (-60, 2, 1), (-180, 1, 2), (-140, 0, 3),
                         (1, 4, 0), (20, 3, 1), (90, 2, 2), (140, 1, 3), (70, 0, 4)]),
]

MAX_P = 6


def num_basis(p):
    """N = (p+1)(p+2)/2 local degrees of freedom (Sec. 2.4.1)."""
    return (p + 1) * (p + 2) // 2


def order_of(N):
    """Inverse of num_basis."""
    p = int(round((np.sqrt(8 * N + 1) - 3) / 2))
    assert num_basis(p) == N
    return p


def _extension_index(i):
    """(a, q) of the function i >= 15: total degree d = a + q, q = 0..d."""
    j = i - len(_TABLE)
    for d in range(5, MAX_P + 1):
        if j <= d:
            return d - j, j
        j -= d + 1
    raise IndexError("basis index %d beyond order %d" % (i, MAX_P))


def _collapsed(i, x1, x2, m=None):
    """psi_{a,q} of basis index i >= 15 (m: None value, 0 d/dx1, 1 d/dx2)."""
    from scipy.special import eval_jacobi, eval_legendre
    a, q = _extension_index(i)
    c = np.sqrt(2.0 * (2 * a + 1) * (a + q + 1))
    x1, x2 = np.broadcast_arrays(np.asarray(x1, np.float64), np.asarray(x2, np.float64))
    t = 1.0 - x2
    top = t == 0.0
    ts = np.where(top, 1.0, t)
    xi = np.where(top, 0.0, 2.0 * x1 / ts - 1.0)
    A = np.where(top, 1.0 if a == 0 else 0.0, eval_legendre(a, xi) * ts ** a)
    B = eval_jacobi(q, 2 * a + 1, 0, 2.0 * x2 - 1.0)
    if m is None:
        return c * A * B
    if np.any(top):
        raise ValueError("gradients of the order-5/6 functions are not taken at the vertex (0, 1)")
    # P_n' = (n + alpha + beta + 1)/2 P_{n-1}^{(alpha+1, beta+1)}
    dL = (a + 1) / 2.0 * eval_jacobi(a - 1, 1, 1, xi) if a > 0 else 0.0 * xi
    if m == 0:
        return c * 2.0 * dL * t ** (a - 1) * B if a > 0 else 0.0 * x1
    dA = (dL * (1.0 + xi) - a * eval_legendre(a, xi)) * t ** (a - 1) if a > 0 else 0.0 * x1
    dB = (q + 2 * a + 2) / 2.0 * eval_jacobi(q - 1, 2 * a + 2, 1, 2.0 * x2 - 1.0) if q > 0 else 0.0 * x1
    return c * (dA * B + A * 2.0 * dB)


def _entry(i):
    if i < len(_TABLE):
        return _TABLE[i]
    raise IndexError(i)


def degree(i):
    """Total polynomial degree of basis function i (0-based)."""
    if i >= len(_TABLE):
        return sum(_extension_index(i))
    return max(a + b for _, a, b in _entry(i)[1])


def phi(i, x1, x2):
    """phi_hat_{i+1}(x1, x2) on the reference triangle."""
    if i >= len(_TABLE):
        return _collapsed(i, x1, x2)
    x1 = np.asarray(x1, dtype=np.float64)
    x2 = np.asarray(x2, dtype=np.float64)
    s, terms = _entry(i)
    out = np.zeros(np.broadcast(x1, x2).shape)
    for c, a, b in terms:
        out = out + c * x1 ** a * x2 ** b
    return s * out


def grad_phi(i, m, x1, x2):
    """Component m (0 -> d/dx1, 1 -> d/dx2) of grad phi_hat_{i+1}."""
    if i >= len(_TABLE):
        return _collapsed(i, x1, x2, m)
    x1 = np.asarray(x1, dtype=np.float64)
    x2 = np.asarray(x2, dtype=np.float64)
    s, terms = _entry(i)
    out = np.zeros(np.broadcast(x1, x2).shape)
    for c, a, b in terms:
        if m == 0 and a > 0:
            out = out + c * a * x1 ** (a - 1) * x2 ** b
        elif m == 1 and b > 0:
            out = out + c * b * x1 ** a * x2 ** (b - 1)
    return s * out


_KIND = ["paper"]


@contextlib.contextmanager
def use(kind):
    """Select "paper" (the listed functions) or "gram-schmidt" inside a with-block."""
    if kind not in ("paper", "gram-schmidt"):
        raise ValueError(kind)
    old = _KIND[0]
    _KIND[0] = kind
    try:
        yield
    finally:
        _KIND[0] = old


def _monomials(N):
    """Exponents (a, b) of x1^a x2^b by total degree, then by power of x2."""
    p = order_of(N)
    return [(d - b, b) for d in range(p + 1) for b in range(d + 1)]


def _gram_schmidt(N):
    """L^{-1} with G = L L^T, G_kl = integral of m_k m_l over the reference
    triangle, whose monomial integrals are a! b! / (a + b + 2)!; the functions
    L^{-1} m are orthonormal."""
    mono = _monomials(N)
    G = np.array([[factorial(a + c) * factorial(b + d) / factorial(a + b + c + d + 2)
                   for (c, d) in mono] for (a, b) in mono])
    return np.linalg.inv(np.linalg.cholesky(G)), mono


def _gs_all(N, x1, x2, m=None):
    Linv, mono = _gram_schmidt(N)
    x1 = np.asarray(x1, dtype=np.float64)
    x2 = np.asarray(x2, dtype=np.float64)
    cols = []
    for a, b in mono:
        if m is None:
            cols.append(x1 ** a * x2 ** b)
        elif m == 0:
            cols.append(a * x1 ** max(a - 1, 0) * x2 ** b if a > 0 else 0.0 * x1)
        else:
            cols.append(b * x1 ** a * x2 ** max(b - 1, 0) if b > 0 else 0.0 * x1)
    M = np.stack(np.broadcast_arrays(*cols), axis=-1)
    return M @ Linv.T


def phi_all(N, x1, x2):
    """[len(x) x N] matrix of all basis functions at the points."""
    if _KIND[0] == "gram-schmidt":
        return _gs_all(N, x1, x2)
    return np.stack([phi(i, x1, x2) for i in range(N)], axis=-1)


def grad_phi_all(N, x1, x2):
    """[len(x) x N x 2] gradients of all basis functions at the points."""
    if _KIND[0] == "gram-schmidt":
        return np.stack([_gs_all(N, x1, x2, 0), _gs_all(N, x1, x2, 1)], axis=-1)
    return np.stack([np.stack([grad_phi(i, m, x1, x2) for m in range(2)], axis=-1)
                     for i in range(N)], axis=-2)
