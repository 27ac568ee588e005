"""Reference-triangle edge maps and reference tensors (Sec. 3.6).

Edges are 0-based here (the paper's E_hat_{n+1}); edge n lies opposite
vertex n of the reference triangle with vertices (0,0), (1,0), (0,1).

Tensors, index order as in the paper (0-based):
  hatM[i,j]              eq:hatM          int phi_i phi_j
  hatH[i,j,m]            eq:hatH          int d_m phi_i phi_j
  hatG[i,j,l,m]          eq:hatG          int d_m phi_i phi_j phi_l
  hatSdiag[i,j,n]        eq:hatSdiag      int_0^1 phi_i(g_n) phi_j(g_n) ds
  hatSoff[i,j,n-,n+]     eq:hatSoffdiag   int_0^1 phi_i(g_n-) phi_j(theta(g_n-)) ds
  hatRdiag[i,j,l,n]      eq:hatRdiag      int_0^1 phi_i phi_l phi_j on edge n
  hatRoff[i,j,l,n-,n+]   eq:hatRoffdiag   int_0^1 phi_i(g_n-) phi_l(theta) phi_j(theta) ds

Policy "exact" integrates every tensor exactly (the integrands are
polynomials of degree <= 3p-1 on the triangle and <= 3p on edges); policy
"paper" uses the rules the paper's routines use (order 2p on the triangle,
2p+1 on edges), which under-integrates hatG and hatR for p >= 2.
"""
import numpy as np

from . import basis
from .quadrature import collapsed_rule, rule_1d, triangle_rule


def gamma(n, s):
    """Parametrisation of reference edge n over s in [0,1] (eq:gammaMap)."""
    s = np.asarray(s, dtype=np.float64)
    if n == 0:
        return 1 - s, s
    if n == 1:
        return np.zeros_like(s), 1 - s
    if n == 2:
        return s, np.zeros_like(s)
    raise ValueError(n)


def theta(nm, npl, x1, x2):
    """Map from reference edge nm onto reference edge npl (eq:mapEE)."""
    x1 = np.asarray(x1, dtype=np.float64)
    x2 = np.asarray(x2, dtype=np.float64)
    z = np.zeros_like(x1)
    table = {
        (0, 0): (1 - x1, 1 - x2), (0, 1): (z, x2), (0, 2): (x1, z),
        (1, 0): (1 - x2, x2), (1, 1): (z, 1 - x2), (1, 2): (x2, z),
        (2, 0): (x1, 1 - x1), (2, 1): (z, x1), (2, 2): (1 - x1, z),
    }
    return table[(nm, npl)]


def _rules(p, policy):
    if policy == "exact":
        tri = collapsed_rule(max(2, (3 * p + 2) // 2 + 1))
        edge = rule_1d(3 * p + 1)
    elif policy == "paper":
        tri = triangle_rule(max(2 * p, 1))
        edge = rule_1d(2 * p + 1)
    else:
        raise ValueError(policy)
    return tri, edge


class RefTensors:
    """All reference tensors of order p under a quadrature policy."""

    def __init__(self, p, policy="exact"):
        self.p = p
        self.N = N = basis.num_basis(p)
        self.policy = policy
        (q1, q2, w), (s, ws) = _rules(p, policy)
        Phi = basis.phi_all(N, q1, q2)                   # [R x N]
        dPhi = basis.grad_phi_all(N, q1, q2)             # [R x N x 2]
        self.hatM = np.einsum("r,ri,rj->ij", w, Phi, Phi)
        self.hatH = np.einsum("r,rim,rj->ijm", w, dPhi, Phi)
        self.hatG = np.einsum("r,rim,rj,rl->ijlm", w, dPhi, Phi, Phi)
        self.hatSdiag = np.zeros((N, N, 3))
        self.hatRdiag = np.zeros((N, N, N, 3))
        self.hatSoff = np.zeros((N, N, 3, 3))
        self.hatRoff = np.zeros((N, N, N, 3, 3))
        for nm in range(3):
            x1, x2 = gamma(nm, s)
            Pin = basis.phi_all(N, x1, x2)               # phi_i(gamma_n(s))
            self.hatSdiag[:, :, nm] = np.einsum("r,ri,rj->ij", ws, Pin, Pin)
            self.hatRdiag[:, :, :, nm] = np.einsum("r,ri,rl,rj->ijl", ws, Pin, Pin, Pin)
            for npl in range(3):
                y1, y2 = theta(nm, npl, x1, x2)
                Pex = basis.phi_all(N, y1, y2)           # phi_j(theta(gamma_n-(s)))
                self.hatSoff[:, :, nm, npl] = np.einsum("r,ri,rj->ij", ws, Pin, Pex)
                self.hatRoff[:, :, :, nm, npl] = np.einsum("r,ri,rl,rj->ijl", ws, Pin, Pex, Pex)
