"""Brute-force pins of the oracle's global blocks.

Every block entry is recomputed here from its component-wise definition in
Sec. 2.4.3-2.4.4 by quadrature on the physical triangles and edges: the
basis of T_k is evaluated through the inverse of the affine map computed
from the vertices, neighbour traces go through the neighbour's own inverse
map (no reference edge maps), normals come from the edge direction and the
opposite vertex.  The oracle instead uses reference tensors, edge maps and
the transformation rules of Sec. 3.6, so a dropped term, a wrong sign, a
wrong normal or a transposed operand in it fails here.
"""
import numpy as np
import pytest

from inputs.meshes import two_triangle_mesh, square_mesh, SOUTH, NORTH, EAST
from oracle import basis
from oracle.ldg import Blocks, boundary_vectors
from oracle.mesh import Grid
from oracle.quadrature import collapsed_rule, gauss_legendre_01, rule_1d
from oracle.refelem import RefTensors


class Brute:
    def __init__(self, coordV, V0T, kind, p):
        self.cV, self.V0T, self.kind, self.p = coordV, V0T, kind, p
        self.N = basis.num_basis(p)
        self.K = V0T.shape[0]

    def verts(self, k):
        return self.cV[self.V0T[k]]

    def ref_coords(self, k, X):
        a = self.verts(k)
        Bm = np.column_stack([a[1] - a[0], a[2] - a[0]])
        return np.linalg.solve(Bm, (X - a[0]).T), Bm

    def phys_phi(self, k, X):
        xh, _ = self.ref_coords(k, X)
        return basis.phi_all(self.N, xh[0], xh[1])               # [R x N]

    def phys_grad(self, k, X):
        xh, Bm = self.ref_coords(k, X)
        g = basis.grad_phi_all(self.N, xh[0], xh[1])             # [R x N x 2] (hat grads)
        return np.einsum("ab,rib->ria", np.linalg.inv(Bm).T, g)  # B^{-T} grad_hat

    def vol_rule(self, k, n=8):
        a = self.verts(k)
        q1, q2, w = collapsed_rule(n)
        X = np.outer(1 - q1 - q2, a[0]) + np.outer(q1, a[1]) + np.outer(q2, a[2])
        e1, e2 = a[1] - a[0], a[2] - a[0]
        area = 0.5 * abs(e1[0] * e2[1] - e1[1] * e2[0])
        return X, 2 * area * w

    def edges(self, k):
        """(n, P, Q, normal, length, neighbour k+ or -1)"""
        out = []
        for n in range(3):
            i1, i2 = self.V0T[k, (n + 1) % 3], self.V0T[k, (n + 2) % 3]
            P, Q = self.cV[i1], self.cV[i2]
            t = Q - P
            L = np.hypot(*t)
            nu = np.array([t[1], -t[0]]) / L
            opp = self.cV[self.V0T[k, n]]
            if np.dot(nu, opp - P) > 0:
                nu = -nu
            kp = -1
            for k2 in range(self.K):
                if k2 != k and {i1, i2} <= set(self.V0T[k2].tolist()):
                    kp = k2
            out.append((n, P, Q, nu, L, kp))
        return out

    def edge_rule(self, P, Q, R=10):
        s, w = gauss_legendre_01(R)
        return P[None] + s[:, None] * (Q - P)[None], w * np.hypot(*(Q - P))


def _dense(sp_mat):
    return np.asarray(sp_mat.todense())


def _meshes():
    out = [two_triangle_mesh()]
    cV, V0T, kind = square_mesh(2, seed=11, neumann_sides=(SOUTH, NORTH))
    out.append((cV, V0T, kind))
    cV, V0T, kind = square_mesh(3, seed=12, neumann_sides=(EAST,))
    out.append((cV, V0T, kind))
    return out


@pytest.mark.parametrize("p", [1, 2, 4, 5])
@pytest.mark.parametrize("mi", [0, 1, 2])
def test_blocks_match_definitions(p, mi):
    cV, V0T, kind = _meshes()[mi]
    rng = np.random.default_rng(100 + p + 10 * mi)
    bf = Brute(cV, V0T, kind, p)
    K, N = bf.K, bf.N
    D = rng.standard_normal((K, N))
    ob = Blocks(Grid(cV, V0T, kind), RefTensors(p, "exact"), D)
    KN = K * N
    M = np.zeros((KN, KN)); S = np.zeros((KN, KN)); SD = np.zeros((KN, KN))
    H = np.zeros((2, KN, KN)); G = np.zeros((2, KN, KN)); Q = np.zeros((2, KN, KN))
    QN = np.zeros((2, KN, KN)); R = np.zeros((2, KN, KN)); RD = np.zeros((2, KN, KN))
    for k in range(K):
        sk = slice(k * N, (k + 1) * N)
        X, w = bf.vol_rule(k)
        P_ = bf.phys_phi(k, X)
        dP = bf.phys_grad(k, X)
        dh = P_ @ D[k]                                           # d_h on T_k
        M[sk, sk] = np.einsum("r,ri,rj->ij", w, P_, P_)
        for m in range(2):
            H[m, sk, sk] = np.einsum("r,ri,rj->ij", w, dP[:, :, m], P_)
            G[m, sk, sk] = np.einsum("r,ri,rj->ij", w * dh, dP[:, :, m], P_)
        for (n, Pa, Qa, nu, L, kp) in bf.edges(k):
            Xe, we = bf.edge_rule(Pa, Qa)
            Pm = bf.phys_phi(k, Xe)
            dm = Pm @ D[k]
            mm = np.einsum("r,ri,rj->ij", we, Pm, Pm)
            mmd = np.einsum("r,ri,rj->ij", we * dm, Pm, Pm)
            if kind[k, n] == 0:
                assert kp >= 0
                spl = slice(kp * N, (kp + 1) * N)
                Pp = bf.phys_phi(kp, Xe)
                dp = Pp @ D[kp]
                mp = np.einsum("r,ri,rj->ij", we, Pm, Pp)
                mpd = np.einsum("r,ri,rj->ij", we * dp, Pm, Pp)
                S[sk, sk] += mm / L
                S[sk, spl] += -mp / L
                for m in range(2):
                    Q[m, sk, sk] += 0.5 * nu[m] * mm
                    Q[m, sk, spl] += 0.5 * nu[m] * mp
                    R[m, sk, sk] += 0.5 * nu[m] * mmd
                    R[m, sk, spl] += 0.5 * nu[m] * mpd
            elif kind[k, n] == 1:
                SD[sk, sk] += mm / L
                for m in range(2):
                    RD[m, sk, sk] += nu[m] * mmd
            else:
                for m in range(2):
                    QN[m, sk, sk] += nu[m] * mm
    tol = 1e-11 * max(1.0, np.abs(D).max())
    np.testing.assert_allclose(_dense(ob.M), M, atol=tol)
    np.testing.assert_allclose(_dense(ob.S), S, atol=tol)
    np.testing.assert_allclose(_dense(ob.SD), SD, atol=tol)
    for m in range(2):
        np.testing.assert_allclose(_dense(ob.H[m]), H[m], atol=tol)
        np.testing.assert_allclose(_dense(ob.G[m]), G[m], atol=tol)
        np.testing.assert_allclose(_dense(ob.Q[m]), Q[m], atol=tol)
        np.testing.assert_allclose(_dense(ob.QN[m]), QN[m], atol=tol)
        np.testing.assert_allclose(_dense(ob.R[m]), R[m], atol=tol)
        np.testing.assert_allclose(_dense(ob.RD[m]), RD[m], atol=tol)


@pytest.mark.parametrize("p", [0, 2, 3])
def test_boundary_vectors_match_definitions(p):
    cV, V0T, kind = square_mesh(3, seed=5, neumann_sides=(SOUTH, NORTH))
    rng = np.random.default_rng(3)
    bf = Brute(cV, V0T, kind, p)
    K, N = bf.K, bf.N
    D = rng.standard_normal((K, N))
    cD = lambda x, y: np.sin(3 * x + 1) * np.cos(2 * y)
    gN = lambda x, y, n1, n2: (x ** 2 + y) * n1 - np.cos(x) * n2
    J1, J2, KD, KN = boundary_vectors(Grid(cV, V0T, kind), p, cD, gN, D)
    s, ws = rule_1d(2 * p + 1)
    eJ = np.zeros((2, K, N)); eKD = np.zeros((K, N)); eKN = np.zeros((K, N))
    for k in range(K):
        for (n, Pa, Qa, nu, L, kp) in bf.edges(k):
            Xe = Pa[None] + s[:, None] * (Qa - Pa)[None]
            we = ws * L
            Pm = bf.phys_phi(k, Xe)
            if kind[k, n] == 1:
                cv = cD(Xe[:, 0], Xe[:, 1])
                for m in range(2):
                    eJ[m, k] += nu[m] * (we * cv) @ Pm                 # eq:globJm:D
                eKD[k] += (we * cv) @ Pm / L                           # eq:globK:D
            elif kind[k, n] == 2:
                gv = gN(Xe[:, 0], Xe[:, 1], nu[0], nu[1])
                eKN[k] += (we * gv * (Pm @ D[k])) @ Pm                 # K_N
    np.testing.assert_allclose(J1, eJ[0], atol=1e-13)
    np.testing.assert_allclose(J2, eJ[1], atol=1e-13)
    np.testing.assert_allclose(KD, eKD, atol=1e-13)
    np.testing.assert_allclose(KN, eKN, atol=1e-12)
