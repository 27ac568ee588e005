"""Grid lists of Table 1 (Sec. 3.1) built from vertex coordinates and the
counter-clockwise triangle vertex list.

Local edge n (0-based) of T_k joins local vertices n+1 and n+2 (mod 3), the
edge opposite vertex n, traversed counter-clockwise, exactly as reference
edge n is traversed by gamma_n.  The exterior unit normal of that edge is
its direction vector rotated by -pi/2.
"""
import numpy as np

INTERIOR, DIRICHLET, NEUMANN = 0, 1, 2


class MeshError(ValueError):
    pass


class Grid:
    def __init__(self, coordV, V0T, kind):
        self.coordV = np.asarray(coordV, dtype=np.float64)
        self.V0T = np.asarray(V0T, dtype=np.int64)
        self.kind = np.asarray(kind, dtype=np.int64)
        K = self.numT = self.V0T.shape[0]
        a = self.coordV[self.V0T]                        # coordV0T [K x 3 x 2]
        self.coordV0T = a
        # B_k = [a2 - a1 | a3 - a1]  (eq:affinemappings:Fk); B[k, r, c]
        self.B = np.stack([a[:, 1] - a[:, 0], a[:, 2] - a[:, 0]], axis=2)
        detB = self.B[:, 0, 0] * self.B[:, 1, 1] - self.B[:, 0, 1] * self.B[:, 1, 0]
        if np.any(detB <= 0):
            raise MeshError("triangle with non-positive orientation (must be CCW)")
        self.areaT = detB / 2                            # det B_k = 2 |T_k|
        vs = self.V0T[:, [1, 2, 0]]                      # start vertex of local edge n
        ve = self.V0T[:, [2, 0, 1]]                      # end vertex of local edge n
        vec = self.coordV[ve] - self.coordV[vs]          # [K x 3 x 2]
        self.areaE0T = np.sqrt(vec[..., 0] ** 2 + vec[..., 1] ** 2)
        self.nuE0T = np.stack([vec[..., 1], -vec[..., 0]], axis=-1) / self.areaE0T[..., None]
        # neighbours: local edges with the same vertex pair (sorted by a pair key)
        self.kp = -np.ones((K, 3), dtype=np.int64)
        self.np_ = -np.ones((K, 3), dtype=np.int64)
        lo = np.minimum(vs, ve).reshape(-1)
        hi = np.maximum(vs, ve).reshape(-1)
        key = lo * (self.coordV.shape[0] + 1) + hi
        order = np.argsort(key, kind="stable")
        ks = key[order]
        same = ks[1:] == ks[:-1]
        if np.any(same[1:] & same[:-1]):
            raise MeshError("edge shared by more than two triangles")
        first, second = order[:-1][same], order[1:][same]
        k1, n1 = first // 3, first % 3
        k2, n2 = second // 3, second % 3
        if np.any(vs[k1, n1] != ve[k2, n2]):
            raise MeshError("neighbouring triangles with inconsistent orientation")
        self.kp[k1, n1], self.np_[k1, n1] = k2, n2
        self.kp[k2, n2], self.np_[k2, n2] = k1, n1
        interior = self.kp >= 0
        if np.any(interior != (self.kind == INTERIOR)):
            raise MeshError("edge kinds disagree with the topology")

    def map_to_physical(self, x1, x2, elems=None):
        """F_k(x_hat) for all k (or the triangles `elems`): X1, X2 of shape [K x len(x1)]."""
        x1 = np.atleast_1d(x1)
        x2 = np.atleast_1d(x2)
        el = slice(None) if elems is None else np.asarray(elems)
        B, a = self.B[el], self.coordV0T[el]
        X1 = B[:, 0, 0:1] * x1 + B[:, 0, 1:2] * x2 + a[:, 0, 0:1]
        X2 = B[:, 1, 0:1] * x1 + B[:, 1, 1:2] * x2 + a[:, 0, 1:2]
        return X1, X2
