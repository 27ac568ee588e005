"""Input and output of the method, written out plainly (test infrastructure).

This module belongs to the FP64 CPU oracle: only the tests and the benchmark's
CPU baseline use it; the library never imports it.

- `lagrange_values`: the change from the modal DG representation to values at
  the Lagrange points of each triangle used for visualization (Sec. 3.8): the
  barycentre for p = 0, the vertices for p = 1, the vertices and the edge
  barycentres for p >= 2 (for p > 2 the order-p function sampled at those six
  points, the visualization holding at most quadratics).
- `read_medit`: the MEDIT ".mesh" format of Gmsh as the paper's circle-domain
  generator reads it (Sec. 4): vertex coordinates, triangles, and the boundary
  ID of every listed boundary edge, returned per local edge.
"""
import numpy as np

from . import basis

# reference coordinates of the Lagrange points (Sec. 3.8): vertices a1, a2, a3
# of the reference triangle, then the barycentres of the edges opposite a1, a2, a3
LAGRANGE_POINTS = {
    1: (np.array([1.0 / 3.0]), np.array([1.0 / 3.0])),
    3: (np.array([0.0, 1.0, 0.0]), np.array([0.0, 0.0, 1.0])),
    6: (np.array([0.0, 1.0, 0.0, 0.5, 0.0, 0.5]), np.array([0.0, 0.0, 1.0, 0.5, 0.5, 0.0])),
}


def lagrange_values(C):
    """K x nL values of the functions with modal coefficients C (K x N)."""
    N = C.shape[1]
    nL = N if N in (1, 3) else 6
    x1, x2 = LAGRANGE_POINTS[nL]
    return C @ basis.phi_all(N, x1, x2).T


def read_medit(path):
    """(coordV numV x 2, V0T K x 3 0-based counter-clockwise, edge_id K x 3)."""
    with open(path) as fh:
        words = []
        for line in fh:
            words += line.split("#", 1)[0].split()
    pos, dim = 0, 3
    coordV = V0T = None
    edges = []
    while pos < len(words):
        w = words[pos]
        pos += 1
        if w == "Dimension":
            dim = int(words[pos])
            pos += 1
        elif w == "Vertices":
            nv = int(words[pos])
            pos += 1
            rows = []
            for _ in range(nv):
                rows.append([float(words[pos]), float(words[pos + 1])])
                pos += dim + 1
            coordV = np.array(rows)
        elif w == "Edges":
            ne = int(words[pos])
            pos += 1
            for _ in range(ne):
                a, b, i = (int(x) for x in words[pos:pos + 3])
                edges.append((a - 1, b - 1, i))
                pos += 3
        elif w == "Triangles":
            nt = int(words[pos])
            pos += 1
            rows = []
            for _ in range(nt):
                rows.append([int(x) - 1 for x in words[pos:pos + 3]])
                pos += 4
            V0T = np.array(rows, dtype=np.int64)
        elif w == "End":
            break
    # counter-clockwise: swap the last two vertices where det B_k < 0
    for t in V0T:
        a, b, c = coordV[t[0]], coordV[t[1]], coordV[t[2]]
        if (b[0] - a[0]) * (c[1] - a[1]) - (c[0] - a[0]) * (b[1] - a[1]) < 0:
            t[1], t[2] = t[2], t[1]
    # edge_id per local edge n (vertices n+1, n+2): 0 interior, listed ID, or -1
    count = {}
    for t in V0T:
        for n in range(3):
            e = frozenset((int(t[(n + 1) % 3]), int(t[(n + 2) % 3])))
            count[e] = count.get(e, 0) + 1
    ids = {frozenset((a, b)): i for a, b, i in edges}
    edge_id = np.zeros(V0T.shape, dtype=np.int64)
    for k, t in enumerate(V0T):
        for n in range(3):
            e = frozenset((int(t[(n + 1) % 3]), int(t[(n + 2) % 3])))
            if count[e] == 1:
                edge_id[k, n] = ids.get(e, -1)
    return coordV, V0T, edge_id
