"""Structured (Friedrichs-Keller) triangulations of the unit square.

The vertex and triangle numbering follows the paper's ``domainSquare``
description (Sec. 3.1.2 and the routine register): vertices on an
(n+1) x (n+1) grid numbered with the y index fastest, every square cell
split along the diagonal from (x+h, y) to (x, y+h), all "lower-left"
triangles first and all "upper-right" triangles after them, every triangle
counter-clockwise.  Boundary kinds are given per local edge, local edge n
lying opposite local vertex n (Fig. 3, eq:gammaMap).
"""
import numpy as np

INTERIOR, DIRICHLET, NEUMANN = 0, 1, 2

# side ids as in the paper's domainSquare: 1 south, 2 east, 3 north, 4 west
SOUTH, EAST, NORTH, WEST = 1, 2, 3, 4


def fk_square(n):
    """Return (coordV [numV x 2], V0T [K x 3] int32, 0-based) for n x n cells."""
    h = 1.0 / n
    g = np.arange(n + 1) * h
    # vertex index v = i + (n+1) j  <->  (x_j, y_i)
    X, Y = np.meshgrid(g, g, indexing="xy")          # X[i, j] = x_j, Y[i, j] = y_i
    coordV = np.stack([X.T.reshape(-1), Y.T.reshape(-1)], axis=1)
    i, j = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    base = (i + (n + 1) * j).T.reshape(-1)          # j outer, i inner
    lower = np.stack([base, base + n + 1, base + 1], axis=1)
    upper = np.stack([base + n + 1, base + n + 2, base + 1], axis=1)
    V0T = np.concatenate([lower, upper], axis=0).astype(np.int32)
    return coordV.astype(np.float64), V0T


def fk_cells(n):
    """(ix, iy): the square cell of every triangle of fk_square(n) (x index, y index)."""
    i, j = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    iy = i.T.reshape(-1)                              # j outer, i inner
    ix = j.T.reshape(-1)
    return np.concatenate([ix, ix]), np.concatenate([iy, iy])


def jitter(coordV, n, seed, amp=0.2):
    """Move every interior vertex by i.i.d. U[-amp*h, amp*h] per coordinate."""
    h = 1.0 / n
    rng = np.random.default_rng(seed)
    c = coordV.copy()
    xs, ys = c[:, 0], c[:, 1]
    interior = (xs > 0.5 * h) & (xs < 1 - 0.5 * h) & (ys > 0.5 * h) & (ys < 1 - 0.5 * h)
    d = rng.uniform(-amp * h, amp * h, size=c.shape)
    c[interior] += d[interior]
    return c


def boundary_sides(coordV, V0T):
    """Per local edge: 0 if interior, else the side id (1..4) of the boundary edge.

    Local edge n joins local vertices n+1 and n+2 (mod 3)."""
    K = V0T.shape[0]
    a = V0T[:, [1, 2, 0]]
    b = V0T[:, [2, 0, 1]]
    lo = np.minimum(a, b).astype(np.int64)
    hi = np.maximum(a, b).astype(np.int64)
    key = lo * (coordV.shape[0] + 1) + hi
    flat = key.reshape(-1)
    _, inv, cnt = np.unique(flat, return_inverse=True, return_counts=True)
    bnd = (cnt[inv] == 1).reshape(K, 3)
    mid = 0.5 * (coordV[a] + coordV[b])              # K x 3 x 2
    side = np.zeros((K, 3), dtype=np.int8)
    tol = 1e-12
    side[bnd & (np.abs(mid[..., 1]) < tol)] = SOUTH
    side[bnd & (np.abs(mid[..., 0] - 1) < tol)] = EAST
    side[bnd & (np.abs(mid[..., 1] - 1) < tol)] = NORTH
    side[bnd & (np.abs(mid[..., 0]) < tol)] = WEST
    if np.any(bnd & (side == 0)):
        raise ValueError("boundary edge not on a side of the unit square")
    return side


def edge_kinds(coordV, V0T, neumann_sides=()):
    """Per local edge kind: 0 interior, 1 Dirichlet, 2 Neumann (int8, K x 3)."""
    side = boundary_sides(coordV, V0T)
    kind = np.where(side > 0, DIRICHLET, INTERIOR).astype(np.int8)
    for s in neumann_sides:
        kind[side == s] = NEUMANN
    return kind


def square_mesh(n, seed=None, neumann_sides=(), amp=0.2):
    """FK mesh of the unit square with n x n cells, optionally jittered."""
    coordV, V0T = fk_square(n)
    if seed is not None:
        coordV = jitter(coordV, n, seed, amp)
    return coordV, V0T, edge_kinds(coordV, V0T, neumann_sides)


def two_triangle_mesh():
    """The two-triangle grid of the visualization example (Sec. 3.8, Fig. 6).

    Returns 0-based (coordV, V0T); all edges are boundary edges (Dirichlet)."""
    s3 = np.sqrt(3.0)
    coordV = np.array([[0.0, -1.0], [s3, 0.0], [0.0, 1.0], [-s3, 0.0]])
    V0T = np.array([[3, 0, 2], [0, 1, 2]], dtype=np.int32)
    kind = np.ones((2, 3), dtype=np.int8)
    # the shared edge (vertices 0 and 2) is interior in both triangles
    for k in range(2):
        for n in range(3):
            e = {int(V0T[k, (n + 1) % 3]), int(V0T[k, (n + 2) % 3])}
            if e == {0, 2}:
                kind[k, n] = INTERIOR
    return coordV, V0T, kind


def rotate_local_numbering(V0T, kind, seed, fraction=0.5):
    """Start the counter-clockwise vertex list of a random subset of triangles
    at another vertex: the mesh is unchanged, the local vertex and edge numbers
    (and hence the neighbour edge index n+) vary from triangle to triangle."""
    rng = np.random.default_rng(seed)
    K = V0T.shape[0]
    shift = np.where(rng.random(K) < fraction, rng.integers(1, 3, K), 0)
    idx = (np.arange(3)[None, :] + shift[:, None]) % 3
    return (np.take_along_axis(V0T, idx, axis=1).astype(np.int32),
            np.take_along_axis(kind, idx, axis=1).astype(np.int8))


def delaunay_square(n, seed, amp=0.35):
    """Unstructured triangulation of the unit square: the Delaunay
    triangulation (scipy.spatial) of an (n+1) x (n+1) point grid whose interior
    points are moved by i.i.d. U[-amp*h, amp*h] per coordinate.  Boundary
    points stay on the sides.  Returns (coordV, V0T) with counter-clockwise
    triangles; the connectivity is not the Friedrichs-Keller pattern."""
    from scipy.spatial import Delaunay
    h = 1.0 / n
    g = np.arange(n + 1) * h
    X, Y = np.meshgrid(g, g, indexing="ij")
    pts = np.stack([X.reshape(-1), Y.reshape(-1)], axis=1)
    rng = np.random.default_rng(seed)
    interior = (pts[:, 0] > 0.5 * h) & (pts[:, 0] < 1 - 0.5 * h) & \
               (pts[:, 1] > 0.5 * h) & (pts[:, 1] < 1 - 0.5 * h)
    d = rng.uniform(-amp * h, amp * h, size=pts.shape)
    pts[interior] += d[interior]
    tri = Delaunay(pts).simplices.astype(np.int32)
    a, b, c = pts[tri[:, 0]], pts[tri[:, 1]], pts[tri[:, 2]]
    det = (b[:, 0] - a[:, 0]) * (c[:, 1] - a[:, 1]) - (c[:, 0] - a[:, 0]) * (b[:, 1] - a[:, 1])
    tri[det < 0] = tri[det < 0][:, [0, 2, 1]]
    keep = np.abs(det) > 1e-14                       # drop degenerate hull slivers
    return pts, np.ascontiguousarray(tri[keep])


def write_medit(path, coordV, V0T, side_ids, reverse=(), dim=3, comment=None):
    """Write a triangulation as an ASCII MEDIT .mesh file (the format Gmsh
    writes): 1-based vertices, the boundary edges with their side ids in
    "Edges" (side_ids: K x 3 per local edge, 0 interior), the triangles with
    reference 0; triangles listed in `reverse` are written clockwise."""
    rev = np.zeros(V0T.shape[0], bool)
    rev[list(reverse)] = True
    lines = []
    if comment:
        lines.append("# " + comment)
    lines += ["MeshVersionFormatted 2", "Dimension", str(dim), "Vertices", str(len(coordV))]
    for x, y in coordV:
        lines.append(("%r %r 0 0" if dim == 3 else "%r %r 0") % (float(x), float(y)))
    edges = []
    for k in range(V0T.shape[0]):
        for n in range(3):
            if side_ids[k, n] > 0:
                edges.append((V0T[k, (n + 1) % 3] + 1, V0T[k, (n + 2) % 3] + 1, side_ids[k, n]))
    lines += ["Edges", str(len(edges))] + ["%d %d %d" % e for e in edges]
    lines += ["Triangles", str(V0T.shape[0])]
    for k, t in enumerate(V0T + 1):
        t = t[[0, 2, 1]] if rev[k] else t
        lines.append("%d %d %d 0" % tuple(t))
    lines.append("End")
    with open(path, "w") as fh:
        fh.write("\n".join(lines) + "\n")


def pair_numbering(V0T, kind):
    """Renumber the triangles so that most follow a neighbour: walk the triangles
    in their order and put each unplaced one right after the previous, followed
    by its first unplaced neighbour (local edges 0, 1, 2).  On fk_square meshes
    this pairs the two triangles of every cell (the diagonal is local edge 0 of
    the lower one), cells in their original order.  Returns (V0T, kind, order)
    with row i of the result = row order[i] of the input."""
    V0T = np.asarray(V0T)
    K = V0T.shape[0]
    owner = {}
    nbr = -np.ones((K, 3), dtype=np.int64)
    for k in range(K):
        for n in range(3):
            a, b = int(V0T[k, (n + 1) % 3]), int(V0T[k, (n + 2) % 3])
            key = (min(a, b), max(a, b))
            if key in owner:
                j = owner.pop(key)
                nbr[k, n], nbr[j[0], j[1]] = j[0], k
            else:
                owner[key] = (k, n)
    placed = np.zeros(K, dtype=bool)
    order = []
    for k in range(K):
        if placed[k]:
            continue
        placed[k] = True
        order.append(k)
        for n in range(3):
            j = nbr[k, n]
            if j >= 0 and not placed[j]:
                placed[j] = True
                order.append(int(j))
                break
    order = np.array(order, dtype=np.int64)
    return (np.ascontiguousarray(V0T[order]).astype(np.int32),
            np.ascontiguousarray(np.asarray(kind)[order]).astype(np.int8), order)


def split_at_centroids(coordV, V0T, which):
    """Split the listed triangles at their centroids into three triangles each
    (counter-clockwise, the new vertex last): every split adds an interior
    vertex of degree three, whose three triangles are pairwise neighbours.
    Returns (coordV, V0T) with the unsplit triangles first, in order."""
    coordV = np.asarray(coordV, dtype=np.float64)
    V0T = np.asarray(V0T)
    which = np.asarray(sorted(set(int(k) for k in which)))
    keep = np.setdiff1d(np.arange(V0T.shape[0]), which)
    cen = coordV[V0T[which]].mean(axis=1)
    base = coordV.shape[0]
    new = []
    for i, k in enumerate(which):
        a, b, c = (int(v) for v in V0T[k])
        m = base + i
        new += [[a, b, m], [b, c, m], [c, a, m]]
    return (np.concatenate([coordV, cen]),
            np.concatenate([V0T[keep], np.array(new, dtype=V0T.dtype).reshape(-1, 3)]).astype(np.int32))
