"""Mesh input and Lagrange output: the oracle pinned, and the library's host
reader against it (host code only, no GPU needed).

Pins of the oracle:
- the reader returns the Fig. 6 grid of Sec. 3.8 from a hand-written file
  (2D vertex lines, comments, a clockwise triangle, the example's boundary IDs);
- Lagrange values of a projected polynomial of degree <= p equal the
  polynomial at the physical Lagrange points (the projection is exact there),
  for p = 1..4, and the p = 0 value is the triangle mean.
"""
import json
import os

import numpy as np
import pytest

from inputs.meshes import EAST, boundary_sides, delaunay_square, square_mesh, write_medit
from oracle import io as oio
from oracle.ldg import project
from oracle.mesh import Grid
from oracle.refelem import RefTensors

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _fixture():
    with open(os.path.join(GOLDEN, "fig6_two_triangles.json")) as fh:
        return json.load(fh)


def test_oracle_reader_on_the_fig6_file():
    want = _fixture()
    cV, V0T, ids = oio.read_medit(os.path.join(GOLDEN, "fig6_two_triangles.mesh"))
    assert np.array_equal(cV, np.array(want["coordV"]))
    assert np.array_equal(V0T, np.array(want["V0T"]))
    assert np.array_equal(ids, np.array(want["edge_id"]))


def test_oracle_reader_roundtrip_of_an_unstructured_mesh(tmp_path):
    cV, V0T = delaunay_square(9, 31)
    side = boundary_sides(cV, V0T)
    path = str(tmp_path / "d.mesh")
    write_medit(path, cV, V0T, side, reverse=range(0, V0T.shape[0], 3), comment="test mesh")
    rc, rV, rid = oio.read_medit(path)
    assert np.array_equal(rc, cV) and np.array_equal(rV, V0T) and np.array_equal(rid, side)


def _poly(deg):
    rng = np.random.default_rng(deg)
    coef = rng.standard_normal((deg + 1, deg + 1))
    return lambda x, y: sum(coef[a, b] * x ** a * y ** b
                            for a in range(deg + 1) for b in range(deg + 1 - a))


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_lagrange_values_of_projected_polynomials(p):
    cV, V0T, kind = square_mesh(3, seed=41)
    g = Grid(cV, V0T, kind)
    f = _poly(p)
    C = project(g, p, f, RefTensors(p).hatM, order=2 * p + 2)
    L = oio.lagrange_values(C)
    x1, x2 = oio.LAGRANGE_POINTS[L.shape[1]]
    X, Y = g.map_to_physical(x1, x2)
    assert np.abs(L - f(X, Y)).max() < 1e-12


def test_lagrange_value_of_p0_is_the_mean():
    cV, V0T, kind = square_mesh(3, seed=42)
    g = Grid(cV, V0T, kind)
    f = lambda x, y: 1.0 + x + 2.0 * y       # linear: the mean is the value at the barycentre
    C = project(g, 0, f, RefTensors(0).hatM, order=2)
    X, Y = g.map_to_physical(np.array([1 / 3]), np.array([1 / 3]))
    assert np.abs(oio.lagrange_values(C) - f(X, Y)).max() < 1e-13


# ---- the library's host reader (libldg.so, no device calls) -------------------

@pytest.fixture(scope="module")
def lib_io():
    from paper_1408_3877_amd import build
    from paper_1408_3877_amd.ldg import library_path
    if not os.path.exists(library_path()):
        build.build()
    from paper_1408_3877_amd import ldg
    return ldg


def test_library_reader_on_the_fig6_file(lib_io):
    want = _fixture()
    cV, V0T, ids = lib_io.read_mesh_medit(os.path.join(GOLDEN, "fig6_two_triangles.mesh"))
    assert np.array_equal(cV, np.array(want["coordV"]))
    assert np.array_equal(V0T, np.array(want["V0T"]))
    assert np.array_equal(ids, np.array(want["edge_id"]))


@pytest.mark.parametrize("n,seed,dim", [(7, 51, 3), (12, 52, 2), (20, 53, 3)])
def test_library_reader_matches_the_oracle(lib_io, tmp_path, n, seed, dim):
    cV, V0T = delaunay_square(n, seed)
    side = boundary_sides(cV, V0T)
    if n == 12:
        side[side == EAST] = 0                 # the east side's edges listed without an ID
    path = str(tmp_path / "m.mesh")
    write_medit(path, cV, V0T, side, reverse=range(1, V0T.shape[0], 2), dim=dim)
    want = oio.read_medit(path)
    got = lib_io.read_mesh_medit(path)
    for a, b in zip(got, want):
        assert np.array_equal(a, b)
    if n == 12:
        assert np.sum(got[2] == -1) == np.sum(boundary_sides(cV, V0T) == EAST)


def test_edge_kinds_from_ids(lib_io):
    ids = np.array([[0, 3, 1], [4, 0, 2], [2, 2, 0]], np.int32)
    kind = lib_io.edge_kinds_from_ids(ids, neumann_ids=(1, 3))
    assert np.array_equal(kind, np.array([[0, 2, 2], [1, 0, 1], [1, 1, 0]], np.int8))
    with pytest.raises(lib_io.LdgError) as e:
        lib_io.edge_kinds_from_ids(np.array([[0, -1, 1]], np.int32))
    assert e.value.code == -2


def test_library_reader_errors(lib_io, tmp_path):
    with pytest.raises(lib_io.LdgError) as e:
        lib_io.read_mesh_medit(str(tmp_path / "missing.mesh"))
    assert e.value.code == -7
    bad = tmp_path / "bad.mesh"
    bad.write_text("MeshVersionFormatted 2\nDimension 3\nVertices\n3\n0 0 0 0\n1 0 0 0\n0 1 0 0\n"
                   "Triangles\n1\n1 2 4 0\nEnd\n")
    with pytest.raises(lib_io.LdgError) as e:
        lib_io.read_mesh_medit(str(bad))
    assert e.value.code == -2 and "out of range" in str(e.value)
