"""Input and output through the library on the GPU.

- Lagrange values (Sec. 3.8) computed on the device match the oracle's, for
  the state and for given coefficients, p = 0..4;
- the .vtu files (ASCII and base64) hold the triangles' points, the cell
  types and the values the oracle gives, rounded to FP32;
- an unstructured (Delaunay) mesh written as a MEDIT file, read back by the
  library and stepped on the device, matches the oracle's steps on the mesh
  the oracle's own reader returns.
"""
import base64
import xml.etree.ElementTree as ET

import numpy as np
import pytest

from inputs.fields import SMOOTH2, Workload
from inputs.meshes import NORTH, SOUTH, boundary_sides, delaunay_square, square_mesh, write_medit
from oracle import io as oio
from oracle.ldg import Problem
from tests.gpu_common import rel_l2, to_np

pytestmark = pytest.mark.gpu


def _solver(cV, V0T, kind, p, **kw):
    from paper_1408_3877_amd import Solver
    return Solver(cV, V0T, kind, p, rtol=1e-13, max_iters=50000, restart=60, **kw)


@pytest.mark.parametrize("p", [0, 1, 2, 3, 4])
def test_lagrange_values_match_the_oracle(p):
    cV, V0T, kind = square_mesh(9, seed=600 + p)     # K = 162: several tiles and a ragged tail
    s = _solver(cV, V0T, kind, p)
    rng = np.random.default_rng(p)
    C = rng.standard_normal((s.K, s.N))
    want = oio.lagrange_values(C)
    got = to_np(s.lagrange(C))
    assert got.shape == want.shape
    assert np.abs(got - want).max() <= 1e-14 * np.abs(want).max()
    s.set_state(C, 0.0)                             # the state goes through the tiled layout
    assert np.abs(to_np(s.lagrange()) - want).max() <= 1e-14 * np.abs(want).max()


def _arrays(root, binary):
    out = {}
    for da in root.iter("DataArray"):
        name = da.get("Name") or "Points"
        typ = {"Float32": np.float32, "Int32": np.int32, "UInt8": np.uint8}[da.get("type")]
        text = da.text.strip()
        if binary:
            raw = base64.b64decode(text)
            nb = np.frombuffer(raw[:4], np.uint32)[0]
            vals = np.frombuffer(raw[4:4 + nb], typ)
        else:
            vals = np.array(text.split(), dtype=np.float64).astype(typ)
        out[name] = vals
    return out


@pytest.mark.parametrize("p,binary", [(0, False), (1, True), (2, False), (4, True)])
def test_vtu_files_hold_the_lagrange_values(tmp_path, p, binary):
    cV, V0T, kind = square_mesh(5, seed=610)
    s = _solver(cV, V0T, kind, p)
    C = np.random.default_rng(610 + p).standard_normal((s.K, s.N))
    s.set_state(C, 0.0)
    path = str(tmp_path / "c.1.vtu")
    s.write_vtu(path, "c_h", s.lagrange(), binary=binary)
    root = ET.parse(path).getroot()
    piece = root.find("UnstructuredGrid/Piece")
    K = s.K
    nL = oio.lagrange_values(C).shape[1]
    np_ = 6 if nL == 6 else 3
    assert int(piece.get("NumberOfCells")) == K and int(piece.get("NumberOfPoints")) == np_ * K
    a = _arrays(root, binary)
    assert np.array_equal(a["connectivity"], np.arange(np_ * K))
    assert np.array_equal(a["offsets"], np_ * np.arange(1, K + 1))
    assert np.all(a["types"] == (22 if nL == 6 else 5))
    # points: the corners, then the midpoints of (v1 v2), (v2 v3), (v3 v1)
    corners = cV[V0T]                                 # K x 3 x 2
    pts = [corners[:, 0], corners[:, 1], corners[:, 2]]
    if np_ == 6:
        pts += [0.5 * (corners[:, 0] + corners[:, 1]), 0.5 * (corners[:, 1] + corners[:, 2]),
                0.5 * (corners[:, 2] + corners[:, 0])]
    want_pts = np.stack(pts, axis=1).reshape(-1, 2).astype(np.float32)
    got_pts = a["Points"].reshape(-1, 3)
    assert np.array_equal(got_pts[:, :2], want_pts) and np.all(got_pts[:, 2] == 0)
    # values in the cell's point order; p = 0 repeats the barycentre value
    L = oio.lagrange_values(C)
    if nL == 1:
        L = np.repeat(L, 3, axis=1)
    elif nL == 6:
        L = L[:, [0, 1, 2, 5, 3, 4]]
    assert np.array_equal(a["c_h"], L.reshape(-1).astype(np.float32))


@pytest.mark.parametrize("n,seed,p", [(10, 621, 2), (7, 622, 3)])
def test_steps_on_an_unstructured_mesh_read_from_a_file(tmp_path, n, seed, p):
    from paper_1408_3877_amd import edge_kinds_from_ids, read_mesh_medit
    cV0, V00 = delaunay_square(n, seed)
    path = str(tmp_path / "u.mesh")
    write_medit(path, cV0, V00, boundary_sides(cV0, V00), reverse=range(0, V00.shape[0], 4))
    cV, V0T, ids = read_mesh_medit(path)
    kind = edge_kinds_from_ids(ids, neumann_ids=(SOUTH, NORTH))
    ocV, oV0T, oids = oio.read_medit(path)
    okind = np.where(oids == 0, 0, np.where(np.isin(oids, (SOUTH, NORTH)), 2, 1)).astype(np.int8)
    pr = Problem(ocV, oV0T, okind, p)
    s = _solver(cV, V0T, kind, p)
    print("[io-steps] n=%d p=%d K=%d" % (n, p, s.K), flush=True)
    w = Workload(SMOOTH2)
    s.set_initial_samples(s.sample_workload(SMOOTH2, 0.0, want=("c0",))["c0"], 0.0)
    C = pr.initial(w)
    dt, t = 0.02, 0.0
    for _ in range(2):
        t += dt
        smp = s.sample_workload(SMOOTH2, t)
        info = s.step_sampled(dt, smp["d"], smp["f"], smp["cD"], smp["gN"])
        C, Z1, Z2, _ = pr.step(C, t, dt, w)
        Cg, Z1g, Z2g = (to_np(x) for x in s.get_solution())
        a = pr.grid.areaT
        errs = (rel_l2(a, Cg, C), rel_l2(a, Z1g, Z1), rel_l2(a, Z2g, Z2))
        print("[io-steps] %s errs %s" % (info, errs), flush=True)
        assert info["rel_residual"] <= 1e-13 and max(errs) < 1e-10
