"""CPU checks of the library's P1 mesh construction (host code behind
st_mesh_level and st_mg_setup_mesh): refinement, interior numbering and the
assembled M_h, K_h agree with the oracle's independent construction; invalid
meshes and parameter combinations are rejected before any device work."""
import ctypes

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import mesh
from paper_1411_0519_amd import stmg, workloads


def node_map(lib_points, oracle_points):
    """pm[j] = oracle index of the library's node j (coordinates match exactly)."""
    index = {tuple(p): i for i, p in enumerate(oracle_points)}
    assert len(index) == len(lib_points)
    return np.array([index[tuple(p)] for p in lib_points])


def z_order(points, coarse_coords):
    """Morton keys of the points in the coarse mesh's bounding box, written out
    bit by bit (first coordinate lowest; 21 bits in 3-D, 31 in 2-D); the
    position in the node list breaks ties."""
    d = points.shape[1]
    bits = 21 if d == 3 else 31
    lo, hi = coarse_coords.min(axis=0), coarse_coords.max(axis=0)
    q = np.rint((points - lo) / (hi - lo) * (2 ** bits - 1)).astype(np.int64)
    keys = []
    for j, row in enumerate(q):
        key = 0
        for b in range(bits - 1, -1, -1):
            for i in range(d - 1, -1, -1):
                key = (key << 1) | int((row[i] >> b) & 1)
        keys.append(key * len(q) + j)
    return np.array(keys, dtype=object)


@pytest.mark.parametrize("kind,levels", [("square4", 4), ("cube12", 2)])
def test_library_mesh_matches_oracle(kind, levels):
    c, t = workloads.coarse_mesh(kind)
    ms = mesh.hierarchy(c, t, levels)
    for L in range(levels + 1):
        g = stmg.mesh_level(c, t, L)
        o = ms[L]
        pm = node_map(g["points"], o.points)                        # the same node set
        M = sp.csr_matrix((g["mval"], g["col"], g["rowptr"]), shape=(o.nx, o.nx))
        K = sp.csr_matrix((g["kval"], g["col"], g["rowptr"]), shape=(o.nx, o.nx))
        assert abs(M - o.Mh[pm][:, pm]).max() <= 1e-15 * abs(o.Mh).max()
        assert abs(K - o.Kh[pm][:, pm]).max() <= 1e-14 * abs(o.Kh).max()
        assert np.all(np.diff(z_order(g["points"], c)) > 0)          # numbered along the Z-order curve
        assert np.all(np.diff(g["rowptr"]) > 0)
        for i in range(o.nx):                                       # columns ascending per row
            row = g["col"][g["rowptr"][i]:g["rowptr"][i + 1]]
            assert np.all(np.diff(row) > 0)


def test_library_mesh_on_an_unstructured_coarse_mesh():
    # a coarse mesh that is not one of the built-in ones: an L-shaped domain of 6 triangles
    c = np.array([[0, 0], [1, 0], [2, 0], [0, 1], [1, 1], [2, 1], [0, 2], [1, 2]], dtype=np.float64)
    t = np.array([[0, 1, 4], [0, 4, 3], [1, 2, 5], [1, 5, 4], [3, 4, 7], [3, 7, 6]])
    ms = mesh.hierarchy(c, t, 3)
    g = stmg.mesh_level(c, t, 3)
    o = ms[3]
    pm = node_map(g["points"], o.points)
    K = sp.csr_matrix((g["kval"], g["col"], g["rowptr"]), shape=(o.nx, o.nx))
    assert abs(K - o.Kh[pm][:, pm]).max() <= 1e-14 * abs(o.Kh).max()


def _mesh(coords, cells):
    return stmg._mesh_struct(coords, cells)


@pytest.mark.parametrize("bad", ["index", "degenerate", "level"])
def test_invalid_meshes_are_rejected(bad):
    c, t = workloads.coarse_mesh("square4")
    t = t.copy()
    level = 1
    if bad == "index":
        t[2, 1] = 7
    elif bad == "degenerate":
        c = c.copy()
        c[4] = [0.5, 0.0]       # centre moved onto the bottom edge: the first triangle is flat
    else:
        level = -1
    m, keep = _mesh(c, t)
    nx = ctypes.c_longlong()
    rc = stmg.lib().st_mesh_level(ctypes.byref(m), level, ctypes.byref(nx), None, None, None, None, None, None)
    assert rc == stmg.ST_EINVAL


def test_mesh_setup_validates_before_device_work():
    L = stmg.lib()
    c, t = workloads.coarse_mesh("cube12")
    m, keep = _mesh(c, t)
    for field, value in (("smoother", 0), ("dim", 2), ("precision", stmg.PRECISION["mixed_bf16"]), ("pt", 4)):
        p = stmg.Params()
        L.st_mg_default_params(ctypes.byref(p))
        p.dim, p.N, p.smoother = 3, 8, 1
        setattr(p, field, value)
        h = ctypes.c_void_p(0)
        assert L.st_mg_setup_mesh(ctypes.byref(p), ctypes.byref(m), 1, ctypes.byref(h)) == stmg.ST_EINVAL, field
        assert L.st_mg_last_error(h)
        L.st_mg_destroy(h)
