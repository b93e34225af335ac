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


@pytest.mark.parametrize("kind,levels", [("square4", 4), ("cube12", 2)])
def test_library_mesh_matches_oracle(kind, levels):
    c, t = workloads.coarse_mesh(kind)
    ms = mesh.hierarchy(c, t, levels)
    for L in range(levels + 1):
        g = stmg.mesh_level(c, t, L)
        o = ms[L]
        assert np.array_equal(g["points"], o.points), L            # same nodes in the same order
        M = sp.csr_matrix((g["mval"], g["col"], g["rowptr"]), shape=(o.nx, o.nx))
        K = sp.csr_matrix((g["kval"], g["col"], g["rowptr"]), shape=(o.nx, o.nx))
        assert abs(M - o.Mh).max() <= 1e-15 * abs(o.Mh).max()
        assert abs(K - o.Kh).max() <= 1e-14 * abs(o.Kh).max()
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
    assert np.array_equal(g["points"], o.points)
    K = sp.csr_matrix((g["kval"], g["col"], g["rowptr"]), shape=(o.nx, o.nx))
    assert abs(K - o.Kh).max() <= 1e-14 * abs(o.Kh).max()


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
    for field, value in (("smoother", 0), ("dim", 2), ("precision", stmg.PRECISION["mixed"]), ("pt", 4)):
        p = stmg.Params()
        L.st_mg_default_params(ctypes.byref(p))
        p.dim, p.N, p.smoother = 3, 8, 1
        setattr(p, field, value)
        h = ctypes.c_void_p(0)
        assert L.st_mg_setup_mesh(ctypes.byref(p), ctypes.byref(m), 1, ctypes.byref(h)) == stmg.ST_EINVAL, field
        assert L.st_mg_last_error(h)
        L.st_mg_destroy(h)
