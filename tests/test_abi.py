"""CPU checks of the C ABI: the library loads and exports every symbol that
include/st_mg.h declares; parameter validation reports errors before any
device work.  No compute calls (no GPU here)."""
import ctypes
import os
import re

import pytest

from paper_1411_0519_amd import stmg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "st_mg.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(st_(?:mg|mesh)_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("st_mg_setup", "st_mg_vcycle", "st_mg_solve", "st_mg_adjoint", "st_mg_destroy"):
        assert required in names


def test_library_exports_every_declared_symbol():
    L = stmg.lib()
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, missing
    # the binding's signature table covers the header exactly
    assert sorted(stmg.SIGNATURES) == declared_functions()


def test_params_struct_layout_matches_header():
    # the ctypes struct mirrors st_mg_params field by field
    text = open(HEADER).read()
    body = text[text.index("typedef struct {"):text.index("} st_mg_params;")]
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    fields = re.findall(r"\b(int|double)\s+([a-zA-Z_0-9, ]+);", body)
    names = []
    for typ, group in fields:
        for name in group.split(","):
            names.append(name.strip())
    assert names == [f[0] for f in stmg.Params._fields_]


def test_default_params():
    L = stmg.lib()
    p = stmg.Params()
    L.st_mg_default_params(ctypes.byref(p))
    assert (p.dim, p.n, p.N, p.pt, p.nu1, p.nu2, p.batch) == (1, 31, 16, 1, 2, 2, 1)
    assert p.omega == 0.5 and p.precision == 0
    assert (p.smoother, p.nu1x, p.nu2x, p.gamma) == (0, 2, 2, 1) and abs(p.omega_x - 2.0 / 3.0) < 1e-15


@pytest.mark.parametrize("field,value,msg", [
    ("dim", 4, "dim"), ("n", 30, "n must"), ("N", 12, "N must"), ("pt", -1, "p_t"),
    ("omega", 0.0, "omega"), ("batch", 0, "batch"), ("T", -1.0, "T must"), ("nu1", -1, "nu1"), ("pt", 48, "p_t"),
    ("smoother", 2, "smoother"), ("gamma", 3, "gamma"), ("gamma", 0, "gamma"),
])
def test_setup_rejects_invalid_parameters(field, value, msg):
    L = stmg.lib()
    p = stmg.Params()
    L.st_mg_default_params(ctypes.byref(p))
    setattr(p, field, value)
    h = ctypes.c_void_p(0)
    rc = L.st_mg_setup(ctypes.byref(p), ctypes.byref(h))
    assert rc == stmg.ST_EINVAL
    assert h.value
    assert msg in L.st_mg_last_error(h).decode()
    assert L.st_mg_destroy(h) == 0


@pytest.mark.parametrize("field,value", [("nu1x", -1), ("nu2x", 17), ("omega_x", 0.0), ("omega_x", 1.5)])
def test_setup_rejects_invalid_spatial_cycle(field, value):
    L = stmg.lib()
    p = stmg.Params()
    L.st_mg_default_params(ctypes.byref(p))
    p.smoother = 1
    setattr(p, field, value)
    h = ctypes.c_void_p(0)
    assert L.st_mg_setup(ctypes.byref(p), ctypes.byref(h)) == stmg.ST_EINVAL
    assert "spatial cycle" in L.st_mg_last_error(h).decode()
    assert L.st_mg_destroy(h) == 0


@pytest.mark.gpu
def test_spatial_cycle_workspace_is_counted():
    # the spatial-cycle smoother needs its own vectors on every level with n > 1
    # (setup uploads the level tables, so this needs a device)
    L = stmg.lib()
    sizes = []
    for sm in (0, 1):
        p = stmg.Params()
        L.st_mg_default_params(ctypes.byref(p))
        p.smoother = sm
        h = ctypes.c_void_p(0)
        assert L.st_mg_setup(ctypes.byref(p), ctypes.byref(h)) == 0
        b = ctypes.c_size_t()
        assert L.st_mg_workspace_bytes(h, ctypes.byref(b)) == 0
        sizes.append(b.value)
        assert L.st_mg_destroy(h) == 0
    assert sizes[1] > sizes[0]


def test_spatial_smoother_rejects_high_orders():
    L = stmg.lib()
    p = stmg.Params()
    L.st_mg_default_params(ctypes.byref(p))
    p.smoother = 1
    p.pt = 4
    h = ctypes.c_void_p(0)
    assert L.st_mg_setup(ctypes.byref(p), ctypes.byref(h)) == stmg.ST_EINVAL
    assert "p_t <= 3" in L.st_mg_last_error(h).decode()
    assert L.st_mg_destroy(h) == 0
