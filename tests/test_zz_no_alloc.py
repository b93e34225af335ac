"""The allocation-free residual entry point (st_mg_residual_noalloc) against
st_mg_residual: same residual and norms, bit for bit (same kernels, same
reduction order), on two calls in a row with the second one smaller, with
and without a bound workspace, FP64 and FP32, forward and transposed; sizes
beyond the static scratch are rejected before any device work."""
import numpy as np
import pytest
import torch

from gpu_util import DEV

pytestmark = pytest.mark.gpu

stmg = pytest.importorskip("paper_1411_0519_amd.stmg")

# (dim, n, N, pt, batch, precision): the first case of each pair is the larger one
PAIRS = [
    ((2, 127, 64, 1, 2, "fp64"), (1, 31, 16, 1, 1, "fp64")),
    ((3, 31, 32, 1, 1, "fp64"), (2, 15, 8, 2, 3, "fp64")),
    ((2, 63, 32, 1, 4, "fp32"), (3, 7, 4, 1, 1, "fp32")),
]


def _inputs(S, seed):
    g = torch.Generator(device=DEV).manual_seed(seed)
    dt = S.dtype
    u = torch.rand(S.level_dof(0), dtype=dt, device=DEV, generator=g) * 2 - 1
    F = torch.rand(S.level_dof(0), dtype=dt, device=DEV, generator=g) * 2 - 1
    return u, F


def _check(case, seed, transpose):
    d, n, N, pt, b, prec = case
    print(f"noalloc residual {case} transpose={transpose}", flush=True)
    ref = stmg.Solver(d, n, N, pt=pt, batch=b, precision=prec, device=DEV)
    bare = stmg.Solver(d, n, N, pt=pt, batch=b, precision=prec, device=DEV, workspace=False)
    u, F = _inputs(ref, seed)
    r_ref, n_ref = ref.residual(u, F, transpose=transpose, norms=True)
    r1, n1 = ref.residual_noalloc(u, F, transpose=transpose, norms=True)
    r2, n2 = bare.residual_noalloc(u, F, transpose=transpose, norms=True)
    r3 = bare.residual_noalloc(u, F, transpose=transpose)
    torch.cuda.synchronize()
    assert torch.equal(r1, r_ref) and torch.equal(r2, r_ref) and torch.equal(r3, r_ref)
    assert n1 == n_ref and n2 == n_ref
    # the norms are the norms of the residual (not stale scratch contents)
    nr = np.linalg.norm(r_ref.view(b, -1).double().cpu().numpy(), axis=1)
    assert np.allclose(n1, nr, rtol=1e-5 if prec == "fp32" else 1e-12)
    ref.close()
    bare.close()


@pytest.mark.parametrize("pair", PAIRS, ids=["2d-1d", "3d-2d", "fp32"])
@pytest.mark.parametrize("transpose", [False, True])
def test_noalloc_residual_matches_residual(pair, transpose):
    big, small = pair
    _check(big, 11, transpose)
    _check(small, 12, transpose)


def test_noalloc_residual_coarse_level_without_norms():
    print("noalloc residual coarse level", flush=True)
    S = stmg.Solver(2, 63, 16, pt=1, device=DEV)
    g = torch.Generator(device=DEV).manual_seed(3)
    nd = S.level_dof(1)
    u = torch.rand(nd, dtype=torch.float64, device=DEV, generator=g)
    F = torch.rand(nd, dtype=torch.float64, device=DEV, generator=g)
    a = S.residual(u, F, level=1)
    b = S.residual_noalloc(u, F, level=1)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    with pytest.raises(stmg.STMGError):
        S.residual_noalloc(u, F, level=1, norms=True)
    S.close()


def test_noalloc_residual_rejects_sizes_beyond_the_scratch():
    print("noalloc residual limits", flush=True)
    # 1-D n = 1: one residual workgroup per slab; 2^20 slabs x 2 right-hand sides = 2^21 partial sums > 2^20
    S = stmg.Solver(1, 1, 1 << 20, pt=1, batch=2, device=DEV, workspace=False)
    u = S.zeros()
    with pytest.raises(stmg.STMGError) as ei:
        S.residual_noalloc(u, u, norms=True)
    assert ei.value.code == stmg.ST_EINVAL and "static scratch too small" in str(ei.value)
    r = S.residual_noalloc(u, u)          # without norms the scratch is not used
    torch.cuda.synchronize()
    assert not r.abs().max().item()
    S.close()
    B = stmg.Solver(1, 7, 2, pt=0, batch=257, device=DEV, workspace=False)
    v = B.zeros()
    with pytest.raises(stmg.STMGError) as ei:
        B.residual_noalloc(v, v, norms=True)
    assert ei.value.code == stmg.ST_EINVAL and "static scratch too small" in str(ei.value)
    B.close()
