"""Launch shapes of the twice-folded passes (waves per workgroup, persistent
grids, column groups of the fused pass): every shape transforms each line
with the same arithmetic, so block solves and smoothing steps must equal the
default shape's bit for bit; the autotuned shapes of a batched level keep the
V-cycle iterates on the oracle's."""
import numpy as np
import pytest
import torch

from gpu_util import DEV, rel_err, to_gpu, to_oracle
from oracle import multigrid

pytestmark = pytest.mark.gpu

stmg = pytest.importorskip("paper_1411_0519_amd.stmg")

# (dim, n, N, pt, batch, precision)
CASES = [(2, 127, 16, 1, 1, "fp64"), (3, 63, 2, 1, 1, "fp64"), (2, 255, 4, 2, 2, "fp32"),
         (2, 63, 8, 0, 2, "fp64"), (2, 127, 8, 1, 2, "mixed_bf16"), (1, 127, 64, 3, 1, "fp64")]
# (wpg, pass_per_cu, fused_cg, fused_per_cu); caps of one or a few workgroups per
# compute unit make every wave and workgroup loop over many groups
SHAPES = [(1, 0, 0, 0), (2, 0, 0, 0), (4, 1, 0, 0), (2, 3, 0, 0), (4, 0, 1, 0), (4, 0, 2, 0), (4, 0, 0, 1),
          (4, 0, 0, 3), (1, 1, 1, 1)]


def cid(c):
    return "d{}n{}N{}p{}b{}-{}".format(*c)


@pytest.mark.parametrize("case", CASES, ids=cid)
def test_shapes_give_identical_results(case):
    d, n, N, pt, b, prec = case
    print(f"shapes {case}", flush=True)
    S = stmg.Solver(d, n, N, pt=pt, batch=b, device=DEV, precision=prec)
    dt = torch.float64 if prec == "fp64" else torch.float32
    lp = stmg.FP64 if prec == "fp64" else stmg.FP32
    nd = S.level_dof(0)
    g = torch.Generator(device=DEV).manual_seed(3)
    r = torch.rand(nd, dtype=dt, device=DEV, generator=g) * 2 - 1
    u0 = torch.rand(nd, dtype=dt, device=DEV, generator=g) * 2 - 1
    x_ref = S.block_solve(r, prec=lp)
    xt_ref = S.block_solve(r, prec=lp, transpose=True)
    u_ref = u0.clone()
    S.smooth(u_ref, r, prec=lp)
    cgmax = 1 if pt >= 2 else 4 // (pt + 1)
    for sh in SHAPES:
        if sh[2] > cgmax:
            continue
        S.set_level_shape(0, *sh)
        x = S.block_solve(r, prec=lp)
        xt = S.block_solve(r, prec=lp, transpose=True)
        u = u0.clone()
        S.smooth(u, r, prec=lp)
        torch.cuda.synchronize()
        assert torch.equal(x, x_ref), sh
        assert torch.equal(xt, xt_ref), sh
        assert torch.equal(u, u_ref), sh
    S.close()


def test_shape_arguments_are_checked():
    S = stmg.Solver(2, 63, 4, pt=1, device=DEV)
    for bad in [(3, 0, 0, 0), (4, -1, 0, 0), (4, 0, 3, 0), (4, 0, 4, 0), (4, 0, 0, -2)]:
        with pytest.raises(stmg.STMGError):
            S.set_level_shape(0, *bad)
    S.set_level_shape(0, 2, 4, 1, 2)
    assert S.level_shape(0) == dict(wpg=2, pass_per_cu=4, fused_cg=1, fused_per_cu=2)
    S.close()


def test_autotuned_batched_shapes_keep_iterates():
    d, n, N, pt, b = 2, 127, 16, 1, 4
    print("autotuned batched shapes", flush=True)
    S = stmg.Solver(d, n, N, pt=pt, batch=b, device=DEV)
    S.autotune()
    shapes = [S.level_shape(k) for k in range(S.nlev)]
    print("  tuned shapes", shapes[:2], flush=True)
    H = multigrid.Hierarchy(d, n, N, pt)
    F = np.random.default_rng(8).uniform(-1, 1, (H.fine.dof, b))
    _, _, its = H.solve(F, rtol=0.0, maxit=3, keep_iterates=True)
    stream = torch.cuda.Stream(device=DEV)
    with torch.cuda.stream(stream):
        S.set_graph(True)
        Fg = to_gpu(F)
        u = torch.zeros_like(Fg)
        for k in range(1, 4):
            S.solve(Fg, u=u, rtol=0.0, maxit=1, raise_on_noconv=False)
            torch.cuda.synchronize()
            assert rel_err(to_oracle(u, b), its[k]) < 1e-12, k
    # a persistent shape set after the graph was recorded replaces it
    with torch.cuda.stream(stream):
        S.set_level_shape(0, 2, 1, 1, 1)
        u2 = torch.zeros_like(Fg)
        for k in range(1, 4):
            S.solve(Fg, u=u2, rtol=0.0, maxit=1, raise_on_noconv=False)
            torch.cuda.synchronize()
            assert rel_err(to_oracle(u2, b), its[k]) < 1e-12, k
    S.close()
