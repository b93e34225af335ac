"""GPU parity of the twice-folded transforms (FP64: n = 63, 127; FP32: n = 63,
127, 255; forced with STMG_TRANSFORM=3) against the oracle's exact slab solves
and the once-folded kernels, through the C ABI."""
import numpy as np
import pytest
import torch

from gpu_util import DEV, rel_err, to_gpu, to_oracle
from oracle import multigrid, spacetime

pytestmark = pytest.mark.gpu

stmg = pytest.importorskip("paper_1411_0519_amd.stmg")

CASES = [(1, 63, 8, 1, 2), (1, 127, 4, 3, 1), (2, 63, 4, 1, 1), (2, 127, 4, 1, 2), (2, 127, 2, 2, 1),
         (2, 63, 2, 0, 1), (3, 63, 2, 1, 1), (2, 127, 2, 3, 1)]


def cid(c):
    return "d{}n{}N{}p{}b{}".format(*c)


def solvers(case, monkeypatch, **kw):
    d, n, N, pt, b = case
    monkeypatch.setenv("STMG_TRANSFORM", "3")
    S2 = stmg.Solver(d, n, N, pt=pt, batch=b, device=DEV, **kw)
    monkeypatch.setenv("STMG_TRANSFORM", "2")
    S1 = stmg.Solver(d, n, N, pt=pt, batch=b, device=DEV, **kw)
    monkeypatch.delenv("STMG_TRANSFORM")
    return S2, S1


@pytest.mark.parametrize("case", CASES, ids=cid)
@pytest.mark.parametrize("transpose", [False, True])
def test_twice_folded_block_solve(case, transpose, monkeypatch):
    print(f"twice folded block solve {case} transpose={transpose}", flush=True)
    d, n, N, pt, b = case
    S2, S1 = solvers(case, monkeypatch)
    r = np.random.default_rng(3).uniform(-1, 1, (S2.level_dof(0) // b, b))
    x2 = S2.block_solve(to_gpu(r), transpose=transpose)
    x1 = S1.block_solve(to_gpu(r), transpose=transpose)
    assert rel_err(to_oracle(x2, b), to_oracle(x1, b)) < 1e-13
    if d < 3:   # a 3-D 63^3 slab is beyond the oracle's sparse LU in test time
        H = multigrid.Hierarchy(d, n, N, pt, transpose=transpose)
        assert rel_err(to_oracle(x2, b), H.block_solve(len(H.levels) - 1, r)) < 1e-12


@pytest.mark.parametrize("case", [(2, 127, 16, 1, 1), (2, 63, 32, 2, 2), (1, 127, 64, 3, 1)], ids=cid)
def test_twice_folded_iterates_match_oracle(case, monkeypatch):
    d, n, N, pt, b = case
    S2, _ = solvers(case, monkeypatch)
    H = multigrid.Hierarchy(d, n, N, pt)
    F = np.random.default_rng(5).uniform(-1, 1, (H.fine.dof, b))
    _, _, its = H.solve(F, rtol=0.0, maxit=3, keep_iterates=True)
    u = torch.zeros(S2.level_dof(0), dtype=torch.float64, device=DEV)
    for k in range(1, 4):
        S2.solve(to_gpu(F), u=u, rtol=0.0, maxit=1, raise_on_noconv=False)
        assert rel_err(to_oracle(u, b), its[k]) < 1e-12, k


def test_twice_folded_smoothing_update_modes(monkeypatch):
    # the inverse x pass writes u += omega x (smoothing step); 3-D checked against the once-folded kernels
    case = (3, 63, 4, 1, 1)
    S2, S1 = solvers(case, monkeypatch)
    rng = np.random.default_rng(7)
    u = to_gpu(rng.uniform(-1, 1, (S2.level_dof(0), 1)))
    F = to_gpu(rng.uniform(-1, 1, (S2.level_dof(0), 1)))
    u2, u1 = u.clone(), u.clone()
    S2.smooth(u2, F)
    S1.smooth(u1, F)
    assert ((u2 - u1).abs().max() / u1.abs().max()).item() < 1e-13


FP32_CASES = [(1, 63, 8, 1, 2), (1, 255, 4, 1, 1), (2, 63, 4, 1, 1), (2, 127, 4, 1, 2), (2, 255, 2, 2, 1),
              (2, 127, 2, 3, 1), (2, 63, 2, 0, 1)]


@pytest.mark.parametrize("case", FP32_CASES, ids=cid)
@pytest.mark.parametrize("transpose", [False, True])
def test_twice_folded_fp32_block_solve(case, transpose, monkeypatch):
    # FP32 twice-folded slab solves: backward error against the slab matrix
    # within 8 d n u32 per slab, and agreement with the once-folded FP32
    # register kernels to the same order
    print(f"twice folded fp32 block solve {case} transpose={transpose}", flush=True)
    d, n, N, pt, b = case
    S2, S1 = solvers(case, monkeypatch, precision="fp32")
    lev = spacetime.SpaceTimeLevel(d, n, N, pt, 1.0 / N)
    r = np.random.default_rng(3).uniform(-1, 1, (lev.dof, b)).astype(np.float32).astype(np.float64)
    x2 = to_oracle(S2.block_solve(to_gpu(r, torch.float32), transpose=transpose), b)
    x1 = to_oracle(S1.block_solve(to_gpu(r, torch.float32), transpose=transpose), b)
    A = (lev.A.T if transpose else lev.A).tocsr()
    normA = abs(A).sum(axis=1).max()
    xs = x2.reshape(N, lev.slab, b).transpose(1, 0, 2).reshape(lev.slab, -1)
    rs = r.reshape(N, lev.slab, b).transpose(1, 0, 2).reshape(lev.slab, -1)
    be = np.abs(A @ xs - rs).max(axis=0) / (normA * np.abs(xs).max(axis=0))
    assert np.all(be < 8 * d * n * 2.0 ** -24), be.max()
    assert rel_err(x2, x1) < 64 * d * n * 2.0 ** -24


def test_twice_folded_fp32_3d_and_update_modes(monkeypatch):
    # 3-D FP32 (two x/y passes, fused z pass) and the smoothing update u += omega x,
    # against the once-folded FP32 register kernels
    case = (3, 63, 2, 1, 1)
    S2, S1 = solvers(case, monkeypatch, precision="fp32")
    rng = np.random.default_rng(7)
    dof = S2.level_dof(0)
    u = to_gpu(rng.uniform(-1, 1, (dof, 1)), torch.float32)
    F = to_gpu(rng.uniform(-1, 1, (dof, 1)), torch.float32)
    x2 = S2.block_solve(F)
    x1 = S1.block_solve(F)
    assert ((x2 - x1).abs().max() / x1.abs().max()).item() < 64 * 3 * 63 * 2.0 ** -24
    u2, u1 = u.clone(), u.clone()
    S2.smooth(u2, F)
    S1.smooth(u1, F)
    assert ((u2 - u1).abs().max() / u1.abs().max()).item() < 64 * 3 * 63 * 2.0 ** -24


# Slab-resident block solve (STMG_TRANSFORM=4): 2-D, FP64 n = 63, FP32 n = 63, 127, N_t <= 2
SLAB_CASES = [(2, 63, 4, 1, 1), (2, 63, 2, 0, 2), (2, 127, 2, 1, 1), (2, 127, 4, 0, 1), (2, 63, 8, 1, 2)]


def slab_solvers(case, monkeypatch, **kw):
    d, n, N, pt, b = case
    monkeypatch.setenv("STMG_TRANSFORM", "4")
    S4 = stmg.Solver(d, n, N, pt=pt, batch=b, device=DEV, **kw)
    monkeypatch.setenv("STMG_TRANSFORM", "2")
    S1 = stmg.Solver(d, n, N, pt=pt, batch=b, device=DEV, **kw)
    monkeypatch.delenv("STMG_TRANSFORM")
    return S4, S1


@pytest.mark.parametrize("case", [c for c in SLAB_CASES if c[1] == 63], ids=cid)
@pytest.mark.parametrize("transpose", [False, True])
def test_slab_block_solve_fp64(case, transpose, monkeypatch):
    print(f"slab block solve fp64 {case} transpose={transpose}", flush=True)
    d, n, N, pt, b = case
    S4, S1 = slab_solvers(case, monkeypatch)
    r = np.random.default_rng(11).uniform(-1, 1, (S4.level_dof(0) // b, b))
    x4 = S4.block_solve(to_gpu(r), transpose=transpose)
    x1 = S1.block_solve(to_gpu(r), transpose=transpose)
    assert rel_err(to_oracle(x4, b), to_oracle(x1, b)) < 1e-13
    H = multigrid.Hierarchy(d, n, N, pt, transpose=transpose)
    assert rel_err(to_oracle(x4, b), H.block_solve(len(H.levels) - 1, r)) < 1e-12


@pytest.mark.parametrize("case", SLAB_CASES, ids=cid)
@pytest.mark.parametrize("transpose", [False, True])
def test_slab_block_solve_fp32(case, transpose, monkeypatch):
    print(f"slab block solve fp32 {case} transpose={transpose}", flush=True)
    d, n, N, pt, b = case
    S4, S1 = slab_solvers(case, monkeypatch, precision="fp32")
    lev = spacetime.SpaceTimeLevel(d, n, N, pt, 1.0 / N)
    r = np.random.default_rng(13).uniform(-1, 1, (lev.dof, b)).astype(np.float32).astype(np.float64)
    x4 = to_oracle(S4.block_solve(to_gpu(r, torch.float32), transpose=transpose), b)
    x1 = to_oracle(S1.block_solve(to_gpu(r, torch.float32), transpose=transpose), b)
    A = (lev.A.T if transpose else lev.A).tocsr()
    normA = abs(A).sum(axis=1).max()
    xs = x4.reshape(N, lev.slab, b).transpose(1, 0, 2).reshape(lev.slab, -1)
    rs = r.reshape(N, lev.slab, b).transpose(1, 0, 2).reshape(lev.slab, -1)
    be = np.abs(A @ xs - rs).max(axis=0) / (normA * np.abs(xs).max(axis=0))
    assert np.all(be < 8 * d * n * 2.0 ** -24), be.max()
    assert rel_err(x4, x1) < 64 * d * n * 2.0 ** -24


def test_slab_smoothing_and_iterates(monkeypatch):
    # the slab kernel inside smoothing steps (u += omega D^{-1} r) and in whole V-cycles on
    # 63^2 x 16 (level 0 slab-resident, coarser levels the default family): oracle iterates to 1e-12
    case = (2, 63, 16, 1, 1)
    d, n, N, pt, b = case
    S4, S1 = slab_solvers(case, monkeypatch)
    rng = np.random.default_rng(17)
    u = to_gpu(rng.uniform(-1, 1, (S4.level_dof(0), 1)))
    F = to_gpu(rng.uniform(-1, 1, (S4.level_dof(0), 1)))
    u4, u1 = u.clone(), u.clone()
    S4.smooth(u4, F)
    S1.smooth(u1, F)
    assert ((u4 - u1).abs().max() / u1.abs().max()).item() < 1e-13
    H = multigrid.Hierarchy(d, n, N, pt)
    Fo = np.random.default_rng(5).uniform(-1, 1, (H.fine.dof, b))
    _, _, its = H.solve(Fo, rtol=0.0, maxit=3, keep_iterates=True)
    uu = torch.zeros(S4.level_dof(0), dtype=torch.float64, device=DEV)
    for k in range(1, 4):
        S4.solve(to_gpu(Fo), u=uu, rtol=0.0, maxit=1, raise_on_noconv=False)
        assert rel_err(to_oracle(uu, b), its[k]) < 1e-12, k


def test_slab_mixed_reaches_fp64_tolerance(monkeypatch):
    # mixed precision with every qualifying FP32 level slab-resident: same 1e-10 as FP64
    d, n, N, pt = 2, 127, 16, 1
    monkeypatch.setenv("STMG_TRANSFORM", "4")
    M = stmg.Solver(d, n, N, pt=pt, device=DEV, precision="mixed")
    monkeypatch.delenv("STMG_TRANSFORM")
    S = stmg.Solver(d, n, N, pt=pt, device=DEV)
    F = to_gpu(np.random.default_rng(19).uniform(-1, 1, (S.level_dof(0), 1)))
    u64, it64, _ = S.solve(F, rtol=1e-10, maxit=60)
    um, itm, hist = M.solve(F, rtol=1e-10, maxit=60)
    assert hist[-1][0] < 1e-10
    assert abs(itm - it64) <= 2
    assert (torch.linalg.vector_norm(um - u64) / torch.linalg.vector_norm(u64)).item() < 1e-8


# Residual fused with the forward x pass (STMG_RX=1): 2-D, N_t = 2, n = 63, 127
RX_CASES = [(2, 63, 4, 1, 1), (2, 127, 2, 1, 2), (2, 63, 8, 1, 2)]


def rx_solvers(case, monkeypatch, **kw):
    d, n, N, pt, b = case
    monkeypatch.setenv("STMG_RX", "1")
    Sx = stmg.Solver(d, n, N, pt=pt, batch=b, device=DEV, **kw)
    monkeypatch.setenv("STMG_RX", "0")
    S0 = stmg.Solver(d, n, N, pt=pt, batch=b, device=DEV, **kw)
    monkeypatch.delenv("STMG_RX")
    return Sx, S0


@pytest.mark.parametrize("case", RX_CASES, ids=cid)
@pytest.mark.parametrize("transpose", [False, True])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_fused_residual_smoothing_step(case, transpose, precision, monkeypatch):
    # one smoothing step u += omega D^{-1}(F - L u) with and without the fused residual
    print(f"fused residual step {case} transpose={transpose} {precision}", flush=True)
    d, n, N, pt, b = case
    Sx, S0 = rx_solvers(case, monkeypatch, precision=precision)
    dt = torch.float64 if precision == "fp64" else torch.float32
    rng = np.random.default_rng(23)
    dof = Sx.level_dof(0) // b
    u = to_gpu(rng.uniform(-1, 1, (dof, b)), dt)
    F = to_gpu(rng.uniform(-1, 1, (dof, b)), dt)
    ux, u0 = u.clone(), u.clone()
    Sx.smooth(ux, F, transpose=transpose)
    S0.smooth(u0, F, transpose=transpose)
    tol = 1e-13 if precision == "fp64" else 64 * d * n * 2.0 ** -24
    assert ((ux - u0).abs().max() / u0.abs().max()).item() < tol


def test_fused_residual_iterates_match_oracle(monkeypatch):
    # whole V-cycles with the fused residual on every qualifying level: oracle iterates to 1e-12
    case = (2, 127, 8, 1, 1)
    d, n, N, pt, b = case
    Sx, _ = rx_solvers(case, monkeypatch)
    H = multigrid.Hierarchy(d, n, N, pt)
    F = np.random.default_rng(29).uniform(-1, 1, (H.fine.dof, b))
    _, _, its = H.solve(F, rtol=0.0, maxit=3, keep_iterates=True)
    u = torch.zeros(Sx.level_dof(0), dtype=torch.float64, device=DEV)
    for k in range(1, 4):
        Sx.solve(to_gpu(F), u=u, rtol=0.0, maxit=1, raise_on_noconv=False)
        assert rel_err(to_oracle(u, b), its[k]) < 1e-12, k


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_fused_residual_norms_and_solve(precision, monkeypatch):
    # the fine residual norm kernel leaves the x-transformed residual for the next cycle's first
    # smoothing step: residual histories and solutions with and without the fused path agree
    case = (2, 63, 16, 1, 2)
    d, n, N, pt, b = case
    Sx, S0 = rx_solvers(case, monkeypatch, precision=precision)
    dt = torch.float64 if precision == "fp64" else torch.float32
    F = to_gpu(np.random.default_rng(31).uniform(-1, 1, (Sx.level_dof(0) // b, b)), dt)
    rtol = 1e-10 if precision == "fp64" else 1e-5
    ux, itx, hx = Sx.solve(F, rtol=rtol, maxit=40)
    u0, it0, h0 = S0.solve(F, rtol=rtol, maxit=40)
    assert itx == it0
    tol = 1e-12 if precision == "fp64" else 1e-4
    assert np.allclose(np.asarray(hx), np.asarray(h0), rtol=tol, atol=0)
    assert ((ux - u0).abs().max() / u0.abs().max()).item() < (1e-12 if precision == "fp64" else 1e-5)


def test_fused_residual_adjoint_and_graph(monkeypatch):
    # the transposed (backward-in-time) system through the fused residual and its norm path, and the
    # same forward solve replayed from a hipGraph: both agree with the separate-kernel path
    case = (2, 127, 8, 1, 1)
    d, n, N, pt, b = case
    Sx, S0 = rx_solvers(case, monkeypatch)
    rng = np.random.default_rng(37)
    g = to_gpu(rng.uniform(-1, 1, (Sx.level_dof(0), 1)))
    lx, gfx, gux, itx, hx = Sx.adjoint(g, rtol=1e-10, maxit=40)
    l0, gf0, gu0, it0, h0 = S0.adjoint(g, rtol=1e-10, maxit=40)
    assert itx == it0
    assert np.allclose(np.asarray(hx), np.asarray(h0), rtol=1e-10, atol=0)
    assert ((lx - l0).abs().max() / l0.abs().max()).item() < 1e-12
    assert ((gfx - gf0).abs().max() / gf0.abs().max()).item() < 1e-12
    F = to_gpu(rng.uniform(-1, 1, (Sx.level_dof(0), 1)))
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        Sx.set_graph(True)
        ug, itg, hg = Sx.solve(F, rtol=1e-10, maxit=40)
        Sx.set_graph(False)
        ue, ite, he = Sx.solve(F, rtol=1e-10, maxit=40)
    stream.synchronize()
    assert itg == ite
    assert ((ug - ue).abs().max() / ue.abs().max()).item() < 1e-13
