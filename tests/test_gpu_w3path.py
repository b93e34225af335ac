"""GPU parity on the path of the 3-D workload (Q1 63^3 x 1024 slabs, p_t = 1,
mu = tau/h^2 = 4): the z-marching 3-D residual against the oracle's sparse L
(several y tiles and z chunks, ragged last tiles), the twice-folded 3-D n = 63
block solve against the oracle's slab matrix A (backward error, FP64 and
FP32, forward and transposed), and FP64 V-cycle iterates against the oracle
on reduced members of the same family: the same mu = 4 (15^3 x 64, 7^3 x 16)
and a 15^3 x 256 instance at mu = 1 whose schedule has the semi-then-full
step of the full-size hierarchy (ffffsfssss); the x-mode-major 3-D family
against the separate passes; and the batched workload's family (2-D, p_t = 2,
mu = 128, 64 right-hand sides) at reduced N."""
import functools

import numpy as np
import pytest
import torch

from gpu_util import DEV, rel_err, to_gpu, to_oracle
from oracle import multigrid, spacetime

pytestmark = pytest.mark.gpu

stmg = pytest.importorskip("paper_1411_0519_amd.stmg")


def cid(c):
    return "d{}n{}N{}p{}b{}".format(*c[:5])


# (dim, n, N, pt, batch): 31^3 x 8 -> 2 y tiles of 16 rows (the second ragged) x 4 z chunks;
# N_t = 4 -> 4 y tiles of 8 rows; 15^3 x 64, b = 2 -> one tile per slab; 63^3 x 2 -> the
# full-size slab shape (8 y tiles of 8 rows, the last one 7, 8 z chunks)
RES_CASES = [(3, 31, 8, 1, 1), (3, 31, 4, 3, 1), (3, 15, 64, 1, 2), (3, 63, 2, 1, 1), (3, 3, 4, 2, 1)]


@functools.lru_cache(maxsize=2)
def slab_level(d, n, pt, tau):
    """The oracle's slab matrices A and B = -N_tau (x) M_h (one-slab level)."""
    lev = spacetime.SpaceTimeLevel(d, n, 1, pt, tau)
    return lev, lev.A.tocsr(), lev.B.tocsr()


def oracle_residual(d, n, N, pt, u, F, transpose):
    """F - L u slab by slab with the oracle's A and B (L block lower bidiagonal)."""
    lev, A, B = slab_level(d, n, pt, 1.0 / N)
    S = lev.slab
    r = np.empty_like(F)
    for k in range(N):
        sl = slice(k * S, (k + 1) * S)
        if not transpose:
            r[sl] = F[sl] - A @ u[sl] - (B @ u[(k - 1) * S:k * S] if k > 0 else 0.0)
        else:
            r[sl] = F[sl] - A.T @ u[sl] - (B.T @ u[(k + 1) * S:(k + 2) * S] if k < N - 1 else 0.0)
    return r


@pytest.mark.parametrize("case", RES_CASES, ids=cid)
@pytest.mark.parametrize("transpose", [False, True])
def test_residual3d_parity(case, transpose):
    d, n, N, pt, b = case
    print(f"3-D residual {case} transpose={transpose}", flush=True)
    S = stmg.Solver(d, n, N, pt=pt, batch=b, device=DEV)
    dof = S.level_dof(0) // b
    rng = np.random.default_rng(17)
    u = rng.uniform(-1, 1, (dof, b))
    F = rng.uniform(-1, 1, (dof, b))
    r_ref = oracle_residual(d, n, N, pt, u, F, transpose)
    r, nrm = S.residual(to_gpu(u), to_gpu(F), transpose=transpose, norms=True)
    torch.cuda.synchronize()
    assert rel_err(to_oracle(r, b), r_ref) < 1e-13
    assert np.allclose(nrm, np.linalg.norm(r_ref, axis=0), rtol=1e-12)
    # FP32 arithmetic on the same data (inner cycle of the mixed solver)
    S32 = stmg.Solver(d, n, N, pt=pt, batch=b, device=DEV, precision="fp32")
    r32 = S32.residual(to_gpu(u, torch.float32), to_gpu(F, torch.float32), transpose=transpose)
    torch.cuda.synchronize()
    assert rel_err(to_oracle(r32, b), r_ref) < 2e-6
    S.close()
    S32.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("transpose", [False, True])
@pytest.mark.parametrize("impl", ["0", "1", "2", "3", "6"], ids=["auto", "lds", "reg", "reg2", "xslab"])
def test_block_solve_3d_n63_backward_error(precision, transpose, impl, monkeypatch):
    """x = D^{-1} r on 63^3 slabs: ||A x - r||_inf <= 8 d n u ||A||_inf ||x||_inf with the
    oracle's assembled slab matrix A (2d length-n transform passes and one N_t x N_t solve
    per mode, each with relative rounding <= n u)."""
    d, n, N, pt, b = 3, 63, 2, 1, 1
    print(f"3-D n=63 block solve {precision} transpose={transpose} impl={impl}", flush=True)
    monkeypatch.setenv("STMG_TRANSFORM", impl)
    S = stmg.Solver(d, n, N, pt=pt, batch=b, device=DEV, precision=precision)
    monkeypatch.delenv("STMG_TRANSFORM")
    lev, A, _ = slab_level(d, n, pt, 1.0 / N)
    A = A.T.tocsr() if transpose else A
    normA = abs(A).sum(axis=1).max()
    dt = torch.float64 if precision == "fp64" else torch.float32
    u_r = 2.0 ** -53 if precision == "fp64" else 2.0 ** -24
    r = np.random.default_rng(23).uniform(-1, 1, (N * lev.slab, b))
    x = S.block_solve(to_gpu(r, dt), transpose=transpose)
    torch.cuda.synchronize()
    xg = to_oracle(x, b)
    rq = to_oracle(to_gpu(r, dt), b)           # the right-hand side the GPU saw
    for s in range(N):
        xs = xg[s * lev.slab:(s + 1) * lev.slab, 0]
        rs = rq[s * lev.slab:(s + 1) * lev.slab, 0]
        be = np.abs(A @ xs - rs).max() / (normA * np.abs(xs).max())
        assert be < 8 * d * n * u_r, (s, be)
    S.close()


def iterate_parity(d, n, N, pt, T, seed, expect_schedule, cycles):
    S = stmg.Solver(d, n, N, pt=pt, T=T, device=DEV)
    H = multigrid.Hierarchy(d, n, N, pt, T=T)
    assert S.schedule == H.schedule == expect_schedule
    rng = np.random.default_rng(seed)
    f = rng.uniform(-1, 1, (1, N, n ** d))
    u0 = np.zeros((1, n ** d))
    F = spacetime.rhs(H.fine, f, u0)
    _, _, its = H.solve(F, rtol=0.0, maxit=cycles, keep_iterates=True)
    Fg = to_gpu(F)
    u = torch.zeros_like(Fg)
    for k in range(1, cycles + 1):
        S.vcycle(u, Fg)
        torch.cuda.synchronize()
        err = rel_err(to_oracle(u, 1), its[k])
        assert err < 1e-12, (k, err)
    S.close()


@pytest.mark.parametrize("case", [
    (3, 15, 64, 1, 1.0, "fffsss", 6),          # mu = 4, like the 63^3 x 1024 workload
    (3, 7, 16, 1, 1.0, "ffss", 8),             # mu = 4
    (3, 15, 256, 1, 1.0, "ffsfssss", 4),       # mu = 1: a full step after a semi step
], ids=lambda c: f"n{c[1]}N{c[2]}T{c[4]}")
def test_w3_family_iterate_parity(case):
    d, n, N, pt, T, sched, cycles = case
    print(f"W3 family iterates {case}", flush=True)
    iterate_parity(d, n, N, pt, T, 31, sched, cycles)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("transpose", [False, True])
@pytest.mark.parametrize("rx", ["0", "1"], ids=["resid", "resid_xfwd"])
@pytest.mark.parametrize("pt", [1, 0])
def test_xslab_smoothing_matches_twice_folded(precision, transpose, rx, pt, monkeypatch):
    """The x-mode-major family (x pass, one (z, y) block solve per (slab, kx) in
    LDS, inverse x pass; with STMG_RX=1 the residual kernel applies the x pass
    and writes that layout itself) against the separate twice-folded passes:
    smoothing step u += omega D^{-1}(F - L u) on 63^3 x 4 slabs, forward and
    adjoint, N_t = 2 and 1."""
    d, n, N = 3, 63, 4
    print(f"xslab smoothing {precision} transpose={transpose} rx={rx} pt={pt}", flush=True)
    monkeypatch.setenv("STMG_TRANSFORM", "6")
    monkeypatch.setenv("STMG_RX", rx)
    X = stmg.Solver(d, n, N, pt=pt, device=DEV, precision=precision)
    monkeypatch.setenv("STMG_TRANSFORM", "3")
    monkeypatch.setenv("STMG_RX", "0")
    R = stmg.Solver(d, n, N, pt=pt, device=DEV, precision=precision)
    monkeypatch.delenv("STMG_TRANSFORM")
    monkeypatch.delenv("STMG_RX")
    dt = torch.float64 if precision == "fp64" else torch.float32
    g = torch.Generator(device=DEV).manual_seed(5)
    u = torch.rand(X.level_dof(0), dtype=dt, device=DEV, generator=g) * 2 - 1
    F = torch.rand(X.level_dof(0), dtype=dt, device=DEV, generator=g) * 2 - 1
    ux, ur = u.clone(), u.clone()
    X.smooth(ux, F, transpose=transpose)
    R.smooth(ur, F, transpose=transpose)
    xr = X.block_solve(F, transpose=transpose)
    rr = R.block_solve(F, transpose=transpose)
    torch.cuda.synchronize()
    tol = 1e-13 if precision == "fp64" else 2e-5
    assert ((ux - ur).abs().max() / ur.abs().max()).item() < tol
    assert ((xr - rr).abs().max() / rr.abs().max()).item() < tol
    X.close()
    R.close()


def test_batched_family_iterate_parity():
    """The batched workload's family (2-D, p_t = 2, mu = 128, 64 right-hand
    sides with the workload's data recipe) at 63^2 x 8 slabs on T = 1/4: FP64
    V-cycle iterates of every right-hand side against the oracle's."""
    from paper_1411_0519_amd import workloads
    d, n, N, pt, b, T = 2, 63, 8, 2, 64, 0.25
    print("batched family iterates", flush=True)
    S = stmg.Solver(d, n, N, pt=pt, T=T, batch=b, device=DEV)
    S.autotune()
    H = multigrid.Hierarchy(d, n, N, pt, T=T)
    assert S.schedule == H.schedule == "fff" and abs(H.fine.mu - 128.0) < 1e-12
    f, u0 = workloads.make(d, n, N, batch=b, seed=4, f="uniform", u0="series16")
    F = spacetime.rhs(H.fine, f, u0)
    _, _, its = H.solve(F, rtol=0.0, maxit=3, keep_iterates=True)
    Fg = to_gpu(F)
    u = torch.zeros_like(Fg)
    for k in range(1, 4):
        S.vcycle(u, Fg)
        torch.cuda.synchronize()
        err = rel_err(to_oracle(u, b), its[k])
        assert err < 1e-12, (k, err)
    S.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_xslab_resid_xfwd_vcycles_match_twice_folded(precision, monkeypatch):
    """Three V-cycles with the residual kernel writing the x-mode-major layout
    (STMG_TRANSFORM=6, STMG_RX=1) against the twice-folded passes on 63^3 x 8
    slabs (a fully coarsened fine level, the headline's smoothing steps)."""
    d, n, N, pt = 3, 63, 8, 1
    print(f"xslab + residual/x-pass V-cycles {precision}", flush=True)
    monkeypatch.setenv("STMG_TRANSFORM", "6")
    monkeypatch.setenv("STMG_RX", "1")
    X = stmg.Solver(d, n, N, pt=pt, device=DEV, precision=precision)
    monkeypatch.setenv("STMG_TRANSFORM", "3")
    monkeypatch.setenv("STMG_RX", "0")
    R = stmg.Solver(d, n, N, pt=pt, device=DEV, precision=precision)
    monkeypatch.delenv("STMG_TRANSFORM")
    monkeypatch.delenv("STMG_RX")
    dt = torch.float64 if precision == "fp64" else torch.float32
    g = torch.Generator(device=DEV).manual_seed(12)
    F = torch.rand(X.level_dof(0), dtype=dt, device=DEV, generator=g) * 2 - 1
    ux, ur = torch.zeros_like(F), torch.zeros_like(F)
    X.profile_start()
    for _ in range(3):
        # the residual norm of the fused kernel (its partial sums) against the plain residual kernel's
        relx = X.vcycle(ux, F)
        relr = R.vcycle(ur, F)
        assert abs(relx[0] - relr[0]) <= (1e-10 if precision == "fp64" else 1e-4) * relr[0], (relx, relr)
    torch.cuda.synchronize()
    assert X.profile_read("resid_x", level=0)[1] > 0
    X.profile_stop()
    tol = 1e-12 if precision == "fp64" else 1e-4
    assert ((ux - ur).abs().max() / ur.abs().max()).item() < tol
    X.close()
    R.close()
