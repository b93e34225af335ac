"""GPU checks of the extensions: FP32 arithmetic, mixed-precision iterative
refinement, batched right-hand sides, hipGraph replay, and the adjoint /
autograd gradients (finite differences, oracle's direct adjoint, dot-product
test)."""
import numpy as np
import pytest
import torch

from gpu_util import DEV, nodal_to_gpu, norm_rel, rel_err, to_gpu, to_oracle
from oracle import multigrid, spacetime
from paper_1411_0519_amd import workloads

pytestmark = pytest.mark.gpu

stmg = pytest.importorskip("paper_1411_0519_amd.stmg")


def rvec(dof, b, seed):
    return np.random.default_rng(seed).uniform(-1, 1, (dof, b))


# ------------------------------------------------------------------- FP32
@pytest.mark.parametrize("d,n,N,pt", [(1, 63, 16, 1), (2, 31, 8, 2), (2, 127, 4, 1), (3, 15, 4, 1)])
def test_fp32_operators(d, n, N, pt):
    # FP32 level operators against the FP64 oracle: rounding of float arithmetic
    # over O(n) terms per pass (u32 = 2^-24): tolerance 64 d n u32.
    print(f"fp32 operators {(d, n, N, pt)}", flush=True)
    S = stmg.Solver(d, n, N, pt=pt, precision="fp32", device=DEV)
    H = multigrid.Hierarchy(d, n, N, pt)
    k = len(H.levels) - 1
    u = rvec(H.fine.dof, 1, 1)
    F = rvec(H.fine.dof, 1, 2)
    tol = 64 * d * n * 2.0 ** -24
    r = S.residual(to_gpu(u, torch.float32), to_gpu(F, torch.float32))
    assert rel_err(to_oracle(r, 1), H.residual(k, u, F)) < 1e-5
    x = S.block_solve(to_gpu(F, torch.float32))
    assert rel_err(to_oracle(x, 1), H.block_solve(k, F)) < tol
    if S.nlev > 1:
        Fc = S.restrict(to_gpu(u, torch.float32))
        assert rel_err(to_oracle(Fc, 1), H.P[k].T @ u) < 1e-6


FP32_SOLVE_CASES = [(1, 255, 8, 1, 2), (1, 63, 4, 3, 1), (2, 255, 2, 1, 1), (2, 127, 4, 2, 1),
                    (2, 31, 8, 0, 2), (3, 15, 4, 1, 1), (3, 31, 2, 2, 1)]


@pytest.mark.parametrize("case", FP32_SOLVE_CASES, ids=lambda c: "d{}n{}N{}p{}b{}".format(*c))
@pytest.mark.parametrize("transpose", [False, True])
@pytest.mark.parametrize("impl", ["0", "1", "2", "3"], ids=["auto", "lds", "reg", "reg2"])
def test_fp32_block_solve_families(case, transpose, impl, monkeypatch):
    # Every FP32 transform family (LDS-staged, register-resident with the LDS
    # re-layout between the time solve and the inverse product, twice folded
    # where n = 63, 127, 255) against the slab matrix, with the FP32
    # backward-error bound 8 d n u32 per slab.
    d, n, N, pt, b = case
    print(f"fp32 block solve {case} transpose={transpose} impl={impl}", flush=True)
    monkeypatch.setenv("STMG_TRANSFORM", impl)
    S = stmg.Solver(d, n, N, pt=pt, batch=b, precision="fp32", device=DEV)
    lev = spacetime.SpaceTimeLevel(d, n, N, pt, 1.0 / N)
    r = rvec(lev.dof, b, 3).astype(np.float32).astype(np.float64)
    x = to_oracle(S.block_solve(to_gpu(r, torch.float32), transpose=transpose), b)
    A = (lev.A.T if transpose else lev.A).tocsr()
    normA = abs(A).sum(axis=1).max()
    xs = x.reshape(N, lev.slab, b).transpose(1, 0, 2).reshape(lev.slab, -1)
    rs = r.reshape(N, lev.slab, b).transpose(1, 0, 2).reshape(lev.slab, -1)
    be = np.abs(A @ xs - rs).max(axis=0) / (normA * np.abs(xs).max(axis=0))
    assert np.all(be < 8 * d * n * 2.0 ** -24), be.max()


def test_fp32_solve_reaches_float_accuracy():
    d, n, N, pt = 2, 31, 32, 1
    S = stmg.Solver(d, n, N, pt=pt, precision="fp32", device=DEV)
    H = multigrid.Hierarchy(d, n, N, pt)
    f, u0 = workloads.make(d, n, N, seed=3, f="uniform", u0="sine1")
    F = spacetime.rhs(H.fine, f, u0)
    u, its, hist = S.solve(to_gpu(F, torch.float32), rtol=1e-5, maxit=30)
    exact = spacetime.forward_substitution(H.fine, F)
    assert hist[-1][0] <= 1e-5
    assert norm_rel(to_oracle(u, 1), exact) < 1e-4


# ------------------------------------------------------- mixed precision
@pytest.mark.parametrize("d,n,N,pt,b", [(2, 31, 32, 1, 1), (3, 15, 16, 1, 1), (2, 15, 16, 2, 2), (1, 31, 16, 1, 1)])
def test_mixed_precision_reaches_fp64_tolerance(d, n, N, pt, b):
    print(f"mixed {(d, n, N, pt, b)}", flush=True)
    M = stmg.Solver(d, n, N, pt=pt, batch=b, precision="mixed", device=DEV)
    S = stmg.Solver(d, n, N, pt=pt, batch=b, device=DEV)
    H = multigrid.Hierarchy(d, n, N, pt)
    f, u0 = workloads.make(d, n, N, batch=b, seed=4, f="uniform", u0="series16")
    F = spacetime.rhs(H.fine, f, u0)
    Fg = to_gpu(F)
    um, itm, histm = M.solve(Fg, rtol=1e-10, maxit=40)
    u64, it64, hist64 = S.solve(Fg, rtol=1e-10, maxit=40)
    assert max(histm[-1]) <= 1e-10
    assert itm <= it64 + 2
    # the FP64 residual of the mixed result, recomputed by the oracle
    r = F - H.fine.L @ to_oracle(um, b)
    assert np.all(np.linalg.norm(r, axis=0) <= 1.01e-10 * np.linalg.norm(F, axis=0))
    exact = spacetime.forward_substitution(H.fine, F)
    assert norm_rel(to_oracle(um, b), exact) < 1e-8
    assert norm_rel(to_oracle(um, b), to_oracle(u64, b)) < 1e-8


# ----------------------------------------------------------------- batching
def test_batch_equals_single_rhs():
    d, n, N, pt, b = 2, 31, 16, 2, 3
    f, u0 = workloads.make(d, n, N, batch=b, seed=8, f="uniform", u0="series16")
    B = stmg.Solver(d, n, N, pt=pt, batch=b, device=DEV)
    Fb = B.rhs(nodal_to_gpu(f), nodal_to_gpu(u0))
    ub = torch.zeros_like(Fb)
    B.solve(Fb, u=ub, rtol=0.0, maxit=6, raise_on_noconv=False)
    S = stmg.Solver(d, n, N, pt=pt, batch=1, device=DEV)
    for i in range(b):
        Fi = S.rhs(nodal_to_gpu(f[i:i + 1]), nodal_to_gpu(u0[i:i + 1]))
        ui = torch.zeros_like(Fi)
        S.solve(Fi, u=ui, rtol=0.0, maxit=6, raise_on_noconv=False)
        seg = ub[i * S.level_dof(0):(i + 1) * S.level_dof(0)]
        assert torch.equal(Fi, Fb[i * S.level_dof(0):(i + 1) * S.level_dof(0)])
        assert (seg - ui).abs().max().item() <= 1e-14 * ui.abs().max().item()


# --------------------------------------------------------------- hipGraph
@pytest.mark.parametrize("precision", ["fp64", "mixed", "fp32"])
def test_graph_replay_matches_eager(precision):
    d, n, N, pt = 2, 31, 16, 1
    dt = torch.float32 if precision == "fp32" else torch.float64
    f, u0 = workloads.make(d, n, N, seed=12, f="uniform", u0="sine1")
    stream = torch.cuda.Stream(device=DEV)
    with torch.cuda.stream(stream):
        E = stmg.Solver(d, n, N, pt=pt, precision=precision, device=DEV)
        G = stmg.Solver(d, n, N, pt=pt, precision=precision, device=DEV)
        G.set_graph(True)
        F = E.rhs(nodal_to_gpu(f, dt), nodal_to_gpu(u0, dt))
        ue = torch.zeros_like(F)
        ug = torch.zeros_like(F)
        for rep in range(4):
            # replays separated by unrelated eager work and synchronisation
            _, _, he = E.solve(F, u=ue, rtol=0.0, maxit=2, raise_on_noconv=False)
            _, _, hg = G.solve(F, u=ug, rtol=0.0, maxit=2, raise_on_noconv=False)
            junk = torch.randn(1 << 16, device=DEV).sum()
            torch.cuda.synchronize()
            assert torch.equal(ue, ug), rep
            assert np.allclose(np.array(he), np.array(hg), rtol=0, atol=0)
            del junk


def test_graph_mode_needs_stream():
    S = stmg.Solver(1, 15, 8, device=DEV)
    S.set_graph(True)
    F = torch.ones(S.level_dof(0), dtype=torch.float64, device=DEV)
    with torch.cuda.stream(torch.cuda.default_stream(DEV)):
        if torch.cuda.current_stream(DEV).cuda_stream == 0:
            with pytest.raises(stmg.STMGError):
                S.solve(F, maxit=2)


# ------------------------------------------------------------------ adjoint
def test_adjoint_dot_product_and_direct_adjoint():
    d, n, N, pt, b = 2, 15, 16, 1, 2
    S = stmg.Solver(d, n, N, pt=pt, batch=b, device=DEV)
    lev = spacetime.SpaceTimeLevel(d, n, N, pt, 1.0 / N)
    # <L^T x, y> = <x, L y> with the GPU residual operator (F = 0)
    x = rvec(lev.dof, b, 1)
    y = rvec(lev.dof, b, 2)
    zero = torch.zeros(S.level_dof(0), dtype=torch.float64, device=DEV)
    LTx = -to_oracle(S.residual(to_gpu(x), zero, transpose=True), b)
    Ly = -to_oracle(S.residual(to_gpu(y), zero), b)
    assert abs(np.sum(LTx * y) - np.sum(x * Ly)) < 1e-12 * np.sqrt(np.sum(LTx ** 2) * np.sum(y ** 2))
    # adjoint solve against the oracle's backward block substitution
    g = rvec(lev.dof, b, 3)
    lam, gf, gu0, its, hist = S.adjoint(to_gpu(g), rtol=1e-12, maxit=40)
    ref = spacetime.forward_substitution(lev, g, transpose=True)
    assert norm_rel(to_oracle(lam, b), ref) < 1e-10
    gf_ref, gu0_ref = spacetime.rhs_adjoint(lev, ref)
    assert rel_err(gf.cpu().numpy().reshape(gf_ref.shape), gf_ref) < 1e-10
    assert rel_err(gu0.cpu().numpy().reshape(gu0_ref.shape), gu0_ref) < 1e-10


def test_autograd_gradients_match_finite_differences():
    from paper_1411_0519_amd.autograd import heat_solve
    d, n, N, pt = 2, 15, 16, 1
    S = stmg.Solver(d, n, N, pt=pt, device=DEV)
    f, u0 = workloads.make(d, n, N, seed=21, f="uniform", u0="sine1")
    ud_nodal = workloads.target_state(d, n, seed=55)
    # target in coefficient space: time-constant, only the l = 0 coefficient
    ud = np.zeros((N, pt + 1, n ** d))
    ud[:, 0, :] = ud_nodal
    ud_g = torch.from_numpy(ud.ravel()).to(DEV)
    fg = nodal_to_gpu(f).requires_grad_(True)
    u0g = nodal_to_gpu(u0).requires_grad_(True)

    def J(fv, u0v):
        u = heat_solve(fv, u0v, S, rtol=1e-13)
        return 0.5 * torch.sum((u - ud_g) ** 2)

    loss = J(fg, u0g)
    loss.backward()
    gf, gu0 = fg.grad.detach().clone(), u0g.grad.detach().clone()
    # oracle: lambda = L^{-T}(u - u_d), gradients by the transposed load map
    lev = spacetime.SpaceTimeLevel(d, n, N, pt, 1.0 / N)
    F = spacetime.rhs(lev, f, u0)
    u_ex = spacetime.forward_substitution(lev, F)
    lam = spacetime.forward_substitution(lev, u_ex - ud.reshape(-1, 1), transpose=True)
    gf_ref, gu0_ref = spacetime.rhs_adjoint(lev, lam)
    assert rel_err(gf.cpu().numpy().reshape(gf_ref.shape), gf_ref) < 1e-9
    assert rel_err(gu0.cpu().numpy().reshape(gu0_ref.shape), gu0_ref) < 1e-9
    # central differences: J is quadratic, so they are exact up to the solve tolerance
    rng = np.random.default_rng(5)
    with torch.no_grad():
        for _ in range(3):
            df = torch.from_numpy(rng.normal(size=f.size)).to(DEV)
            du = torch.from_numpy(rng.normal(size=u0.size)).to(DEV)
            eps = 1e-2
            jp = J(fg + eps * df, u0g + eps * du).item()
            jm = J(fg - eps * df, u0g - eps * du).item()
            fd = (jp - jm) / (2 * eps)
            an = (torch.sum(gf * df) + torch.sum(gu0 * du)).item()
            assert abs(fd - an) <= 1e-7 * max(1.0, abs(an)), (fd, an)


# ------------------------------------------------------------------ W-cycle
@pytest.mark.parametrize("smoother", ["exact", "spatial_mg"])
@pytest.mark.parametrize("case", [(1, 31, 32, 1, 1), (2, 15, 16, 2, 2), (3, 7, 8, 1, 1)],
                         ids=lambda c: "d{}n{}N{}p{}b{}".format(*c))
def test_w_cycle_iterates_match_oracle(case, smoother):
    d, n, N, pt, b = case
    print(f"W-cycle {case} {smoother}", flush=True)
    S = stmg.Solver(d, n, N, pt=pt, batch=b, gamma=2, smoother=smoother, device=DEV)
    H = multigrid.Hierarchy(d, n, N, pt, gamma=2, smoother="inexact" if smoother == "spatial_mg" else "exact")
    f, u0 = workloads.make(d, n, N, batch=b, seed=15, f="uniform", u0="sine1")
    F = spacetime.rhs(H.fine, f, u0)
    _, _, its = H.solve(F, rtol=0.0, maxit=3, keep_iterates=True)
    ug = torch.zeros(S.level_dof(0), dtype=torch.float64, device=DEV)
    for k in range(1, 4):
        S.solve(to_gpu(F), u=ug, rtol=0.0, maxit=1, raise_on_noconv=False)
        assert rel_err(to_oracle(ug, b), its[k]) < 1e-12, k


def test_w_cycle_graph_replay_matches_eager():
    d, n, N, pt = 2, 31, 16, 1
    f, u0 = workloads.make(d, n, N, seed=16, f="uniform", u0="sine1")
    stream = torch.cuda.Stream(device=DEV)
    with torch.cuda.stream(stream):
        E = stmg.Solver(d, n, N, pt=pt, gamma=2, device=DEV)
        G = stmg.Solver(d, n, N, pt=pt, gamma=2, device=DEV)
        G.set_graph(True)
        F = E.rhs(nodal_to_gpu(f), nodal_to_gpu(u0))
        ue, ug = torch.zeros_like(F), torch.zeros_like(F)
        for rep in range(3):
            E.solve(F, u=ue, rtol=0.0, maxit=2, raise_on_noconv=False)
            G.solve(F, u=ug, rtol=0.0, maxit=2, raise_on_noconv=False)
            torch.cuda.synchronize()
            assert torch.equal(ue, ug), rep


# ------------------------------------------------- BF16 inner-cycle transforms
BF16_CASES = [(1, 31, 8, 1, 1), (2, 31, 4, 1, 2), (2, 127, 2, 2, 1), (2, 255, 2, 1, 1), (3, 15, 2, 1, 1)]


@pytest.mark.parametrize("case", BF16_CASES, ids=lambda c: "d{}n{}N{}p{}b{}".format(*c))
@pytest.mark.parametrize("transpose", [False, True])
def test_bf16_block_solve_accuracy(case, transpose):
    # Each folded product rounds its operands (data and sine matrix) to bfloat16
    # (unit roundoff 2^-9) and accumulates in FP32; a d-dimensional block solve
    # has 2d products, so its relative error is bounded by about 2d * 2 * 2^-9.
    d, n, N, pt, b = case
    print(f"bf16 block solve {case} transpose={transpose}", flush=True)
    S = stmg.Solver(d, n, N, pt=pt, batch=b, precision="mixed_bf16", device=DEV)
    lev = spacetime.SpaceTimeLevel(d, n, N, pt, 1.0 / N)
    r = rvec(lev.dof, b, 3).astype(np.float32).astype(np.float64)
    x = to_oracle(S.block_solve(to_gpu(r, torch.float32), prec="fp32", transpose=transpose), b)
    A = (lev.A.T if transpose else lev.A).tocsc()
    import scipy.sparse.linalg as spla
    lu = spla.splu(A)
    rs = r.reshape(N, lev.slab, b).transpose(1, 0, 2).reshape(lev.slab, -1)
    xs = x.reshape(N, lev.slab, b).transpose(1, 0, 2).reshape(lev.slab, -1)
    ref = lu.solve(np.ascontiguousarray(rs))
    err = np.linalg.norm(xs - ref, axis=0) / np.linalg.norm(ref, axis=0)
    print("bf16 relative errors", err.max(), flush=True)
    assert np.all(err <= 4 * d * 2.0 ** -9), err.max()
    assert err.max() > 2.0 ** -24          # the bf16 path really ran (FP32 transforms are far more accurate)


@pytest.mark.parametrize("d,n,N,pt,b", [(2, 31, 32, 1, 1), (3, 15, 16, 1, 1), (2, 63, 32, 2, 2)])
def test_mixed_bf16_reaches_fp64_tolerance(d, n, N, pt, b):
    print(f"mixed bf16 {(d, n, N, pt, b)}", flush=True)
    M = stmg.Solver(d, n, N, pt=pt, batch=b, precision="mixed_bf16", device=DEV)
    S = stmg.Solver(d, n, N, pt=pt, batch=b, device=DEV)
    lev = spacetime.SpaceTimeLevel(d, n, N, pt, 1.0 / N)
    f, u0 = workloads.make(d, n, N, batch=b, seed=4, f="uniform", u0="series16")
    F = spacetime.rhs(lev, f, u0)
    Fg = to_gpu(F)
    um, itm, histm = M.solve(Fg, rtol=1e-10, maxit=40)
    u64, it64, hist64 = S.solve(Fg, rtol=1e-10, maxit=40)
    assert max(histm[-1]) <= 1e-10
    assert itm <= it64 + 4, (itm, it64)
    r = F - lev.L @ to_oracle(um, b)
    assert np.all(np.linalg.norm(r, axis=0) <= 1.01e-10 * np.linalg.norm(F, axis=0))
    assert norm_rel(to_oracle(um, b), spacetime.forward_substitution(lev, F)) < 1e-8


def test_mixed_bf16_graph_replay_matches_eager():
    d, n, N, pt = 2, 31, 16, 1
    f, u0 = workloads.make(d, n, N, seed=17, f="uniform", u0="sine1")
    stream = torch.cuda.Stream(device=DEV)
    with torch.cuda.stream(stream):
        E = stmg.Solver(d, n, N, pt=pt, precision="mixed_bf16", device=DEV)
        G = stmg.Solver(d, n, N, pt=pt, precision="mixed_bf16", device=DEV)
        G.set_graph(True)
        F = E.rhs(nodal_to_gpu(f), nodal_to_gpu(u0))
        ue, ug = torch.zeros_like(F), torch.zeros_like(F)
        for rep in range(3):
            E.solve(F, u=ue, rtol=0.0, maxit=2, raise_on_noconv=False)
            G.solve(F, u=ug, rtol=0.0, maxit=2, raise_on_noconv=False)
            torch.cuda.synchronize()
            assert torch.equal(ue, ug), rep
