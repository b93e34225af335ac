"""GPU parity of the inexact smoother (one spatial multigrid cycle per slab,
Remark V-cycleApproxSpace) against the oracle's SpatialCycle / Hierarchy on
the same seeded inputs, through the C ABI."""
import numpy as np
import pytest
import torch

from gpu_util import DEV, nodal_to_gpu, norm_rel, rel_err, to_gpu, to_oracle
from oracle import multigrid, spacetime
from oracle.spatial_mg import SpatialCycle
from paper_1411_0519_amd import workloads

pytestmark = pytest.mark.gpu

stmg = pytest.importorskip("paper_1411_0519_amd.stmg")

CASES = [
    (1, 31, 8, 1, 1),
    (1, 255, 4, 2, 2),
    (2, 15, 4, 1, 2),
    (2, 63, 4, 0, 1),
    (2, 127, 2, 1, 1),
    (3, 15, 2, 1, 1),
    (3, 7, 4, 3, 1),
    (2, 1, 4, 1, 1),
]


def cid(c):
    return "d{}n{}N{}p{}b{}".format(*c)


def oracle_cycle(d, n, N, pt, tau, r, b, transpose=False, **kw):
    sc = SpatialCycle(d, n, pt, tau, transpose=transpose, **kw)
    slab = (pt + 1) * n ** d
    cols = r.reshape(N, slab, b).transpose(1, 0, 2).reshape(slab, N * b)
    x = sc.cycle(cols)
    return x.reshape(slab, N, b).transpose(1, 0, 2).reshape(N * slab, b)


@pytest.mark.parametrize("case", CASES, ids=cid)
@pytest.mark.parametrize("transpose", [False, True])
def test_spatial_cycle_parity(case, transpose):
    d, n, N, pt, b = case
    print(f"spatial cycle {case} transpose={transpose}", flush=True)
    S = stmg.Solver(d, n, N, pt=pt, batch=b, smoother="spatial_mg", device=DEV)
    dof = N * (pt + 1) * n ** d
    r = np.random.default_rng(5).uniform(-1, 1, (dof, b))
    x = S.spatial_cycle(to_gpu(r), transpose=transpose)
    ref = oracle_cycle(d, n, N, pt, 1.0 / N, r, b, transpose)
    assert rel_err(to_oracle(x, b), ref) < 1e-13


@pytest.mark.parametrize("nu", [(1, 0), (0, 1), (0, 0), (3, 1)])
@pytest.mark.parametrize("omega_x", [2.0 / 3.0, 0.8])
def test_spatial_cycle_parameters(nu, omega_x):
    d, n, N, pt, b = 2, 31, 4, 1, 1
    print(f"spatial cycle nu={nu} omega_x={omega_x}", flush=True)
    S = stmg.Solver(d, n, N, pt=pt, batch=b, smoother="spatial_mg", nu1x=nu[0], nu2x=nu[1], omega_x=omega_x,
                    device=DEV)
    dof = N * (pt + 1) * n ** d
    r = np.random.default_rng(6).uniform(-1, 1, (dof, b))
    x = S.spatial_cycle(to_gpu(r))
    ref = oracle_cycle(d, n, N, pt, 1.0 / N, r, b, nu1=nu[0], nu2=nu[1], omega=omega_x)
    assert rel_err(to_oracle(x, b), ref) < 1e-13


@pytest.mark.skip(reason="the one-kernel LDS tail of the spatial cycle ended in a GPU memory-aperture fault "
                         "with nu1x = 1, nu2x = 0 (2-D n = 31); the cause was not found, so the library runs the "
                         "tail only for nu1x, nu2x >= 2 and this configuration takes the kernel-per-step path")
def test_spatial_tail_with_single_pre_step_and_no_post_step():
    pass


def test_spatial_cycle_on_every_level():
    d, n, N, pt, b = 2, 31, 16, 1, 1
    S = stmg.Solver(d, n, N, pt=pt, batch=b, smoother="spatial_mg", device=DEV)
    for lvl in range(S.nlev):
        L = S.levels[lvl]
        dof = L["N"] * (pt + 1) * L["n"] ** d
        r = np.random.default_rng(10 + lvl).uniform(-1, 1, (dof, b))
        x = S.spatial_cycle(to_gpu(r), level=lvl)
        ref = oracle_cycle(d, L["n"], L["N"], pt, L["tau"], r, b)
        assert rel_err(to_oracle(x, b), ref) < 1e-13, lvl


def test_smoothing_step_parity():
    # st_mg_smooth with the spatial cycle: u + omega D-tilde^{-1} (F - L u)
    d, n, N, pt, b = 2, 15, 8, 2, 2
    S = stmg.Solver(d, n, N, pt=pt, batch=b, smoother="spatial_mg", device=DEV)
    H = multigrid.Hierarchy(d, n, N, pt, smoother="inexact")
    k = len(H.levels) - 1
    rng = np.random.default_rng(7)
    u = rng.uniform(-1, 1, (H.fine.dof, b))
    F = rng.uniform(-1, 1, (H.fine.dof, b))
    ug = to_gpu(u)
    for transpose in (False, True):
        Ht = multigrid.Hierarchy(d, n, N, pt, smoother="inexact", transpose=transpose)
        ug = to_gpu(u)
        S.smooth(ug, to_gpu(F), transpose=transpose)
        assert rel_err(to_oracle(ug, b), Ht.smooth(k, u, F)) < 1e-13


@pytest.mark.parametrize("case", [(1, 63, 32, 1, 1), (2, 31, 16, 1, 2), (3, 15, 8, 1, 1), (2, 15, 16, 0, 1)],
                         ids=cid)
def test_inexact_vcycle_iterates_match_oracle(case):
    d, n, N, pt, b = case
    print(f"inexact iterates {case}", flush=True)
    S = stmg.Solver(d, n, N, pt=pt, batch=b, smoother="spatial_mg", device=DEV)
    H = multigrid.Hierarchy(d, n, N, pt, smoother="inexact")
    assert S.schedule == H.schedule
    f, u0 = workloads.make(d, n, N, batch=b, seed=9, f="uniform", u0="sine1")
    F = spacetime.rhs(H.fine, f, u0)
    _, _, its = H.solve(F, rtol=0.0, maxit=4, keep_iterates=True)
    ug = torch.zeros(S.level_dof(0), dtype=torch.float64, device=DEV)
    Fg = to_gpu(F)
    for k in range(1, 5):
        S.solve(Fg, u=ug, rtol=0.0, maxit=1, raise_on_noconv=False)
        assert rel_err(to_oracle(ug, b), its[k]) < 1e-12, k


def test_inexact_adjoint_iterates_match_oracle():
    d, n, N, pt, b = 2, 15, 16, 1, 1
    S = stmg.Solver(d, n, N, pt=pt, batch=b, smoother="spatial_mg", device=DEV)
    H = multigrid.Hierarchy(d, n, N, pt, smoother="inexact", transpose=True)
    g = np.random.default_rng(11).uniform(-1, 1, (H.fine.dof, b))
    _, _, its = H.solve(g, rtol=0.0, maxit=3, keep_iterates=True)
    lam = torch.zeros(S.level_dof(0), dtype=torch.float64, device=DEV)
    for k in range(1, 4):
        S.adjoint(to_gpu(g), lam=lam, rtol=0.0, maxit=1, gradients=False, raise_on_noconv=False)
        assert rel_err(to_oracle(lam, b), its[k]) < 1e-12, k


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_inexact_solve_reaches_direct_solution(precision):
    d, n, N, pt, b = 2, 31, 32, 1, 2
    S = stmg.Solver(d, n, N, pt=pt, batch=b, smoother="spatial_mg", precision=precision, device=DEV)
    lev = spacetime.SpaceTimeLevel(d, n, N, pt, 1.0 / N)
    f, u0 = workloads.make(d, n, N, batch=b, seed=13, f="uniform", u0="series16")
    F = spacetime.rhs(lev, f, u0)
    u, its, hist = S.solve(to_gpu(F), rtol=1e-10, maxit=40)
    assert max(hist[-1]) <= 1e-10
    assert norm_rel(to_oracle(u, b), spacetime.forward_substitution(lev, F)) < 1e-8


def test_inexact_fp32_cycle():
    d, n, N, pt, b = 2, 63, 4, 1, 1
    S = stmg.Solver(d, n, N, pt=pt, batch=b, smoother="spatial_mg", precision="fp32", device=DEV)
    dof = N * (pt + 1) * n ** d
    r = np.random.default_rng(14).uniform(-1, 1, (dof, b)).astype(np.float32).astype(np.float64)
    x = S.spatial_cycle(to_gpu(r, torch.float32))
    ref = oracle_cycle(d, n, N, pt, 1.0 / N, r, b)
    # float rounding through ~20 stencil/Jacobi/transfer sweeps on values of O(cond) size
    assert rel_err(to_oracle(x, b), ref) < 1e-4


def test_inexact_graph_replay_matches_eager():
    d, n, N, pt = 2, 31, 16, 1
    f, u0 = workloads.make(d, n, N, seed=12, f="uniform", u0="sine1")
    stream = torch.cuda.Stream(device=DEV)
    with torch.cuda.stream(stream):
        E = stmg.Solver(d, n, N, pt=pt, smoother="spatial_mg", device=DEV)
        G = stmg.Solver(d, n, N, pt=pt, smoother="spatial_mg", device=DEV)
        G.set_graph(True)
        F = E.rhs(nodal_to_gpu(f), nodal_to_gpu(u0))
        ue = torch.zeros_like(F)
        ug = torch.zeros_like(F)
        for rep in range(3):
            E.solve(F, u=ue, rtol=0.0, maxit=2, raise_on_noconv=False)
            G.solve(F, u=ug, rtol=0.0, maxit=2, raise_on_noconv=False)
            junk = torch.randn(1 << 16, device=DEV).sum()
            torch.cuda.synchronize()
            assert torch.equal(ue, ug), rep
            del junk


def test_spatial_cycle_needs_spatial_handle():
    S = stmg.Solver(1, 15, 4, device=DEV)
    r = torch.ones(S.level_dof(0), dtype=torch.float64, device=DEV)
    with pytest.raises(stmg.STMGError) as ei:
        S.spatial_cycle(r)
    assert ei.value.code == stmg.ST_ESTATE


def test_inexact_full_size_heat2d_n127_N256():
    # the 127^2 x 256, p_t = 1 workload with the paper's smoother: converges to
    # 1e-10 and sampled slabs satisfy the oracle's slab equations
    w, f, u0 = workloads.workload(2)
    d, n, N, pt = w["dim"], w["n"], w["N"], w["pt"]
    print("inexact W2 full size", flush=True)
    stream = torch.cuda.Stream(device=DEV)
    with torch.cuda.stream(stream):
        S = stmg.Solver(d, n, N, pt=pt, smoother="spatial_mg", device=DEV)
        S.set_graph(True)
        F = S.rhs(nodal_to_gpu(f), nodal_to_gpu(u0))
        u, its, hist = S.solve(F, rtol=1e-10, maxit=30)
        torch.cuda.synchronize()
    assert hist[-1][0] <= 1e-10 and its <= 14
    lev = spacetime.SpaceTimeLevel(d, n, 1, pt, 1.0 / N)
    A, B = lev.A.tocsr(), lev.B.tocsr()
    sz = (pt + 1) * n ** d
    nF = torch.linalg.vector_norm(F).item()
    Fh, uh = F.cpu().numpy(), u.cpu().numpy()
    for k in (0, 77, N - 1):
        r = Fh[k * sz:(k + 1) * sz] - A @ uh[k * sz:(k + 1) * sz]
        if k > 0:
            r -= B @ uh[(k - 1) * sz:k * sz]
        assert np.linalg.norm(r) <= 1e-10 * nF, k
