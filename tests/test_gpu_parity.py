"""GPU parity: the HIP path (through the C ABI) against the CPU oracle on the
same seeded inputs.  FP64 tolerances: level operators 1e-13, V-cycle iterates
1e-12 relative (elementwise against the oracle's max)."""
import numpy as np
import pytest
import torch

from gpu_util import DEV, nodal_to_gpu, norm_rel, rel_err, to_gpu, to_oracle
from oracle import multigrid, spacetime
from paper_1411_0519_amd import workloads

pytestmark = pytest.mark.gpu

stmg = pytest.importorskip("paper_1411_0519_amd.stmg")

# (dim, n, N, pt, batch): several transform tiles, ragged tails (n = 2^m - 1
# is never a multiple of the 16-wide MFMA blocks), every supported order.
OPERATOR_CASES = [
    (1, 31, 16, 1, 1),
    (1, 255, 8, 1, 2),
    (2, 15, 8, 1, 2),
    (2, 31, 8, 0, 1),
    (2, 31, 4, 2, 1),
    (2, 63, 4, 3, 1),
    (2, 127, 4, 1, 1),
    (3, 7, 4, 2, 1),
    (3, 15, 4, 1, 2),
    (2, 1, 4, 1, 1),
    (3, 1, 2, 0, 1),
]


def case_id(c):
    return "d{}n{}N{}p{}b{}".format(*c)


def make_solver(d, n, N, pt, b, **kw):
    return stmg.Solver(d, n, N, pt=pt, batch=b, device=DEV, **kw)


def random_vec(dof, b, seed):
    return np.random.default_rng(seed).uniform(-1, 1, (dof, b))


@pytest.mark.parametrize("case", OPERATOR_CASES, ids=case_id)
@pytest.mark.parametrize("transpose", [False, True])
def test_residual_parity(case, transpose):
    d, n, N, pt, b = case
    print(f"residual {case} transpose={transpose}", flush=True)
    S = make_solver(d, n, N, pt, b)
    lev = spacetime.SpaceTimeLevel(d, n, N, pt, 1.0 / N)
    u = random_vec(lev.dof, b, 1)
    F = random_vec(lev.dof, b, 2)
    r_ref = F - lev.apply(u, transpose)
    r, nrm = S.residual(to_gpu(u), to_gpu(F), transpose=transpose, norms=True)
    torch.cuda.synchronize()
    assert rel_err(to_oracle(r, b), r_ref) < 1e-13
    assert np.allclose(nrm, np.linalg.norm(r_ref, axis=0), rtol=1e-12)


# The widest 2-D grid: the residual tile shrinks to 4 rows so that its
# staged rows fit one set of prefetched loads.
@pytest.mark.parametrize("case", [(2, 255, 2, 1, 1), (2, 255, 4, 3, 1)], ids=case_id)
def test_residual_parity_wide(case):
    test_residual_parity(case, False)


@pytest.mark.parametrize("case", OPERATOR_CASES, ids=case_id)
@pytest.mark.parametrize("transpose", [False, True])
@pytest.mark.parametrize("impl", ["0", "1", "2"], ids=["auto", "lds", "reg"])
def test_block_solve_parity(case, transpose, impl, monkeypatch):
    d, n, N, pt, b = case
    print(f"block solve {case} transpose={transpose} impl={impl}", flush=True)
    monkeypatch.setenv("STMG_TRANSFORM", impl)      # read at setup: transform kernel family
    S = make_solver(d, n, N, pt, b)
    H = multigrid.Hierarchy(d, n, N, pt, transpose=transpose)
    k = len(H.levels) - 1
    r = random_vec(H.fine.dof, b, 3)
    x_ref = H.block_solve(k, r)
    x = S.block_solve(to_gpu(r), transpose=transpose)
    torch.cuda.synchronize()
    xg = to_oracle(x, b)
    # Backward error of the fast-diagonalisation solve: 2d length-n transform
    # passes and one N_t x N_t solve per mode, each with relative rounding
    # <= n u in the worst case (u = 2^-53): ||A x - r|| <= 8 d n u ||A|| ||x||.
    A = (H.fine.A.T if transpose else H.fine.A).tocsr()
    u_r = 2.0 ** -53
    normA = abs(A).sum(axis=1).max()
    for n_slab in range(H.fine.N * b):
        xs = xg.reshape(H.fine.N, H.fine.slab, b).transpose(1, 0, 2).reshape(H.fine.slab, -1)[:, n_slab]
        rs = r.reshape(H.fine.N, H.fine.slab, b).transpose(1, 0, 2).reshape(H.fine.slab, -1)[:, n_slab]
        be = np.abs(A @ xs - rs).max() / (normA * np.abs(xs).max())
        assert be < 8 * d * n * u_r, (n_slab, be)
    # forward error against the oracle's sparse LU (both carry cond(A) u)
    assert rel_err(xg, x_ref) < 1e-12


TRANSFER_CASES = [
    (1, 31, 16, 1, 1, "auto"), (2, 15, 8, 1, 2, "auto"), (2, 15, 8, 2, 1, "semi"),
    (3, 15, 4, 1, 1, "auto"), (3, 7, 4, 3, 2, "semi"), (2, 127, 4, 1, 1, "auto"),
    (2, 3, 4, 0, 1, "full"),
]


@pytest.mark.parametrize("case", TRANSFER_CASES, ids=lambda c: case_id(c[:5]) + c[5])
def test_transfer_parity(case):
    d, n, N, pt, b, rule = case
    print(f"transfers {case}", flush=True)
    S = make_solver(d, n, N, pt, b, coarsen=rule)
    H = multigrid.Hierarchy(d, n, N, pt, rule={"auto": 0, "semi": 1, "full": 2}[rule])
    assert S.schedule == H.schedule
    for lvl in range(S.nlev - 1):
        k = len(H.levels) - 1 - lvl          # oracle index of this level
        P = H.P[k]
        rf = random_vec(H.levels[k].dof, b, 10 + lvl)
        ec = random_vec(H.levels[k - 1].dof, b, 20 + lvl)
        uf = random_vec(H.levels[k].dof, b, 30 + lvl)
        Fc = S.restrict(to_gpu(rf), level=lvl)
        ug = to_gpu(uf)
        S.prolong_add(to_gpu(ec), ug, level=lvl)
        torch.cuda.synchronize()
        assert rel_err(to_oracle(Fc, b), P.T @ rf) < 1e-13
        assert rel_err(to_oracle(ug, b), uf + P @ ec) < 1e-13


@pytest.mark.parametrize("d,n,N,pt", [(1, 31, 16, 1), (2, 15, 8, 2), (3, 7, 4, 1), (2, 7, 4, 0)])
def test_rhs_parity(d, n, N, pt):
    print(f"rhs {(d, n, N, pt)}", flush=True)
    b = 2
    S = make_solver(d, n, N, pt, b)
    lev = spacetime.SpaceTimeLevel(d, n, N, pt, 1.0 / N)
    f, u0 = workloads.make(d, n, N, batch=b, seed=5, f="uniform", u0="series16")
    F_ref = spacetime.rhs(lev, f, u0)
    F = S.rhs(nodal_to_gpu(f), nodal_to_gpu(u0))
    lam = random_vec(lev.dof, b, 6)
    gf_ref, gu0_ref = spacetime.rhs_adjoint(lev, lam)
    gf, gu0 = S.rhs_adjoint(to_gpu(lam))
    torch.cuda.synchronize()
    assert rel_err(to_oracle(F, b), F_ref) < 1e-13
    assert rel_err(gf.cpu().numpy().reshape(gf_ref.shape), gf_ref) < 1e-13
    assert rel_err(gu0.cpu().numpy().reshape(gu0_ref.shape), gu0_ref) < 1e-13


def run_iterate_parity(d, n, N, pt, b, f_kind, u0_kind, seed, rule="auto", maxit=12, transpose=False,
                       autotune=False):
    S = make_solver(d, n, N, pt, b, coarsen=rule)
    if autotune:
        S.autotune()
    H = multigrid.Hierarchy(d, n, N, pt, rule={"auto": 0, "semi": 1, "full": 2}[rule], transpose=transpose)
    assert S.schedule == H.schedule
    f, u0 = workloads.make(d, n, N, batch=b, seed=seed, f=f_kind, u0=u0_kind)
    F = spacetime.rhs(H.fine, f, u0)
    u_ref, hist_ref, its_ref = H.solve(F, rtol=1e-10, maxit=maxit, keep_iterates=True)
    Fg = to_gpu(F)
    u = torch.zeros_like(Fg)
    worst = 0.0
    for k in range(1, len(its_ref)):
        if transpose:
            lam, _, _, _, _ = S.adjoint(Fg, lam=u, rtol=0.0, maxit=1, gradients=False, raise_on_noconv=False)
        else:
            S.vcycle(u, Fg)
        torch.cuda.synchronize()
        err = rel_err(to_oracle(u, b), its_ref[k])
        worst = max(worst, err)
        assert err < 1e-12, (k, err)
    return worst, len(its_ref) - 1


@pytest.mark.parametrize("case", [
    (1, 31, 16, 1, 1, "uniform", "sine1", 1),     # workload W1 at full size
    (2, 31, 32, 1, 1, "bumps", "sine1", 2),       # W2 family, reduced (mu = 32)
    (2, 63, 64, 1, 1, "bumps", "sine1", 2),       # W2 family, reduced (mu = 64)
    (3, 15, 16, 1, 1, "uniform", "zero", 3),      # W3 family, reduced (mu = 16)
    (2, 15, 16, 2, 3, "uniform", "series16", 4),  # W4 family, reduced, batched
    (1, 15, 64, 0, 1, "uniform", "sine1", 7),     # p_t = 0 with semi steps
], ids=lambda c: case_id(c[:5]))
@pytest.mark.parametrize("small", ["1", "0"], ids=["small-on", "small-off"])
def test_vcycle_iterate_parity(case, small, monkeypatch):
    d, n, N, pt, b, fk, uk, seed = case
    print(f"vcycle iterates {case} small={small}", flush=True)
    monkeypatch.setenv("STMG_SMALL", small)     # one-kernel smoothing on levels that fit in LDS
    worst, its = run_iterate_parity(d, n, N, pt, b, fk, uk, seed)
    assert its >= 5


@pytest.mark.parametrize("case", [(2, 63, 64, 1, 1), (3, 15, 16, 2, 1), (1, 255, 32, 1, 2)], ids=case_id)
def test_autotuned_iterate_parity(case):
    d, n, N, pt, b = case
    print(f"autotuned iterates {case}", flush=True)
    run_iterate_parity(d, n, N, pt, b, "uniform", "sine1", 13, autotune=True)


@pytest.mark.parametrize("small", ["1", "0"], ids=["small-on", "small-off"])
def test_adjoint_iterate_parity(small, monkeypatch):
    print(f"adjoint iterates small={small}", flush=True)
    monkeypatch.setenv("STMG_SMALL", small)
    run_iterate_parity(2, 31, 32, 1, 1, "uniform", "sine1", 5, transpose=True)


@pytest.mark.parametrize("rule", ["semi", "full"])
def test_vcycle_parity_other_rules(rule):
    print(f"vcycle rule {rule}", flush=True)
    run_iterate_parity(2, 15, 16, 1, 1, "uniform", "sine1", 9, rule=rule, maxit=30)


def test_solve_matches_oracle_and_direct():
    d, n, N, pt, b = 2, 31, 32, 1, 2
    print("solve", flush=True)
    S = make_solver(d, n, N, pt, b)
    H = multigrid.Hierarchy(d, n, N, pt)
    f, u0 = workloads.make(d, n, N, batch=b, seed=11, f="uniform", u0="series16")
    F = spacetime.rhs(H.fine, f, u0)
    u_ref, hist_ref, _ = H.solve(F, rtol=1e-10)
    u, its, hist = S.solve(to_gpu(F), rtol=1e-10)
    assert its == len(hist_ref) - 1
    assert np.allclose(np.array(hist), hist_ref, rtol=1e-8, atol=1e-15)
    assert rel_err(to_oracle(u, b), u_ref) < 1e-12
    exact = spacetime.forward_substitution(H.fine, F)
    assert norm_rel(to_oracle(u, b), exact) < 1e-8


def test_single_slab_and_single_node():
    # N = 1: the fine level is the coarsest, one V-cycle is an exact solve.
    for (d, n, N) in ((2, 15, 1), (1, 1, 8), (3, 1, 1)):
        print(f"edge {(d, n, N)}", flush=True)
        S = make_solver(d, n, N, 1, 1)
        lev = spacetime.SpaceTimeLevel(d, n, N, 1, 1.0 / N)
        F = random_vec(lev.dof, 1, 4)
        u, its, hist = S.solve(to_gpu(F), rtol=1e-12, maxit=50)
        exact = spacetime.forward_substitution(lev, F)
        assert norm_rel(to_oracle(u, 1), exact) < 1e-11
        if N == 1:
            assert its == 1


def test_zero_rhs_gives_zero():
    S = make_solver(2, 15, 8, 1, 1)
    F = torch.zeros(S.level_dof(0), dtype=torch.float64, device=DEV)
    u, its, hist = S.solve(F)
    assert its == 0 and hist[0][0] == 0.0 and torch.count_nonzero(u) == 0


def test_error_paths():
    S = make_solver(2, 15, 8, 1, 1)
    F = torch.ones(S.level_dof(0), dtype=torch.float64, device=DEV)
    u = torch.zeros_like(F)
    with pytest.raises(stmg.STMGError) as e:
        S.solve(F, u=u, rtol=1e-14, maxit=1)
    assert e.value.code == stmg.ST_ENOCONV
    F[5] = float("nan")
    with pytest.raises(stmg.STMGError) as e:
        S.solve(F, u=torch.zeros_like(F), maxit=3)
    assert e.value.code == stmg.ST_ENAN
    with pytest.raises(ValueError):
        S.solve(F[:-1])
    with pytest.raises(ValueError):
        S.residual(u, F, level=S.nlev)
    # the C ABI checks the level itself
    rc = stmg.lib().st_mg_residual(S._h, S.nlev, stmg.FP64, 0, stmg._ptr(u), stmg._ptr(F), stmg._ptr(u),
                                   None, None)
    assert rc == stmg.ST_EINVAL
