"""The coarse end of the cycle in one workgroup (levels whose vectors fit in
LDS) gives the same iterates as the kernel-per-step path, and the oracle's."""
import numpy as np
import pytest
import torch

from gpu_util import DEV, rel_err, to_gpu, to_oracle
from oracle import multigrid

pytestmark = pytest.mark.gpu

stmg = pytest.importorskip("paper_1411_0519_amd.stmg")

CASES = [(2, 63, 64, 1, 1, 1), (2, 31, 32, 1, 2, 2), (1, 255, 64, 2, 1, 1), (3, 15, 16, 1, 1, 2),
         (2, 63, 256, 0, 1, 1), (2, 15, 8, 3, 1, 1)]


def cid(c):
    return "d{}n{}N{}p{}b{}g{}".format(*c)


def pair(case, monkeypatch, **kw):
    d, n, N, pt, b, gamma = case
    T = stmg.Solver(d, n, N, pt=pt, batch=b, gamma=gamma, device=DEV, **kw)
    monkeypatch.setenv("STMG_COARSE_TAIL", "0")
    R = stmg.Solver(d, n, N, pt=pt, batch=b, gamma=gamma, device=DEV, **kw)
    monkeypatch.delenv("STMG_COARSE_TAIL")
    return T, R


@pytest.mark.parametrize("case", CASES, ids=cid)
@pytest.mark.parametrize("transpose", [False, True])
def test_tail_matches_kernel_per_step_path(case, transpose, monkeypatch):
    print(f"coarse tail {case} transpose={transpose}", flush=True)
    d, n, N, pt, b, gamma = case
    T, R = pair(case, monkeypatch)
    dof = T.level_dof(0)
    F = torch.from_numpy(np.random.default_rng(3).uniform(-1, 1, dof)).to(DEV)
    ut = torch.zeros_like(F)
    ur = torch.zeros_like(F)
    for k in range(3):
        if transpose:
            T.adjoint(F, lam=ut, rtol=0.0, maxit=1, gradients=False, raise_on_noconv=False)
            R.adjoint(F, lam=ur, rtol=0.0, maxit=1, gradients=False, raise_on_noconv=False)
        else:
            T.solve(F, u=ut, rtol=0.0, maxit=1, raise_on_noconv=False)
            R.solve(F, u=ur, rtol=0.0, maxit=1, raise_on_noconv=False)
        err = ((ut - ur).abs().max() / ur.abs().max()).item()
        assert err < 1e-13, (k, err)


def test_tail_iterates_match_oracle():
    d, n, N, pt = 2, 31, 64, 1
    S = stmg.Solver(d, n, N, pt=pt, device=DEV)
    H = multigrid.Hierarchy(d, n, N, pt)
    F = np.random.default_rng(4).uniform(-1, 1, (H.fine.dof, 1))
    _, _, its = H.solve(F, rtol=0.0, maxit=3, keep_iterates=True)
    u = torch.zeros(S.level_dof(0), dtype=torch.float64, device=DEV)
    for k in range(1, 4):
        S.solve(to_gpu(F), u=u, rtol=0.0, maxit=1, raise_on_noconv=False)
        assert rel_err(to_oracle(u, 1), its[k]) < 1e-12, k


def test_tail_fp32(monkeypatch):
    T, R = pair((2, 63, 64, 1, 1, 1), monkeypatch, precision="fp32")
    F = torch.from_numpy(np.random.default_rng(5).uniform(-1, 1, T.level_dof(0))).to(DEV, torch.float32)
    ut, _, ht = T.solve(F, rtol=1e-5, maxit=30)
    ur, _, hr = R.solve(F, rtol=1e-5, maxit=30)
    assert len(ht) == len(hr)
    assert ((ut - ur).abs().max() / ur.abs().max()).item() < 1e-5


def test_tail_in_graph_replay():
    S = stmg.Solver(2, 63, 64, pt=1, device=DEV)
    E = stmg.Solver(2, 63, 64, pt=1, device=DEV)
    stream = torch.cuda.Stream(device=DEV)
    with torch.cuda.stream(stream):
        S.set_graph(True)
        F = torch.from_numpy(np.random.default_rng(6).uniform(-1, 1, S.level_dof(0))).to(DEV)
        ug = torch.zeros_like(F)
        ue = torch.zeros_like(F)
        for rep in range(3):
            S.solve(F, u=ug, rtol=0.0, maxit=2, raise_on_noconv=False)
            E.solve(F, u=ue, rtol=0.0, maxit=2, raise_on_noconv=False)
            torch.cuda.synchronize()
            assert torch.equal(ug, ue), rep
