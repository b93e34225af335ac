"""Pins of the oracle's inexact smoother (one spatial multigrid cycle per slab,
Remark V-cycleApproxSpace) against what the mathematics and the paper fix:
the single-node cycle is exact, the Galerkin identity of the spatial
transfers, the rigorous Fourier analysis of the spatial two-grid cycle on the
Dirichlet grid (sine modes are invariant pairs), the remark's LFA claims, the
measured contraction against the LFA, and the iteration range of the paper's
numerical example."""
import json
import os

import numpy as np
import pytest

from oracle import dg_time, lfa, multigrid, spacetime
from oracle.spatial_mg import SpatialCycle, spatial_sizes

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
XOPTS = dict(nu1x=2, nu2x=2, omega_x=2.0 / 3.0)


def test_spatial_sizes():
    assert spatial_sizes(127) == [127, 63, 31, 15, 7, 3, 1]
    assert spatial_sizes(1) == [1]
    assert spatial_sizes(31, depth=1) == [31, 15]


@pytest.mark.parametrize("d,pt", [(1, 0), (2, 1), (3, 2)])
def test_single_node_cycle_is_exact(d, pt):
    # n = 1: the cycle is the coarsest-level exact solve, so (I - M^x) A^{-1} = A^{-1}
    lev = spacetime.SpaceTimeLevel(d, 1, 1, pt, 0.25)
    sc = SpatialCycle(d, 1, pt, 0.25)
    f = np.random.default_rng(1).normal(size=(lev.slab, 3))
    x = sc.cycle(f)
    assert np.abs(lev.A @ x - f).max() < 1e-14 * np.abs(f).max()


@pytest.mark.parametrize("d", [1, 2, 3])
def test_spatial_galerkin_identity(d):
    # P_x^T A_h P_x = A_{2h} for Q1 (nested spaces), per time block
    pt, tau = 1, 0.01
    n = 7 if d == 3 else 15
    sc = SpatialCycle(d, n, pt, tau, depth=1)
    P = sc.P[0]
    G = (P.T @ sc.A[0] @ P).toarray()
    assert np.abs(G - sc.A[1].toarray()).max() < 1e-13 * np.abs(G).max()


def test_spatial_galerkin_in_symbol_space():
    sym = lfa.Symbols(1, 0.37 / 64 ** 2, 1 / 64)
    n = sym.nt
    for tx in (0.1, 0.7, -1.3, np.pi / 2):
        gx = lfa.gamma(tx)
        I = np.eye(n)
        Rt = np.concatenate([sym.Rx(tx) * I, sym.Rx(gx) * I], axis=1)
        Pt = np.concatenate([sym.Px(tx) * I, sym.Px(gx) * I], axis=0)
        At = np.zeros((2 * n, 2 * n))
        At[:n, :n] = sym.Ahat(tx)
        At[n:, n:] = sym.Ahat(gx)
        Ac = sym.Ahat(2 * tx, h=2 * sym.h)
        assert np.abs(Rt @ At @ Pt - Ac).max() < 1e-12 * np.abs(Ac).max()


@pytest.mark.parametrize("pt", [0, 1, 2])
@pytest.mark.parametrize("mu", [1e-3, 1.0, 1e3])
def test_spatial_two_grid_equals_fourier_symbols(pt, mu):
    # Dirichlet grid, d = 1: sin(k pi x) and sin((n+1-k) pi x) span invariant
    # pairs of the two-grid cycle (mass/stiffness/Jacobi are diagonal in the
    # sine basis, full weighting and linear interpolation couple exactly the
    # pair).  So the eigenvalues of the assembled M^x are those of
    # M-tilde(theta_k), theta_k = k pi h, k = 1..(n-1)/2, plus those of the
    # pure smoother S_x(pi/2)^(nu1+nu2) on the mode k = (n+1)/2 that vanishes at
    # the coarse nodes.
    n = 31
    h = 1.0 / (n + 1)
    tau = mu * h * h
    sc = SpatialCycle(1, n, pt, tau, nu1=2, nu2=2, omega=2.0 / 3.0, depth=1)
    ev_dense = np.linalg.eigvals(sc.iteration_matrix())
    sym = lfa.Symbols(pt, tau, h)
    ev_sym = []
    for k in range(1, (n - 1) // 2 + 1):
        ev_sym.extend(np.linalg.eigvals(sym.Mx(k * np.pi * h, **XOPTS)))
    ev_sym.extend(np.linalg.eigvals(np.linalg.matrix_power(sym.Sx(np.pi / 2, 2.0 / 3.0), 4)))
    ev_sym = np.array(ev_sym)
    assert len(ev_sym) == len(ev_dense)
    rho_d, rho_s = np.abs(ev_dense).max(), np.abs(ev_sym).max()
    assert abs(rho_d - rho_s) <= 1e-10 * max(rho_s, 1e-3), (rho_d, rho_s)
    assert np.allclose(np.sort(np.abs(ev_dense)), np.sort(np.abs(ev_sym)), rtol=1e-7, atol=1e-12)
    assert rho_d < 0.2         # a working spatial two-grid cycle


def test_inexact_lfa_claims():
    # Remark V-cycleApproxSpace: with nu1x = nu2x = 2, omega_x = 2/3 the
    # semi-coarsening factors stay <= 1/2 for every mu, are a little larger than
    # with the exact inverse for small mu, and full coarsening is very close to
    # the exact-inverse case.
    g = dict(nx_grid=64, nt_grid=16)
    for pt in (0, 1):
        for nu in (1, 2):
            for mu in (1e-6, 1e-2, 1.0, 1e2, 1e6):
                inex = lfa.two_grid_factor(pt, mu, "s", nu, nu, xopts=XOPTS, **g)
                ex = lfa.two_grid_factor(pt, mu, "s", nu, nu, **g)
                assert inex <= 0.5 + 1e-9, (pt, nu, mu, inex)
                assert inex >= ex - 1e-3, (pt, nu, mu, inex, ex)     # never markedly better
    assert lfa.two_grid_factor(1, 1e-6, "s", 1, 1, xopts=XOPTS, **g) > \
        lfa.two_grid_factor(1, 1e-6, "s", 1, 1, **g) + 0.05
    for pt in (0, 1):
        ms = dg_time.mu_star(pt)
        for mu in (2 * ms, 10 * ms):
            inex = lfa.two_grid_factor(pt, mu, "f", 1, 1, xopts=XOPTS, **g)
            ex = lfa.two_grid_factor(pt, mu, "f", 1, 1, **g)
            assert abs(inex - ex) < 0.01, (pt, mu, inex, ex)


@pytest.mark.slow
@pytest.mark.parametrize("mu,kind", [(64.0, "s"), (1e-2, "s"), (64.0, "f")])
def test_measured_inexact_two_grid_matches_lfa(mu, kind):
    # The remark reports that the numerical factors coincide with the theory:
    # f = 0, random u0 in [0, 1], space-time two-grid cycle, spatial two-grid
    # inside the smoother (depth 1, as in the analysis), p_t = 1, nu = 1.
    n, N, pt = 127, 64, 1
    h = 1.0 / (n + 1)
    T = mu * h ** 2 * N
    rule = multigrid.FULL if kind == "f" else multigrid.SEMI
    H = multigrid.Hierarchy(1, n, N, pt, T=T, nu1=1, nu2=1, rule=rule, smoother="inexact", depth_x=1)
    rng = np.random.default_rng(0)
    u0 = rng.uniform(0, 1, (H.fine.dof, 1))
    meas = multigrid.measured_contraction(H, u0, np.zeros_like(u0), iters=60)
    theory = lfa.two_grid_factor(pt, mu, kind, 1, 1, nx_grid=256, nt_grid=64, xopts=XOPTS)
    assert abs(meas - theory) <= 0.05 * theory, (meas, theory)


@pytest.mark.parametrize("d,n,N", [(1, 63, 64), (2, 15, 16), (2, 31, 32), (3, 7, 8)])
def test_inexact_iterations_in_paper_range(d, n, N):
    # Sec. 4 example protocol (f = 0, random u0 in [0,1], eps_MG = 1e-8, nu = 2,
    # omega_t = 1/2, one spatial V-cycle with nu_x = 2, omega_x = 2/3, p_t = 1):
    # the printed counts lie in 7..9.  Their meshes are P1 simplices, ours Q1,
    # so this is a range check.
    with open(os.path.join(GOLDEN, "iterations.json")) as fh:
        lo, hi = json.load(fh)["table1_range"]
    H = multigrid.Hierarchy(d, n, N, 1, smoother="inexact")
    u0 = np.random.default_rng(3).uniform(0, 1, (H.fine.dof, 1))
    _, hist, _ = H.solve(np.zeros_like(u0), u=u0, rtol=1e-8, maxit=40)
    its = len(hist) - 1
    assert lo - 1 <= its <= hi + 1, its


def test_inexact_solver_converges_to_direct_solution():
    d, n, N, pt = 2, 15, 8, 2
    H = multigrid.Hierarchy(d, n, N, pt, smoother="inexact")
    F = np.random.default_rng(4).normal(size=(H.fine.dof, 2))
    u, hist, _ = H.solve(F, rtol=1e-12, maxit=60)
    ref = spacetime.forward_substitution(H.fine, F)
    assert np.abs(u - ref).max() <= 1e-9 * np.abs(ref).max()


def test_inexact_adjoint_cycle_uses_transposed_blocks():
    # the transposed cycle applied to g equals the transpose of the forward
    # cycle's matrix applied to g (the spatial transfers are symmetric pairs)
    d, n, pt, tau = 2, 7, 1, 0.05
    fw = SpatialCycle(d, n, pt, tau)
    bw = SpatialCycle(d, n, pt, tau, transpose=True)
    m = fw.A[0].shape[0]
    C = fw.cycle(np.eye(m))
    Ct = bw.cycle(np.eye(m))
    assert np.abs(Ct - C.T).max() < 1e-12 * np.abs(C).max()
