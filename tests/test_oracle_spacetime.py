"""Pins of the oracle's space-time system against exact or textbook results."""
import math

import numpy as np
import pytest
import scipy.sparse.linalg as spla
from numpy.polynomial import Legendre
from numpy.polynomial import legendre as npleg

from oracle import dg_time, fe_space, spacetime


def pade(p, z):
    m, n = p, p + 1
    num = sum(math.factorial(m + n - j) * math.factorial(m)
              / (math.factorial(m + n) * math.factorial(j) * math.factorial(m - j)) * z ** j
              for j in range(m + 1))
    den = sum(math.factorial(m + n - j) * math.factorial(n)
              / (math.factorial(m + n) * math.factorial(j) * math.factorial(n - j)) * (-z) ** j
              for j in range(n + 1))
    return num / den


@pytest.mark.parametrize("d,n", [(1, 15), (2, 7)])
def test_pt0_equals_backward_euler(d, n):
    # Sec. 1: p_t = 0 is backward Euler: (M + tau K) u_n = M u_{n-1} + tau M f_n.
    N, tau = 8, 0.05
    lev = spacetime.SpaceTimeLevel(d, n, N, 0, tau)
    rng = np.random.default_rng(3)
    f = rng.uniform(-1, 1, (1, N, lev.nx))
    u0 = rng.uniform(-1, 1, (1, lev.nx))
    F = spacetime.rhs(lev, f, u0)
    u = spla.spsolve(lev.L.tocsc(), F[:, 0]).reshape(N, lev.nx)
    M, K = fe_space.q1_matrices(d, n)
    prev = u0[0]
    for k in range(N):
        ref = spla.spsolve((M + tau * K).tocsc(), M @ prev + tau * (M @ f[0, k]))
        assert np.allclose(u[k], ref, rtol=1e-12, atol=1e-13)
        prev = ref


@pytest.mark.parametrize("d,pt", [(1, 1), (2, 2), (3, 1)])
def test_forward_substitution_matches_direct(d, pt):
    n, N = 3, 4
    lev = spacetime.SpaceTimeLevel(d, n, N, pt, 0.1)
    rng = np.random.default_rng(5)
    F = rng.normal(size=(lev.dof, 2))
    for tr in (False, True):
        u = spacetime.forward_substitution(lev, F, transpose=tr)
        Lm = (lev.L.T if tr else lev.L).tocsc()
        ref = np.stack([spla.spsolve(Lm, F[:, i]) for i in range(2)], axis=1)
        assert np.allclose(u, ref, rtol=1e-12, atol=1e-13)


@pytest.mark.parametrize("d,pt", [(1, 0), (1, 1), (2, 1), (2, 2), (3, 1)])
def test_end_of_slab_closed_form(d, pt):
    # f = 0, u0 = prod sin(pi x_i): the fully discrete solution stays in the
    # first sine mode and its end-of-slab trace is R(-lam_h tau)^n u0_h with
    # lam_h = d * (6/h^2)(1 - cos pi h)/(2 + cos pi h) (Lemma chap4_theorem2).
    n, N, tau = 7, 6, 0.02
    h = 1.0 / (n + 1)
    lev = spacetime.SpaceTimeLevel(d, n, N, pt, tau)
    x = fe_space.node_coordinates(d, n)
    u0 = np.prod(np.sin(np.pi * x), axis=1)
    F = spacetime.rhs(lev, np.zeros((1, N, lev.nx)), u0[None])
    u = spla.spsolve(lev.L.tocsc(), F[:, 0]).reshape(N, lev.nt, lev.nx)
    lam = d * 6 / h ** 2 * (1 - math.cos(math.pi * h)) / (2 + math.cos(math.pi * h))
    R = pade(pt, -lam * tau)
    bvec = dg_time.right_trace(pt)
    for k in range(N):
        end = np.tensordot(bvec, u[k], axes=(0, 0))
        assert np.allclose(end, R ** (k + 1) * u0, rtol=1e-12, atol=1e-14)


def _mms_error(n, N, pt, T=0.5):
    """1-D MMS: u = e^{-t} sin(pi x), f = (pi^2 - 1) u.  Load vector by exact
    space integrals of sin against hats and Gauss quadrature in time; returns
    the max end-of-slab nodal error."""
    h = 1.0 / (n + 1)
    tau = T / N
    lev = spacetime.SpaceTimeLevel(1, n, N, pt, tau)
    x = fe_space.node_coordinates(1, n)[:, 0]
    sx = np.sin(np.pi * x) * 2 * (1 - math.cos(math.pi * h)) / (math.pi ** 2 * h)   # int sin(pi x) phi_j
    s, w = npleg.leggauss(12)
    F = np.zeros((N, pt + 1, n))
    for k in range(N):
        t = k * tau + 0.5 * tau * (s + 1)
        for l in range(pt + 1):
            tl = np.sum(w * np.exp(-t) * Legendre.basis(l)(s)) * 0.5 * tau
            F[k, l] = (math.pi ** 2 - 1) * tl * sx
    u0 = np.sin(np.pi * x)
    a = dg_time.left_trace(pt)
    for l in range(pt + 1):
        F[0, l] += a[l] * (lev.Mh @ u0)
    u = spla.spsolve(lev.L.tocsc(), F.ravel()).reshape(N, pt + 1, n)
    ends = u.sum(axis=1)                     # psi_l(t_n^-) = 1
    exact = np.exp(-tau * np.arange(1, N + 1))[:, None] * np.sin(np.pi * x)[None]
    return np.abs(ends - exact).max()


@pytest.mark.parametrize("pt", [0, 1])
def test_mms_time_order_at_slab_ends(pt):
    # DG(p_t) is superconvergent at slab ends, order 2 p_t + 1 (textbook; the
    # paper cites Thomee).  Fine space grid so the time error dominates.
    n = 255
    e1 = _mms_error(n, 4, pt)
    e2 = _mms_error(n, 8, pt)
    rate = math.log2(e1 / e2)
    assert abs(rate - (2 * pt + 1)) < 0.35, rate


def test_mms_space_order():
    # Q1/P1 in 1-D: second order at the nodes; p_t = 2 so time error is negligible.
    e1 = _mms_error(7, 16, 2)
    e2 = _mms_error(15, 16, 2)
    rate = math.log2(e1 / e2)
    assert abs(rate - 2.0) < 0.25, rate


@pytest.mark.parametrize("d,pt", [(1, 1), (2, 0), (2, 2)])
def test_rhs_adjoint_is_transpose(d, pt):
    lev = spacetime.SpaceTimeLevel(d, 3, 4, pt, 0.2)
    rng = np.random.default_rng(11)
    f = rng.normal(size=(2, 4, lev.nx))
    u0 = rng.normal(size=(2, lev.nx))
    lam = rng.normal(size=(lev.dof, 2))
    F = spacetime.rhs(lev, f, u0)
    gf, gu0 = spacetime.rhs_adjoint(lev, lam)
    lhs = np.sum(F * lam)
    rhs = np.sum(f * gf) + np.sum(u0 * gu0)
    assert abs(lhs - rhs) < 1e-12 * (abs(lhs) + 1)


def test_L_is_block_lower_bidiagonal():
    # eq. chap4_generalLinearSystem
    lev = spacetime.SpaceTimeLevel(2, 3, 3, 1, 0.1)
    Ld = lev.L.toarray()
    S = lev.slab
    A = lev.A.toarray()
    B = lev.B.toarray()
    for i in range(3):
        for j in range(3):
            blk = Ld[i * S:(i + 1) * S, j * S:(j + 1) * S]
            ref = A if i == j else (B if i == j + 1 else np.zeros_like(A))
            assert np.allclose(blk, ref)
