"""Pins of the oracle's DG-in-time pieces against the paper and textbook facts."""
import json
import math
import os

import numpy as np
import pytest
from numpy.polynomial import Legendre

from oracle import dg_time

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def pade_subdiagonal(p, z):
    """Textbook (p, p+1) Pade approximant of e^z (numerator degree p,
    denominator degree p+1), written from the classical coefficient formula."""
    m, n = p, p + 1
    num = sum(math.factorial(m + n - j) * math.factorial(m)
              / (math.factorial(m + n) * math.factorial(j) * math.factorial(m - j)) * z ** j
              for j in range(m + 1))
    den = sum(math.factorial(m + n - j) * math.factorial(n)
              / (math.factorial(m + n) * math.factorial(j) * math.factorial(n - j)) * (-z) ** j
              for j in range(n + 1))
    return num / den


def test_pt0_is_backward_euler():
    # Sec. 1: p_t = 0 gives backward Euler: K = 1, M = tau, N = 1.
    for tau in (1.0, 0.25, 1e-3):
        K, M, N = dg_time.time_matrices(0, tau)
        assert K.shape == (1, 1)
        assert abs(K[0, 0] - 1.0) < 1e-15
        assert abs(M[0, 0] - tau) < 1e-15 * max(1, tau)
        assert abs(N[0, 0] - 1.0) < 1e-15


@pytest.mark.parametrize("pt", range(6))
def test_stability_function_is_subdiagonal_pade(pt):
    # Lemma chap4_theorem2: the nonzero eigenvalue of (K + lam M)^{-1} N is the
    # (p_t, p_t+1) subdiagonal Pade approximation of e^z at z = -lam tau.
    zs = list(-np.logspace(-3, 3, 25)) + [-0.5 + 2j, 1.5j, -3 - 1j]
    for z in zs:
        r = dg_time.stability_function(pt, z)
        ref = pade_subdiagonal(pt, z)
        assert abs(r - ref) <= 1e-12 * max(1.0, abs(ref)), (pt, z, r, ref)


@pytest.mark.parametrize("pt", range(4))
def test_spectrum_is_zero_and_R(pt):
    # Lemma chap4_theorem2: sigma((K + lam M)^{-1} N) = {0, R(-lam tau)}.
    tau = 0.37
    K, M, N = dg_time.time_matrices(pt, tau)
    for lam in (0.1, 3.0, 250.0):
        ev = np.sort_complex(np.linalg.eigvals(np.linalg.solve(K + lam * M, N)))
        nz = ev[np.argmax(np.abs(ev))]
        assert abs(nz - pade_subdiagonal(pt, -lam * tau)) < 1e-12
        assert np.sum(np.abs(ev) > 1e-12) <= 1


def test_pt1_poles():
    # Eigenvalues of M^{-1} K are the poles of R at z = -lam tau: for p_t = 1,
    # 1 - 2z/3 + z^2/6 = 0, i.e. lam = -(2 +- i sqrt 2)/tau in -lam convention.
    tau = 0.5
    K, M, _ = dg_time.time_matrices(1, tau)
    ev = np.sort_complex(np.linalg.eigvals(np.linalg.solve(M, K)))
    ref = np.sort_complex(np.array([2 - 1j * math.sqrt(2), 2 + 1j * math.sqrt(2)]) / tau)
    assert np.allclose(ev, ref, atol=1e-12)


def test_mu_star_printed_values():
    gold = json.load(open(os.path.join(GOLD, "mu_star.json")))
    for p, v in gold["mu_star"].items():
        assert abs(dg_time.mu_star(int(p)) - v) < 1e-10 / 2 + 1e-12, (p, dg_time.mu_star(int(p)), v)
    assert abs(dg_time.mu_star(0) - math.sqrt(2) / 3) < 1e-12
    assert abs(dg_time.mu_star(1) - (-3 - math.sqrt(2) + math.sqrt(11 + 12 * math.sqrt(2))) / 3) < 1e-12
    # mu*_p tends to the exp-based value (R -> e^z as p -> inf)
    mu_inf = math.log(math.sqrt(2) - 1) / -3.0
    assert abs(mu_inf - gold["mu_star_inf"]) < 1e-10
    assert abs(dg_time.mu_star(6) - mu_inf) < 1e-6


@pytest.mark.parametrize("pt", range(5))
def test_time_prolongation_embeds_coarse_polynomials(pt):
    # eq. chap4_restrictionTime: R_s^T = M^{-1} Mtilde^s is the L2 projection of
    # the coarse basis onto the fine slabs; coarse polynomials lie in the fine
    # space, so the fine expansion must reproduce them pointwise.
    tau = 0.3
    R1T, R2T = dg_time.time_prolongation_blocks(pt, tau)
    rng = np.random.default_rng(7)
    c = rng.normal(size=pt + 1)
    coarse = lambda t: sum(c[l] * Legendre.basis(l)(t / tau - 1.0) for l in range(pt + 1))
    for half, RT in ((0, R1T), (1, R2T)):
        f = RT @ c
        t = np.linspace(half * tau, (half + 1) * tau, 11)
        s = 2 * (t - half * tau) / tau - 1
        fine = sum(f[k] * Legendre.basis(k)(s) for k in range(pt + 1))
        assert np.allclose(fine, coarse(t), atol=1e-13)


def test_pt1_prolongation_blocks_values():
    R1T, R2T = dg_time.time_prolongation_blocks(1, 1.0)
    assert np.allclose(R1T, [[1, -0.5], [0, 0.5]], atol=1e-15)
    assert np.allclose(R2T, [[1, 0.5], [0, 0.5]], atol=1e-15)


@pytest.mark.parametrize("pt", range(4))
def test_slab_integrals_and_traces(pt):
    tau = 0.7
    ints = dg_time.slab_integrals(pt, tau)
    assert abs(ints[0] - tau) < 1e-15 and np.all(np.abs(ints[1:]) < 1e-15)
    a = dg_time.left_trace(pt)
    b = dg_time.right_trace(pt)
    assert np.allclose(a, [(-1) ** k for k in range(pt + 1)])
    assert np.allclose(b, 1.0)
    _, _, N = dg_time.time_matrices(pt, tau)
    assert np.allclose(N, np.outer(a, b))
