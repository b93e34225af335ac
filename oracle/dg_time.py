"""DG-in-time matrices and the time transfer operators (oracle, test-only).

Time basis on a slab (t_{n-1}, t_n) of length tau: shifted Legendre
polynomials psi_l(t) = P_l(2 (t - t_{n-1}) / tau - 1), l = 0..p_t.  The paper
leaves the basis open (Sec. 1, definition of the time matrices); the Legendre
choice is a reading recorded with the other readings of the method.

Everything here is computed from the defining integrals by Gauss-Legendre
quadrature, not from closed forms, so the closed forms can pin it.
"""
import numpy as np
from numpy.polynomial import legendre as npleg
from numpy.polynomial import Legendre


def _basis(pt):
    return [Legendre.basis(l) for l in range(pt + 1)]


def _quad(nq):
    x, w = npleg.leggauss(nq)
    return x, w


def time_matrices(pt, tau):
    """K_tau, M_tau, N_tau of Sec. 1 (definitions following eq. (equation1)).

    K[k,l] = -int_slab psi_l d/dt psi_k dt + psi_l(t_n) psi_k(t_n)
    M[k,l] =  int_slab psi_l psi_k dt
    N[k,l] =  psi_l^{n-1}(t_{n-1}) psi_k^{n}(t_{n-1})   (trace of the previous slab)
    """
    P = _basis(pt)
    s, w = _quad(pt + 2)               # exact for degree <= 2 pt + 3
    jac = 0.5 * tau                     # dt = tau/2 ds
    nt = pt + 1
    K = np.zeros((nt, nt))
    M = np.zeros((nt, nt))
    N = np.zeros((nt, nt))
    for k in range(nt):
        dk = P[k].deriv()               # d/ds; d/dt = (2/tau) d/ds
        for l in range(nt):
            M[k, l] = np.sum(w * P[l](s) * P[k](s)) * jac
            K[k, l] = -np.sum(w * P[l](s) * dk(s) * (2.0 / tau)) * jac \
                + P[l](1.0) * P[k](1.0)
            # previous slab's psi_l evaluated at its right end (s=+1),
            # this slab's psi_k at its left end (s=-1)
            N[k, l] = P[l](1.0) * P[k](-1.0)
    return K, M, N


def slab_integrals(pt, tau):
    """int_slab psi_l dt for l = 0..p_t (load vector of a time-constant f)."""
    P = _basis(pt)
    s, w = _quad(pt + 2)
    return np.array([np.sum(w * P[l](s)) * 0.5 * tau for l in range(pt + 1)])


def left_trace(pt):
    """psi_k(t_{n-1}^+) for k = 0..p_t: how the previous slab's trace enters slab n."""
    return np.array([b(-1.0) for b in _basis(pt)])


def right_trace(pt):
    """psi_l(t_n^-) for l = 0..p_t: end-of-slab value functional."""
    return np.array([b(1.0) for b in _basis(pt)])


def time_prolongation_blocks(pt, tau_fine):
    """R1^T, R2^T of eq. (chap4_restrictionTime): R_s^T = M_tau^{-1} Mtilde^s.

    Mtilde^1[k,l] = int_0^tau      psit_l(t) psi_k(t)        dt
    Mtilde^2[k,l] = int_tau^{2tau} psit_l(t) psi_k(t - tau)  dt
    with psit_l the coarse basis on (0, 2 tau) and psi_k the fine basis on
    (0, tau).  The paper prints psi_k(t + tau) in Mtilde^2; the fine basis
    has to be shifted onto (tau, 2 tau), i.e. psi_k(t - tau).
    """
    P = _basis(pt)
    nt = pt + 1
    s, w = _quad(pt + 2)
    _, Mt, _ = time_matrices(pt, tau_fine)
    blocks = []
    for half in (0, 1):
        t = half * tau_fine + 0.5 * tau_fine * (s + 1.0)      # points in the fine slab
        sc = t / tau_fine - 1.0                                # coarse reference coordinate on (0, 2tau)
        sf = 2.0 * (t - half * tau_fine) / tau_fine - 1.0      # fine reference coordinate
        Mtil = np.zeros((nt, nt))
        for k in range(nt):
            for l in range(nt):
                Mtil[k, l] = np.sum(w * P[l](sc) * P[k](sf)) * 0.5 * tau_fine
        blocks.append(np.linalg.solve(Mt, Mtil))
    return blocks[0], blocks[1]


def stability_function(pt, z, _mats=None):
    """R(z): the nonzero eigenvalue of (K_tau + lam M_tau)^{-1} N_tau with lam tau = -z
    (Lemma chap4_theorem2, read with R(-lam tau); N_tau has rank one, so the
    nonzero eigenvalue equals the trace)."""
    K, M, N = _mats if _mats is not None else time_matrices(pt, 1.0)
    z = np.atleast_1d(np.asarray(z, dtype=complex))
    out = np.empty(z.shape, dtype=complex)
    for i, zi in enumerate(z):
        out[i] = np.trace(np.linalg.solve(K - zi * M, N))
    if np.all(np.abs(out.imag) < 1e-13 * (1 + np.abs(out.real))):
        out = out.real
    return out if out.size > 1 else out[0]


def mu_star(pt):
    """Critical discretisation parameter of Remark
    chap4_remarkCriticalDiscretizationParameter: smallest mu > 0 with
    R(-3 mu) = sqrt(2) - 1 (scan for the first sign change, then bisection)."""
    target = np.sqrt(2.0) - 1.0
    mats = time_matrices(pt, 1.0)
    g = lambda mu: float(np.real(stability_function(pt, -3.0 * mu, mats))) - target
    grid = np.linspace(0.0, 5.0, 5001)
    vals = [g(m) for m in grid]
    for i in range(len(grid) - 1):
        if vals[i] > 0.0 >= vals[i + 1]:
            lo, hi = grid[i], grid[i + 1]
            break
    else:
        raise RuntimeError("no root of R(-3mu) = sqrt(2)-1 on (0, 5]")
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if g(mid) > 0.0:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)
