"""Inexact block-Jacobi smoother: one geometric multigrid cycle in space per
time slab in place of the exact inverse of A (Remark V-cycleApproxSpace,
Sec. 3; numerical setting of Sec. 4).  Oracle, test-only.

The slab matrix A = K_tau (x) M_h + M_tau (x) K_h acts on [l][space] vectors.
Its spatial hierarchy halves h down to one interior node: n, (n-1)/2, ..., 1.
One cycle from the zero initial guess maps f to x = (I - M^x) A^{-1} f, where
M^x is the cycle's iteration matrix:
  * nu1x damped block-Jacobi steps  x <- x + omega_x (D^x)^{-1} (f - A x),
    D^x = K_tau (x) diag(M_h) + M_tau (x) diag(K_h), i.e. the N_t x N_t
    blocks of A at each spatial node;
  * defect restriction with R_x (x) I_{N_t}, R_x = P_x^T, P_x the
    (bi/tri)linear interpolation;
  * the same cycle for the re-discretised coarse matrix A_{tau,2h} (gamma_x =
    1), an exact solve on the coarsest spatial level of the cycle;
  * prolongation P_x (x) I_{N_t}, nu2x damped block-Jacobi steps.
The paper's setting is nu1x = nu2x = 2, omega_x = 2/3.  `depth` limits the
number of coarsenings (depth = 1 is the spatial two-grid cycle of the local
Fourier analysis).
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import dg_time, fe_space


def spatial_sizes(n, depth=None):
    """n, (n-1)/2, ..., 1 (at most depth + 1 entries)."""
    ns = [n]
    while ns[-1] > 1 and (depth is None or len(ns) <= depth):
        ns.append((ns[-1] - 1) // 2)
    return ns


class SpatialCycle:
    """One spatial multigrid cycle for A_{tau,h} on every column of a [l][space] block."""

    def __init__(self, d, n, pt, tau, nu1=2, nu2=2, omega=2.0 / 3.0, transpose=False, depth=None, space=None):
        """space = (mats, prolongations) gives the spatial hierarchy explicitly
        (P1 meshes): mats[j] = (M_j, K_j) from fine to coarse, prolongations[j-1]
        the interpolation from sub-level j to j-1."""
        self.d, self.n, self.pt, self.tau = d, n, pt, tau
        self.nu1, self.nu2, self.omega = nu1, nu2, omega
        if space is None:
            self.ns = spatial_sizes(n, depth)
            mats = [fe_space.q1_matrices(d, nj) for nj in self.ns]
            pros = [fe_space.space_prolongation(d, nj) for nj in self.ns[1:]]
        else:
            mats, pros = space
            self.ns = [M.shape[0] for M, _ in mats]
        Kt, Mt, _ = dg_time.time_matrices(pt, tau)
        nt = pt + 1
        self.A, self.Dlu, self.P = [], [], []
        for j, (Mh, Kh) in enumerate(mats):
            A = sp.kron(Kt, Mh) + sp.kron(Mt, Kh)
            D = sp.kron(Kt, sp.diags(Mh.diagonal())) + sp.kron(Mt, sp.diags(Kh.diagonal()))
            if transpose:
                A, D = A.T, D.T
            self.A.append(A.tocsr())
            self.Dlu.append(spla.splu(D.tocsc()))
            if j > 0:
                self.P.append(sp.kron(sp.identity(nt), pros[j - 1], format="csr"))
        self.coarse_lu = spla.splu(self.A[-1].tocsc())

    def cycle(self, f, j=0):
        """x = cycle applied to A_j x = f from x = 0 (columns independent)."""
        if j == len(self.ns) - 1:
            return self.coarse_lu.solve(np.ascontiguousarray(f))
        A, Dlu, w = self.A[j], self.Dlu[j], self.omega
        x = np.zeros_like(f)
        for _ in range(self.nu1):
            x = x + w * Dlu.solve(np.ascontiguousarray(f - A @ x))
        P = self.P[j]
        x = x + P @ self.cycle(P.T @ (f - A @ x), j + 1)
        for _ in range(self.nu2):
            x = x + w * Dlu.solve(np.ascontiguousarray(f - A @ x))
        return x

    def iteration_matrix(self):
        """M^x = I - C A (dense), C the cycle's linear map."""
        m = self.A[0].shape[0]
        C = self.cycle(np.eye(m))
        return np.eye(m) - C @ self.A[0].toarray()
