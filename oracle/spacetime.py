"""The all-at-once space-time system (oracle, test-only).

Sec. 1, eq. (equation1) and eq. (chap4_generalLinearSystem):
    A = K_tau (x) M_h + M_tau (x) K_h,    B = -N_tau (x) M_h,
    L = block lower-bidiagonal with A on the diagonal and B below it.
Vector layout: u[(n*N_t + l)*N_x + j] (time-slab outer, time dof, then space),
the ordering of Sec. 1.  Batched vectors are arrays of shape (dof, b).
"""
import numpy as np
import scipy.sparse as sp

from . import dg_time, fe_space


class SpaceTimeLevel:
    """Matrices of one space-time level (d, n interior nodes, N slabs of length tau)."""

    def __init__(self, d, n, N, pt, tau, space=None):
        """space = (M_h, K_h, h) replaces the Q1 matrices of the n^d grid (P1 meshes)."""
        self.d, self.n, self.N, self.pt, self.tau = d, n, N, pt, tau
        self.nt = pt + 1
        if space is None:
            self.h = 1.0 / (n + 1)
            self.nx = n ** d
            self.Mh, self.Kh = fe_space.q1_matrices(d, n)
        else:
            self.Mh, self.Kh, self.h = space
            self.nx = self.Mh.shape[0]
        self.Kt, self.Mt, self.Nt = dg_time.time_matrices(pt, tau)
        self.A = (sp.kron(self.Kt, self.Mh) + sp.kron(self.Mt, self.Kh)).tocsc()
        self.B = (-sp.kron(self.Nt, self.Mh)).tocsr()
        self.L = (sp.kron(sp.identity(N), self.A)
                  + sp.kron(sp.eye(N, N, k=-1), self.B)).tocsr()
        self.mu = tau / self.h ** 2
        self.slab = self.nt * self.nx
        self.dof = N * self.slab

    def apply(self, u, transpose=False):
        """L u (or L^T u) by sparse matrix-vector product."""
        return (self.L.T @ u) if transpose else (self.L @ u)


def rhs(level, f_nodal, u0_nodal):
    """Right-hand side of Sec. 1 for data that is Q1-interpolated in space and
    constant in time on every slab (reading of the load vector, whose indices
    are garbled in the text):
        F_n[l] = (int_slab psi_l dt) M_h f_n,
        F_1   += (N_tau (x) M_h) applied to the initial trace, i.e.
        F_1[l] += psi_l(t_0^+) M_h u0_h     (eq. (equation1) with n = 0).
    f_nodal: (b, N, N_x); u0_nodal: (b, N_x).  Returns F of shape (dof, b).
    """
    f_nodal = np.asarray(f_nodal, dtype=np.float64)
    u0_nodal = np.asarray(u0_nodal, dtype=np.float64)
    b = f_nodal.shape[0]
    N, nt, nx = level.N, level.nt, level.nx
    ints = dg_time.slab_integrals(level.pt, level.tau)
    a = dg_time.left_trace(level.pt)
    F = np.zeros((N, nt, nx, b))
    for ib in range(b):
        for n in range(N):
            mf = level.Mh @ f_nodal[ib, n]
            for l in range(nt):
                F[n, l, :, ib] = ints[l] * mf
        mu0 = level.Mh @ u0_nodal[ib]
        for l in range(nt):
            F[0, l, :, ib] += a[l] * mu0
    return F.reshape(level.dof, b)


def rhs_adjoint(level, lam):
    """Transpose of the linear map (f, u0) -> F of `rhs`:
    grad_f[b,n] = sum_l (int psi_l) M_h lam_{n,l},  grad_u0[b] = sum_l psi_l(t_0^+) M_h lam_{1,l}."""
    b = lam.shape[1]
    N, nt, nx = level.N, level.nt, level.nx
    ints = dg_time.slab_integrals(level.pt, level.tau)
    a = dg_time.left_trace(level.pt)
    lam4 = lam.reshape(N, nt, nx, b)
    gf = np.zeros((b, N, nx))
    gu0 = np.zeros((b, nx))
    for ib in range(b):
        for n in range(N):
            acc = np.zeros(nx)
            for l in range(nt):
                acc += ints[l] * lam4[n, l, :, ib]
            gf[ib, n] = level.Mh @ acc
        acc = np.zeros(nx)
        for l in range(nt):
            acc += a[l] * lam4[0, l, :, ib]
        gu0[ib] = level.Mh @ acc
    return gf, gu0


def forward_substitution(level, F, transpose=False):
    """Exact solve of L u = F slab by slab (Sec. 1: "forward substitution with
    respect to the blocks"), or of L^T u = F backwards in time."""
    import scipy.sparse.linalg as spla
    b = F.shape[1]
    N, S = level.N, level.slab
    Fb = F.reshape(N, S, b)
    u = np.zeros_like(Fb)
    if not transpose:
        lu = spla.splu(level.A.tocsc())
        for n in range(N):
            rhs_n = Fb[n].copy()
            if n > 0:
                rhs_n -= level.B @ u[n - 1]
            u[n] = lu.solve(rhs_n)
    else:
        lu = spla.splu(level.A.T.tocsc())
        BT = level.B.T.tocsr()
        for n in range(N - 1, -1, -1):
            rhs_n = Fb[n].copy()
            if n < N - 1:
                rhs_n -= BT @ u[n + 1]
            u[n] = lu.solve(rhs_n)
    return u.reshape(level.dof, b)
