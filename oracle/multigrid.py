"""Space-time multigrid of Sec. 2 and Sec. 4 (oracle, test-only).

Plain, unfused and unblocked: sparse L from element assembly, one sparse LU of
the slab block A per level (all slabs and right-hand sides solved as columns),
sparse prolongation P and restriction R = P^T.  The V-cycle follows the order
of Sec. 2: nu1 damped block-Jacobi steps (eq. chap4_smoother with the exact
block inverse, eq. chap4_smootherExact), residual, restriction, recursive
coarse correction from a zero initial guess, prolongation, nu2 steps; the
coarsest level (one time slab) is solved exactly by LU.

smoother="inexact" replaces the exact block inverse by one geometric
multigrid cycle in space per slab (eq. chap4_smootherApprox of Remark
V-cycleApproxSpace, module spatial_mg); the coarsest level stays exact.
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import dg_time, fe_space
from .spatial_mg import SpatialCycle
from .spacetime import SpaceTimeLevel, forward_substitution

AUTO, SEMI, FULL = 0, 1, 2


def coarsening_schedule(n, N, T, pt, rule=AUTO, mu_star=None):
    """Level list fine -> coarse and the transition kinds.

    Sec. 4: full space-time coarsening if mu_L >= mu*, otherwise semi-coarsening
    in time; semi doubles mu, full halves it.  Space is coarsened down to one
    interior node; once it cannot be coarsened, only time is.  Coarsening stops
    at a single time slab (Sec. 2: the coarsest level has one time step).
    Ties mu_L = mu* count as full (relative tolerance 1e-12).
    Returns ([(n_L, N_L, tau_L, mu_L) fine->coarse], "fs..." per transition).
    """
    if mu_star is None or mu_star <= 0:
        mu_star = dg_time.mu_star(pt)
    levels = []
    kinds = []
    tau = T / N
    while True:
        h = 1.0 / (n + 1)
        mu = tau / h ** 2
        levels.append((n, N, tau, mu))
        if N == 1:
            break
        if rule == FULL:
            full = n > 1
        elif rule == SEMI:
            full = False
        else:
            full = (n > 1) and (mu >= mu_star * (1.0 - 1e-12))
        kinds.append("f" if full else "s")
        if full:
            n = (n - 1) // 2
        N //= 2
        tau *= 2.0
    return levels, "".join(kinds)


def transfer(fine, coarse, kind):
    """Prolongation P from `coarse` to `fine` (eq. chap4_restrictionTime and
    eq. chap4_spaceRestrictionProlongation): P = P_t (x) P_x for full
    coarsening, P_t (x) I for semi-coarsening, in the slab-outer layout."""
    R1T, R2T = dg_time.time_prolongation_blocks(fine.pt, fine.tau)
    Nc, nt = coarse.N, fine.nt
    Pt = sp.lil_matrix((fine.N * nt, Nc * nt))
    for m in range(Nc):
        for s, blk in ((0, R1T), (1, R2T)):
            fs = 2 * m + s
            for l in range(nt):
                for k in range(nt):
                    if blk[l, k] != 0.0:
                        Pt[fs * nt + l, m * nt + k] = blk[l, k]
    Pt = Pt.tocsr()
    if kind == "f":
        Px = fe_space.space_prolongation(fine.d, coarse.n)
    else:
        Px = sp.identity(fine.nx, format="csr")
    return sp.kron(Pt, Px, format="csr")


class Hierarchy:
    """All levels of the space-time multigrid (index 0 = coarsest)."""

    def __init__(self, d, n, N, pt, T=1.0, omega=0.5, nu1=2, nu2=2,
                 rule=AUTO, mu_star=None, transpose=False, smoother="exact",
                 nu1x=2, nu2x=2, omega_x=2.0 / 3.0, depth_x=None, gamma=1):
        lv, kinds = coarsening_schedule(n, N, T, pt, rule, mu_star)
        self.schedule = kinds                                  # fine -> coarse
        self.levels = [SpaceTimeLevel(d, nL, NL, pt, tauL) for (nL, NL, tauL, _) in lv][::-1]
        self.kinds = kinds[::-1]                               # kinds[k-1]: level k-1 -> k
        self.omega, self.nu1, self.nu2 = omega, nu1, nu2
        self.gamma = gamma
        self.transpose = transpose
        self.P = [None] + [transfer(self.levels[k], self.levels[k - 1], self.kinds[k - 1])
                           for k in range(1, len(self.levels))]
        self._lu = [None] * len(self.levels)
        if smoother not in ("exact", "inexact"):
            raise ValueError(smoother)
        self.smoother = smoother
        self.xopts = dict(nu1=nu1x, nu2=nu2x, omega=omega_x, depth=depth_x)
        self._sc = [None] * len(self.levels)

    @property
    def fine(self):
        return self.levels[-1]

    def lu(self, k):
        if self._lu[k] is None:
            A = self.levels[k].A
            self._lu[k] = spla.splu((A.T if self.transpose else A).tocsc())
        return self._lu[k]

    def residual(self, k, u, F):
        """r = F - L u (eq. chap4_smoother's defect)."""
        return F - self.levels[k].apply(u, self.transpose)

    def block_solve(self, k, r):
        """x = D^{-1} r, D = diag{A}: one LU solve per time slab and RHS."""
        lev = self.levels[k]
        b = r.shape[1]
        cols = r.reshape(lev.N, lev.slab, b).transpose(1, 0, 2).reshape(lev.slab, lev.N * b)
        x = self.lu(k).solve(np.ascontiguousarray(cols))
        return x.reshape(lev.slab, lev.N, b).transpose(1, 0, 2).reshape(lev.dof, b)

    def spatial_cycle(self, k):
        if self._sc[k] is None:
            lev = self.levels[k]
            self._sc[k] = SpatialCycle(lev.d, lev.n, lev.pt, lev.tau, transpose=self.transpose, **self.xopts)
        return self._sc[k]

    def approx_block_solve(self, k, r):
        """x = (I - M^x) D^{-1} r: one spatial cycle per slab and RHS from zero."""
        lev = self.levels[k]
        b = r.shape[1]
        cols = r.reshape(lev.N, lev.slab, b).transpose(1, 0, 2).reshape(lev.slab, lev.N * b)
        x = self.spatial_cycle(k).cycle(cols)
        return x.reshape(lev.slab, lev.N, b).transpose(1, 0, 2).reshape(lev.dof, b)

    def smooth(self, k, u, F):
        """One damped block-Jacobi step, eq. chap4_smoother (exact inverse) or
        eq. chap4_smootherApprox (one spatial cycle per slab)."""
        r = self.residual(k, u, F)
        x = self.approx_block_solve(k, r) if self.smoother == "inexact" else self.block_solve(k, r)
        return u + self.omega * x

    def coarsest_solve(self, F):
        """Exact solve on the coarsest level (one slab: L_0 = A_0)."""
        lev = self.levels[0]
        if lev.N == 1:
            return self.block_solve(0, F)
        return forward_substitution(lev, F, self.transpose)

    def vcycle(self, k, u, F):
        """One multigrid cycle on level k (Sec. 2): gamma = 1 is the V-cycle,
        gamma = 2 the W-cycle (the coarse problem is approximated by gamma
        cycles from a zero initial guess)."""
        if k == 0:
            return self.coarsest_solve(F)
        for _ in range(self.nu1):
            u = self.smooth(k, u, F)
        r = self.residual(k, u, F)
        P = self.P[k]
        Fc = P.T @ r                                   # R = P^T
        ec = np.zeros((self.levels[k - 1].dof, F.shape[1]))
        for _ in range(self.gamma):
            ec = self.vcycle(k - 1, ec, Fc)
        u = u + P @ ec
        for _ in range(self.nu2):
            u = self.smooth(k, u, F)
        return u

    def two_grid(self, u, F):
        """Two-grid cycle on the finest level with an exact coarse solve
        (iteration matrices M^s, M^f of Sec. 3.2)."""
        k = len(self.levels) - 1
        for _ in range(self.nu1):
            u = self.smooth(k, u, F)
        r = self.residual(k, u, F)
        P = self.P[k]
        ec = forward_substitution(self.levels[k - 1], P.T @ r, self.transpose)
        u = u + P @ ec
        for _ in range(self.nu2):
            u = self.smooth(k, u, F)
        return u

    def solve(self, F, u=None, rtol=1e-10, maxit=100, keep_iterates=False, cycle=None):
        """Repeat cycles until ||F - L u_k||_2 / ||F - L u_0||_2 <= rtol for every
        right-hand side (reading of the relative error reduction eps_MG)."""
        k = len(self.levels) - 1
        F = np.asarray(F, dtype=np.float64)
        if F.ndim == 1:
            F = F[:, None]
        u = np.zeros_like(F) if u is None else np.array(u, dtype=np.float64).reshape(F.shape)
        cyc = cycle or (lambda uu, FF: self.vcycle(k, uu, FF))
        r0 = np.linalg.norm(self.residual(k, u, F), axis=0)
        scale = np.where(r0 > 0, r0, 1.0)
        hist = [np.where(r0 > 0, 1.0, 0.0)]
        its = [u.copy()] if keep_iterates else None
        for _ in range(maxit):
            if np.all(hist[-1] <= rtol):
                break
            u = cyc(u, F)
            if keep_iterates:
                its.append(u.copy())
            hist.append(np.linalg.norm(self.residual(k, u, F), axis=0) / scale)
        return u, np.array(hist), its


def measured_contraction(hier, u0, F, iters=120, stop=1e-140, cycle="two_grid"):
    """Measured convergence factor max_k ||r^{k+1}|| / ||r^k|| (Sec. 3.2,
    protocol of the numerical test: zero right-hand side, random start)."""
    k = len(hier.levels) - 1
    u = u0.copy()
    r = np.linalg.norm(hier.residual(k, u, F))
    r_first = r
    worst = 0.0
    for _ in range(iters):
        u = hier.two_grid(u, F) if cycle == "two_grid" else hier.vcycle(k, u, F)
        rn = np.linalg.norm(hier.residual(k, u, F))
        worst = max(worst, rn / r)
        r = rn
        if r <= stop * r_first:
            break
    return worst
