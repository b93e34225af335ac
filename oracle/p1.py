"""Space-time multigrid on P1 simplicial meshes (oracle, test-only).

The setting of the numerical examples of Sec. 4: P1 elements in space on a
uniformly refined coarse mesh, DG(p_t) in time, the damped block-Jacobi
smoother with one spatial multigrid cycle per slab (Remark
V-cycleApproxSpace), full space-time or time-only coarsening by the rule of
Sec. 4.  Everything else (smoothing, residual, restriction R = P^T, coarse
correction, exact solve on one slab) is the Q1 hierarchy's code in
`multigrid.Hierarchy`; this module supplies the levels, the transfers and the
spatial cycles.

Reading of the mesh size in mu = tau / h^2: h_L = h_0 2^{-L} on refinement
level L, h_0 the longest edge of the coarse mesh (1 for the square of 4
triangles, sqrt(2) for the cube of 12 tetrahedra).  With h_0 = 1/2 (the
spacing of the Q1 grid whose single interior node is the centre) the rule
picks full coarsening at mu too small for these tetrahedra and the counts of
Table chap4_TableExample1 grow with N; with the longest edge they stay
bounded.
"""
import numpy as np
import scipy.sparse as sp

from . import dg_time, mesh as meshmod
from .multigrid import AUTO, FULL, SEMI, Hierarchy
from .spacetime import SpaceTimeLevel
from .spatial_mg import SpatialCycle


def coarsening_schedule(refinements, N, T, pt, h0, rule=AUTO, mu_star=None):
    """As multigrid.coarsening_schedule with the refinement level in place of
    the grid size: space can be coarsened while the level is above 0.
    Returns ([(L_x, N_L, tau_L, mu_L) fine->coarse], "fs..." per transition)."""
    if mu_star is None or mu_star <= 0:
        mu_star = dg_time.mu_star(pt)
    levels, kinds = [], []
    lx, tau = refinements, T / N
    while True:
        h = h0 * 2.0 ** (-lx)
        mu = tau / h ** 2
        levels.append((lx, N, tau, mu))
        if N == 1:
            break
        if rule == FULL:
            full = lx > 0
        elif rule == SEMI:
            full = False
        else:
            full = lx > 0 and mu >= mu_star * (1.0 - 1e-12)
        kinds.append("f" if full else "s")
        if full:
            lx -= 1
        N //= 2
        tau *= 2.0
    return levels, "".join(kinds)


def time_prolongation(fine_N, pt, tau):
    """P_t: coarse slab m feeds fine slabs 2m, 2m+1 through R_1^T, R_2^T
    (eq. chap4_restrictionTime)."""
    R1T, R2T = dg_time.time_prolongation_blocks(pt, tau)
    nt = pt + 1
    Nc = fine_N // 2
    Pt = sp.lil_matrix((fine_N * nt, Nc * nt))
    for m in range(Nc):
        for s, blk in ((0, R1T), (1, R2T)):
            for l in range(nt):
                for k in range(nt):
                    if blk[l, k] != 0.0:
                        Pt[(2 * m + s) * nt + l, m * nt + k] = blk[l, k]
    return Pt.tocsr()


def longest_edge(level):
    """Longest cell edge of a mesh level."""
    best = 0.0
    for c in level.cells:
        for a in range(len(c)):
            for b in range(a + 1, len(c)):
                best = max(best, float(np.linalg.norm(level.coords[c[a]] - level.coords[c[b]])))
    return best


class P1Hierarchy(Hierarchy):
    """Space-time hierarchy on a refined coarse mesh (index 0 = coarsest)."""

    def __init__(self, coarse_coords, coarse_cells, refinements, N, pt, T=1.0, h0=None, omega=0.5, nu1=2,
                 nu2=2, rule=AUTO, mu_star=None, transpose=False, smoother="inexact", nu1x=2, nu2x=2,
                 omega_x=2.0 / 3.0, gamma=1, meshes=None):
        self.meshes = meshes or meshmod.hierarchy(coarse_coords, coarse_cells, refinements)
        self.Px = [None] + [meshmod.prolongation(self.meshes[j - 1], self.meshes[j])
                            for j in range(1, len(self.meshes))]
        d = self.meshes[0].d
        if h0 is None:
            h0 = longest_edge(self.meshes[0])
        self.h0 = h0
        lv, kinds = coarsening_schedule(refinements, N, T, pt, h0, rule, mu_star)
        self.schedule = kinds
        self.space_level = [lx for (lx, _, _, _) in lv][::-1]
        self.levels = [SpaceTimeLevel(d, None, NL, pt, tauL,
                                      space=(self.meshes[lx].Mh, self.meshes[lx].Kh, h0 * 2.0 ** (-lx)))
                       for (lx, NL, tauL, _) in lv][::-1]
        self.kinds = kinds[::-1]
        self.omega, self.nu1, self.nu2 = omega, nu1, nu2
        self.gamma = gamma
        self.transpose = transpose
        self.P = [None]
        for k in range(1, len(self.levels)):
            fine = self.levels[k]
            Pt = time_prolongation(fine.N, pt, fine.tau)
            if self.kinds[k - 1] == "f":
                Px = self.Px[self.space_level[k]]
            else:
                Px = sp.identity(fine.nx, format="csr")
            self.P.append(sp.kron(Pt, Px, format="csr"))
        self._lu = [None] * len(self.levels)
        if smoother not in ("exact", "inexact"):
            raise ValueError(smoother)
        self.smoother = smoother
        self.xopts = dict(nu1=nu1x, nu2=nu2x, omega=omega_x)
        self._sc = [None] * len(self.levels)

    def spatial_cycle(self, k):
        """The spatial cycle of level k runs over refinement levels L_x .. 0."""
        if self._sc[k] is None:
            lev = self.levels[k]
            lx = self.space_level[k]
            mats = [(self.meshes[j].Mh, self.meshes[j].Kh) for j in range(lx, -1, -1)]
            pros = [self.Px[j] for j in range(lx, 0, -1)]
            self._sc[k] = SpatialCycle(lev.d, None, lev.pt, lev.tau, transpose=self.transpose,
                                       space=(mats, pros), **self.xopts)
        return self._sc[k]
