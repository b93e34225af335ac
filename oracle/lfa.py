"""Local Fourier mode analysis of Sec. 3 (oracle, test-only).

1-D in space (Omega = (0,1), uniform h), DG(p_t) in time, periodic
space-time boundary conditions as assumed by the analysis.  Symbols are
formed as N_t x N_t matrices exactly as in the lemmas; two-grid factors are
spectral radii of the 4 N_t x 4 N_t iteration matrices of Theorems
cahp4_theorem5 / cahp4_theorem6, maximised over the low frequencies with
theta_x != 0 (Definition of the asymptotic two-grid convergence factors).

The inexact smoother of Remark V-cycleApproxSpace replaces D^{-1} by
(I - M^x) D^{-1}, M^x the spatial two-grid iteration matrix; on the four
harmonics it acts as M-tilde(theta_x) on the pair (theta_x, gamma(theta_x))
for each of the two time frequencies.

Readings where the text is ambiguous:
  * gamma(theta) = theta - sign(theta) pi with sign(0) := +1;
  * the second block of the semi-coarsening coarse symbol is taken at
    (gamma(theta_x), 2 theta_t);
  * the nonzero eigenvalue of (K + lam M)^{-1} N is R(-lam tau);
  * M-tilde = S^nu2 K^x S^nu1 (post-smoothing applied last; the printed order
    S^nu1 K^x S^nu2 is the same matrix when nu1 = nu2), R-tilde_x is N_t x 2N_t
    and P-tilde_x is 2N_t x N_t (the printed shapes are swapped).
"""
import numpy as np

from . import dg_time


def beta(theta_x):
    """beta(theta_x) = 6 (1 - cos) / (2 + cos)  (Lemma chap4_lemma17)."""
    c = np.cos(theta_x)
    return 6.0 * (1.0 - c) / (2.0 + c)


def gamma(theta):
    """Harmonic shift theta - sign(theta) pi, sign(0) := +1 (Lemma chap4_lemma9)."""
    s = np.where(np.asarray(theta) >= 0.0, 1.0, -1.0)
    return theta - s * np.pi


class Symbols:
    """Fourier symbols for one (p_t, tau, h, omega)."""

    def __init__(self, pt, tau, h, omega=0.5):
        self.pt, self.tau, self.h, self.omega = pt, tau, h, omega
        self.K, self.M, self.N = dg_time.time_matrices(pt, tau)
        self.R1T, self.R2T = dg_time.time_prolongation_blocks(pt, tau)
        self.R1, self.R2 = self.R1T.T, self.R2T.T
        self.nt = pt + 1
        self._tm = {tau: (self.K, self.M, self.N)}

    def _time(self, tau):
        if tau not in self._tm:
            self._tm[tau] = dg_time.time_matrices(self.pt, tau)
        return self._tm[tau]

    def L(self, tx, tt, tau=None, h=None):
        """L-hat of Lemma chap4_lemma17 on the level (tau, h)."""
        tau = self.tau if tau is None else tau
        h = self.h if h is None else h
        K, M, N = self._time(tau)
        return (h / 3.0) * (2.0 + np.cos(tx)) * (
            K + beta(tx) / h ** 2 * M - np.exp(-1j * tt) * N)

    def S(self, tx, tt):
        """S-hat of Lemma chap4_lemma18 (exact block inverse)."""
        Ablk = self.K + beta(tx) / self.h ** 2 * self.M
        return (1.0 - self.omega) * np.eye(self.nt) + \
            self.omega * np.exp(-1j * tt) * np.linalg.solve(Ablk, self.N)

    def Ahat(self, tx, h=None):
        """A-hat_{tau,h}(theta_x) = h/3 (2 + cos) K + 2/h (1 - cos) M (Remark V-cycleApproxSpace)."""
        h = self.h if h is None else h
        c = np.cos(tx)
        return (h / 3.0) * (2.0 + c) * self.K + (2.0 / h) * (1.0 - c) * self.M

    def Dx(self):
        """Block diagonal of A in space: 2h/3 K + 2/h M."""
        return (2.0 * self.h / 3.0) * self.K + (2.0 / self.h) * self.M

    def Sx(self, tx, omega_x):
        """Damped block-Jacobi symbol in space, I - omega_x Dx^{-1} A-hat(theta_x)."""
        return np.eye(self.nt) - omega_x * np.linalg.solve(self.Dx(), self.Ahat(tx))

    def Mx(self, tx, nu1x=2, nu2x=2, omega_x=2.0 / 3.0):
        """M-tilde(theta_x): spatial two-grid iteration symbol on (theta_x, gamma(theta_x))."""
        n = self.nt
        gx = gamma(tx)
        I = np.eye(n)
        At = np.zeros((2 * n, 2 * n))
        At[:n, :n] = self.Ahat(tx)
        At[n:, n:] = self.Ahat(gx)
        Rt = np.concatenate([self.Rx(tx) * I, self.Rx(gx) * I], axis=1)
        Pt = np.concatenate([self.Px(tx) * I, self.Px(gx) * I], axis=0)
        Ac = self.Ahat(2 * tx, h=2 * self.h)
        Kx = np.eye(2 * n) - Pt @ np.linalg.solve(Ac, Rt @ At)

        def Sp(nu):
            out = np.zeros((2 * n, 2 * n))
            out[:n, :n] = np.linalg.matrix_power(self.Sx(tx, omega_x), nu)
            out[n:, n:] = np.linalg.matrix_power(self.Sx(gx, omega_x), nu)
            return out
        return Sp(nu2x) @ Kx @ Sp(nu1x)

    def S_inexact(self, tx, tt, nu1x=2, nu2x=2, omega_x=2.0 / 3.0):
        """S-bar = I - omega (I - M) D^{-1} L on the four harmonics (eq. chap4_smootherApprox)."""
        n = self.nt
        H = self.harmonics(tx, tt)
        DinvL = self.blockdiag([np.linalg.solve(self.Ahat(a), self.L(a, b)) for a, b in H])
        M = np.zeros((4 * n, 4 * n), dtype=complex)
        Mt = self.Mx(tx, nu1x, nu2x, omega_x)
        M[:2 * n, :2 * n] = Mt
        M[2 * n:, 2 * n:] = Mt
        return np.eye(4 * n) - self.omega * (np.eye(4 * n) - M) @ DinvL

    def Rt(self, tt):
        """Time restriction symbol e^{-i theta} R1 + R2 (Lemma chap4_lemma12)."""
        return np.exp(-1j * tt) * self.R1 + self.R2

    def Pt(self, tt):
        """Time prolongation symbol 1/2 [e^{i theta} R1^T + R2^T] (Lemma chap4_lemma13)."""
        return 0.5 * (np.exp(1j * tt) * self.R1T + self.R2T)

    @staticmethod
    def Rx(tx):
        """Space restriction symbol 1 + cos(theta_x) (Lemma chap4_lemma25)."""
        return 1.0 + np.cos(tx)

    @staticmethod
    def Px(tx):
        return 0.5 * (1.0 + np.cos(tx))

    def harmonics(self, tx, tt):
        gx, gt = gamma(tx), gamma(tt)
        return [(tx, tt), (gx, tt), (tx, gt), (gx, gt)]

    def blockdiag(self, mats):
        n = self.nt
        out = np.zeros((4 * n, 4 * n), dtype=complex)
        for i, m in enumerate(mats):
            out[i * n:(i + 1) * n, i * n:(i + 1) * n] = m
        return out

    def two_grid_matrix(self, tx, tt, kind, nu1, nu2, xopts=None):
        """M-tilde of Theorem cahp4_theorem5 (kind 's') or cahp4_theorem6 (kind 'f');
        with xopts (dict nu1x, nu2x, omega_x) the smoother is the inexact one,
        giving the matrices of eq. chap4_twoGridIterationMatrixApprox."""
        n = self.nt
        H = self.harmonics(tx, tt)
        Lt = self.blockdiag([self.L(a, b) for a, b in H])
        if xopts is None:
            St = self.blockdiag([self.S(a, b) for a, b in H])
        else:
            St = self.S_inexact(tx, tt, **xopts)
        gt = gamma(tt)
        if kind == "s":
            Rs = np.zeros((2 * n, 4 * n), dtype=complex)
            Rs[:n, 0:n] = self.Rt(tt)
            Rs[:n, 2 * n:3 * n] = self.Rt(gt)
            Rs[n:, n:2 * n] = self.Rt(tt)
            Rs[n:, 3 * n:] = self.Rt(gt)
            Ps = np.zeros((4 * n, 2 * n), dtype=complex)
            Ps[0:n, :n] = self.Pt(tt)
            Ps[2 * n:3 * n, :n] = self.Pt(gt)
            Ps[n:2 * n, n:] = self.Pt(tt)
            Ps[3 * n:, n:] = self.Pt(gt)
            Lc = np.zeros((2 * n, 2 * n), dtype=complex)
            Lc[:n, :n] = self.L(tx, 2 * tt, tau=2 * self.tau)
            Lc[n:, n:] = self.L(gamma(tx), 2 * tt, tau=2 * self.tau)
            Kc = np.eye(4 * n) - Ps @ np.linalg.solve(Lc, Rs @ Lt)
        elif kind == "f":
            Rf = np.concatenate([self.Rx(a) * self.Rt(b) for a, b in H], axis=1)
            Pf = np.concatenate([self.Px(a) * self.Pt(b) for a, b in H], axis=0)
            Lc = self.L(2 * tx, 2 * tt, tau=2 * self.tau, h=2 * self.h)
            Kc = np.eye(4 * n) - Pf @ np.linalg.solve(Lc, Rf @ Lt)
        else:
            raise ValueError(kind)
        return np.linalg.matrix_power(St, nu2) @ Kc @ np.linalg.matrix_power(St, nu1)

    def galerkin_defect(self, tx, tt, kind):
        """|| R-tilde L-tilde P-tilde - L-coarse || in symbol space (should vanish)."""
        n = self.nt
        H = self.harmonics(tx, tt)
        Lt = self.blockdiag([self.L(a, b) for a, b in H])
        gt = gamma(tt)
        if kind == "f":
            Rf = np.concatenate([self.Rx(a) * self.Rt(b) for a, b in H], axis=1)
            Pf = np.concatenate([self.Px(a) * self.Pt(b) for a, b in H], axis=0)
            Lc = self.L(2 * tx, 2 * tt, tau=2 * self.tau, h=2 * self.h)
            return np.abs(Rf @ Lt @ Pf - Lc).max()
        Rs = np.zeros((2 * n, 4 * n), dtype=complex)
        Rs[:n, 0:n] = self.Rt(tt)
        Rs[:n, 2 * n:3 * n] = self.Rt(gt)
        Rs[n:, n:2 * n] = self.Rt(tt)
        Rs[n:, 3 * n:] = self.Rt(gt)
        Ps = np.zeros((4 * n, 2 * n), dtype=complex)
        Ps[0:n, :n] = self.Pt(tt)
        Ps[2 * n:3 * n, :n] = self.Pt(gt)
        Ps[n:2 * n, n:] = self.Pt(tt)
        Ps[3 * n:, n:] = self.Pt(gt)
        Lc = np.zeros((2 * n, 2 * n), dtype=complex)
        Lc[:n, :n] = self.L(tx, 2 * tt, tau=2 * self.tau)
        Lc[n:, n:] = self.L(gamma(tx), 2 * tt, tau=2 * self.tau)
        return np.abs(Rs @ Lt @ Ps - Lc).max()


def low_frequencies(nl):
    """Theta_L^low = {2 k pi / N_L} cap (-pi/2, pi/2]."""
    k = np.arange(1 - nl // 2, nl // 2 + 1)
    th = 2.0 * np.pi * k / nl
    return th[(th > -np.pi / 2) & (th <= np.pi / 2 + 1e-15)]


def two_grid_factor(pt, mu, kind, nu1=1, nu2=1, omega=0.5, nx_grid=1024, nt_grid=256, h=1.0 / 1024,
                    xopts=None):
    """rho(M-hat_mu^{s|f}) (or rho(M-bar) with the inexact smoother when xopts is
    given): max spectral radius over low frequencies, theta_x != 0."""
    tau = mu * h ** 2
    sym = Symbols(pt, tau, h, omega)
    best = 0.0
    for tx in low_frequencies(nx_grid):
        if tx == 0.0:
            continue
        for tt in low_frequencies(nt_grid):
            ev = np.linalg.eigvals(sym.two_grid_matrix(tx, tt, kind, nu1, nu2, xopts))
            best = max(best, np.abs(ev).max())
    return best


def smoothing_symbol_radius(sym, tx, tt):
    """Spectral radius of S-hat(theta_x, theta_t) from the matrix symbol."""
    return np.abs(np.linalg.eigvals(sym.S(tx, tt))).max()


def smoothing_factor(pt, mu, kind, omega=0.5, ngrid=257, h=1.0 / 64):
    """Smoothing factor: sup of rho(S-hat) over the high frequencies of the
    coarsening (semi: theta_t in [pi/2, pi]; full: theta_x in [pi/2, pi])."""
    sym = Symbols(pt, mu * h ** 2, h, omega)
    th = np.linspace(0.0, np.pi, ngrid)
    hi = np.linspace(np.pi / 2, np.pi, ngrid)
    if kind == "s":
        txs, tts = th, hi
    else:
        txs, tts = hi, th
    best = 0.0
    for tx in txs:
        for tt in tts:
            best = max(best, smoothing_symbol_radius(sym, tx, tt))
    return best
