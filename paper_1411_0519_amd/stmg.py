"""ctypes binding of libstmg.so (C ABI in include/st_mg.h).

Argument marshalling only: every step of the solver runs in the HIP library.
PyTorch supplies device memory (vectors and the workspace) and the stream.
The library must be built (``__graft_entry__.build()``); loading fails loudly
otherwise, and nothing here falls back to a CPU implementation.
"""
import ctypes
import os

import torch

ST_OK, ST_EINVAL, ST_ENOMEM, ST_EHIP, ST_ENOCONV, ST_ESTATE, ST_EWORKSPACE, ST_ENAN = 0, -1, -2, -3, -4, -5, -6, -7
COARSEN = {"auto": 0, "semi": 1, "full": 2}
PRECISION = {"fp64": 0, "fp32": 1, "mixed": 2, "mixed_bf16": 3}
SMOOTHER = {"exact": 0, "spatial_mg": 1}
FP64, FP32 = 0, 1

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libstmg.so")


class Params(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int), ("n", ctypes.c_int), ("T", ctypes.c_double), ("N", ctypes.c_int),
        ("pt", ctypes.c_int), ("omega", ctypes.c_double), ("nu1", ctypes.c_int), ("nu2", ctypes.c_int),
        ("coarsen", ctypes.c_int), ("mu_star", ctypes.c_double), ("precision", ctypes.c_int),
        ("batch", ctypes.c_int), ("smoother", ctypes.c_int), ("nu1x", ctypes.c_int), ("nu2x", ctypes.c_int),
        ("omega_x", ctypes.c_double), ("gamma", ctypes.c_int),
    ]


class Mesh(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int), ("nnodes", ctypes.c_int), ("ncells", ctypes.c_int),
        ("coords", ctypes.POINTER(ctypes.c_double)), ("cells", ctypes.POINTER(ctypes.c_int)), ("h0", ctypes.c_double),
    ]


class STMGError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"st_mg error {code}: {msg}")
        self.code = code


_lib = None
_vp, _i, _d, _sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_size_t
_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)
_llp = ctypes.POINTER(ctypes.c_longlong)

SIGNATURES = {
    "st_mg_default_params": (None, [ctypes.POINTER(Params)]),
    "st_mg_setup": (_i, [ctypes.POINTER(Params), ctypes.POINTER(_vp)]),
    "st_mg_setup_mesh": (_i, [ctypes.POINTER(Params), ctypes.POINTER(Mesh), _i, ctypes.POINTER(_vp)]),
    "st_mesh_level": (_i, [ctypes.POINTER(Mesh), _i, _llp, _llp, _dp, _ip, _ip, _dp, _dp]),
    "st_mg_level_nx": (_i, [_vp, _i, _llp]),
    "st_mg_destroy": (_i, [_vp]),
    "st_mg_last_error": (ctypes.c_char_p, [_vp]),
    "st_mg_workspace_bytes": (_i, [_vp, ctypes.POINTER(_sz)]),
    "st_mg_bind_workspace": (_i, [_vp, _vp, _sz]),
    "st_mg_levels": (_i, [_vp, _ip, ctypes.c_char_p, _i]),
    "st_mg_level_info": (_i, [_vp, _i, _ip, _ip, _dp, _dp]),
    "st_mg_sizes": (_i, [_vp, _llp, _llp, _llp]),
    "st_mg_rhs": (_i, [_vp, _vp, _vp, _vp, _vp]),
    "st_mg_rhs_adjoint": (_i, [_vp, _vp, _vp, _vp, _vp]),
    "st_mg_residual": (_i, [_vp, _i, _i, _i, _vp, _vp, _vp, _dp, _vp]),
    "st_mg_residual_noalloc": (_i, [_vp, _i, _i, _i, _vp, _vp, _vp, _dp, _vp]),
    "st_mg_block_solve": (_i, [_vp, _i, _i, _i, _vp, _vp, _vp]),
    "st_mg_spatial_cycle": (_i, [_vp, _i, _i, _i, _vp, _vp, _vp]),
    "st_mg_smooth": (_i, [_vp, _i, _i, _i, _vp, _vp, _vp]),
    "st_mg_restrict": (_i, [_vp, _i, _i, _vp, _vp, _vp]),
    "st_mg_residual_restrict": (_i, [_vp, _i, _i, _i, _vp, _vp, _vp, _vp]),
    "st_mg_prolong_add": (_i, [_vp, _i, _i, _vp, _vp, _vp]),
    "st_mg_vcycle": (_i, [_vp, _vp, _vp, _dp, _vp]),
    "st_mg_solve": (_i, [_vp, _vp, _vp, _d, _i, _ip, _dp, _vp]),
    "st_mg_adjoint": (_i, [_vp, _vp, _vp, _vp, _vp, _d, _i, _ip, _dp, _vp]),
    "st_mg_set_graph": (_i, [_vp, _i]),
    "st_mg_autotune": (_i, [_vp, _vp, _vp, _vp]),
    "st_mg_level_tuning": (_i, [_vp, _i, _ip, _ip, ctypes.POINTER(ctypes.c_float)]),
    "st_mg_level_shape": (_i, [_vp, _i, _ip, _ip, _ip, _ip]),
    "st_mg_set_level_shape": (_i, [_vp, _i, _i, _i, _i, _i]),
    "st_mg_profile_start": (_i, [_vp]),
    "st_mg_profile_stop": (_i, [_vp]),
    "st_mg_profile_read": (_i, [_vp, _i, _i, _dp, _ip]),
}

PROF_KINDS = {"residual": 0, "pass_fwd": 1, "pass_inv": 2, "fused": 3, "small": 4, "restrict": 5,
              "prolong": 6, "other": 7, "jacobi": 8, "xfer_x": 9, "resid_x": 10, "pass_fwd_y": 11, "pass_inv_y": 12,
              "resid_restrict": 13}


def lib():
    """Load libstmg.so (raises if it is not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() first")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _mesh_struct(coords, cells, h0=0.0):
    """(Mesh, keep-alive arrays) for a coarse mesh given as numpy arrays."""
    import numpy as np
    c = np.ascontiguousarray(coords, dtype=np.float64)
    t = np.ascontiguousarray(cells, dtype=np.int32)
    if c.ndim != 2 or t.ndim != 2 or t.shape[1] != c.shape[1] + 1:
        raise ValueError("coords must be (nodes, dim) and cells (cells, dim + 1)")
    m = Mesh(c.shape[1], c.shape[0], t.shape[0], c.ctypes.data_as(_dp), t.ctypes.data_as(_ip), float(h0))
    return m, (c, t)


def mesh_level(coords, cells, level):
    """Refinement `level` of a coarse P1 mesh as the library builds it (host
    only, no GPU): interior node coordinates and the interior M_h, K_h in CSR."""
    import numpy as np
    m, keep = _mesh_struct(coords, cells)
    L = lib()
    nx, nnz = ctypes.c_longlong(), ctypes.c_longlong()
    rc = L.st_mesh_level(ctypes.byref(m), level, ctypes.byref(nx), ctypes.byref(nnz), None, None, None, None, None)
    if rc != ST_OK:
        raise STMGError(rc, "st_mesh_level failed")
    pts = np.zeros((nx.value, m.dim))
    rowptr = np.zeros(nx.value + 1, dtype=np.int32)
    col = np.zeros(nnz.value, dtype=np.int32)
    mval = np.zeros(nnz.value)
    kval = np.zeros(nnz.value)
    rc = L.st_mesh_level(ctypes.byref(m), level, None, None, pts.ctypes.data_as(_dp), rowptr.ctypes.data_as(_ip),
                         col.ctypes.data_as(_ip), mval.ctypes.data_as(_dp), kval.ctypes.data_as(_dp))
    if rc != ST_OK:
        raise STMGError(rc, "st_mesh_level failed")
    return dict(points=pts, rowptr=rowptr, col=col, mval=mval, kval=kval)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _stream(device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


class Solver:
    """One space-time multigrid hierarchy on one GPU.

    dim, n, N, pt, T: Omega = (0,1)^dim with n interior nodes per dimension,
    N slabs on (0, T), DG order pt.  omega, nu1, nu2, coarsen ('auto' = the
    mu >= mu* rule, 'semi', 'full'), precision ('fp64', 'fp32', 'mixed', 'mixed_bf16':
    FP64 refinement around an FP32 inner cycle whose transforms use bf16 matrix cores),
    batch = number of right-hand sides.  smoother: 'exact' (fast
    diagonalisation) or 'spatial_mg' (one spatial multigrid cycle per slab with
    nu1x/nu2x damped block-Jacobi steps, damping omega_x).  gamma: cycle index
    (1 = V-cycle, 2 = W-cycle).

    mesh = (coords, cells): P1 elements on that coarse triangle/tetrahedron mesh
    refined n times (n then counts refinements; smoother 'spatial_mg', precision
    'fp64', 'fp32' or 'mixed'); h0 = its mesh size in mu = tau/h^2 (0: longest edge).
    """

    def __init__(self, dim, n, N, pt=1, T=1.0, omega=0.5, nu1=2, nu2=2, coarsen="auto",
                 mu_star=0.0, precision="fp64", batch=1, device="cuda:0", workspace=True,
                 smoother="exact", nu1x=2, nu2x=2, omega_x=2.0 / 3.0, gamma=1, mesh=None, h0=0.0):
        if not torch.cuda.is_available():
            raise RuntimeError("stmg needs a ROCm GPU (torch.cuda.is_available() is False)")
        self.device = torch.device(device)
        self._h = ctypes.c_void_p(0)
        L = lib()
        p = Params(dim, n, float(T), N, pt, float(omega), nu1, nu2, COARSEN[coarsen], float(mu_star),
                   PRECISION[precision], batch, SMOOTHER[smoother], nu1x, nu2x, float(omega_x), gamma)
        with torch.cuda.device(self.device):
            if mesh is None:
                rc = L.st_mg_setup(ctypes.byref(p), ctypes.byref(self._h))
            else:
                ms, keep = _mesh_struct(*mesh, h0=h0)
                rc = L.st_mg_setup_mesh(ctypes.byref(p), ctypes.byref(ms), n, ctypes.byref(self._h))
        if rc != ST_OK:
            msg = L.st_mg_last_error(self._h).decode() if self._h.value else "setup failed"
            if self._h.value:
                L.st_mg_destroy(self._h)
                self._h = ctypes.c_void_p(0)
            raise STMGError(rc, msg)
        self.params = dict(dim=dim, n=n, N=N, pt=pt, T=T, omega=omega, nu1=nu1, nu2=nu2,
                           coarsen=coarsen, precision=precision, batch=batch, smoother=smoother,
                           nu1x=nu1x, nu2x=nu2x, omega_x=omega_x, gamma=gamma)
        self.dim, self.n, self.N, self.pt, self.batch = dim, n, N, pt, batch
        self.mesh = mesh
        self.nt = pt + 1
        self.precision = precision
        self.dtype = torch.float32 if precision == "fp32" else torch.float64
        dof, flen, ulen = ctypes.c_longlong(), ctypes.c_longlong(), ctypes.c_longlong()
        self._check(L.st_mg_sizes(self._h, ctypes.byref(dof), ctypes.byref(flen), ctypes.byref(ulen)))
        self.dof, self.f_len, self.u0_len = dof.value, flen.value, ulen.value
        nl = ctypes.c_int()
        buf = ctypes.create_string_buffer(64)
        self._check(L.st_mg_levels(self._h, ctypes.byref(nl), buf, 64))
        self.nlev = nl.value
        self.schedule = buf.value.decode()
        self.levels = []
        for k in range(self.nlev):
            nn, NN, tau, mu = ctypes.c_int(), ctypes.c_int(), ctypes.c_double(), ctypes.c_double()
            self._check(L.st_mg_level_info(self._h, k, ctypes.byref(nn), ctypes.byref(NN),
                                           ctypes.byref(tau), ctypes.byref(mu)))
            nx = ctypes.c_longlong()
            self._check(L.st_mg_level_nx(self._h, k, ctypes.byref(nx)))
            self.levels.append(dict(n=nn.value, N=NN.value, tau=tau.value, mu=mu.value, nx=nx.value))
        self._ws = None
        if workspace:
            self.bind_workspace()

    # ------------------------------------------------------------------ basics
    def _check(self, rc, allow=()):
        if rc != ST_OK and rc not in allow:
            raise STMGError(rc, lib().st_mg_last_error(self._h).decode())
        return rc

    def workspace_bytes(self):
        b = ctypes.c_size_t()
        self._check(lib().st_mg_workspace_bytes(self._h, ctypes.byref(b)))
        return b.value

    def bind_workspace(self):
        nbytes = self.workspace_bytes()
        ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        off = (-ws.data_ptr()) % 256
        self._ws = ws
        self._check(lib().st_mg_bind_workspace(self._h, ctypes.c_void_p(ws.data_ptr() + off), nbytes))

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().st_mg_destroy(self._h)
            self._h = ctypes.c_void_p(0)
        self._ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def level_dof(self, level):
        if not 0 <= level < self.nlev:
            raise ValueError(f"level {level} out of range 0..{self.nlev - 1}")
        lv = self.levels[level]
        return self.batch * lv["N"] * self.nt * lv["nx"]

    def _vec(self, t, numel, dtype, name):
        if not isinstance(t, torch.Tensor):
            raise TypeError(f"{name} must be a torch.Tensor")
        if t.device != self.device:
            raise ValueError(f"{name} must live on {self.device}")
        if t.dtype != dtype:
            raise TypeError(f"{name} must have dtype {dtype}, got {t.dtype}")
        if not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous")
        if t.numel() != numel:
            raise ValueError(f"{name} has {t.numel()} elements, expected {numel}")
        return t

    def empty(self, level=0, dtype=None):
        return torch.empty(self.level_dof(level), dtype=dtype or self.dtype, device=self.device)

    def zeros(self, level=0, dtype=None):
        return torch.zeros(self.level_dof(level), dtype=dtype or self.dtype, device=self.device)

    # ------------------------------------------------------------- right-hand side
    def rhs(self, f, u0=None, out=None):
        """F from nodal data f [b][N][n^d] and u0 [b][n^d] (Sec. 1 load vector)."""
        f = self._vec(f, self.batch * self.f_len, self.dtype, "f")
        if u0 is not None:
            u0 = self._vec(u0, self.batch * self.u0_len, self.dtype, "u0")
        F = out if out is not None else self.empty()
        self._check(lib().st_mg_rhs(self._h, _ptr(f), _ptr(u0), _ptr(F), _stream(self.device)))
        return F

    def rhs_adjoint(self, lam):
        lam = self._vec(lam, self.dof * self.batch, self.dtype, "lam")
        gf = torch.empty(self.batch * self.f_len, dtype=self.dtype, device=self.device)
        gu0 = torch.empty(self.batch * self.u0_len, dtype=self.dtype, device=self.device)
        self._check(lib().st_mg_rhs_adjoint(self._h, _ptr(lam), _ptr(gf), _ptr(gu0), _stream(self.device)))
        return gf, gu0

    # ------------------------------------------------------------- level operators
    def _prec(self, prec):
        if prec is None:
            return FP64 if self.precision == "fp64" else FP32
        return {"fp64": FP64, "fp32": FP32}[prec] if isinstance(prec, str) else prec

    def _pdtype(self, prec):
        return torch.float64 if prec == FP64 else torch.float32

    def residual(self, u, F, level=0, prec=None, transpose=False, out=None, norms=False):
        p = self._prec(prec)
        dt = self._pdtype(p)
        nd = self.level_dof(level)
        u = self._vec(u, nd, dt, "u")
        F = self._vec(F, nd, dt, "F")
        r = out if out is not None else torch.empty(nd, dtype=dt, device=self.device)
        nrm = (ctypes.c_double * self.batch)() if norms else None
        self._check(lib().st_mg_residual(self._h, level, p, int(transpose), _ptr(u), _ptr(F), _ptr(r),
                                         nrm, _stream(self.device)))
        return (r, [x ** 0.5 for x in nrm]) if norms else r

    def residual_noalloc(self, u, F, level=0, prec=None, transpose=False, out=None, norms=False):
        """As `residual`, through st_mg_residual_noalloc (norm partial sums in the
        library's static device array; no workspace needed)."""
        p = self._prec(prec)
        dt = self._pdtype(p)
        nd = self.level_dof(level)
        u = self._vec(u, nd, dt, "u")
        F = self._vec(F, nd, dt, "F")
        r = out if out is not None else torch.empty(nd, dtype=dt, device=self.device)
        nrm = (ctypes.c_double * self.batch)() if norms else None
        self._check(lib().st_mg_residual_noalloc(self._h, level, p, int(transpose), _ptr(u), _ptr(F), _ptr(r),
                                                 nrm, _stream(self.device)))
        return (r, [x ** 0.5 for x in nrm]) if norms else r

    def block_solve(self, r, level=0, prec=None, transpose=False, out=None):
        p = self._prec(prec)
        dt = self._pdtype(p)
        nd = self.level_dof(level)
        r = self._vec(r, nd, dt, "r")
        x = out if out is not None else torch.empty(nd, dtype=dt, device=self.device)
        self._check(lib().st_mg_block_solve(self._h, level, p, int(transpose), _ptr(r), _ptr(x),
                                            _stream(self.device)))
        return x

    def spatial_cycle(self, r, level=0, prec=None, transpose=False, out=None):
        """x = (I - M^x) A^{-1} r per slab: one spatial multigrid cycle from zero."""
        p = self._prec(prec)
        dt = self._pdtype(p)
        nd = self.level_dof(level)
        r = self._vec(r, nd, dt, "r")
        x = out if out is not None else torch.empty(nd, dtype=dt, device=self.device)
        self._check(lib().st_mg_spatial_cycle(self._h, level, p, int(transpose), _ptr(r), _ptr(x),
                                              _stream(self.device)))
        return x

    def smooth(self, u, F, level=0, prec=None, transpose=False):
        p = self._prec(prec)
        dt = self._pdtype(p)
        nd = self.level_dof(level)
        self._check(lib().st_mg_smooth(self._h, level, p, int(transpose),
                                       _ptr(self._vec(u, nd, dt, "u")), _ptr(self._vec(F, nd, dt, "F")),
                                       _stream(self.device)))
        return u

    def restrict(self, r, level=0, prec=None, out=None):
        p = self._prec(prec)
        dt = self._pdtype(p)
        r = self._vec(r, self.level_dof(level), dt, "r")
        Fc = out if out is not None else torch.empty(self.level_dof(level + 1), dtype=dt, device=self.device)
        self._check(lib().st_mg_restrict(self._h, level, p, _ptr(r), _ptr(Fc), _stream(self.device)))
        return Fc

    def residual_restrict(self, u, F, level=0, prec=None, transpose=False, out=None):
        """F_c = P^T (F - L u) on level + 1 (the cycle's pre-restriction defect)."""
        p = self._prec(prec)
        dt = self._pdtype(p)
        nd = self.level_dof(level)
        u = self._vec(u, nd, dt, "u")
        F = self._vec(F, nd, dt, "F")
        Fc = out if out is not None else torch.empty(self.level_dof(level + 1), dtype=dt, device=self.device)
        self._check(lib().st_mg_residual_restrict(self._h, level, p, int(transpose), _ptr(u), _ptr(F), _ptr(Fc),
                                                  _stream(self.device)))
        return Fc

    def prolong_add(self, e, u, level=0, prec=None):
        p = self._prec(prec)
        dt = self._pdtype(p)
        e = self._vec(e, self.level_dof(level + 1), dt, "e")
        u = self._vec(u, self.level_dof(level), dt, "u")
        self._check(lib().st_mg_prolong_add(self._h, level, p, _ptr(e), _ptr(u), _stream(self.device)))
        return u

    # ------------------------------------------------------------------ cycles
    def vcycle(self, u, F):
        nd = self.level_dof(0)
        u = self._vec(u, nd, self.dtype, "u")
        F = self._vec(F, nd, self.dtype, "F")
        rel = (ctypes.c_double * self.batch)()
        self._check(lib().st_mg_vcycle(self._h, _ptr(u), _ptr(F), rel, _stream(self.device)))
        return list(rel)

    def solve(self, F, u=None, rtol=1e-10, maxit=100, raise_on_noconv=True):
        """Returns (u, iterations, history[iters+1][batch])."""
        nd = self.level_dof(0)
        F = self._vec(F, nd, self.dtype, "F")
        if u is None:
            u = torch.zeros(nd, dtype=self.dtype, device=self.device)
        u = self._vec(u, nd, self.dtype, "u")
        its = ctypes.c_int()
        hist = (ctypes.c_double * ((maxit + 1) * self.batch))()
        rc = lib().st_mg_solve(self._h, _ptr(u), _ptr(F), float(rtol), int(maxit), ctypes.byref(its),
                               hist, _stream(self.device))
        self._check(rc, allow=() if raise_on_noconv else (ST_ENOCONV,))
        k = its.value
        h = [list(hist[i * self.batch:(i + 1) * self.batch]) for i in range(k + 1)]
        return u, k, h

    def adjoint(self, g, lam=None, rtol=1e-10, maxit=100, gradients=True, raise_on_noconv=True):
        """Solve L^T lam = g; returns (lam, grad_f, grad_u0, iterations, history)."""
        nd = self.level_dof(0)
        g = self._vec(g, nd, self.dtype, "g")
        if lam is None:
            lam = torch.zeros(nd, dtype=self.dtype, device=self.device)
        lam = self._vec(lam, nd, self.dtype, "lam")
        gf = gu0 = None
        if gradients:
            gf = torch.empty(self.batch * self.f_len, dtype=self.dtype, device=self.device)
            gu0 = torch.empty(self.batch * self.u0_len, dtype=self.dtype, device=self.device)
        its = ctypes.c_int()
        hist = (ctypes.c_double * ((maxit + 1) * self.batch))()
        rc = lib().st_mg_adjoint(self._h, _ptr(g), _ptr(lam), _ptr(gf), _ptr(gu0), float(rtol),
                                 int(maxit), ctypes.byref(its), hist, _stream(self.device))
        self._check(rc, allow=() if raise_on_noconv else (ST_ENOCONV,))
        k = its.value
        h = [list(hist[i * self.batch:(i + 1) * self.batch]) for i in range(k + 1)]
        return lam, gf, gu0, k, h

    def set_graph(self, enable=True):
        self._check(lib().st_mg_set_graph(self._h, int(bool(enable))))

    # ---------------------------------------------------------------- autotune
    def autotune(self):
        """Pick the fastest kernel family per level by timing smoothing steps.
        Returns [(small, impl, ms) per level]."""
        if self.precision in ("mixed", "mixed_bf16"):
            us = fs = None
        else:
            us, fs = self.empty(), self.empty()
        self._check(lib().st_mg_autotune(self._h, _ptr(us), _ptr(fs), _stream(self.device)))
        return self.tuning()

    def tuning(self):
        out = []
        for k in range(self.nlev):
            sm, im, ms = ctypes.c_int(), ctypes.c_int(), ctypes.c_float()
            self._check(lib().st_mg_level_tuning(self._h, k, ctypes.byref(sm), ctypes.byref(im), ctypes.byref(ms)))
            out.append((sm.value, im.value, ms.value))
        return out

    # --------------------------------------------------------------- profiling
    def level_shape(self, level):
        """Launch shape of the twice-folded passes on a level: dict(wpg, pass_per_cu, fused_cg, fused_per_cu)."""
        v = [ctypes.c_int() for _ in range(4)]
        self._check(lib().st_mg_level_shape(self._h, level, *[ctypes.byref(x) for x in v]))
        return dict(zip(("wpg", "pass_per_cu", "fused_cg", "fused_per_cu"), (x.value for x in v)))

    def set_level_shape(self, level, wpg=4, pass_per_cu=0, fused_cg=0, fused_per_cu=0):
        self._check(lib().st_mg_set_level_shape(self._h, level, wpg, pass_per_cu, fused_cg, fused_per_cu))

    def profile_start(self):
        self._check(lib().st_mg_profile_start(self._h))

    def profile_stop(self):
        self._check(lib().st_mg_profile_stop(self._h))

    def profile_read(self, kind, level=-1):
        """(total_ms, launches) of one kernel kind on one level (-1 = all)."""
        ms, cnt = ctypes.c_double(), ctypes.c_int()
        k = PROF_KINDS[kind] if isinstance(kind, str) else kind
        self._check(lib().st_mg_profile_read(self._h, k, level, ctypes.byref(ms), ctypes.byref(cnt)))
        return ms.value, cnt.value
