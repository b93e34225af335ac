"""Seeded synthetic inputs for the heat-equation workloads.

This module only draws and evaluates data (nodal source values per time slab,
nodal initial data, target states).  It holds none of the method's
arithmetic: turning nodal data into the space-time right-hand side is done
separately by the HIP library and by the CPU reference.

Nodal arrays use the interior-node numbering j = x + n*y + n*n*z (x fastest);
node i along an axis sits at (i+1) h, h = 1/(n+1).

Workloads (d, n interior nodes per dimension, N slabs on (0,T), DG order p_t):
  W1  1-D, n=31,  N=16,   p_t=1, T=1: f ~ U[-1,1] per (node, slab), u0 = sin(pi x)
  W2  2-D, n=127, N=256,  p_t=1, T=1: f = sum of 8 Gaussian bumps (width 0.05,
      centres ~ U[0.1,0.9]^2, constant in time), u0 = sin(pi x) sin(pi y)
  W3  3-D, n=63,  N=1024, p_t=1, T=1: f ~ U[-1,1] per (node, slab), u0 = 0
  W4  2-D, n=255, N=512,  p_t=2, T=1, 64 right-hand sides: f ~ U[-1,1] per
      (rhs, node, slab), u0 = 16-mode sine series per rhs
  W5  2-D, n=255, N=1024, p_t=1, T=1: f ~ U[-1,1], u0 = sin sin, target u_d =
      16-mode sine series (constant in time)

Coarse simplicial meshes of the numerical examples (Sec. 4), refined by the
method's own code:
  square4  (0,1)^2 as 4 triangles around the centre (Example 2)
  cube12   (0,1)^3 as 12 tetrahedra: every face cut along the diagonal through
           its corner nearest the origin, each half joined to the centre
           (Example 1; four uniform refinements give the 49,152 tetrahedra of
           the parallel example)
"""
import numpy as np

WORKLOADS = {
    1: dict(name="heat1d_n31_N16_p1", dim=1, n=31, N=16, pt=1, T=1.0, batch=1, seed=1,
            f="uniform", u0="sine1"),
    2: dict(name="heat2d_n127_N256_p1", dim=2, n=127, N=256, pt=1, T=1.0, batch=1, seed=2,
            f="bumps", u0="sine1"),
    3: dict(name="heat3d_n63_N1024_p1", dim=3, n=63, N=1024, pt=1, T=1.0, batch=1, seed=3,
            f="uniform", u0="zero"),
    4: dict(name="heat2d_n255_N512_p2_b64", dim=2, n=255, N=512, pt=2, T=1.0, batch=64, seed=4,
            f="uniform", u0="series16"),
    5: dict(name="heat2d_n255_N1024_p1_adjoint", dim=2, n=255, N=1024, pt=1, T=1.0, batch=1, seed=5,
            f="uniform", u0="sine1", target_seed=55),
}


def coordinates(dim, n):
    """Interior node coordinates, list of dim arrays broadcastable to (n,)*dim in (z, y, x) order."""
    h = 1.0 / (n + 1)
    g = h * np.arange(1, n + 1)
    if dim == 1:
        return [g]
    if dim == 2:
        y, x = np.meshgrid(g, g, indexing="ij")
        return [x.ravel(), y.ravel()]
    z, y, x = np.meshgrid(g, g, g, indexing="ij")
    return [x.ravel(), y.ravel(), z.ravel()]


def sine1(dim, n):
    xs = coordinates(dim, n)
    out = np.ones_like(xs[0])
    for c in xs:
        out = out * np.sin(np.pi * c)
    return out


def sine_series(dim, n, rng, modes=16, kmax=16):
    """sum_m a_m prod_i sin(pi k_{m,i} x_i), k ~ U{1..kmax}, a ~ U[-1,1]."""
    xs = coordinates(dim, n)
    out = np.zeros_like(xs[0])
    for _ in range(modes):
        k = rng.integers(1, kmax + 1, size=dim)
        a = rng.uniform(-1.0, 1.0)
        term = np.full_like(xs[0], a)
        for i, c in enumerate(xs):
            term = term * np.sin(np.pi * k[i] * c)
        out += term
    return out


def gaussian_bumps(dim, n, rng, count=8, width=0.05):
    xs = coordinates(dim, n)
    out = np.zeros_like(xs[0])
    for _ in range(count):
        c = rng.uniform(0.1, 0.9, size=dim)
        r2 = sum((xs[i] - c[i]) ** 2 for i in range(dim))
        out += np.exp(-r2 / (2.0 * width ** 2))
    return out


def make(dim, n, N, batch=1, seed=0, f="uniform", u0="sine1", dtype=np.float64, **_):
    """Nodal data: f of shape (batch, N, n^dim) and u0 of shape (batch, n^dim)."""
    rng = np.random.default_rng(seed)
    nx = n ** dim
    if f == "uniform":
        fa = rng.uniform(-1.0, 1.0, size=(batch, N, nx))
    elif f == "bumps":
        bumps = gaussian_bumps(dim, n, rng)
        fa = np.broadcast_to(bumps, (batch, N, nx)).copy()
    elif f == "zero":
        fa = np.zeros((batch, N, nx))
    else:
        raise ValueError(f)
    if u0 == "sine1":
        ua = np.broadcast_to(sine1(dim, n), (batch, nx)).copy()
    elif u0 == "series16":
        ua = np.stack([sine_series(dim, n, rng) for _ in range(batch)])
    elif u0 == "zero":
        ua = np.zeros((batch, nx))
    elif u0 == "uniform01":
        ua = rng.uniform(0.0, 1.0, size=(batch, nx))
    else:
        raise ValueError(u0)
    return fa.astype(dtype, copy=False), ua.astype(dtype, copy=False)


def make_streamed(dim, n, N, batch=1, seed=0, f="uniform", u0="series16", **_):
    """The nodal data of `make` for f = "uniform", one right-hand side at a
    time (for batches too large to hold as one float64 array): returns an
    iterator over the batch's f[b] of shape (N, n^dim) and a function that,
    called after the iterator is exhausted, returns u0 of shape (batch,
    n^dim).  The values equal make()'s: the generator draws the same stream in
    the same order."""
    if f != "uniform":
        raise ValueError(f)
    rng = np.random.default_rng(seed)
    nx = n ** dim

    def f_iter():
        for _ in range(batch):
            yield rng.uniform(-1.0, 1.0, size=(N, nx))

    def u0_fn():
        if u0 == "series16":
            return np.stack([sine_series(dim, n, rng) for _ in range(batch)])
        if u0 == "sine1":
            return np.broadcast_to(sine1(dim, n), (batch, nx)).copy()
        if u0 == "zero":
            return np.zeros((batch, nx))
        raise ValueError(u0)

    return f_iter(), u0_fn


def workload(idx, **overrides):
    """Parameters and nodal data of workload idx; overrides shrink it (n, N, batch)."""
    w = dict(WORKLOADS[idx])
    w.update(overrides)
    f, u0 = make(**w)
    return w, f, u0


def target_state(dim, n, seed):
    """Tracking target u_d: 16-mode sine series, constant in time (nodal)."""
    return sine_series(dim, n, np.random.default_rng(seed))


def random_start(dof, batch, seed):
    """Random initial iterate with values in [0,1] (paper's contraction protocol)."""
    return np.random.default_rng(seed).uniform(0.0, 1.0, size=(batch, dof))


def coarse_mesh(kind):
    """(coords, cells): vertex coordinates (float64, rows x dim) and cells (int32,
    rows of dim+1 vertex indices) of a built-in coarse mesh."""
    if kind == "square4":
        coords = np.array([[0, 0], [1, 0], [1, 1], [0, 1], [0.5, 0.5]], dtype=np.float64)
        cells = np.array([[0, 1, 4], [1, 2, 4], [2, 3, 4], [3, 0, 4]], dtype=np.int32)
        return coords, cells
    if kind == "cube12":
        corners = [[x, y, z] for z in (0, 1) for y in (0, 1) for x in (0, 1)]   # index x + 2y + 4z
        coords = np.array(corners + [[0.5, 0.5, 0.5]], dtype=np.float64)
        faces = [(0, 2, 6), (0, 6, 4), (1, 3, 7), (1, 7, 5), (0, 1, 5), (0, 5, 4),
                 (2, 3, 7), (2, 7, 6), (0, 1, 3), (0, 3, 2), (4, 5, 7), (4, 7, 6)]
        cells = np.array([list(f) + [8] for f in faces], dtype=np.int32)
        return coords, cells
    raise ValueError(kind)


def mesh_data(points, N, batch=1, seed=0, f="uniform", u0="sine1"):
    """Nodal data at given node coordinates (rows x dim): f of shape (batch, N,
    nodes), u0 of shape (batch, nodes); the same recipes as `make`."""
    rng = np.random.default_rng(seed)
    pts = np.asarray(points, dtype=np.float64)
    nx = pts.shape[0]
    if f == "uniform":
        fa = rng.uniform(-1.0, 1.0, size=(batch, N, nx))
    elif f == "zero":
        fa = np.zeros((batch, N, nx))
    else:
        raise ValueError(f)
    if u0 == "sine1":
        ua = np.broadcast_to(np.prod(np.sin(np.pi * pts), axis=1), (batch, nx)).copy()
    elif u0 == "uniform01":
        ua = rng.uniform(0.0, 1.0, size=(batch, nx))
    elif u0 == "zero":
        ua = np.zeros((batch, nx))
    else:
        raise ValueError(u0)
    return fa, ua
