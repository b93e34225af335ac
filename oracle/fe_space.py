"""Q1 finite elements on the uniform tensor grid of (0,1)^d (oracle, test-only).

M_h[i,j] = int phi_j phi_i dx and K_h[i,j] = int grad phi_j . grad phi_i dx
(Sec. 1), with the nodal basis of the interior nodes (homogeneous Dirichlet
boundary).  The paper uses P1 on simplices for its experiments and prints the
1-D matrices in Sec. 3; the tensor-product Q1 element is the reading used for
d = 2, 3 here.  Assembly is element by element: element matrices come from
Gauss quadrature of the bilinear/trilinear shape functions on one element,
then are scattered into the global matrix; boundary rows/columns are dropped.

Interior node numbering: j = x + n*y + n*n*z (x fastest), 0-based.
"""
import itertools

import numpy as np
import scipy.sparse as sp
from numpy.polynomial import legendre as npleg


def _element_matrices(d, h):
    """Element mass and stiffness of the Q1 element [0,h]^d by 2-point Gauss."""
    g, gw = npleg.leggauss(2)
    g = 0.5 * (g + 1.0)                 # points on (0,1)
    gw = 0.5 * gw
    corners = list(itertools.product((0, 1), repeat=d))   # corner a = (a_0,..,a_{d-1}), a_0 = x
    nloc = len(corners)
    Me = np.zeros((nloc, nloc))
    Ke = np.zeros((nloc, nloc))
    for qp in itertools.product(range(2), repeat=d):
        xi = np.array([g[q] for q in qp])
        wq = np.prod([gw[q] for q in qp]) * h ** d
        val = np.zeros(nloc)
        grad = np.zeros((nloc, d))
        for a, c in enumerate(corners):
            f1 = [xi[i] if c[i] else 1.0 - xi[i] for i in range(d)]
            df = [1.0 if c[i] else -1.0 for i in range(d)]
            val[a] = np.prod(f1)
            for i in range(d):
                grad[a, i] = df[i] / h * np.prod([f1[j] for j in range(d) if j != i])
        Me += wq * np.outer(val, val)
        Ke += wq * grad @ grad.T
    return corners, Me, Ke


def q1_matrices(d, n):
    """Global interior M_h, K_h (CSR) for n interior nodes per dimension."""
    if n < 1:
        raise ValueError("n >= 1")
    h = 1.0 / (n + 1)
    corners, Me, Ke = _element_matrices(d, h)
    # elements: lower-corner index e_i in 0..n along each dimension (n+1 elements per dim)
    ne = n + 1
    E = np.array(list(itertools.product(range(ne), repeat=d)))[:, ::-1]   # columns (x, y, z)
    rows, cols, vm, vk = [], [], [], []
    gidx = []
    valid = []
    for c in corners:
        node = E + np.array(c)[None, :]               # full-grid coordinates 0..n+1
        inside = np.all((node >= 1) & (node <= n), axis=1)
        idx = np.zeros(len(E), dtype=np.int64)
        stride = 1
        for i in range(d):
            idx += (node[:, i] - 1) * stride
            stride *= n
        gidx.append(idx)
        valid.append(inside)
    for a in range(len(corners)):
        for b in range(len(corners)):
            m = valid[a] & valid[b]
            rows.append(gidx[a][m])
            cols.append(gidx[b][m])
            vm.append(np.full(m.sum(), Me[a, b]))
            vk.append(np.full(m.sum(), Ke[a, b]))
    rows = np.concatenate(rows)
    cols = np.concatenate(cols)
    nx = n ** d
    M = sp.coo_matrix((np.concatenate(vm), (rows, cols)), shape=(nx, nx)).tocsr()
    K = sp.coo_matrix((np.concatenate(vk), (rows, cols)), shape=(nx, nx)).tocsr()
    M.sum_duplicates()
    K.sum_duplicates()
    return M, K


def node_coordinates(d, n):
    """Coordinates of the interior nodes, shape (n^d, d), columns (x, y, z)."""
    h = 1.0 / (n + 1)
    g = h * np.arange(1, n + 1)
    pts = np.array(list(itertools.product(g, repeat=d)))[:, ::-1]
    return pts


def space_prolongation_1d(n_coarse):
    """Linear interpolation P_x = R_x^T from n_c to n_f = 2 n_c + 1 interior nodes
    (eq. chap4_spaceRestrictionProlongation, read as standard full weighting
    R_x: coarse i <- 1/2 u_{2i-1} + u_{2i} + 1/2 u_{2i+1}, 1-based)."""
    nc = n_coarse
    nf = 2 * nc + 1
    P = sp.lil_matrix((nf, nc))
    for i in range(nc):
        f = 2 * i + 1                 # 0-based fine index of coarse node i
        P[f, i] = 1.0
        P[f - 1, i] = 0.5
        P[f + 1, i] = 0.5
    return P.tocsr()


def space_prolongation(d, n_coarse):
    """Tensor-product interpolation for the x-fastest numbering."""
    P1 = space_prolongation_1d(n_coarse)
    P = P1
    for _ in range(d - 1):
        P = sp.kron(P1, P, format="csr")   # slower dimension on the left
    return P.tocsr()
