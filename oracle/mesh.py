"""Simplicial meshes and P1 finite elements (oracle, test-only).

The numerical examples of Sec. 4 discretise space with conforming P1 elements
on uniformly refined triangulations of (0,1)^2 and tetrahedral meshes of
(0,1)^3.  This module refines a coarse mesh, assembles the P1 mass and
stiffness matrices of the interior nodes (homogeneous Dirichlet boundary) and
builds the interpolation between consecutive refinement levels, in plain
loops over cells.

Readings (the paper gives only the cell counts):
  * uniform refinement is red refinement: every edge is halved; a triangle
    gives 4 children, a tetrahedron its 4 corner tetrahedra plus the inner
    octahedron cut into 4 along its shortest diagonal (ties: the diagonal whose
    endpoints have the lexicographically smallest coordinates, compared as
    (smaller endpoint, larger endpoint));
  * new nodes are numbered after the old ones, in the order in which a sweep
    over the cells (in order) meets their edges, local edges in the order
    (0,1), (0,2), (0,3), (1,2), (1,3), (2,3) (triangles: the first three);
  * a node lies on the boundary when it is a vertex of a boundary face (a face
    of exactly one cell); interior nodes keep the order of the node numbers.
"""
import itertools
import math

import numpy as np
import scipy.sparse as sp

LOCAL_EDGES = {2: [(0, 1), (0, 2), (1, 2)], 3: [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)]}


def _key(p):
    return tuple(float(v) for v in p)


def refine(coords, cells):
    """One red refinement.  Returns (coords, cells, parents): parents[i] is the
    pair of old vertices whose edge node i halves (None for old vertices)."""
    coords = [np.asarray(c, dtype=np.float64) for c in coords]
    cells = [tuple(int(v) for v in c) for c in cells]
    d = len(cells[0]) - 1
    nv = len(coords)
    mid = {}
    parents = [None] * nv
    for c in cells:
        for a, b in LOCAL_EDGES[d]:
            e = (min(c[a], c[b]), max(c[a], c[b]))
            if e not in mid:
                mid[e] = len(coords)
                coords.append(0.5 * (coords[e[0]] + coords[e[1]]))
                parents.append(e)
    out = []
    for c in cells:
        m = {}
        for a, b in LOCAL_EDGES[d]:
            m[(a, b)] = m[(b, a)] = mid[(min(c[a], c[b]), max(c[a], c[b]))]
        if d == 2:
            out += [(c[0], m[0, 1], m[0, 2]), (m[0, 1], c[1], m[1, 2]),
                    (m[0, 2], m[1, 2], c[2]), (m[0, 1], m[1, 2], m[0, 2])]
            continue
        out += [(c[0], m[0, 1], m[0, 2], m[0, 3]), (m[0, 1], c[1], m[1, 2], m[1, 3]),
                (m[0, 2], m[1, 2], c[2], m[2, 3]), (m[0, 3], m[1, 3], m[2, 3], c[3])]
        # inner octahedron: the three diagonals join midpoints of opposite edges
        best = None
        for (a, b), (cc, dd) in (((0, 1), (2, 3)), ((0, 2), (1, 3)), ((0, 3), (1, 2))):
            p, q = m[a, b], m[cc, dd]
            kp, kq = _key(coords[p]), _key(coords[q])
            rank = (float(np.sum((coords[p] - coords[q]) ** 2)), min(kp, kq), max(kp, kq))
            if best is None or rank < best[0]:
                best = (rank, (a, b, cc, dd))
        a, b, cc, dd = best[1]
        ring = [m[a, cc], m[a, dd], m[b, dd], m[b, cc]]    # consecutive ring nodes share an old vertex
        p, q = m[a, b], m[cc, dd]
        out += [(p, q, ring[i], ring[(i + 1) % 4]) for i in range(4)]
    return np.array(coords), np.array(out, dtype=np.int64), parents


def boundary_nodes(cells, nnodes):
    """Mask of the nodes on boundary faces (faces that belong to one cell)."""
    d = cells.shape[1] - 1
    count = {}
    for c in cells:
        for f in itertools.combinations(sorted(int(v) for v in c), d):
            count[f] = count.get(f, 0) + 1
    mask = np.zeros(nnodes, dtype=bool)
    for f, k in count.items():
        if k == 1:
            mask[list(f)] = True
    return mask


def p1_element(x):
    """Element mass and stiffness of the P1 simplex with vertex rows x:
    M_e[i,j] = |T| (1 + delta_ij) / ((d+1)(d+2)),  K_e = |T| G G^T, with G the
    constant gradients of the barycentric coordinates."""
    d = x.shape[1]
    B = (x[1:] - x[0]).T                         # columns x_i - x_0
    vol = abs(np.linalg.det(B)) / math.factorial(d)
    Binv = np.linalg.inv(B)
    G = np.zeros((d + 1, d))
    G[1:] = Binv                                  # grad lambda_i = row i-1 of B^{-1}
    G[0] = -Binv.sum(axis=0)
    Me = vol / ((d + 1) * (d + 2)) * (np.ones((d + 1, d + 1)) + np.eye(d + 1))
    Ke = vol * G @ G.T
    return Me, Ke


def p1_matrices(coords, cells, interior):
    """Interior M_h, K_h (CSR), assembled cell by cell and restricted to the
    interior nodes (in node order)."""
    nn = coords.shape[0]
    M = sp.lil_matrix((nn, nn))
    K = sp.lil_matrix((nn, nn))
    for c in cells:
        Me, Ke = p1_element(coords[c])
        for a in range(len(c)):
            for b in range(len(c)):
                M[c[a], c[b]] += Me[a, b]
                K[c[a], c[b]] += Ke[a, b]
    idx = np.flatnonzero(interior)
    M = M.tocsr()[idx][:, idx]
    K = K.tocsr()[idx][:, idx]
    return M.tocsr(), K.tocsr()


class MeshLevel:
    """One refinement level: nodes, cells, interior numbering, P1 matrices."""

    def __init__(self, coords, cells, parents=None):
        self.coords, self.cells = coords, cells
        self.d = coords.shape[1]
        self.parents = parents
        self.boundary = boundary_nodes(cells, coords.shape[0])
        self.interior = np.flatnonzero(~self.boundary)
        self.nx = len(self.interior)
        self.points = coords[self.interior]
        self.Mh, self.Kh = p1_matrices(coords, cells, ~self.boundary)


def hierarchy(coords, cells, refinements):
    """Levels 0 (the coarse mesh) .. refinements."""
    levels = [MeshLevel(np.asarray(coords, dtype=np.float64), np.asarray(cells, dtype=np.int64))]
    for _ in range(refinements):
        c, t, par = refine(levels[-1].coords, levels[-1].cells)
        levels.append(MeshLevel(c, t, par))
    return levels


def prolongation(coarse, fine):
    """Interpolation of coarse interior P1 functions at the fine interior nodes:
    an old vertex keeps its value, an edge node takes the mean of the edge's
    two ends (a boundary end contributes zero)."""
    cpos = -np.ones(coarse.coords.shape[0], dtype=np.int64)
    cpos[coarse.interior] = np.arange(coarse.nx)
    P = sp.lil_matrix((fine.nx, coarse.nx))
    for r, i in enumerate(fine.interior):
        par = fine.parents[i]
        if par is None:
            if cpos[i] >= 0:
                P[r, cpos[i]] = 1.0
            continue
        for v in par:
            if cpos[v] >= 0:
                P[r, cpos[v]] += 0.5
    return P.tocsr()
