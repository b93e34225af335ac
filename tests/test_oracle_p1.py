"""Pins of the P1 mesh oracle (oracle/mesh.py, oracle/p1.py) against the
paper's printed values (cell counts, Tables chap4_TableExample1 and
chap4_TableExample2), exact integrals of P1 functions, closed-form element
matrices, the Galerkin identities of nested P1 spaces and brute-force point
evaluation."""
import json
import math
import os

import numpy as np
import pytest

from oracle import mesh, p1
from paper_1411_0519_amd import workloads

SQ = workloads.coarse_mesh("square4")
CU = workloads.coarse_mesh("cube12")


@pytest.fixture(scope="module")
def square_levels():
    return mesh.hierarchy(*SQ, 3)


@pytest.fixture(scope="module")
def cube_levels():
    return mesh.hierarchy(*CU, 3)


def volumes(level):
    d = level.d
    return np.array([abs(np.linalg.det((level.coords[c[1:]] - level.coords[c[0]]).T)) / math.factorial(d)
                     for c in level.cells])


def test_cell_counts(square_levels, cube_levels):
    # 4 triangles and 12 tetrahedra (Examples chap4_example2 and chap4_example1); red refinement
    # multiplies by 2^d
    assert [len(m.cells) for m in square_levels] == [4 * 4 ** L for L in range(4)]
    assert [len(m.cells) for m in cube_levels] == [12 * 8 ** L for L in range(4)]


def test_parallel_example_cell_count():
    # the parallel example's cube is decomposed into 49,152 tetrahedra: four
    # uniform refinements of the 12-tetrahedron cube
    c, t, _ = mesh.refine(*mesh.refine(*mesh.refine(*mesh.refine(*CU)[:2])[:2])[:2])
    assert len(t) == 49152
    # every node is a vertex of the uniform grid of spacing 1/32 (dyadic coordinates)
    assert np.all(np.abs(c * 32 - np.round(c * 32)) == 0)


@pytest.mark.parametrize("which", ["square", "cube"])
def test_red_refinement_halves_every_cell(which, square_levels, cube_levels):
    levels = square_levels if which == "square" else cube_levels
    d = levels[0].d
    for L in range(len(levels)):
        v = volumes(levels[L])
        assert abs(v.sum() - 1.0) < 1e-13
        if L > 0:
            # children come in groups of 2^d per parent, each of 1/2^d of its volume
            vp = volumes(levels[L - 1])
            assert np.allclose(v.reshape(-1, 2 ** d), np.repeat(vp / 2 ** d, 2 ** d).reshape(-1, 2 ** d))


@pytest.mark.parametrize("which", ["square", "cube"])
def test_boundary_nodes_are_on_the_box(which, square_levels, cube_levels):
    levels = square_levels if which == "square" else cube_levels
    for m in levels:
        on_box = np.any((m.coords == 0.0) | (m.coords == 1.0), axis=1)
        assert np.array_equal(m.boundary, on_box)


def test_interior_node_counts(square_levels, cube_levels):
    # square: (2^L + 1)^2 + 4^L nodes, of which 2^(L+2) on the boundary
    assert [m.nx for m in square_levels] == [(2 ** L + 1) ** 2 + 4 ** L - 2 ** (L + 2) for L in range(4)]
    assert [m.nx for m in cube_levels][:2] == [1, 9]


def test_element_matrices_closed_form():
    # reference triangle: K = 1/2 [[2,-1,-1],[-1,1,0],[-1,0,1]], M = 1/24 [[2,1,1],[1,2,1],[1,1,2]]
    Me, Ke = mesh.p1_element(np.array([[0.0, 0.0], [1.0, 0.0], [0.0, 1.0]]))
    assert np.allclose(Ke, 0.5 * np.array([[2, -1, -1], [-1, 1, 0], [-1, 0, 1]]), atol=1e-15)
    assert np.allclose(Me, np.array([[2, 1, 1], [1, 2, 1], [1, 1, 2]]) / 24.0, atol=1e-15)
    # reference tetrahedron: |T| = 1/6, M = |T|/20 (1 + delta), K row of vertex 0 = |T| [3,-1,-1,-1]
    Me, Ke = mesh.p1_element(np.array([[0.0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]]))
    assert np.allclose(Me, (np.ones((4, 4)) + np.eye(4)) / 120.0, atol=1e-15)
    assert np.allclose(Ke[0], np.array([3, -1, -1, -1]) / 6.0, atol=1e-15)
    assert np.allclose(Ke[1:, 1:], np.eye(3) / 6.0, atol=1e-15)


@pytest.mark.parametrize("which", ["square", "cube"])
def test_full_matrices_integrate_p1_functions_exactly(which, square_levels, cube_levels):
    m = (square_levels if which == "square" else cube_levels)[2]
    M, K = mesh.p1_matrices(m.coords, m.cells, np.ones(m.coords.shape[0], dtype=bool))
    one = np.ones(m.coords.shape[0])
    x = m.coords[:, 0]
    y = m.coords[:, 1]
    assert abs(one @ M @ one - 1.0) < 1e-13           # |Omega|
    assert abs(x @ M @ x - 1.0 / 3.0) < 1e-13         # int x^2
    assert abs(x @ M @ y - 0.25) < 1e-13              # int x y
    assert np.abs(K @ one).max() < 1e-12             # constants have no energy
    assert abs(x @ K @ x - 1.0) < 1e-12               # int |grad x|^2
    assert abs((x + 2 * y) @ K @ (x + 2 * y) - 5.0) < 1e-12
    # a linear function is discretely harmonic at every interior node
    assert np.abs((K @ (x - 3 * y))[m.interior]).max() < 1e-12


@pytest.mark.parametrize("which", ["square", "cube"])
def test_galerkin_identities(which, square_levels, cube_levels):
    levels = square_levels if which == "square" else cube_levels
    for j in range(1, len(levels)):
        P = mesh.prolongation(levels[j - 1], levels[j])
        assert abs(P.T @ levels[j].Kh @ P - levels[j - 1].Kh).max() < 1e-12
        assert abs(P.T @ levels[j].Mh @ P - levels[j - 1].Mh).max() < 1e-15


def evaluate(level, values, points):
    """Brute force: locate each point in a cell by barycentric coordinates and
    interpolate the nodal values (full node numbering)."""
    out = np.zeros(len(points))
    for i, p in enumerate(points):
        for c in level.cells:
            x = level.coords[c]
            B = (x[1:] - x[0]).T
            lam = np.linalg.solve(B, p - x[0])
            bary = np.concatenate([[1.0 - lam.sum()], lam])
            if np.all(bary >= -1e-12):
                out[i] = bary @ values[c]
                break
        else:
            raise AssertionError("point outside the mesh")
    return out


@pytest.mark.parametrize("which", ["square", "cube"])
def test_prolongation_is_interpolation(which, square_levels, cube_levels):
    levels = square_levels if which == "square" else cube_levels
    c, f = levels[1], levels[2]
    rng = np.random.default_rng(3)
    uc = rng.uniform(-1, 1, c.nx)
    full = np.zeros(c.coords.shape[0])
    full[c.interior] = uc
    ref = evaluate(c, full, f.points)
    assert np.abs(mesh.prolongation(c, f) @ uc - ref).max() < 1e-13


def test_schedule_rule():
    # full coarsening while mu >= mu* and space can be coarsened, then time only
    _, kinds = p1.coarsening_schedule(3, 1024, 1024.0, 1, 1.0)
    assert kinds == "fff" + "s" * 7
    _, kinds = p1.coarsening_schedule(3, 64, 1.0, 1, 2 ** 0.5, rule=p1.SEMI)
    assert kinds == "ssssss"
    lv, kinds = p1.coarsening_schedule(2, 256, 1.0, 1, 2 ** 0.5)
    for (lx, N, tau, mu), k in zip(lv, kinds):
        assert (k == "f") == (lx > 0 and mu >= p1.dg_time.mu_star(1) * (1 - 1e-12))
        assert abs(mu - tau / (2 ** 0.5 * 2.0 ** -lx) ** 2) < 1e-12 * mu


def test_longest_edge_reading(square_levels, cube_levels):
    assert p1.longest_edge(square_levels[0]) == 1.0
    assert abs(p1.longest_edge(cube_levels[0]) - 2 ** 0.5) < 1e-15


def iterations(coarse, refinements, N, pt, T, smoother, meshes=None, seed=0):
    H = p1.P1Hierarchy(*coarse, refinements, N, pt, T=T, smoother=smoother, meshes=meshes)
    u = np.random.default_rng(seed).uniform(0, 1, (H.fine.dof, 1))
    _, hist, _ = H.solve(np.zeros_like(u), u=u, rtol=1e-8, maxit=30)
    assert hist[-1][0] <= 1e-8
    return len(hist) - 1


with open(os.path.join(os.path.dirname(__file__), "golden", "tables_p1.json")) as _fh:
    TABLES = json.load(_fh)


@pytest.mark.parametrize("space_level", [0, 1, 2])
def test_table1_iterations(space_level, cube_levels):
    # zero right-hand side, random start in [0,1], reduction 1e-8.  The exact
    # block inverse reproduces the printed counts within one; the paper's
    # spatial cycle (nu_x = 2) needs at most two more on these meshes
    ms = cube_levels[:space_level + 1]
    lts = range(0, 8) if space_level < 2 else range(0, 7)
    exact = [iterations(CU, space_level, 2 ** lt, 1, 1.0, "exact", ms) for lt in lts]
    inexact = [iterations(CU, space_level, 2 ** lt, 1, 1.0, "inexact", ms) for lt in lts]
    printed = TABLES["table1"][f"space_level_{space_level}"][:len(exact)]
    assert all(abs(a - b) <= 1 for a, b in zip(exact, printed)), (exact, printed)
    assert all(b <= a <= b + 2 for a, b in zip(inexact, printed)), (inexact, printed)
    assert exact[0] == inexact[0] == 1          # one time step: the coarsest level is solved exactly


@pytest.mark.parametrize("pt", [0, 1, 3, 10])
def test_table2_iterations(pt, square_levels):
    # Table chap4_TableExample2: 2-D, 4 triangles refined once, T = 1024,
    # tau = 1, printed 7 for every p_t on every space level >= 1
    its = iterations(SQ, 1, 1024, pt, 1024.0, "inexact", square_levels[:2])
    assert abs(its - TABLES["table2"]["space_levels_1_to_7"]) <= 1, its
