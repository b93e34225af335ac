"""Pins of the oracle's Q1 space discretisation."""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import fe_space


def tridiag(n, lo, di, up):
    return sp.diags([np.full(n - 1, lo), np.full(n, di), np.full(n - 1, up)], [-1, 0, 1]).toarray()


@pytest.mark.parametrize("n", [1, 3, 7, 31])
def test_1d_matches_printed_stencils(n):
    # Sec. 3: M_h = h/6 tridiag(1,4,1), K_h = 1/h tridiag(-1,2,-1).
    h = 1.0 / (n + 1)
    M, K = fe_space.q1_matrices(1, n)
    assert np.allclose(M.toarray(), h / 6 * tridiag(n, 1, 4, 1), atol=1e-15)
    assert np.allclose(K.toarray(), 1 / h * tridiag(n, -1, 2, -1), rtol=1e-14, atol=1e-12)


@pytest.mark.parametrize("d,n", [(2, 3), (2, 7), (3, 3), (3, 5)])
def test_tensor_product_structure(d, n):
    # Q1 on a tensor grid: M = (x) M1, K = sum over directions of K1 in that slot.
    M1, K1 = fe_space.q1_matrices(1, n)
    M1, K1 = M1.toarray(), K1.toarray()
    M, K = fe_space.q1_matrices(d, n)

    def kron_list(ms):
        out = ms[0]
        for m in ms[1:]:
            out = np.kron(out, m)
        return out

    Mref = kron_list([M1] * d)
    Kref = sum(kron_list([K1 if i == j else M1 for i in range(d)]) for j in range(d))
    assert np.abs(M.toarray() - Mref).max() < 1e-15
    assert np.abs(K.toarray() - Kref).max() < 1e-12


@pytest.mark.parametrize("d,n", [(1, 15), (2, 7), (3, 3)])
def test_sine_modes_diagonalise(d, n):
    # DST-I vectors are eigenvectors: m_k = h/3 (2 + cos k pi h), kappa_k = 2/h (1 - cos k pi h).
    h = 1.0 / (n + 1)
    M, K = fe_space.q1_matrices(d, n)
    x = fe_space.node_coordinates(d, n)
    rng = np.random.default_rng(0)
    for _ in range(5):
        k = rng.integers(1, n + 1, size=d)
        v = np.prod([np.sin(k[i] * np.pi * x[:, i]) for i in range(d)], axis=0)
        m = h / 3 * (2 + np.cos(k * np.pi * h))
        kap = 2 / h * (1 - np.cos(k * np.pi * h))
        mu = np.prod(m)
        nu = sum(kap[i] * np.prod([m[j] for j in range(d) if j != i]) for i in range(d))
        assert np.allclose(M @ v, mu * v, atol=1e-14)
        assert np.allclose(K @ v, nu * v, atol=1e-11)


@pytest.mark.parametrize("d", [1, 2, 3])
def test_mass_row_sums_equal_basis_integrals(d):
    # int phi_j dx = h^d for every interior hat function: full-support rows of M sum to h^d.
    n = 5
    h = 1.0 / (n + 1)
    M, K = fe_space.q1_matrices(d, n)
    x = fe_space.node_coordinates(d, n)
    interior = np.all((x > 1.5 * h) & (x < 1 - 1.5 * h), axis=1)
    rs = np.asarray(M.sum(axis=1)).ravel()
    assert np.allclose(rs[interior], h ** d, rtol=1e-13)
    ks = np.asarray(K.sum(axis=1)).ravel()
    assert np.allclose(ks[interior], 0.0, atol=1e-12)


def hat_expansion_1d(coef, n, x):
    """Evaluate sum_i coef_i phi_i(x) for the n interior hats (brute force)."""
    h = 1.0 / (n + 1)
    out = np.zeros_like(x)
    for i in range(n):
        xi = (i + 1) * h
        out += coef[i] * np.clip(1 - np.abs(x - xi) / h, 0, None)
    return out


@pytest.mark.parametrize("d", [1, 2, 3])
def test_prolongation_is_exact_interpolation(d):
    # eq. chap4_spaceRestrictionProlongation: P_x interpolates the coarse
    # piecewise (multi)linear function at the fine nodes.
    nc = 3
    nf = 2 * nc + 1
    rng = np.random.default_rng(d)
    c = rng.normal(size=nc ** d)
    P = fe_space.space_prolongation(d, nc)
    fine = P @ c
    xf = fe_space.node_coordinates(d, nf)
    # brute-force evaluation of the coarse tensor-hat expansion at fine nodes
    cc = c.reshape([nc] * d)        # index order (z, y, x)
    val = np.zeros(len(xf))
    h = 1.0 / (nc + 1)
    for idx in np.ndindex(*cc.shape):
        w = np.ones(len(xf))
        for axis in range(d):
            coord = xf[:, d - 1 - axis]          # idx[0] is the slowest dimension
            xi = (idx[axis] + 1) * h
            w *= np.clip(1 - np.abs(coord - xi) / h, 0, None)
        val += cc[idx] * w
    assert np.allclose(fine, val, atol=1e-14)


def test_prolongation_1d_transpose_is_full_weighting():
    # R_x = P_x^T: coarse i <- 1/2 u_{2i-1} + u_{2i} + 1/2 u_{2i+1}; symbol 1 + cos(theta).
    P = fe_space.space_prolongation_1d(3).toarray()
    R = P.T
    assert np.allclose(R[1], [0, 0, 0.5, 1, 0.5, 0, 0])
    assert np.allclose(R.sum(axis=1), 2.0)
