"""Pins of the oracle's 1D basis and quadrature against closed forms."""
import numpy as np
import pytest

from oracle.basis import gauss_rule, gll_nodes, lagrange_1d, ref_matrices_1d


def test_gll_closed_forms():
    # Gauss-Lobatto nodes on [0,1] for p <= 4 (textbook values)
    assert np.allclose(gll_nodes(1), [0, 1], atol=1e-15)
    assert np.allclose(gll_nodes(2), [0, 0.5, 1], atol=1e-15)
    s5 = 1 / np.sqrt(5)
    assert np.allclose(gll_nodes(3), [0, 0.5 * (1 - s5), 0.5 * (1 + s5), 1], atol=1e-14)
    s = np.sqrt(3 / 7)
    assert np.allclose(gll_nodes(4), [0, 0.5 * (1 - s), 0.5, 0.5 * (1 + s), 1], atol=1e-14)


@pytest.mark.parametrize("nq", [1, 2, 3, 5, 8])
def test_gauss_exactness(nq):
    x, w = gauss_rule(nq)
    for k in range(2 * nq):
        assert abs(np.sum(w * x ** k) - 1.0 / (k + 1)) < 1e-14
    # one degree more is not integrated exactly
    k = 2 * nq
    assert abs(np.sum(w * x ** k) - 1.0 / (k + 1)) > 1e-13


@pytest.mark.parametrize("p", range(1, 9))
def test_lagrange_derivative_identities(p):
    xi = gll_nodes(p)
    V, D = lagrange_1d(xi, xi)
    assert np.allclose(V, np.eye(p + 1), atol=1e-12)
    assert np.allclose(D @ np.ones(p + 1), 0.0, atol=1e-10)
    assert np.allclose(D @ xi, 1.0, atol=1e-10)
    if p >= 2:
        assert np.allclose(D @ xi ** 2, 2 * xi, atol=1e-9)


@pytest.mark.parametrize("p", range(1, 9))
def test_reference_matrices(p):
    M, K = ref_matrices_1d(p)
    assert abs(M.sum() - 1.0) < 1e-13  # int 1 = 1
    assert np.allclose(K @ np.ones(p + 1), 0.0, atol=1e-10)
    xi = gll_nodes(p)
    # int x * 1 = 1/2 and int (x)'(x)' = 1
    assert abs(np.ones(p + 1) @ M @ xi - 0.5) < 1e-13
    assert abs(xi @ K @ xi - 1.0) < 1e-11
    np.linalg.cholesky(M)


def test_p1_textbook_matrices():
    M, K = ref_matrices_1d(1)
    assert np.allclose(M, [[1 / 3, 1 / 6], [1 / 6, 1 / 3]], atol=1e-15)
    assert np.allclose(K, [[1, -1], [-1, 1]], atol=1e-15)
