"""Pins of the oracle's GLL points, Lagrange basis and 1D element matrices
against closed forms and quadrature exactness (not against itself)."""
import numpy as np
import pytest

from oracle import basis, fcm


@pytest.mark.parametrize("p,nodes,weights", [
    (1, [-1, 1], [1, 1]),
    (2, [-1, 0, 1], [1 / 3, 4 / 3, 1 / 3]),
    (3, [-1, -np.sqrt(1 / 5), np.sqrt(1 / 5), 1], [1 / 6, 5 / 6, 5 / 6, 1 / 6]),
    (4, [-1, -np.sqrt(3 / 7), 0, np.sqrt(3 / 7), 1], [1 / 10, 49 / 90, 32 / 45, 49 / 90, 1 / 10]),
])
def test_gll_closed_forms(p, nodes, weights):
    x, w = basis.gll(p)
    np.testing.assert_allclose(x, nodes, atol=1e-15)
    np.testing.assert_allclose(w, weights, rtol=1e-14)


@pytest.mark.parametrize("p", range(1, 9))
def test_gll_exact_to_degree_2p_minus_1(p):
    x, w = basis.gll(p)
    for k in range(2 * p):
        exact = 0.0 if k % 2 else 2.0 / (k + 1)
        assert abs(np.sum(w * x ** k) - exact) < 1e-13
    # and not exact for degree 2p (the Lobatto rule's known defect)
    assert abs(np.sum(w * x ** (2 * p)) - 2.0 / (2 * p + 1)) > 1e-6


@pytest.mark.parametrize("p", range(1, 9))
def test_lagrange_cardinal_and_partition_of_unity(p):
    x, _ = basis.gll(p)
    np.testing.assert_allclose(basis.lagrange(x, x), np.eye(p + 1), atol=1e-14)
    xi = np.linspace(-1, 1, 37)
    np.testing.assert_allclose(basis.lagrange(x, xi).sum(axis=1), 1.0, atol=1e-13)
    np.testing.assert_allclose(basis.lagrange_deriv(x, xi).sum(axis=1), 0.0, atol=1e-11)
    # derivative reproduces d/dxi of xi^k exactly for k <= p
    for k in range(p + 1):
        d = basis.lagrange_deriv(x, xi) @ (x ** k)
        np.testing.assert_allclose(d, k * xi ** max(k - 1, 0) if k else 0.0, atol=1e-11)


@pytest.mark.parametrize("p", range(1, 8))
def test_1d_reference_matrices(p):
    """Consistent 1D mass rows sum to the GLL weights (GLL is exact to degree
    2p-1); stiffness rows sum to zero; both symmetric positive (semi)definite."""
    xg, wg = basis.gauss_legendre(p + 1)
    Mh, Kh = fcm.quadrature_matrices(p, np.array([-1.0]), np.array([2.0]),
                                     xg[:, None], wg, np.ones(p + 1), np.ones(p + 1))
    _, wl = basis.gll(p)
    np.testing.assert_allclose(Mh.sum(axis=1), wl, rtol=1e-13)
    np.testing.assert_allclose(Kh.sum(axis=1), 0.0, atol=1e-12)
    np.testing.assert_allclose(Mh, Mh.T, atol=1e-15)
    assert np.linalg.eigvalsh(Mh)[0] > 0
    assert np.linalg.eigvalsh(Kh)[0] > -1e-12
    # the stiffness energy of xi is int_{-1}^{1} 1 dxi = 2
    x, _ = basis.gll(p)
    assert abs(x @ Kh @ x - 2.0) < 1e-12
