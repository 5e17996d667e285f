"""Pins of the oracle's condition estimate for the per-block precision choice of the FEM
factorisation (kappa_est = (max L_rr / min L_rr)^2 of the Cholesky factor; FP64 kept for the
stiffest blocks only, the paper not stating its arithmetic).

* Diagonal K: L = sqrt(K), so kappa_est is the ratio of the largest to the smallest diagonal
  entry (a missing square or square root fails it).
* 2 x 2 worked by hand: [[9, 3], [3, 2]] has L = [[3, 0], [1, 1]], kappa_est = 9, and its
  eigenvalues (11 +- sqrt(85)) / 2 give the condition number 11.36 above it; [[4, 2], [2, 5]]
  has L = [[2, 0], [1, 2]], kappa_est = 1.
* The factor itself: L L^T reproduces K and L is lower triangular with a positive diagonal
  (a transposed or mis-indexed update fails it).
* The bound: kappa_est never exceeds the 2-norm condition number (every pivot lies between the
  extreme eigenvalues), over random SPD matrices spanning condition numbers 1e0 to 1e8.
* A matrix that is not positive definite is refused.
"""
import numpy as np
import pytest

from oracle import precision as P


@pytest.mark.parametrize("d", [[1.0, 4.0, 2.0], [5.0], [3.0, 3.0], [1e-3, 7.0, 1e5, 2.0]])
def test_diagonal(d):
    assert P.kappa_est(np.diag(d)) == pytest.approx(max(d) / min(d), rel=1e-14)


def test_two_by_two_by_hand():
    K = np.array([[9.0, 3.0], [3.0, 2.0]])
    np.testing.assert_allclose(P.cholesky_lower(K), [[3.0, 0.0], [1.0, 1.0]], rtol=0, atol=1e-15)
    assert P.kappa_est(K) == pytest.approx(9.0, rel=1e-14)
    lam = np.array([(11 - np.sqrt(85)) / 2, (11 + np.sqrt(85)) / 2])
    assert lam[1] / lam[0] == pytest.approx(11.3564, rel=1e-4) and P.kappa_est(K) <= lam[1] / lam[0]
    assert P.kappa_est(np.array([[4.0, 2.0], [2.0, 5.0]])) == pytest.approx(1.0, rel=1e-14)


@pytest.mark.parametrize("seed,logc", [(1, 0.0), (2, 2.0), (3, 4.0), (4, 6.0), (5, 8.0)])
def test_factor_and_lower_bound(seed, logc):
    rng = np.random.default_rng(seed)
    n = 24
    Q, _ = np.linalg.qr(rng.normal(size=(n, n)))
    ev = np.logspace(0.0, logc, n)
    K = (Q * ev) @ Q.T
    K = (K + K.T) / 2
    L = P.cholesky_lower(K)
    assert np.allclose(np.triu(L, 1), 0.0) and (np.diag(L) > 0).all()
    np.testing.assert_allclose(L @ L.T, K, rtol=0, atol=1e-10 * np.abs(K).max())
    k = P.kappa_est(K)
    assert 1.0 <= k <= ev[-1] / ev[0] * (1 + 1e-6)


def test_block_matrix_order():
    A = np.diag([1.0, 2.0, 3.0])
    J = np.array([[0.0, 0.0, 1.0]])
    K = P.block_matrix(A, J, 10.0, [1, 0, 2])
    np.testing.assert_array_equal(K, np.diag([2.0, 1.0, 13.0]))


def test_not_positive_definite_is_refused():
    with pytest.raises(ValueError):
        P.kappa_est(np.array([[1.0, 2.0], [2.0, 1.0]]))
