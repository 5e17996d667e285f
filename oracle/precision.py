"""Condition estimate behind the precision choice for deformable blocks, written from its
definition on the CPU.  Test infrastructure: used by the tests only.

The paper does not state its arithmetic.  The precision choice read here keeps FP64 for
factorising the stiffest deformable subsystem blocks only, a block's stiffness measured by
  kappa_est = (max_r L_rr / min_r L_rr)^2
of the Cholesky factor K = L L^T of the block's K = A + beta J^T J (beta by Eq. 23), taken
in the order the factorisation uses.  Each pivot L_rr^2 is the last pivot of the leading
r x r block, 1 / ((K_{1:r,1:r})^{-1})_{rr}, which lies between the smallest and largest
eigenvalues of K (interlacing), so kappa_est never exceeds the 2-norm condition number.
Blocks with kappa_est above a threshold are factorised in FP64, the others in FP32.
"""
from __future__ import annotations

import numpy as np


def cholesky_lower(K):
    """Lower Cholesky factor of a symmetric positive definite K, column by column from the
    definition K = L L^T (L_jj = sqrt(K_jj - sum_k<j L_jk^2),
    L_ij = (K_ij - sum_k<j L_ik L_jk) / L_jj for i > j)."""
    K = np.asarray(K, dtype=np.float64)
    n = K.shape[0]
    L = np.zeros_like(K)
    for j in range(n):
        d = K[j, j] - L[j, :j] @ L[j, :j]
        if not d > 0.0:
            raise ValueError("matrix is not positive definite")
        L[j, j] = np.sqrt(d)
        L[j + 1:, j] = (K[j + 1:, j] - L[j + 1:, :j] @ L[j, :j]) / L[j, j]
    return L


def kappa_est(K):
    """(max_r L_rr / min_r L_rr)^2 of the Cholesky factor of K."""
    d = np.diag(cholesky_lower(K))
    return float((d.max() / d.min()) ** 2)


def block_matrix(A_i, J_i, beta, order):
    """K = A_i + beta J_i^T J_i with rows and columns taken in ``order``."""
    K = np.asarray(A_i, np.float64) + beta * np.asarray(J_i, np.float64).T @ np.asarray(J_i, np.float64)
    o = np.asarray(order)
    return K[np.ix_(o, o)]
