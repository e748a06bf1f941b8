"""Dense-matrix forms of the oracle operators on tiny grids (test infrastructure only).

Used to pin the matrix-free oracle: the adjoint against the explicit transpose
of the forward map, CG against a direct Cholesky solve of eq. (normalewi), the
Sherman-Morrison-Woodbury route of Sec. 5.1 and the weighted-residual identity
of Sec. 2.3.
"""
from __future__ import annotations

import numpy as np


def dense_matrix(apply, n_in: int, in_shape) -> np.ndarray:
    """Columns of a linear map from its action on unit vectors."""
    cols = []
    for j in range(n_in):
        e = np.zeros(n_in)
        e[j] = 1.0
        cols.append(np.ravel(apply(e.reshape(in_shape))))
    return np.stack(cols, axis=1)


def cholesky_solve(N: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Solve N x = b for symmetric positive definite N by a Cholesky factorisation."""
    L = np.linalg.cholesky(N)
    y = np.linalg.solve(L, b)
    return np.linalg.solve(L.T, y)


def smw_extended_source(S: np.ndarray, w2: np.ndarray, beta: float, d: np.ndarray) -> np.ndarray:
    """Extended source through data space (Sec. 5.1, eq. (vd), eq. (wv), eq. (q)):

      v = S (B^T B)^{-1} S^T d,  (beta I + S (B^T B)^{-1} S^T) w = v,
      q = (beta B^T B)^{-1} S^T (d - w).
    """
    Winv = 1.0 / w2
    K = S @ (Winv[:, None] * S.T)
    v = K @ d
    w = np.linalg.solve(beta * np.eye(K.shape[0]) + K, v)
    return Winv * (S.T @ (d - w)) / beta
