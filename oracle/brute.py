"""Textbook unblocked Householder QR of a whole m x n matrix (oracle; test
infrastructure only).

The plain definition of the result the tiled method reaches (Sec. 1): R upper
triangular with A = QR and Q orthonormal.  One reflector per column, applied
to the trailing columns; the reflector convention is oracle.kernels.house.
For full-rank A, R is unique up to the signs of its rows, so any tree and any
kernel family give the same |R| rows.

Parity: pinned against numpy.linalg.qr (|R| rows) and LAPACK dgeqrf through
SciPy (tests/test_oracle_kernels.py).
"""

import numpy as np

from .kernels import house


def householder_qr(A):
    """Returns (R, V, tau): R upper n x n, V the unit-lower reflectors."""
    A = np.array(A, dtype=np.float64, copy=True)
    m, n = A.shape
    tau = np.zeros(n)
    for j in range(n):
        beta, t, v = house(A[j, j], A[j + 1:, j])
        A[j, j] = beta
        A[j + 1:, j] = v
        tau[j] = t
        if t != 0.0:
            w = A[j, j + 1:] + v @ A[j + 1:, j + 1:]
            A[j, j + 1:] -= t * w
            A[j + 1:, j + 1:] -= t * np.outer(v, w)
    return np.triu(A[:n, :]), np.tril(A, -1), tau
