"""The six tile kernels as plain unblocked Householder code in FP64 (oracle;
test infrastructure only).

Sec. 2.1 (Table 1) defines the kernels as standard LAPACK-style blocked
algorithms; the blocking (inner block size ib and the compact-WY T factor)
changes neither R, the reflector vectors V, nor the scalars tau in exact
arithmetic, so this oracle applies one reflector at a time and never forms T.

Conventions (LAPACK's elementary reflector, Sec. 2.1 "a la LAPACK"):
  H = I - tau * v v^T with v(1) = 1 implicit.  For a column (alpha, x):
  sigma = ||x||_2; if sigma == 0 then tau = 0 and beta = alpha (H = I);
  otherwise beta = -sign(alpha) * hypot(alpha, sigma) with sign(+0) = +1,
  tau = (beta - alpha) / beta and v = x / (alpha - beta).

Kernel storage (tiles are nb x nb, column-major as NumPy arrays):
  GEQRT(A)          A <- R (upper) and V (strict lower, unit diagonal implicit).
  UNMQR(V, tau, C)  C <- Q^T C with Q from GEQRT.
  TSQRT(R, A2)      [R; A2] -> R (upper of R), V2 full in A2.
  TSMQR(V2, tau, C1, C2)  [C1; C2] <- Q^T [C1; C2] for TSQRT's Q.
  TTQRT(R1, R2)     [R1; R2] (both upper) -> R in R1, V2 upper triangular in
                    R2's upper triangle; R2's strict lower part is untouched.
  TTMQR(V2, tau, C1, C2)  as TSMQR using only rows 0..j of V2 column j.
Q^T applies H_1 first (Q = H_1 H_2 ... H_nb).

Parity: pinned against LAPACK through SciPy (dgeqrf on the tile or on the
stacked pair; dormqr for the updates) in tests/test_oracle_kernels.py.
"""

import numpy as np


def house(alpha, x):
    """Elementary reflector of (alpha, x).  Returns (beta, tau, v)."""
    sigma = float(np.sqrt(np.dot(x, x)))
    if sigma == 0.0:
        return float(alpha), 0.0, np.zeros_like(x)
    beta = -np.copysign(np.hypot(alpha, sigma), alpha if alpha != 0.0 else 1.0)
    tau = (beta - alpha) / beta
    v = x / (alpha - beta)
    return float(beta), float(tau), v


def geqrt(A):
    """Householder QR of one tile, in place.  Returns tau (length nb)."""
    n = A.shape[1]
    m = A.shape[0]
    tau = np.zeros(n)
    for j in range(min(m, n)):
        beta, t, v = house(A[j, j], A[j + 1:, j])
        A[j, j] = beta
        A[j + 1:, j] = v
        tau[j] = t
        if t != 0.0 and j + 1 < n:
            w = A[j, j + 1:] + v @ A[j + 1:, j + 1:]
            A[j, j + 1:] -= t * w
            A[j + 1:, j + 1:] -= t * np.outer(v, w)
    return tau


def unmqr(V, tau, C, trans="T"):
    """C <- Q^T C (trans='T') or Q C (trans='N') for Q from geqrt(V)."""
    n = V.shape[1]
    order = range(n) if trans == "T" else range(n - 1, -1, -1)
    for j in order:
        t = tau[j]
        if t == 0.0:
            continue
        v = V[j + 1:, j]
        w = C[j, :] + v @ C[j + 1:, :]
        C[j, :] -= t * w
        C[j + 1:, :] -= t * np.outer(v, w)


def tsqrt(R, A2):
    """Zero the full tile A2 against the upper triangle R, in place."""
    n = R.shape[1]
    tau = np.zeros(n)
    for j in range(n):
        beta, t, v = house(R[j, j], A2[:, j])
        R[j, j] = beta
        A2[:, j] = v
        tau[j] = t
        if t != 0.0 and j + 1 < n:
            w = R[j, j + 1:] + v @ A2[:, j + 1:]
            R[j, j + 1:] -= t * w
            A2[:, j + 1:] -= t * np.outer(v, w)
    return tau


def tsmqr(V2, tau, C1, C2, trans="T"):
    """[C1; C2] <- Q^T [C1; C2] (or Q [...] for trans='N'), Q from tsqrt."""
    n = V2.shape[1]
    order = range(n) if trans == "T" else range(n - 1, -1, -1)
    for j in order:
        t = tau[j]
        if t == 0.0:
            continue
        v = V2[:, j]
        w = C1[j, :] + v @ C2
        C1[j, :] -= t * w
        C2 -= t * np.outer(v, w)


def ttqrt(R1, R2):
    """Zero the upper triangle R2 against the upper triangle R1, in place.
    Column j's reflector has support on row j of R1 and rows 0..j of R2."""
    n = R1.shape[1]
    tau = np.zeros(n)
    for j in range(n):
        beta, t, v = house(R1[j, j], R2[:j + 1, j].copy())
        R1[j, j] = beta
        R2[:j + 1, j] = v
        tau[j] = t
        if t != 0.0 and j + 1 < n:
            w = R1[j, j + 1:] + v @ R2[:j + 1, j + 1:]
            R1[j, j + 1:] -= t * w
            R2[:j + 1, j + 1:] -= t * np.outer(v, w)
    return tau


def ttmqr(V2, tau, C1, C2, trans="T"):
    """[C1; C2] <- Q^T [C1; C2] (or Q [...]), Q from ttqrt; only the upper
    triangle of V2 is read."""
    n = V2.shape[1]
    order = range(n) if trans == "T" else range(n - 1, -1, -1)
    for j in order:
        t = tau[j]
        if t == 0.0:
            continue
        v = V2[:j + 1, j]
        w = C1[j, :] + v @ C2[:j + 1, :]
        C1[j, :] -= t * w
        C2[:j + 1, :] -= t * np.outer(v, w)
