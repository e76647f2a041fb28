"""The six tile kernels in double-complex arithmetic, as plain unblocked
Householder code (oracle; test infrastructure only).

The paper's experiments run the same kernels in double and double complex
(Sec. 5: the ZGEQRT family).  The algorithms are those of oracle.kernels with
the complex elementary reflector of LAPACK's zlarfg:

  H = I - tau u u^H, u = (1, v), and H^H (alpha, x) = (beta, 0) with beta
  real: beta = -sign(Re alpha) * sqrt(|alpha|^2 + ||x||^2) (sign(+0) = +1),
  tau = (beta - alpha) / beta, v = x / (alpha - beta).  H = I (tau = 0)
  only when x = 0 and alpha is real; a complex alpha over a zero x still
  gets a reflector, which makes the diagonal of R real.

The factorization applies H_j^H from the left: R = H_n^H ... H_1^H A, so
Q = H_1 H_2 ... H_n, and Q^H C applies H_1^H first, H^H c = c - conj(tau)
u (u^H c); Q C applies H_n first with tau.

Storage is that of oracle.kernels (R upper, V below the diagonal or in the
zeroed tile).  On real input every quantity stays real and the kernels do
the arithmetic of oracle.kernels.

Parity: pinned in tests/test_oracle_complex.py by the real oracle on real
input, by numpy.linalg.qr (LAPACK zgeqrf: R equal up to the signs of its
rows), by ||A - QR||_F / ||A||_F and ||Q^H Q - I||_F <= 50 n eps, and by
the closed form of a diagonal complex matrix.
"""

import numpy as np


def zhouse(alpha, x):
    """Complex elementary reflector of (alpha, x): (beta, tau, v)."""
    alpha = complex(alpha)
    sigma = float(np.sqrt(np.vdot(x, x).real))
    if sigma == 0.0 and alpha.imag == 0.0:
        return alpha, 0j, np.zeros_like(x)
    nrm = float(np.sqrt(alpha.real * alpha.real + alpha.imag * alpha.imag + sigma * sigma))
    beta = -np.copysign(nrm, alpha.real if alpha.real != 0.0 else 1.0)
    tau = (beta - alpha) / beta
    v = x / (alpha - beta)
    return complex(beta), complex(tau), v


def _apply(t, top, below, v, trans):
    """[top; below] <- H^H [top; below] (trans 'C') or H [top; below] ('N')
    for H = I - t u u^H, u = (1, v); top is a row, below a block."""
    w = top + np.conj(v) @ below
    s = np.conj(t) if trans == "C" else t
    top -= s * w
    below -= s * np.outer(v, w)


def zgeqrt(A):
    """Householder QR of one complex tile, in place.  Returns tau."""
    m, n = A.shape
    tau = np.zeros(n, dtype=np.complex128)
    for j in range(min(m, n)):
        beta, t, v = zhouse(A[j, j], A[j + 1:, j])
        A[j, j] = beta
        A[j + 1:, j] = v
        tau[j] = t
        if t != 0 and j + 1 < n:
            _apply(t, A[j, j + 1:], A[j + 1:, j + 1:], v, "C")
    return tau


def zunmqr(V, tau, C, trans="C"):
    """C <- Q^H C (trans 'C') or Q C ('N') for Q from zgeqrt(V)."""
    n = V.shape[1]
    for j in (range(n) if trans == "C" else range(n - 1, -1, -1)):
        if tau[j] != 0:
            _apply(tau[j], C[j, :], C[j + 1:, :], V[j + 1:, j], trans)


def ztsqrt(R, A2):
    """Zero the full tile A2 against the upper triangle R, in place."""
    n = R.shape[1]
    tau = np.zeros(n, dtype=np.complex128)
    for j in range(n):
        beta, t, v = zhouse(R[j, j], A2[:, j])
        R[j, j] = beta
        A2[:, j] = v
        tau[j] = t
        if t != 0 and j + 1 < n:
            _apply(t, R[j, j + 1:], A2[:, j + 1:], v, "C")
    return tau


def ztsmqr(V2, tau, C1, C2, trans="C"):
    """[C1; C2] <- Q^H [C1; C2] (or Q [...]), Q from ztsqrt."""
    n = V2.shape[1]
    for j in (range(n) if trans == "C" else range(n - 1, -1, -1)):
        if tau[j] != 0:
            _apply(tau[j], C1[j, :], C2, V2[:, j], trans)


def zttqrt(R1, R2):
    """Zero the upper triangle R2 against the upper triangle R1, in place;
    column j's reflector has support on row j of R1 and rows 0..j of R2."""
    n = R1.shape[1]
    tau = np.zeros(n, dtype=np.complex128)
    for j in range(n):
        beta, t, v = zhouse(R1[j, j], R2[:j + 1, j].copy())
        R1[j, j] = beta
        R2[:j + 1, j] = v
        tau[j] = t
        if t != 0 and j + 1 < n:
            _apply(t, R1[j, j + 1:], R2[:j + 1, j + 1:], v, "C")
    return tau


def zttmqr(V2, tau, C1, C2, trans="C"):
    """[C1; C2] <- Q^H [C1; C2] (or Q [...]), Q from zttqrt; only the upper
    triangle of V2 is read."""
    n = V2.shape[1]
    for j in (range(n) if trans == "C" else range(n - 1, -1, -1)):
        if tau[j] != 0:
            _apply(tau[j], C1[j, :], C2[:j + 1, :], V2[:j + 1, j], trans)
