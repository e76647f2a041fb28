"""Tiled QR driver, application of Q, least squares and iterative refinement
(oracle; test infrastructure only).

The driver runs the kernel tasks of oracle.dag in emission order (a
topological order of the DAG), each on the tiles it names, with the kernels
of oracle.kernels.  The matrix is m x n with m = p*nb, n = q*nb (full tiles,
Remark 1 of Sec. 3.2).

After the factorization, R is the upper triangle of the top n x n block (tile
rows 1..q).  Q is the product of the reflector sets of the panel tasks:
Q^T applies them in task order, Q in reverse task order (Sec. 1: R = U_l ...
U_1 A and Q = U_1^H ... U_l^H).

Least squares (Sec. 1, first use of the QR factorization): x minimizes
||b - A x||_2 and is R^{-1} (Q^T b)(1:n).

Parity: pinned by the unblocked Householder QR (oracle.brute, R equal up to
row signs), by numpy.linalg.qr / numpy.linalg.lstsq, and by the residual and
orthogonality bounds ||A - QR||_F / ||A||_F <= 50 n eps and
||Q^T Q - I||_F <= 50 n eps (tests/test_oracle_tiled.py).  The refinement
loop is pinned on the CPU by planting a perturbed factorization and checking
that it converges to the FP64 solution.  backward_error is pinned by hand
values (square and tall, with ||A||_F != ||A||_2), by the perturbations of
the Rigal-Gaches theorem that attain it, by its zeros (exact and
least-squares solutions, b orthogonal to range(A)) and by its invariance
under A, b -> cA, cb.
"""

import numpy as np
from scipy.linalg import solve_triangular

from . import dag, kernels, trees


def _tile(A, r, c, nb):
    """View of tile (r, c), 1-based."""
    return A[(r - 1) * nb:r * nb, (c - 1) * nb:c * nb]


class Factors:
    def __init__(self, A, nb, tasks, tau_g, tau_p, p, q):
        self.A, self.nb, self.tasks = A, nb, tasks
        self.tau_g, self.tau_p, self.p, self.q = tau_g, tau_p, p, q

    @property
    def m(self):
        return self.p * self.nb

    @property
    def n(self):
        return self.q * self.nb

    def R(self):
        return np.triu(self.A[:self.n, :self.n])


def tiled_qr(A, nb, tree, bs=1, kern=dag.KERN_DEFAULT):
    """Factor A (m x n, m = p nb, n = q nb) with the given tree and kernels."""
    A = np.array(A, dtype=np.float64, order="F", copy=True)
    m, n = A.shape
    if m % nb or n % nb:
        raise ValueError("m and n must be multiples of nb")
    p, q = m // nb, n // nb
    kf = dag.resolve_kernels(tree, kern)
    tasks, _ = dag.build_tasks(p, q, trees.elim_list(p, q, tree, bs), kf)
    tau_g, tau_p = {}, {}
    for (kind, i, piv, k, j) in tasks:
        if kind == dag.GEQRT:
            tau_g[(i, k)] = kernels.geqrt(_tile(A, i, k, nb))
        elif kind == dag.UNMQR:
            kernels.unmqr(_tile(A, i, k, nb), tau_g[(i, k)], _tile(A, i, j, nb))
        elif kind == dag.TSQRT:
            tau_p[(i, k)] = kernels.tsqrt(_tile(A, piv, k, nb), _tile(A, i, k, nb))
        elif kind == dag.TSMQR:
            kernels.tsmqr(_tile(A, i, k, nb), tau_p[(i, k)],
                          _tile(A, piv, j, nb), _tile(A, i, j, nb))
        elif kind == dag.TTQRT:
            tau_p[(i, k)] = kernels.ttqrt(_tile(A, piv, k, nb), _tile(A, i, k, nb))
        elif kind == dag.TTMQR:
            kernels.ttmqr(_tile(A, i, k, nb), tau_p[(i, k)],
                          _tile(A, piv, j, nb), _tile(A, i, j, nb))
    return Factors(A, nb, tasks, tau_g, tau_p, p, q)


def apply_q(F, B, trans="T"):
    """Return Q^T B (trans='T') or Q B (trans='N') for B with m rows."""
    B = np.array(B, dtype=np.float64, order="F", copy=True)
    if B.ndim == 1:
        B = B[:, None]
    nb, A = F.nb, F.A
    panels = [t for t in F.tasks if t[0] in (dag.GEQRT, dag.TSQRT, dag.TTQRT)]
    if trans == "N":
        panels = panels[::-1]
    for (kind, i, piv, k, _) in panels:
        Bi = B[(i - 1) * nb:i * nb, :]
        if kind == dag.GEQRT:
            kernels.unmqr(_tile(A, i, k, nb), F.tau_g[(i, k)], Bi, trans)
            continue
        Bp = B[(piv - 1) * nb:piv * nb, :]
        if kind == dag.TSQRT:
            kernels.tsmqr(_tile(A, i, k, nb), F.tau_p[(i, k)], Bp, Bi, trans)
        else:
            kernels.ttmqr(_tile(A, i, k, nb), F.tau_p[(i, k)], Bp, Bi, trans)
    return B


def thin_q(F):
    """Q (m x n) = Q [I_n; 0]."""
    E = np.zeros((F.m, F.n))
    E[:F.n, :F.n] = np.eye(F.n)
    return apply_q(F, E, "N")


def lstsq(F, B):
    """x = R^{-1} (Q^T B)(1:n)."""
    Y = apply_q(F, B, "T")
    return solve_triangular(F.R(), Y[:F.n, :], lower=False)


def backward_error(A, X, B):
    """Normwise backward error per right-hand side.

    Square systems: ||b - A x||_2 / (||A||_F ||x||_2 + ||b||_2).
    Tall systems (least squares, residual r = b - A x): ||A^T r||_2 /
    (||A||_F ||r||_2) when r != 0, else 0.
    """
    A = np.asarray(A, dtype=np.float64)
    X = np.atleast_2d(np.asarray(X, dtype=np.float64).T).T
    B = np.atleast_2d(np.asarray(B, dtype=np.float64).T).T
    nA = np.linalg.norm(A, "fro")
    R = B - A @ X
    out = []
    for c in range(X.shape[1]):
        r = R[:, c]
        if A.shape[0] == A.shape[1]:
            den = nA * np.linalg.norm(X[:, c]) + np.linalg.norm(B[:, c])
            out.append(np.linalg.norm(r) / den if den else 0.0)
        else:
            nr = np.linalg.norm(r)
            out.append(np.linalg.norm(A.T @ r) / (nA * nr) if nr else 0.0)
    return np.array(out)


def refine(A, B, solve, tol=1e-12, max_iter=30):
    """Classical iterative refinement for a square system.

    solve(Rhs) returns an approximate A^{-1} Rhs (e.g. from a factorization
    held at lower precision).  Iterates x <- x + solve(b - A x) with the
    residual in FP64 until the backward error is <= tol, max_iter is reached,
    or the error stops halving over three iterations.
    Returns (X, iters, converged, eta).
    """
    A = np.asarray(A, dtype=np.float64)
    X = solve(B)
    hist = []
    for it in range(max_iter + 1):
        eta = float(np.max(backward_error(A, X, B)))
        hist.append(eta)
        if eta <= tol:
            return X, it, True, eta
        if it == max_iter:
            break
        if len(hist) > 3 and hist[-1] > 0.5 * hist[-4]:
            break
        X = X + solve(B - A @ X)
    return X, it, False, eta
