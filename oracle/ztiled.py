"""Tiled QR driver and application of Q in double complex (oracle; test
infrastructure only).

The same task lists as oracle.tiled (oracle.dag over the elimination lists
of oracle.trees, run in emission order), with the complex kernels of
oracle.zkernels.  R is the upper triangle of the top n x n block; Q^H
applies the panel tasks' reflector sets in task order, Q in reverse order
(Sec. 1: R = U_l ... U_1 A, Q = U_1^H ... U_l^H).

Parity: pinned in tests/test_oracle_complex.py (see oracle.zkernels).
"""

import numpy as np

from . import dag, trees, zkernels


def _tile(A, r, c, nb):
    return A[(r - 1) * nb:r * nb, (c - 1) * nb:c * nb]


class ZFactors:
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


def ztiled_qr(A, nb, tree, bs=1, kern=dag.KERN_DEFAULT):
    """Factor the complex A (m x n, m = p nb, n = q nb)."""
    A = np.array(A, dtype=np.complex128, order="F", copy=True)
    m, n = A.shape
    if m % nb or n % nb:
        raise ValueError("m and n must be multiples of nb")
    p, q = m // nb, n // nb
    kf = dag.resolve_kernels(tree, kern)
    tasks, _ = dag.build_tasks(p, q, trees.elim_list(p, q, tree, bs), kf)
    tau_g, tau_p = {}, {}
    for (kind, i, piv, k, j) in tasks:
        if kind == dag.GEQRT:
            tau_g[(i, k)] = zkernels.zgeqrt(_tile(A, i, k, nb))
        elif kind == dag.UNMQR:
            zkernels.zunmqr(_tile(A, i, k, nb), tau_g[(i, k)], _tile(A, i, j, nb))
        elif kind == dag.TSQRT:
            tau_p[(i, k)] = zkernels.ztsqrt(_tile(A, piv, k, nb), _tile(A, i, k, nb))
        elif kind == dag.TSMQR:
            zkernels.ztsmqr(_tile(A, i, k, nb), tau_p[(i, k)], _tile(A, piv, j, nb), _tile(A, i, j, nb))
        elif kind == dag.TTQRT:
            tau_p[(i, k)] = zkernels.zttqrt(_tile(A, piv, k, nb), _tile(A, i, k, nb))
        elif kind == dag.TTMQR:
            zkernels.zttmqr(_tile(A, i, k, nb), tau_p[(i, k)], _tile(A, piv, j, nb), _tile(A, i, j, nb))
    return ZFactors(A, nb, tasks, tau_g, tau_p, p, q)


def zapply_q(F, B, trans="C"):
    """Return Q^H B (trans 'C') or Q B ('N') for B with m rows."""
    B = np.array(B, dtype=np.complex128, order="F", copy=True)
    if B.ndim == 1:
        B = B[:, None]
    nb, A = F.nb, F.A
    panels = [t for t in F.tasks if t[0] in (dag.GEQRT, dag.TSQRT, dag.TTQRT)]
    if trans == "N":
        panels = panels[::-1]
    for (kind, i, piv, k, _) in panels:
        Bi = B[(i - 1) * nb:i * nb, :]
        if kind == dag.GEQRT:
            zkernels.zunmqr(_tile(A, i, k, nb), F.tau_g[(i, k)], Bi, trans)
            continue
        Bp = B[(piv - 1) * nb:piv * nb, :]
        if kind == dag.TSQRT:
            zkernels.ztsmqr(_tile(A, i, k, nb), F.tau_p[(i, k)], Bp, Bi, trans)
        else:
            zkernels.zttmqr(_tile(A, i, k, nb), F.tau_p[(i, k)], Bp, Bi, trans)
    return B


def zthin_q(F):
    """Q (m x n) = Q [I_n; 0]."""
    E = np.zeros((F.m, F.n), dtype=np.complex128)
    E[:F.n, :F.n] = np.eye(F.n)
    return zapply_q(F, E, "N")
