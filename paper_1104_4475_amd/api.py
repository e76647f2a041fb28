"""Torch-facing helpers over the C ABI: device memory and the current HIP
stream come from torch; all arithmetic runs in libtiledqr.so."""

import ctypes

from . import _lib
from ._lib import check


def _torch():
    import torch
    return torch


def colmajor(A):
    """Return a float64 CUDA tensor with the same values as A stored in
    column-major order (stride (1, rows))."""
    torch = _torch()
    if A.dtype != torch.float64:
        raise TypeError("tiled QR works on float64 tensors")
    if not A.is_cuda:
        raise ValueError("tensor must live on the GPU")
    if A.dim() == 1:
        A = A[:, None]
    if A.stride(0) == 1 and A.stride(1) >= max(1, A.shape[0]):
        return A
    return A.t().contiguous().t()


def _stream():
    return ctypes.c_void_p(_torch().cuda.current_stream().cuda_stream)


def _ld(A):
    """Leading dimension of a column-major tensor (the column stride is
    meaningless with fewer than two columns, so it is then the row count)."""
    if A.dim() == 2 and A.shape[1] > 1:
        return A.stride(1)
    return max(1, A.shape[0])


class Factors:
    """Owner of a tqr_factors handle."""

    def __init__(self, handle, m, n, nb, opts, owner=None):
        self.handle = handle
        self.m, self.n, self.nb = m, n, nb
        self.opts = opts
        self.owner = owner  # a Batch that owns the handle (then not destroyed here)

    def __del__(self):
        h = getattr(self, "handle", None)
        if h and getattr(self, "owner", None) is None:
            destroy = getattr(_lib, "tiledqr_destroy", None)
            if destroy is not None:  # None once the interpreter tears modules down
                destroy(h)
        self.handle = None

    def sync(self):
        check(_lib.tiledqr_sync(self.handle), "tiledqr_sync")

    def exec_ms(self):
        """Duration of the last factorization's executor kernel (HIP events)."""
        ms = ctypes.c_float()
        check(_lib.tiledqr_exec_time(self.handle, ctypes.byref(ms)), "tiledqr_exec_time")
        return ms.value

    def set_trace(self, enable=True):
        check(_lib.tiledqr_set_trace(self.handle, 1 if enable else 0), "tiledqr_set_trace")

    def trace(self):
        """Per executor subtask (dispatch order): int64 array (n, 10) =
        kind, i, piv, k, j, slab, ticket, ready, end, workgroup (ticks), and
        the tick rate in Hz."""
        import numpy as np
        n = ctypes.c_int64()
        rate = ctypes.c_double()
        check(_lib.tiledqr_get_trace(self.handle, None, ctypes.byref(n), ctypes.byref(rate)), "tiledqr_get_trace")
        out = np.zeros((max(1, n.value), 10), dtype=np.int64)
        check(_lib.tiledqr_get_trace(self.handle, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                     ctypes.byref(n), ctypes.byref(rate)), "tiledqr_get_trace")
        return out[:n.value], rate.value

    def exec_plan(self):
        """Executor subtasks of the factorization in dispatch order: int32
        array (n, 10) = kind, i, piv, k, j, slab, dep_begin, dep_end, sdep,
        pdep, and the int32 predecessor entries (index, stage and early bit:
        _lib.DEP_INDEX, DEP_STAGE_SHIFT, DEP_EARLY; tiledqr_exec_plan)."""
        import numpy as np
        n, nd = ctypes.c_int64(), ctypes.c_int64()
        check(_lib.tiledqr_exec_plan(self.handle, None, ctypes.byref(n), None, ctypes.byref(nd)), "tiledqr_exec_plan")
        sub = np.zeros((max(1, n.value), 10), dtype=np.int32)
        deps = np.zeros(max(1, nd.value), dtype=np.int32)
        P = ctypes.POINTER(ctypes.c_int32)
        check(_lib.tiledqr_exec_plan(self.handle, sub.ctypes.data_as(P), ctypes.byref(n), deps.ctypes.data_as(P),
                                     ctypes.byref(nd)), "tiledqr_exec_plan")
        return sub[:n.value], deps[:nd.value]

    def solve_r(self, X, trans="N"):
        """Return R^{-1} X (trans 'N') or R^{-T} X (trans 'T') for X with n
        rows (tiledqr_solve_r); X is not modified."""
        X = colmajor(X).clone()
        check(_lib.tiledqr_solve_r(self.handle, trans.encode(), X.data_ptr(), _ld(X), X.shape[1], _stream()),
              "tiledqr_solve_r")
        return X

    def refactor(self, A):
        A = colmajor(A)
        check(_lib.tiledqr_refactor(self.handle, A.data_ptr(), _ld(A), _stream()), "tiledqr_refactor")

    def R(self):
        torch = _torch()
        R = torch.empty((self.n, self.n), dtype=torch.float64, device="cuda").t()
        check(_lib.tiledqr_get_r(self.handle, R.data_ptr(), self.n, _stream()), "tiledqr_get_r")
        return R

    def packed(self):
        torch = _torch()
        P = torch.empty((self.n, self.m), dtype=torch.float64, device="cuda").t()
        check(_lib.tiledqr_get_packed(self.handle, P.data_ptr(), self.m, _stream()), "tiledqr_get_packed")
        return P

    def tau(self):
        """(tau_geqrt, tau_pair) each of shape (q, p, nb): [c, r] -> tile (r, c)."""
        torch = _torch()
        p, q = self.m // self.nb, self.n // self.nb
        t = torch.empty(2 * p * q * self.nb, dtype=torch.float64, device="cuda")
        check(_lib.tiledqr_get_tau(self.handle, t.data_ptr(), _stream()), "tiledqr_get_tau")
        t = t.view(2, q, p, self.nb)
        return t[0], t[1]

    def apply_q(self, B, trans="T"):
        """Return Q^T B or Q B (B: m x nrhs float64 CUDA tensor, not modified)."""
        B = colmajor(B).clone()  # preserves the column-major strides
        check(_lib.tiledqr_apply_q(self.handle, trans.encode(), B.data_ptr(), _ld(B), B.shape[1], _stream()),
              "tiledqr_apply_q")
        return B

    def thin_q(self):
        torch = _torch()
        E = torch.zeros((self.n, self.m), dtype=torch.float64, device="cuda").t()
        E[:self.n, :self.n] = torch.eye(self.n, dtype=torch.float64, device="cuda")
        check(_lib.tiledqr_apply_q(self.handle, b"N", E.data_ptr(), self.m, self.n, _stream()), "tiledqr_apply_q")
        return E

    def refactor_qtb(self, A, B):
        """Re-factor A and compute Q^T B in the same executor launch
        (tiledqr_refactor_qtb); returns Q^T B as a new column-major tensor."""
        A = colmajor(A)
        QtB = colmajor(B).clone().t().contiguous().t() if B.dim() == 2 else colmajor(B).clone()
        check(_lib.tiledqr_refactor_qtb(self.handle, A.data_ptr(), _ld(A), QtB.data_ptr(), _ld(QtB), QtB.shape[1],
                                        _stream()), "tiledqr_refactor_qtb")
        return QtB

    def lstsq(self, B, A0=None, tol=0.0, max_iter=30, method=0, raise_on_noconv=False, QtB=None):
        """Solve min ||B - A X||.  With tol > 0 the solution is refined
        against A0 (the original matrix); method: 0 auto (semi-normal
        corrections, then classical for square or the augmented system for
        tall matrices), 1 classical, 2 augmented system, 3 semi-normal only
        (tiledqr_lstsq).  QtB: Q^T B already computed (from refactor_qtb).
        Returns (X, info dict)."""
        torch = _torch()
        B = colmajor(B)
        nrhs = B.shape[1]
        X = torch.empty((nrhs, self.n), dtype=torch.float64, device="cuda").t()
        info = _lib.RefineInfo()
        ref = _lib.RefineOpts(tol, max_iter, method)
        a0p, lda = None, self.m
        if A0 is not None:
            A0 = colmajor(A0)
            a0p, lda = A0.data_ptr(), _ld(A0)
        if QtB is not None:
            QtB = colmajor(QtB)
            st = _lib.tiledqr_lstsq_qtb(self.handle, a0p, lda, B.data_ptr(), _ld(B), QtB.data_ptr(), _ld(QtB), nrhs,
                                        X.data_ptr(), self.n, ctypes.byref(ref), ctypes.byref(info), _stream())
        else:
            st = _lib.tiledqr_lstsq(self.handle, a0p, lda, B.data_ptr(), _ld(B), nrhs, X.data_ptr(), self.n,
                                    ctypes.byref(ref), ctypes.byref(info), _stream())
        if st != _lib.TQR_OK and not (st == _lib.TQR_ENOTCONV and not raise_on_noconv):
            raise _lib.TiledQRError(st, "tiledqr_lstsq")
        return X, {"iters": info.iters, "converged": bool(info.converged),
                   "backward_err": info.backward_err, "semi_normal": info.semi_normal,
                   "augmented": info.augmented, "status": st}


def factor(A, nb, tree=_lib.TREE_GREEDY, bs=1, kernels=_lib.KERN_DEFAULT, upd=_lib.UPD_F64):
    """Factor the m x n float64 CUDA tensor A (m, n multiples of nb)."""
    A = colmajor(A)
    m, n = A.shape
    opts = _lib.Opts(m, n, nb, 0, tree, bs, kernels, upd)
    h = ctypes.c_void_p()
    check(_lib.tiledqr_factor(ctypes.byref(opts), A.data_ptr(), _ld(A), ctypes.byref(h), _stream()),
          "tiledqr_factor")
    return Factors(h, m, n, nb, opts)


def _batch_opts(shapes, nbs, tree, bs, kernels, upd):
    """Per-problem options (tree, bs and kernels: one value for every
    problem, or a list); a PlasmaTree or Hadri domain size larger than a
    problem's tile rows is capped at them."""
    k = len(shapes)
    per = lambda v, i: v[i] if isinstance(v, (list, tuple)) else v  # noqa: E731
    opts = (_lib.Opts * k)()
    for i, ((m, n), nb) in enumerate(zip(shapes, nbs)):
        t, b = per(tree, i), per(bs, i)
        if t in (_lib.TREE_PLASMA, _lib.TREE_HADRI):
            b = min(b, m // nb)
        opts[i] = _lib.Opts(m, n, nb, 0, t, b, per(kernels, i), upd)
    return opts


class Batch:
    """Many factorizations in one persistent launch, replayable as a HIP
    graph (tiledqr_batch_*).  shapes: list of (m, n); nbs: tile sizes (32
    or 64); tree, bs, kernels: one value for all problems or one per
    problem; lds: leading dimensions the runs will use (default m)."""

    def __init__(self, shapes, nbs, tree=_lib.TREE_GREEDY, bs=1, kernels=_lib.KERN_DEFAULT, upd=_lib.UPD_F64,
                 lds=None):
        k = len(shapes)
        self.shapes, self.nbs = list(shapes), list(nbs)
        self.opts = _batch_opts(shapes, nbs, tree, bs, kernels, upd)
        ldas = (ctypes.c_int64 * k)(*[(lds[i] if lds else shapes[i][0]) for i in range(k)])
        self.lds = list(ldas)
        h = ctypes.c_void_p()
        self.handle = None
        check(_lib.tiledqr_batch_create(k, self.opts, ldas, ctypes.byref(h)), "tiledqr_batch_create")
        self.handle = h

    def __del__(self):
        h = getattr(self, "handle", None)
        if h:
            destroy = getattr(_lib, "tiledqr_batch_destroy", None)
            if destroy is not None:  # None once the interpreter tears modules down
                destroy(h)
            self.handle = None

    def run(self, mats):
        """Enqueue one run on the current stream (mats: column-major float64
        CUDA tensors of the batch's shapes and leading dimensions)."""
        k = len(self.shapes)
        ptrs = (ctypes.c_void_p * k)()
        self._mats = mats  # keep alive until the run completes
        for i, A in enumerate(mats):
            if tuple(A.shape) != tuple(self.shapes[i]) or _ld(A) != self.lds[i] or A.stride(0) != 1:
                raise ValueError("matrix %d does not match the batch layout" % i)
            ptrs[i] = A.data_ptr()
        check(_lib.tiledqr_batch_run(self.handle, ptrs, _stream()), "tiledqr_batch_run")

    def sync(self):
        check(_lib.tiledqr_batch_sync(self.handle), "tiledqr_batch_sync")

    def time_ms(self):
        ms = ctypes.c_float()
        check(_lib.tiledqr_batch_time(self.handle, ctypes.byref(ms)), "tiledqr_batch_time")
        return ms.value

    def set_trace(self, enable=True):
        check(_lib.tiledqr_batch_set_trace(self.handle, 1 if enable else 0), "tiledqr_batch_set_trace")

    def trace(self):
        """Per subtask of the merged dispatch order: int64 array (n, 11) =
        kind, i, piv, k, j, slab, ticket, ready, end, workgroup (ticks),
        problem; and the tick rate in Hz."""
        import numpy as np
        n = ctypes.c_int64()
        rate = ctypes.c_double()
        check(_lib.tiledqr_batch_get_trace(self.handle, None, ctypes.byref(n), ctypes.byref(rate)),
              "tiledqr_batch_get_trace")
        out = np.zeros((max(1, n.value), 11), dtype=np.int64)
        check(_lib.tiledqr_batch_get_trace(self.handle, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                           ctypes.byref(n), ctypes.byref(rate)), "tiledqr_batch_get_trace")
        return out[:n.value], rate.value

    def factors(self, i):
        """Borrowed Factors of problem i (valid while the batch lives)."""
        h = ctypes.c_void_p()
        check(_lib.tiledqr_batch_get(self.handle, i, ctypes.byref(h)), "tiledqr_batch_get")
        m, n = self.shapes[i]
        return Factors(h, m, n, self.nbs[i], self.opts[i], owner=self)


class ZFactors:
    """Handle of a double-complex tiled QR (tiledqr_zfactor, nb = 32)."""

    def __init__(self, handle, m, n):
        self.handle, self.m, self.n = handle, m, n

    def __del__(self):
        h = getattr(self, "handle", None)
        if h:
            destroy = getattr(_lib, "tiledqr_zdestroy", None)
            if destroy is not None:
                destroy(h)
            self.handle = None

    def sync(self):
        check(_lib.tiledqr_zsync(self.handle), "tiledqr_zsync")

    def refactor(self, A):
        """Factor a new complex128 matrix of the same shape into the handle."""
        A = A if A.stride(0) == 1 else A.t().contiguous().t()
        self._A = A
        check(_lib.tiledqr_zrefactor(self.handle, A.data_ptr(), _ld(A), _stream()), "tiledqr_zrefactor")

    def apply_q(self, B, trans="C"):
        """Return Q^H B (trans 'C') or Q B ('N') for a complex128 CUDA B with
        m rows (tiledqr_zapply_q); B is not modified."""
        B = B if B.dim() == 2 else B[:, None]
        X = B.t().contiguous().t().clone()
        check(_lib.tiledqr_zapply_q(self.handle, trans.encode(), X.data_ptr(), _ld(X), X.shape[1], _stream()),
              "tiledqr_zapply_q")
        return X

    def lstsq(self, B):
        """Least-squares solution X (n x nrhs, complex128 CUDA) of A X ~ B
        (tiledqr_zlstsq)."""
        import torch
        B = B if B.dim() == 2 else B[:, None]
        B = B.t().contiguous().t()
        X = torch.empty((B.shape[1], self.n), dtype=torch.complex128, device="cuda").t()
        check(_lib.tiledqr_zlstsq(self.handle, B.data_ptr(), _ld(B), B.shape[1], X.data_ptr(), _ld(X), _stream()),
              "tiledqr_zlstsq")
        torch.cuda.current_stream().synchronize()
        return X

    def solve_r(self, X):
        """R^{-1} X for a complex128 CUDA X with n rows (tiledqr_zsolve_r)."""
        X = (X if X.dim() == 2 else X[:, None]).t().contiguous().t().clone()
        check(_lib.tiledqr_zsolve_r(self.handle, X.data_ptr(), _ld(X), X.shape[1], _stream()), "tiledqr_zsolve_r")
        return X

    def packed(self):
        """The factored matrix (R and the reflectors) as an m x n complex128
        column-major CUDA tensor."""
        import torch
        out = torch.empty((self.n, self.m), dtype=torch.complex128, device="cuda").t()
        check(_lib.tiledqr_zget_packed(self.handle, out.data_ptr(), self.m, _stream()), "tiledqr_zget_packed")
        return out

    def tau(self):
        """(taug, taup): complex128 CUDA tensors of p q 32 entries."""
        import torch
        k = (self.m // 32) * (self.n // 32) * 32
        tg = torch.empty(k, dtype=torch.complex128, device="cuda")
        tp = torch.empty(k, dtype=torch.complex128, device="cuda")
        check(_lib.tiledqr_zget_tau(self.handle, tg.data_ptr(), tp.data_ptr(), _stream()), "tiledqr_zget_tau")
        return tg, tp


def zfactor(A, nb=32, tree=_lib.TREE_GREEDY, bs=1, kernels=_lib.KERN_DEFAULT):
    """Tiled QR of a complex128 CUDA matrix (tiledqr_zfactor; nb = 32)."""
    import torch
    if A.dtype != torch.complex128:
        raise ValueError("zfactor takes a complex128 matrix")
    A = A if A.stride(0) == 1 else A.t().contiguous().t()
    m, n = A.shape
    opts = _lib.Opts(m, n, nb, 0, tree, bs, kernels, _lib.UPD_F64)
    h = ctypes.c_void_p()
    check(_lib.tiledqr_zfactor(ctypes.byref(opts), A.data_ptr(), _ld(A), ctypes.byref(h), _stream()),
          "tiledqr_zfactor")
    F = ZFactors(h, m, n)
    F._A = A  # the copy into tiles runs on the stream
    return F


# Candidates of the batch autotuner: (tree, BS, kernel family); BS is capped
# at each problem's tile rows.
BATCH_CANDIDATES = [(_lib.TREE_PLASMA, 16, _lib.KERN_TS), (_lib.TREE_PLASMA, 8, _lib.KERN_TS),
                    (_lib.TREE_PLASMA, 4, _lib.KERN_TS), (_lib.TREE_GREEDY, 1, _lib.KERN_TS),
                    (_lib.TREE_GREEDY, 1, _lib.KERN_TT), (_lib.TREE_FLAT, 1, _lib.KERN_TS)]


def batch_nb_rules(shapes):
    """Tile-size choices of the batch autotuner, one nb per problem: the
    largest of 64 and 32 dividing m and n, and 32 throughout."""
    big = [64 if m % 64 == 0 and n % 64 == 0 else 32 for m, n in shapes]
    return {"nb 64 where it divides": big, "nb 32": [32] * len(shapes)}


def tune_batch(mats, candidates=None, upd=_lib.UPD_F64, reps=2):
    """Exhaustive autotuner of a batched launch: times the replayed graph for
    every candidate (tree, BS, kernel family) under every tile-size rule of
    batch_nb_rules (best of reps runs after one warm-up) and returns
    (best, table): best = (ms, rule, tree, bs, kernels, nbs), table = list of
    (ms, rule, tree, bs, kernels).  mats: column-major float64 CUDA tensors."""
    shapes = [tuple(A.shape) for A in mats]
    table, best = [], None
    for rule, nbs in batch_nb_rules(shapes).items():
        for tree, bs, kern in (candidates or BATCH_CANDIDATES):
            if any(m % nb or n % nb for (m, n), nb in zip(shapes, nbs)):
                continue
            B = Batch(shapes, nbs, tree=tree, bs=bs, kernels=kern, upd=upd, lds=[_ld(A) for A in mats])
            ms = []
            for _ in range(reps + 1):
                B.run(mats)
                B.sync()
                ms.append(B.time_ms())
            del B
            t = min(ms[1:])
            table.append((t, rule, tree, bs, kern))
            if best is None or t < best[0]:
                best = (t, rule, tree, bs, kern, nbs)
    return best, table


def factor_batched(mats, nbs, tree=_lib.TREE_GREEDY, bs=1, kernels=_lib.KERN_DEFAULT, upd=_lib.UPD_F64):
    """Factor a list of matrices in one batched launch (tiledqr_factor_batched);
    returns a list of independent Factors."""
    mats = [colmajor(A) for A in mats]
    k = len(mats)
    opts = _batch_opts([tuple(A.shape) for A in mats], nbs, tree, bs, kernels, upd)
    ptrs = (ctypes.c_void_p * k)()
    ldas = (ctypes.c_int64 * k)()
    for i, A in enumerate(mats):
        ptrs[i] = A.data_ptr()
        ldas[i] = _ld(A)
    hs = (ctypes.c_void_p * k)()
    check(_lib.tiledqr_factor_batched(k, opts, ptrs, ldas, hs, _stream()), "tiledqr_factor_batched")
    return [Factors(ctypes.c_void_p(hs[i]), mats[i].shape[0], mats[i].shape[1], nbs[i], opts[i]) for i in range(k)]
