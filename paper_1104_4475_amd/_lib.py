"""ctypes declarations of libtiledqr.so (names and arguments as in
include/tiledqr.h).  Loading fails loudly if the library has not been built."""

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
lib_path = os.path.join(HERE, "libtiledqr.so")

TREE_FLAT, TREE_SAMEH_KUCK, TREE_BINARY, TREE_FIBONACCI, TREE_GREEDY, TREE_PLASMA, TREE_ASAP, TREE_GRASAP, TREE_HADRI = \
    range(9)
KERN_DEFAULT, KERN_TT, KERN_TS = 0, 1, 2
UPD_F64, UPD_F32, UPD_BF16 = 0, 1, 2
# Fields of an executor predecessor entry (tiledqr_exec_plan): index, stage
# (0 at the start, 1 before the look-ahead, 2 before the rest of the tiles)
# and the early-release bit.
DEP_INDEX, DEP_STAGE_SHIFT, DEP_EARLY = (1 << 28) - 1, 28, 1 << 30
TQR_OK, TQR_EINVAL, TQR_ENOMEM, TQR_EHIP, TQR_ENOTCONV, TQR_EUNSUPPORTED, TQR_EEXEC = 0, -1, -2, -3, -4, -5, -6

if not os.path.exists(lib_path):
    raise ImportError("libtiledqr.so is not built (run python -m paper_1104_4475_amd.build): %s" % lib_path)
# torch ships its own HIP runtime whose soname (libamdhip64.so.7) is the one
# libtiledqr.so asks for.  Loading torch first makes the library bind to that
# copy, so the process holds a single HIP runtime and torch's device memory
# and streams are valid in the library.
try:
    import torch  # noqa: F401
except ImportError:  # plain C-ABI use without torch
    pass
lib = ctypes.CDLL(lib_path)


class Opts(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int64), ("n", ctypes.c_int64), ("nb", ctypes.c_int32), ("ib", ctypes.c_int32),
                ("tree", ctypes.c_int32), ("bs", ctypes.c_int32), ("kernels", ctypes.c_int32),
                ("upd", ctypes.c_int32)]


class RefineOpts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("max_iter", ctypes.c_int32), ("method", ctypes.c_int32)]


class RefineInfo(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("converged", ctypes.c_int32), ("backward_err", ctypes.c_double),
                ("semi_normal", ctypes.c_int32), ("augmented", ctypes.c_int32)]


class TiledQRError(RuntimeError):
    def __init__(self, status, where=""):
        self.status = status
        msg = lib.tiledqr_strerror(status).decode()
        if status in (TQR_EHIP, TQR_ENOMEM):
            msg += " (last hipError %d)" % lib.tiledqr_last_hip_error()
        super().__init__("%s: %s (%d)" % (where, msg, status))


_vp, _i32, _i64, _dp = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p
_P = ctypes.POINTER

_sigs = {
    "tiledqr_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "tiledqr_last_hip_error": (ctypes.c_int, []),
    "tiledqr_factor": (ctypes.c_int, [_P(Opts), _dp, _i64, _P(_vp), _vp]),
    "tiledqr_refactor": (ctypes.c_int, [_vp, _dp, _i64, _vp]),
    "tiledqr_sync": (ctypes.c_int, [_vp]),
    "tiledqr_apply_q": (ctypes.c_int, [_vp, ctypes.c_char, _dp, _i64, _i64, _vp]),
    "tiledqr_get_r": (ctypes.c_int, [_vp, _dp, _i64, _vp]),
    "tiledqr_get_packed": (ctypes.c_int, [_vp, _dp, _i64, _vp]),
    "tiledqr_get_tau": (ctypes.c_int, [_vp, _dp, _vp]),
    "tiledqr_destroy": (ctypes.c_int, [_vp]),
    "tiledqr_exec_plan": (ctypes.c_int, [_vp, _P(_i32), _P(_i64), _P(_i32), _P(_i64)]),
    "tiledqr_solve_r": (ctypes.c_int, [_vp, ctypes.c_char, _dp, _i64, _i64, _vp]),
    "tiledqr_exec_time": (ctypes.c_int, [_vp, _P(ctypes.c_float)]),
    "tiledqr_set_trace": (ctypes.c_int, [_vp, ctypes.c_int]),
    "tiledqr_get_trace": (ctypes.c_int, [_vp, _P(_i64), _P(_i64), _P(ctypes.c_double)]),
    "tiledqr_lstsq": (ctypes.c_int, [_vp, _dp, _i64, _dp, _i64, _i64, _dp, _i64, _P(RefineOpts), _P(RefineInfo),
                                     _vp]),
    "tiledqr_factor_batched": (ctypes.c_int, [_i32, _P(Opts), _P(_vp), _P(_i64), _P(_vp), _vp]),
    "tiledqr_refactor_qtb": (ctypes.c_int, [_vp, _dp, _i64, _dp, _i64, _i64, _vp]),
    "tiledqr_lstsq_qtb": (ctypes.c_int, [_vp, _dp, _i64, _dp, _i64, _dp, _i64, _i64, _dp, _i64, _P(RefineOpts),
                                         _P(RefineInfo), _vp]),
    "tiledqr_zfactor": (ctypes.c_int, [_P(Opts), _vp, _i64, _P(_vp), _vp]),
    "tiledqr_zrefactor": (ctypes.c_int, [_vp, _vp, _i64, _vp]),
    "tiledqr_zapply_q": (ctypes.c_int, [_vp, ctypes.c_char, _vp, _i64, _i64, _vp]),
    "tiledqr_zsolve_r": (ctypes.c_int, [_vp, _vp, _i64, _i64, _vp]),
    "tiledqr_zlstsq": (ctypes.c_int, [_vp, _vp, _i64, _i64, _vp, _i64, _vp]),
    "tiledqr_zget_packed": (ctypes.c_int, [_vp, _vp, _i64, _vp]),
    "tiledqr_zget_tau": (ctypes.c_int, [_vp, _vp, _vp, _vp]),
    "tiledqr_zsync": (ctypes.c_int, [_vp]),
    "tiledqr_zdestroy": (ctypes.c_int, [_vp]),
    "tiledqr_batch_create": (ctypes.c_int, [_i32, _P(Opts), _P(_i64), _P(_vp)]),
    "tiledqr_batch_run": (ctypes.c_int, [_vp, _P(_vp), _vp]),
    "tiledqr_batch_sync": (ctypes.c_int, [_vp]),
    "tiledqr_batch_time": (ctypes.c_int, [_vp, _P(ctypes.c_float)]),
    "tiledqr_batch_set_trace": (ctypes.c_int, [_vp, ctypes.c_int]),
    "tiledqr_batch_get_trace": (ctypes.c_int, [_vp, _P(_i64), _P(_i64), _P(ctypes.c_double)]),
    "tiledqr_batch_get": (ctypes.c_int, [_vp, _i32, _P(_vp)]),
    "tiledqr_batch_destroy": (ctypes.c_int, [_vp]),
    "tiledqr_mlp_nparam": (ctypes.c_int, []),
    "tiledqr_mlp_forward": (ctypes.c_int, [_vp, _vp, _i64, _vp, _vp]),
    "tiledqr_mlp_loss_grad": (ctypes.c_int, [_vp, _vp, _vp, _i64, _vp, _vp, _vp]),
    "tiledqr_mlp_loss_grad_noalloc": (ctypes.c_int, [_vp, _vp, _vp, _i64, _vp, _vp, _vp]),
    "tiledqr_mlp_noalloc_max_samples": (ctypes.c_int, []),
    "tiledqr_mlp_adam": (ctypes.c_int, [_vp, _vp, _vp, _vp, _i64, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                        ctypes.c_float, _i32, _vp]),
    "tiledqr_elim_list": (ctypes.c_int, [_i32, _i32, _i32, _i32, _P(_i32), _P(_i64)]),
    "tiledqr_schedule": (ctypes.c_int, [_i32, _i32, _i32, _i32, _i32, _P(_i32), _P(_i64), _P(_i64)]),
    "tiledqr_task_preds": (ctypes.c_int, [_i32, _i32, _i32, _i32, _i32, _P(_i64), _P(_i32)]),
}
for _name, (_res, _args) in _sigs.items():
    _f = getattr(lib, _name)
    _f.restype = _res
    _f.argtypes = _args
    globals()[_name] = _f


def check(status, where):
    if status != TQR_OK:
        raise TiledQRError(status, where)


def elim_list(p, q, tree, bs=1):
    """Elimination list as an int32 array of shape (nelim, 3), 1-based."""
    n = ctypes.c_int64()
    check(tiledqr_elim_list(p, q, tree, bs, None, ctypes.byref(n)), "tiledqr_elim_list")
    out = np.zeros((max(n.value, 1), 3), dtype=np.int32)
    check(tiledqr_elim_list(p, q, tree, bs, out.ctypes.data_as(_P(_i32)), ctypes.byref(n)), "tiledqr_elim_list")
    return out[:n.value]


def schedule(p, q, tree, bs=1, kernels=KERN_DEFAULT):
    """(tasks int32 (n, 7) = kind, i, piv, k, j, start, finish; critical path)."""
    n, cp = ctypes.c_int64(), ctypes.c_int64()
    check(tiledqr_schedule(p, q, tree, bs, kernels, None, ctypes.byref(n), ctypes.byref(cp)), "tiledqr_schedule")
    out = np.zeros((max(n.value, 1), 7), dtype=np.int32)
    check(tiledqr_schedule(p, q, tree, bs, kernels, out.ctypes.data_as(_P(_i32)), ctypes.byref(n),
                           ctypes.byref(cp)), "tiledqr_schedule")
    return out[:n.value], cp.value


def task_preds(p, q, tree, bs=1, kernels=KERN_DEFAULT):
    """CSR predecessors (ptr int64 (n+1), idx int32)."""
    tasks, _ = schedule(p, q, tree, bs, kernels)
    ptr = np.zeros(len(tasks) + 1, dtype=np.int64)
    check(tiledqr_task_preds(p, q, tree, bs, kernels, ptr.ctypes.data_as(_P(_i64)), None), "tiledqr_task_preds")
    idx = np.zeros(max(int(ptr[-1]), 1), dtype=np.int32)
    check(tiledqr_task_preds(p, q, tree, bs, kernels, ptr.ctypes.data_as(_P(_i64)), idx.ctypes.data_as(_P(_i32))),
          "tiledqr_task_preds")
    return ptr, idx[:int(ptr[-1])]
