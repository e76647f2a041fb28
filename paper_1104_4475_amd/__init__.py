"""MI355X tiled QR factorization (Bouwmeester, Jacquelin, Langou, Robert,
"Tiled QR factorization algorithms", 2011) on hand-written HIP kernels.

The compute library is libtiledqr.so (C ABI in include/tiledqr.h).  This
package is a thin ctypes binding: the functions named tiledqr_* take the same
arguments as their C counterparts, and the helpers below marshal torch
tensors (device memory and the current HIP stream) into them.  Every step of
the factorization runs in the library's kernels; there is no fallback.
"""

from ._lib import (  # noqa: F401
    TREE_FLAT, TREE_SAMEH_KUCK, TREE_BINARY, TREE_FIBONACCI, TREE_GREEDY, TREE_PLASMA, TREE_ASAP, TREE_GRASAP, TREE_HADRI,
    KERN_DEFAULT, KERN_TT, KERN_TS, UPD_F64, UPD_F32, UPD_BF16,
    TQR_OK, TQR_EINVAL, TQR_ENOMEM, TQR_EHIP, TQR_ENOTCONV, TQR_EUNSUPPORTED, TQR_EEXEC,
    TiledQRError, lib, lib_path, Opts, RefineOpts, RefineInfo,
    tiledqr_factor, tiledqr_refactor, tiledqr_sync, tiledqr_apply_q, tiledqr_get_r,
    tiledqr_get_packed, tiledqr_get_tau, tiledqr_destroy, tiledqr_lstsq, tiledqr_exec_time,
    tiledqr_set_trace, tiledqr_get_trace, tiledqr_exec_plan, tiledqr_solve_r,
    tiledqr_factor_batched, tiledqr_refactor_qtb, tiledqr_lstsq_qtb, tiledqr_batch_create, tiledqr_batch_run, tiledqr_batch_sync, tiledqr_batch_time,
    tiledqr_batch_get, tiledqr_batch_destroy, tiledqr_elim_list, tiledqr_schedule, tiledqr_task_preds,
    tiledqr_strerror, elim_list, schedule, task_preds,
)
from .api import BATCH_CANDIDATES, Batch, Factors, ZFactors, colmajor, factor, factor_batched, tune_batch, zfactor  # noqa: F401
