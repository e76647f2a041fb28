"""The C-ABI library loads, exports every function declared in
include/tiledqr.h, and rejects bad arguments on the host before any launch
(no GPU needed)."""

import ctypes
import os
import re

import paper_1104_4475_amd as tqr
from paper_1104_4475_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", fn)).read()
            names |= set(re.findall(r"^\s*(?:const\s+)?\w+\**\s+\**(tiledqr_\w+)\s*\(", txt, re.M))
    return names


def test_every_declared_symbol_is_exported():
    names = _declared()
    assert {"tiledqr_factor", "tiledqr_apply_q", "tiledqr_lstsq"} <= names
    for n in names:
        assert hasattr(_lib.lib, n), n


def test_strerror():
    assert _lib.tiledqr_strerror(0) == b"success"
    assert b"invalid" in _lib.tiledqr_strerror(-1)


def test_factor_rejects_bad_options_before_any_launch():
    h = ctypes.c_void_p()
    fake = ctypes.c_void_p(0x1000)  # never dereferenced: validation fails first
    bad = [
        dict(m=256, n=128, nb=48),          # nb not supported
        dict(m=250, n=128, nb=32),          # m % nb
        dict(m=128, n=256, nb=32),          # m < n
        dict(m=256, n=128, nb=32, ib=16),   # ib
        dict(m=256, n=128, nb=32, tree=9),  # tree
        dict(m=256, n=128, nb=32, tree=5, bs=0),
        dict(m=256, n=128, nb=32, upd=7),
    ]
    for kw in bad:
        o = _lib.Opts(kw["m"], kw["n"], kw["nb"], kw.get("ib", 0), kw.get("tree", 4), kw.get("bs", 1), 0,
                      kw.get("upd", 0))
        assert _lib.tiledqr_factor(ctypes.byref(o), fake, kw["m"], ctypes.byref(h), None) == tqr.TQR_EINVAL
    o = _lib.Opts(256, 128, 32, 0, 4, 1, 0, 0)
    assert _lib.tiledqr_factor(ctypes.byref(o), fake, 100, ctypes.byref(h), None) == tqr.TQR_EINVAL  # lda
    assert _lib.tiledqr_factor(ctypes.byref(o), None, 256, ctypes.byref(h), None) == tqr.TQR_EINVAL
    assert _lib.tiledqr_factor(None, fake, 256, ctypes.byref(h), None) == tqr.TQR_EINVAL
    # nb = 512 is a valid tile size without kernels here
    o = _lib.Opts(1024, 512, 512, 0, 4, 1, 0, 0)
    assert _lib.tiledqr_factor(ctypes.byref(o), fake, 1024, ctypes.byref(h), None) == tqr.TQR_EUNSUPPORTED


def test_other_entry_points_reject_null_handles():
    assert _lib.tiledqr_apply_q(None, b"T", None, 1, 1, None) == tqr.TQR_EINVAL
    assert _lib.tiledqr_lstsq(None, None, 1, None, 1, 1, None, 1, None, None, None) == tqr.TQR_EINVAL
    assert _lib.tiledqr_get_r(None, None, 1, None) == tqr.TQR_EINVAL
    assert _lib.tiledqr_destroy(None) == tqr.TQR_OK
    n = ctypes.c_int64()
    assert _lib.tiledqr_exec_plan(None, None, ctypes.byref(n), None, ctypes.byref(n)) == tqr.TQR_EINVAL
    assert _lib.tiledqr_solve_r(None, b"N", None, 1, 1, None) == tqr.TQR_EINVAL


def test_batch_create_rejects_bad_options_before_allocating():
    b = ctypes.c_void_p()
    ok = _lib.Opts(256, 64, 32, 0, 4, 1, 0, 0)
    big = _lib.Opts(512, 256, 128, 0, 4, 1, 0, 0)   # nb 128: not a batched tile size
    f32 = _lib.Opts(256, 64, 32, 0, 4, 1, 0, 1)     # upd differs from problem 0
    bad = _lib.Opts(250, 64, 32, 0, 4, 1, 0, 0)     # m % nb
    two = lambda a, c: (_lib.Opts * 2)(a, c)  # noqa: E731
    ld2 = (ctypes.c_int64 * 2)(512, 512)
    assert _lib.tiledqr_batch_create(0, two(ok, ok), ld2, ctypes.byref(b)) == tqr.TQR_EINVAL
    assert _lib.tiledqr_batch_create(2, two(ok, big), ld2, ctypes.byref(b)) == tqr.TQR_EUNSUPPORTED
    assert _lib.tiledqr_batch_create(2, two(ok, f32), ld2, ctypes.byref(b)) == tqr.TQR_EINVAL
    assert _lib.tiledqr_batch_create(2, two(ok, bad), ld2, ctypes.byref(b)) == tqr.TQR_EINVAL
    assert _lib.tiledqr_batch_create(2, two(ok, ok), (ctypes.c_int64 * 2)(512, 100), ctypes.byref(b)) == tqr.TQR_EINVAL
    assert _lib.tiledqr_batch_run(None, None, None) == tqr.TQR_EINVAL
    assert _lib.tiledqr_batch_destroy(None) == tqr.TQR_OK
