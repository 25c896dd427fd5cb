"""ctypes loader for libtsqr.so (the C ABI declared in include/tsqr.h).

torch is imported first so that the library binds to the HIP runtime torch already loaded (both
carry the soname libamdhip64.so.7), which lets torch streams and allocations be passed straight
through.  There is no fallback: if the library is missing, loading raises.
"""
from __future__ import annotations

import ctypes
import os

import torch  # noqa: F401  (must precede the CDLL load, see module docstring)

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtsqr.so")

TSQR_OK = 0
STATUS_NAMES = {0: "TSQR_OK", 1: "TSQR_ERR_INVALID_ARG", 2: "TSQR_ERR_SHAPE",
                3: "TSQR_ERR_WORKSPACE", 4: "TSQR_ERR_UNSUPPORTED", 5: "TSQR_ERR_HIP"}
PRECISION = {"fp64": 0, "fp32_refined": 1, "fp32": 2}
OPS = {"r": 0, "qr": 1, "svd": 2, "qr_backward": 3, "svd_backward": 4}

# Exported symbols and their signatures (kept in step with include/tsqr.h).
_i64, _i32, _vp, _sz = ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p, ctypes.c_size_t
SIGNATURES = {
    "tsqr_default_opts": (None, [_vp]),
    "tsqr_workspace_bytes": (_i32, [_i32, _i64, _i64, _vp, ctypes.POINTER(_sz)]),
    "tsqr_r": (_i32, [_i64, _i64, _vp, _i64, _vp, _i64, _vp, _sz, _vp, _vp, _vp]),
    "tsqr_r_f32": (_i32, [_i64, _i64, _vp, _i64, _vp, _i64, _vp, _sz, _vp, _vp, _vp]),
    "tsqr_r_noalloc": (_i32, [_i64, _i64, _vp, _i64, _vp, _i64, _vp, _vp, _vp]),
    "tsqr_qr": (_i32, [_i64, _i64, _vp, _i64, _vp, _i64, _vp, _i64, _vp, _sz, _vp, _vp, _vp]),
    "tsqr_qr_f32": (_i32, [_i64, _i64, _vp, _i64, _vp, _i64, _vp, _i64, _vp, _sz, _vp, _vp,
                           _vp]),
    "tsqr_qr_chunked_workspace_bytes": (_i32, [_i64, _i64, _i64, _vp, ctypes.POINTER(_sz)]),
    "tsqr_qr_chunked": (_i32, [_i64, _i64, _i64, _vp, _i64, _vp, _i64, _vp, _i64, _vp, _sz, _vp,
                               _vp, _vp]),
    "tsqr_svd": (_i32, [_i64, _i64, _vp, _i64, _vp, _i64, _vp, _vp, _i64, _vp, _i64, _vp, _i64,
                        _vp, _sz, _vp, _vp, _vp]),
    "tsqr_svd_f32": (_i32, [_i64, _i64, _vp, _i64, _vp, _i64, _vp, _vp, _i64, _vp, _i64, _vp,
                            _i64, _vp, _sz, _vp, _vp, _vp]),
    "tsqr_qr_backward": (_i32, [_i64, _i64, _vp, _i64, _vp, _i64, _vp, _i64, _vp, _i64, _vp, _sz,
                                 _vp, _vp, _vp]),
    "tsqr_svd_backward": (_i32, [_i64, _i64, _vp, _i64, _vp, _i64, _vp, _vp, _i64, _vp, _i64, _vp,
                                  _sz, _vp, _vp, _vp]),
    "tsqr_batch_plan_create": (_i32, [_i32, _vp, _vp, _vp, _vp, _vp, _i32, _vp, _vp]),
    "tsqr_batch_plan_destroy": (_i32, [_vp]),
    "tsqr_batch_workspace_bytes": (_i32, [_vp, ctypes.POINTER(_sz)]),
    "tsqr_batch_plan_launches": (_i32, [_vp, ctypes.POINTER(_i32)]),
    "tsqr_qr_batched": (_i32, [_vp, _vp, _vp, _vp, _vp, _sz, _vp, _vp]),
    "tsqr_tune_set": (_i32, [_i32, _i64, _i32]),
    "tsqr_tune_get": (_i32, [_i32, _i64, ctypes.POINTER(_i32), ctypes.POINTER(_i32)]),
    "tsqr_tune_variants": (_i32, [_i32, _i64, _i32, ctypes.POINTER(_i32), ctypes.POINTER(_i32)]),
    "tsqr_plan_levels": (_i32, [_i32, _i64, _i64, _vp, _i32, ctypes.POINTER(_i32),
                                 ctypes.POINTER(_i64), ctypes.POINTER(_i32)]),
    "tsqr_profile_enable": (_i32, [_i32]),
    "tsqr_profile_set_mask": (_i32, [ctypes.c_uint32]),
    "tsqr_profile_collect": (_i32, [ctypes.POINTER(ctypes.c_double), ctypes.POINTER(_i64), _i32]),
    "tsqr_profile_num_classes": (_i32, []),
    "tsqr_profile_class_name": (ctypes.c_char_p, [_i32]),
    "tsqr_indirect_workspace_bytes": (_i32, [_i32, _i32, _i64, _i64, _vp, ctypes.POINTER(_sz)]),
    "tsqr_qr_indirect": (_i32, [_i32, _i32, _i64, _i64, _vp, _i64, _vp, _i64, _vp, _i64, _vp, _sz,
                                _vp, _vp, _vp]),
    "tsqr_metric_workspace_bytes": (_i32, [_i64, _i64, ctypes.POINTER(_sz)]),
    "tsqr_metric_gram": (_i32, [_i32, _i64, _i64, _vp, _i64, _vp, _i64, _vp, _i64, _vp, _vp, _sz,
                                _vp]),
    "tsqr_status_string": (ctypes.c_char_p, [_i32]),
    "tsqr_abi_version": (_i32, []),
    "tsqr_last_error": (ctypes.c_char_p, []),
}


class Opts(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("panel_rows", ctypes.c_int32), ("flags", ctypes.c_int32)]


FLAG_REUSE_OUTPUT = 1


def make_opts(precision: str = "fp64", panel_rows: int = 0, reuse_output: bool = False) -> Opts:
    o = Opts()
    o.struct_size = ctypes.sizeof(Opts)
    o.precision = PRECISION[precision]
    o.panel_rows = int(panel_rows)
    o.flags = FLAG_REUSE_OUTPUT if reuse_output else 0
    return o


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libtsqr.so is not built (%s); run __graft_entry__.build()" % LIB_PATH)
        h = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(h, name)
            f.restype = res
            f.argtypes = args
        _lib = h
    return _lib


class TSQRError(RuntimeError):
    def __init__(self, status: int, where: str):
        super().__init__("%s: %s" % (where, STATUS_NAMES.get(status, "status %d" % status)))
        self.status = status


def check(status: int, where: str) -> None:
    if status != TSQR_OK:
        if status == 5:
            where = "%s [%s]" % (where, lib().tsqr_last_error().decode())
        raise TSQRError(status, where)


def profile_enable(on: bool) -> None:
    check(lib().tsqr_profile_enable(1 if on else 0), "tsqr_profile_enable")


def profile_set_mask(classes=None) -> None:
    """Record only the named kernel classes (None: all)."""
    if classes is None:
        mask = 0xFFFFFFFF
    else:
        n = lib().tsqr_profile_num_classes()
        names = [lib().tsqr_profile_class_name(i).decode() for i in range(n)]
        mask = 0
        for c in classes:
            mask |= 1 << names.index(c)
    check(lib().tsqr_profile_set_mask(mask), "tsqr_profile_set_mask")


def profile_collect() -> dict:
    """{kernel class: (total ms, launches)} since the last collect (waits for the events)."""
    n = lib().tsqr_profile_num_classes()
    ms = (ctypes.c_double * n)()
    cnt = (ctypes.c_int64 * n)()
    check(lib().tsqr_profile_collect(ms, cnt, n), "tsqr_profile_collect")
    return {lib().tsqr_profile_class_name(i).decode(): (ms[i], cnt[i]) for i in range(n)}


def plan_levels(op: str, m: int, n: int, precision: str = "fp64", panel_rows: int = 0):
    """[(rows, panel height)] of every level of the recursive tree the library runs."""
    o = make_opts(precision, panel_rows)
    cap = 64
    nl = ctypes.c_int32(0)
    rows = (ctypes.c_int64 * cap)()
    prs = (ctypes.c_int32 * cap)()
    check(lib().tsqr_plan_levels(OPS[op], m, n, ctypes.byref(o), cap, ctypes.byref(nl), rows, prs),
          "tsqr_plan_levels")
    return [(rows[i], prs[i]) for i in range(min(nl.value, cap))]
