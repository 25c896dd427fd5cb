"""CPU checks of the C ABI: the library loads, exports every function include/tsqr.h declares, and
rejects bad arguments synchronously, before anything reaches the GPU."""
import ctypes
import os
import re

import pytest

from paper_1301_1071_amd import _lib
from paper_1301_1071_amd._lib import lib, make_opts

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tsqr.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^[A-Za-z_][\w\s\*]*?\b(tsqr_\w+)\s*\(", src, flags=re.M)
    return sorted(set(names))


def test_header_symbols_exported():
    names = declared_functions()
    assert "tsqr_qr" in names and "tsqr_svd" in names and "tsqr_r" in names
    h = lib()
    for nm in names:
        assert hasattr(h, nm), nm
    # and the binding's signature table covers exactly the declared functions
    assert set(_lib.SIGNATURES) == set(names)


def test_abi_version_and_strings():
    assert lib().tsqr_abi_version() == 1
    for code, name in _lib.STATUS_NAMES.items():
        assert lib().tsqr_status_string(code).decode() == name


def _ws(op, m, n, opts=None):
    out = ctypes.c_size_t(0)
    st = lib().tsqr_workspace_bytes(_lib.OPS[op], m, n, ctypes.byref(opts) if opts else None,
                                    ctypes.byref(out))
    return st, out.value


def test_workspace_query():
    st, b1 = _ws("qr", 100_000, 10)
    assert st == 0 and b1 >= 100_000 * 10 * 8
    st, b2 = _ws("qr", 200_000, 10)
    assert st == 0 and b2 > b1
    st, br = _ws("r", 100_000, 10)
    assert st == 0 and br < b1          # R only keeps no Q1 panels
    st, bs = _ws("svd", 100_000, 10)
    assert st == 0 and bs > b1          # Q and U carried down the tree
    assert _ws("qr", 5, 10)[0] == 2     # m < n
    assert _ws("qr", 1000, 513)[0] == 2  # n > TSQR_NMAX
    assert _ws("qr", 1000, 512)[0] == 0  # the wide path
    assert _ws("qr", 0, 10)[0] == 1
    assert _ws("qr", 1000, 0)[0] == 1
    assert lib().tsqr_workspace_bytes(9, 10, 1, None, ctypes.byref(ctypes.c_size_t())) == 1
    # the adjoints hold the forward's workspace plus the recomputed Q (or U) and n x n partials
    st, bq = _ws("qr_backward", 100_000, 10)
    assert st == 0 and bq >= b1 + 100_000 * 10 * 8
    st, bsv = _ws("svd_backward", 100_000, 10)
    assert st == 0 and bsv >= 100_000 * 10 * 8
    assert _ws("qr_backward", 1000, 129)[0] == 2          # n > TSQR_NMAX_SMALL
    assert _ws("svd_backward", 5, 10)[0] == 2
    assert _ws("qr_backward", 1000, 10, make_opts("fp32"))[0] == 4      # FP64 only


def test_opts_validation():
    o = make_opts("fp64")
    assert _ws("qr", 1000, 10, o)[0] == 0
    o.struct_size = 4
    assert _ws("qr", 1000, 10, o)[0] == 1
    o = make_opts("fp64"); o.precision = 7
    assert _ws("qr", 1000, 10, o)[0] == 1
    o = make_opts("fp64"); o.flags = 4            # not a defined flag
    assert _ws("qr", 1000, 10, o)[0] == 1
    o = make_opts("fp64", panel_rows=5)          # shorter than n
    assert _ws("qr", 1000, 10, o)[0] == 1
    o = make_opts("fp64", panel_rows=512)
    assert _ws("qr", 100_000, 10, o)[0] == 0
    o = make_opts("fp32_refined")
    assert _ws("qr", 100_000, 100, o)[0] == 4    # refinement implemented for n <= 64


FAKE = ctypes.c_void_p(0x1000)   # never dereferenced: every call below fails validation first


def _gpu_visible():
    import torch
    return torch.cuda.is_available()


@pytest.mark.skipif(_gpu_visible(), reason="fake device pointers are only passed where no GPU exists")
def test_entry_points_reject_bad_arguments_without_gpu():
    L = lib()
    info = FAKE
    # NULL input
    assert L.tsqr_qr(100, 10, None, 10, FAKE, 10, FAKE, 10, FAKE, 1 << 30, info, None, None) == 1
    # ld < n
    assert L.tsqr_qr(100, 10, FAKE, 9, FAKE, 10, FAKE, 10, FAKE, 1 << 30, info, None, None) == 1
    assert L.tsqr_r(100, 10, FAKE, 10, FAKE, 9, FAKE, 1 << 30, info, None, None) == 1
    # shapes
    assert L.tsqr_qr(5, 10, FAKE, 10, FAKE, 10, FAKE, 10, FAKE, 1 << 30, info, None, None) == 2
    assert L.tsqr_r(1000, 600, FAKE, 600, FAKE, 600, FAKE, 1 << 30, info, None, None) == 2
    # workspace missing or too small
    assert L.tsqr_qr(100, 10, FAKE, 10, FAKE, 10, FAKE, 10, None, 1 << 30, info, None, None) == 3
    assert L.tsqr_qr(100, 10, FAKE, 10, FAKE, 10, FAKE, 10, FAKE, 16, info, None, None) == 3
    # missing info
    assert L.tsqr_r(100, 10, FAKE, 10, FAKE, 10, FAKE, 1 << 30, None, None, None) == 1
    # svd: missing outputs, bad ld
    assert L.tsqr_svd(100, 10, FAKE, 10, None, 10, FAKE, FAKE, 10, None, 0, None, 0, FAKE,
                      1 << 30, info, None, None) == 1
    assert L.tsqr_svd(100, 10, FAKE, 10, FAKE, 10, FAKE, FAKE, 9, None, 0, None, 0, FAKE,
                      1 << 30, info, None, None) == 1
    # f32 twins
    assert L.tsqr_qr_f32(100, 10, FAKE, 10, FAKE, 10, FAKE, 10, FAKE, 16, info, None, None) == 3
    assert L.tsqr_r_f32(5, 10, FAKE, 10, FAKE, 10, FAKE, 1 << 30, info, None, None) == 2
    # adjoints: NULL input / output, bad ld, shape, workspace, precision
    assert L.tsqr_qr_backward(100, 10, None, 10, FAKE, 10, FAKE, 10, FAKE, 10, FAKE, 1 << 30,
                              info, None, None) == 1
    assert L.tsqr_qr_backward(100, 10, FAKE, 10, FAKE, 9, FAKE, 10, FAKE, 10, FAKE, 1 << 30,
                              info, None, None) == 1
    assert L.tsqr_qr_backward(5, 10, FAKE, 10, FAKE, 10, FAKE, 10, FAKE, 10, FAKE, 1 << 30,
                              info, None, None) == 2
    assert L.tsqr_qr_backward(100, 10, FAKE, 10, FAKE, 10, FAKE, 10, FAKE, 10, FAKE, 16,
                              info, None, None) == 3
    o32 = make_opts("fp32")
    assert L.tsqr_qr_backward(100, 10, FAKE, 10, FAKE, 10, FAKE, 10, FAKE, 10, FAKE, 1 << 30,
                              info, ctypes.byref(o32), None) == 4
    assert L.tsqr_svd_backward(100, 10, FAKE, 10, FAKE, 10, FAKE, FAKE, 10, None, 10, FAKE,
                               1 << 30, info, None, None) == 1
    assert L.tsqr_svd_backward(100, 10, FAKE, 10, FAKE, 10, FAKE, FAKE, 9, FAKE, 10, FAKE,
                               1 << 30, info, None, None) == 1
    assert L.tsqr_svd_backward(100, 10, FAKE, 10, FAKE, 10, FAKE, FAKE, 10, FAKE, 10, FAKE,
                               16, info, None, None) == 3


def test_plan_terminates_for_every_width():
    """The recursive tree (Sec. III-C) must shrink to one panel for every supported n."""
    for n in range(1, 129):
        for m in (n, n + 1, 2 * n + 1, 7 * n + 3, 1000, 4097, 100_000, 1_000_003):
            if m < n:
                continue
            for op in ("r", "qr", "svd"):
                st, nbytes = _ws(op, m, n)
                assert st == 0, (op, m, n, st)
                assert nbytes > 0


def test_plan_levels_shape():
    from paper_1301_1071_amd._lib import plan_levels
    lv = plan_levels("qr", 4_000_000, 50)
    assert lv[0][0] == 4_000_000
    for (rows, b), (rows_next, _) in zip(lv, lv[1:]):
        panels = -(-rows // b)
        assert rows_next == panels * 50          # the stacked R of the level below
        assert rows_next < rows
    assert lv[-1][1] == lv[-1][0]                # the top is one panel


def test_batched_plan_validation_without_gpu():
    """Shape and option errors of tsqr_batch_plan_create return before any device call."""
    L = lib()
    b = 3
    arr = lambda xs: (ctypes.c_int64 * b)(*xs)
    h = ctypes.c_void_p()
    ms, ns = arr([100, 200, 300]), arr([4, 8, 16])
    good = arr([64, 64, 64])
    assert L.tsqr_batch_plan_create(0, ms, ns, good, good, good, 0, None, ctypes.byref(h)) == 1
    assert L.tsqr_batch_plan_create(b, ms, ns, good, good, good, 5, None, ctypes.byref(h)) == 1
    wide = arr([70, 70, 70])
    assert L.tsqr_batch_plan_create(b, ms, arr([4, 8, 65]), wide, wide, wide, 0, None,
                                    ctypes.byref(h)) == 2                        # n > 64
    assert L.tsqr_batch_plan_create(b, arr([100, 5, 300]), ns, good, good, good, 0, None,
                                    ctypes.byref(h)) == 2                        # m < n
    assert L.tsqr_batch_plan_create(b, ms, ns, arr([4, 7, 16]), good, good, 0, None,
                                    ctypes.byref(h)) == 1                        # lda < n
    o = make_opts("fp32")
    assert L.tsqr_batch_plan_create(b, ms, ns, good, good, good, 0, ctypes.byref(o),
                                    ctypes.byref(h)) == 4                        # precision != dtype
    assert L.tsqr_qr_batched(None, FAKE, FAKE, FAKE, FAKE, 1 << 20, FAKE, None) == 1
    assert L.tsqr_batch_plan_destroy(None) == 1


def test_tune_table_queries():
    L = lib()
    buf = (ctypes.c_int32 * 4)()
    c = ctypes.c_int32()
    assert L.tsqr_tune_variants(0, 4, 4, buf, ctypes.byref(c)) == 0 and c.value == 3
    assert buf[0] > buf[1] > 0
    assert L.tsqr_tune_variants(0, 64, 4, buf, ctypes.byref(c)) == 0
    assert buf[0] >= 3 * 64 and buf[1] == 0 and buf[2] == 0    # half height too short at n = 64
    assert L.tsqr_tune_set(0, 64, 1) == 1                        # unusable variant rejected
    assert L.tsqr_tune_set(0, 65, 0) == 1
    v, rows = ctypes.c_int32(), ctypes.c_int32()
    assert L.tsqr_tune_get(1, 16, ctypes.byref(v), ctypes.byref(rows)) == 0
    assert rows.value > 0


@pytest.mark.skipif(_gpu_visible(), reason="fake device pointers are only passed where no GPU exists")
def test_new_entry_points_reject_bad_arguments_without_gpu():
    """tsqr_svd_f32, the refined precision on FP32 entry points, and the metric Gram."""
    L = lib()
    info = FAKE
    assert L.tsqr_svd_f32(100, 10, None, 10, FAKE, 10, FAKE, FAKE, 10, None, 0, None, 0, FAKE,
                          1 << 30, info, None, None) == 1
    assert L.tsqr_svd_f32(5, 10, FAKE, 10, FAKE, 10, FAKE, FAKE, 10, None, 0, None, 0, FAKE,
                          1 << 30, info, None, None) == 2
    assert L.tsqr_svd_f32(100, 10, FAKE, 10, FAKE, 10, FAKE, FAKE, 10, None, 0, None, 0, FAKE,
                          16, info, None, None) == 3
    # the refinement needs FP64 input: FP32 entry points reject it (the FP64 workspace query of
    # the refined form would not cover the FP32 path)
    ref = make_opts("fp32_refined")
    for fn in (L.tsqr_qr_f32,):
        assert fn(100, 10, FAKE, 10, FAKE, 10, FAKE, 10, FAKE, 1 << 30, info, ctypes.byref(ref),
                  None) == 4
    assert L.tsqr_r_f32(100, 10, FAKE, 10, FAKE, 10, FAKE, 1 << 30, info, ctypes.byref(ref),
                        None) == 4
    assert L.tsqr_svd_f32(100, 10, FAKE, 10, FAKE, 10, FAKE, FAKE, 10, None, 0, None, 0, FAKE,
                          1 << 30, info, ctypes.byref(ref), None) == 4
    # FP32 entry points accept the FP32 and FP64 precision codes alike
    o32 = make_opts("fp32")
    assert L.tsqr_qr_f32(100, 10, FAKE, 10, FAKE, 10, FAKE, 10, FAKE, 16, info,
                         ctypes.byref(o32), None) == 3
    # metric Gram: bad mode, missing inputs, shape, workspace
    G = FAKE
    assert L.tsqr_metric_gram(3, 100, 10, FAKE, 10, None, 0, None, 0, G, FAKE, 1 << 30, None) == 1
    assert L.tsqr_metric_gram(1, 100, 10, FAKE, 10, None, 0, FAKE, 10, G, FAKE, 1 << 30, None) == 1
    assert L.tsqr_metric_gram(0, 100, 200, FAKE, 200, None, 0, None, 0, G, FAKE, 1 << 30, None) == 2
    assert L.tsqr_metric_gram(0, 100, 10, FAKE, 10, None, 0, None, 0, G, FAKE, 8, None) == 3


def test_fp32_wide_panels_are_blocked():
    """FP32 panels wider than 64 columns run the blocked kernel with many panels (no single
    m-row panel), and the recursion shrinks every level."""
    from paper_1301_1071_amd._lib import plan_levels
    lv = plan_levels("qr", 16_000_000, 100, "fp32")
    assert len(lv) > 1
    assert lv[0] == (16_000_000, 256)
    for (rows, b), (rows_next, _) in zip(lv, lv[1:]):
        assert rows_next == -(-rows // b) * 100 and rows_next < rows


def test_svd_workspace_covers_both_outputs_and_refined_forms():
    st, b = _ws("svd", 200_000, 25)
    assert st == 0
    st, bref = _ws("svd", 200_000, 25, make_opts("fp32_refined"))
    assert st == 0 and bref >= 200_000 * 25 * 8         # holds Q when the caller gives none
    st, bq = _ws("qr", 200_000, 25, make_opts("fp32_refined"))
    assert st == 0 and bq < 200_000 * 25 * 8            # no m x n intermediate is stored
    st, b32 = _ws("qr", 200_000, 25, make_opts("fp32"))
    assert st == 0 and b32 < _ws("qr", 200_000, 25)[1]  # FP32 level-0 panels
    nb = ctypes.c_size_t()
    assert lib().tsqr_metric_workspace_bytes(1000, 10, ctypes.byref(nb)) == 0 and nb.value > 0
    assert lib().tsqr_metric_workspace_bytes(1000, 129, ctypes.byref(nb)) == 2


@pytest.mark.parametrize("n", [129, 256, 512])
def test_wide_plan_quarters_each_level(n):
    """Widths above 128 factor panels of 4 n rows at every level (Sec. III-C recursion), so each
    level's stacked R holds a quarter of the rows below it; the top is one panel; every level
    of the tree is a whole number of n-row blocks."""
    from paper_1301_1071_amd._lib import plan_levels
    m = 200 * n
    lv = plan_levels("qr", m, n)
    assert lv[0] == (m, 4 * n)
    for (rows, b), (rows_next, _) in zip(lv, lv[1:]):
        assert b == min(4 * n, rows)
        assert rows_next == -(-rows // b) * n and rows_next < rows
    assert lv[-1][1] == lv[-1][0]
    for op in ("r", "qr", "svd"):
        st, nbytes = _ws(op, m, n)
        assert st == 0 and nbytes > 0
    assert _ws("qr", m, n, make_opts("fp32_refined"))[0] == 4
    assert _ws("svd_backward", m, n)[0] == 2


def test_reuse_output_workspace_and_limits():
    """TSQR_FLAG_REUSE_OUTPUT drops the m x n level-0 factor buffer from the workspace where one
    work-group can cover all output columns; elsewhere the query returns TSQR_ERR_UNSUPPORTED."""
    def ws(op, m, n, prec="fp64", reuse=True):
        o = make_opts(prec, 0, reuse)
        out = ctypes.c_size_t(0)
        st = lib().tsqr_workspace_bytes(_lib.OPS[op], m, n, ctypes.byref(o), ctypes.byref(out))
        return st, out.value
    for m, n in [(600_000_000, 25), (4_000_000, 50), (100_000, 10), (20_000, 100)]:
        st0, b0 = ws("qr", m, n, reuse=False)
        st1, b1 = ws("qr", m, n)
        assert st0 == 0 and st1 == 0 and b0 - b1 >= 8 * m * n
    # A, Q and the workspace of the paper's 600M x 25 QR within 288 GB of HBM
    assert 2 * 8 * 600_000_000 * 25 + ws("qr", 600_000_000, 25)[1] < 288e9 - 4e9
    assert ws("qr", 20_000, 128)[0] == 4          # W image of 128 columns past one LDS
    assert ws("qr", 20_000, 256)[0] == 4          # the wide path runs in column chunks
    assert ws("qr", 20_000, 25, "fp32")[0] == 0   # FP32 input
    st, b = ws("svd", 20_000, 100)                # only U: the layout without Q
    assert st == 0 and b < ws("svd", 20_000, 100, reuse=False)[1]
    assert ws("r", 20_000, 256)[0] == 0           # ignored without Q
    assert ws("qr", 20_000, 25, "fp32_refined")[0] == 0
    o = make_opts("fp64")
    o.flags = 2
    assert lib().tsqr_workspace_bytes(1, 1000, 10, ctypes.byref(o), ctypes.byref(ctypes.c_size_t())) == 1


def test_chunked_workspace_and_limits():
    def ws(m, n, h, prec="fp64"):
        o = make_opts(prec)
        out = ctypes.c_size_t(0)
        st = lib().tsqr_qr_chunked_workspace_bytes(m, n, h, ctypes.byref(o), ctypes.byref(out))
        return st, out.value
    st, b = ws(150_000_000, 100, 15_000_000)
    assert st == 0
    # A, Q and the workspace of the paper's 150M x 100 QR within 288 GB of HBM
    assert 2 * 8 * 150_000_000 * 100 + b < 288e9 - 10e9
    st1, b1 = ws(1_000_000, 50, 100_000)
    st2, b2 = ws(1_000_000, 50, 500_000)
    assert st1 == 0 and st2 == 0 and b1 < b2                # about one chunk's workspace
    assert ws(1000, 0, 100)[0] == 1
    assert ws(1000, 10, 0)[0] == 1
    assert ws(5, 10, 100)[0] == 2                           # m < n
    assert ws(100_000, 200, 10_000)[0] == 4                 # the wide path keeps no factors in Q
    assert ws(100_000, 20, 10_000, "fp32")[0] == 4           # FP64 only
