"""tsqr_r_noalloc (the entry point for callers that cannot allocate) against tsqr_r, through the
C ABI: two calls in a row, the second on a smaller input, each bit-identical to tsqr_r on the
same input (the same kernels, the workspace in the library's fixed device array)."""
import ctypes

import numpy as np
import pytest
import torch

from paper_1301_1071_amd import _lib
from paper_1301_1071_amd._lib import lib, make_opts

pytestmark = pytest.mark.gpu


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _r_with_ws(A):
    m, n = A.shape
    o = make_opts("fp64")
    nb = ctypes.c_size_t()
    assert lib().tsqr_workspace_bytes(_lib.OPS["r"], m, n, ctypes.byref(o), ctypes.byref(nb)) == 0
    ws = torch.empty(nb.value, dtype=torch.uint8, device=A.device)
    R = torch.empty((n, n), dtype=torch.float64, device=A.device)
    info = torch.zeros(1, dtype=torch.int32, device=A.device)
    assert lib().tsqr_r(m, n, _ptr(A), A.stride(0), _ptr(R), n, _ptr(ws), ws.numel(), _ptr(info),
                        ctypes.byref(o), _stream()) == 0
    return R, info


def _r_noalloc(A):
    m, n = A.shape
    o = make_opts("fp64")
    R = torch.full((n, n), np.nan, dtype=torch.float64, device=A.device)
    info = torch.full((1,), 7, dtype=torch.int32, device=A.device)
    st = lib().tsqr_r_noalloc(m, n, _ptr(A), A.stride(0), _ptr(R), n, _ptr(info),
                              ctypes.byref(o), _stream())
    assert st == 0, lib().tsqr_last_error()
    return R, info


def test_noalloc_matches_tsqr_r_two_calls():
    dev = torch.device("cuda:0")
    g = np.random.default_rng(2024)
    for m, n in [(1_000_000, 50), (70_001, 17)]:      # the second call is smaller
        A = torch.from_numpy(g.standard_normal((m, n))).to(dev)
        R0, i0 = _r_with_ws(A)
        R1, i1 = _r_noalloc(A)
        torch.cuda.synchronize()
        assert int(i0.item()) == 0 and int(i1.item()) == 0
        assert torch.equal(R0, R1)
        assert bool(torch.all(torch.diagonal(R1) > 0))


def test_noalloc_rejects_inputs_beyond_its_scratch():
    dev = torch.device("cuda:0")
    A = torch.zeros((64, 64), dtype=torch.float64, device=dev)      # never read
    R = torch.zeros((64, 64), dtype=torch.float64, device=dev)
    info = torch.zeros(1, dtype=torch.int32, device=dev)
    o = make_opts("fp64")
    # 40M x 64: the level-0 stacked R alone is far above the scratch size
    st = lib().tsqr_r_noalloc(40_000_000, 64, _ptr(A), 64, _ptr(R), 64, _ptr(info),
                              ctypes.byref(o), _stream())
    assert st == 3
