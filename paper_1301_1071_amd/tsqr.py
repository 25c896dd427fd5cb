"""Python entry points over libtsqr.so: argument marshalling only.

Every step of the factorization runs in the library's HIP kernels; this module allocates the
outputs and the workspace with torch on the input's device, passes raw pointers and the current
HIP stream, and turns non-OK statuses into exceptions.  Inputs must be CUDA (HIP) tensors; there
is no CPU path.
"""
from __future__ import annotations

import ctypes

import torch

from . import _lib
from ._lib import check, lib, make_opts


def _require_gpu_matrix(A: torch.Tensor, dtypes=(torch.float64,)) -> None:
    if not isinstance(A, torch.Tensor) or A.dim() != 2:
        raise TypeError("A must be a 2-D torch tensor")
    if A.device.type != "cuda":
        raise TypeError("A must live on the GPU (device 'cuda'); the library has no CPU path")
    if A.dtype not in dtypes:
        raise TypeError("unsupported dtype %s" % A.dtype)
    if A.stride(1) != 1:
        raise ValueError("A must be row-major with unit column stride")


def _stream(dev: torch.device) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)


def _p(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def workspace_bytes(op: str, m: int, n: int, precision: str = "fp64", panel_rows: int = 0,
                    reuse_output: bool = False) -> int:
    o = make_opts(precision, panel_rows, reuse_output)
    out = ctypes.c_size_t(0)
    check(lib().tsqr_workspace_bytes(_lib.OPS[op], m, n, ctypes.byref(o), ctypes.byref(out)),
          "tsqr_workspace_bytes")
    return int(out.value)


def _workspace(op, m, n, precision, panel_rows, device, reuse_output=False):
    nbytes = workspace_bytes(op, m, n, precision, panel_rows, reuse_output)
    return torch.empty(nbytes, dtype=torch.uint8, device=device)


def _info_check(info: torch.Tensor, check_info: bool, where: str) -> None:
    if check_info:
        v = int(info.item())
        if v != 0:
            raise torch.linalg.LinAlgError("%s: info = %d (%s)" % (
                where, v, "non-finite input" if v == -1 else
                "refinement breakdown" if v == -2 else
                "adjoint undefined (zero pivot or repeated singular value)" if v == -3 else
                "R[%d][%d] == 0 (rank deficient)" % (v - 1, v - 1)))


def r(A: torch.Tensor, panel_rows: int = 0, ws: torch.Tensor | None = None,
      check_info: bool = True) -> torch.Tensor:
    """R factor of A (steps 1-2 of direct TSQR), diag(R) > 0.  FP64 or FP32 input."""
    _require_gpu_matrix(A, (torch.float64, torch.float32))
    m, n = A.shape
    f32 = A.dtype == torch.float32
    R = torch.empty((n, n), dtype=A.dtype, device=A.device)
    info = torch.zeros(1, dtype=torch.int32, device=A.device)
    o = make_opts("fp64", panel_rows)
    if ws is None:
        ws = _workspace("r", m, n, "fp32" if f32 else "fp64", panel_rows, A.device)
    fn = lib().tsqr_r_f32 if f32 else lib().tsqr_r
    check(fn(m, n, _p(A), A.stride(0), _p(R), n, _p(ws), ws.numel(), _p(info), ctypes.byref(o),
             _stream(A.device)), fn.__name__)
    _info_check(info, check_info, "tsqr_r")
    return R


def qr(A: torch.Tensor, precision: str = "fp64", panel_rows: int = 0,
       ws: torch.Tensor | None = None, out=None, check_info: bool = True,
       info: torch.Tensor | None = None, reuse_output: bool = False):
    """Thin QR by direct TSQR: returns (Q, R).  precision in {"fp64", "fp32", "fp32_refined"}
    for FP64 input; FP32 input always runs the FP32 path.  reuse_output keeps the level-0 panel
    factors in Q instead of the workspace (m x n elements less; Q must be contiguous)."""
    _require_gpu_matrix(A, (torch.float64, torch.float32))
    m, n = A.shape
    f32 = A.dtype == torch.float32
    if out is None:
        Q = torch.empty((m, n), dtype=A.dtype, device=A.device)
        R = torch.empty((n, n), dtype=A.dtype, device=A.device)
    else:
        Q, R = out
    if info is None:
        info = torch.zeros(1, dtype=torch.int32, device=A.device)
    prec = "fp32" if f32 else precision
    o = make_opts(prec, panel_rows, reuse_output)
    if ws is None:
        ws = _workspace("qr", m, n, prec, panel_rows, A.device, reuse_output)
    fn = lib().tsqr_qr_f32 if f32 else lib().tsqr_qr
    check(fn(m, n, _p(A), A.stride(0), _p(Q), Q.stride(0), _p(R), R.stride(0), _p(ws), ws.numel(),
             _p(info), ctypes.byref(o), _stream(A.device)), fn.__name__)
    _info_check(info, check_info, "tsqr_qr")
    return Q, R


def qr_chunked_workspace_bytes(m: int, n: int, chunk_rows: int) -> int:
    out = ctypes.c_size_t(0)
    o = make_opts("fp64")
    check(lib().tsqr_qr_chunked_workspace_bytes(m, n, chunk_rows, ctypes.byref(o),
                                                ctypes.byref(out)), "tsqr_qr_chunked_workspace_bytes")
    return int(out.value)


def qr_chunked(A: torch.Tensor, chunk_rows: int, ws: torch.Tensor | None = None, out=None,
               check_info: bool = True, info: torch.Tensor | None = None):
    """Row-chunked thin QR (tsqr_qr_chunked): the same (Q, R) as qr() with a workspace of about
    one chunk's.  FP64, n <= 128; Q must be contiguous."""
    _require_gpu_matrix(A, (torch.float64,))
    m, n = A.shape
    if out is None:
        Q = torch.empty((m, n), dtype=A.dtype, device=A.device)
        R = torch.empty((n, n), dtype=A.dtype, device=A.device)
    else:
        Q, R = out
    if info is None:
        info = torch.zeros(1, dtype=torch.int32, device=A.device)
    o = make_opts("fp64")
    if ws is None:
        ws = torch.empty(qr_chunked_workspace_bytes(m, n, chunk_rows), dtype=torch.uint8,
                         device=A.device)
    check(lib().tsqr_qr_chunked(m, n, chunk_rows, _p(A), A.stride(0), _p(Q), Q.stride(0), _p(R),
                                R.stride(0), _p(ws), ws.numel(), _p(info), ctypes.byref(o),
                                _stream(A.device)), "tsqr_qr_chunked")
    _info_check(info, check_info, "tsqr_qr_chunked")
    return Q, R


def svd(A: torch.Tensor, want_qr: bool = False, precision: str = "fp64", panel_rows: int = 0,
        ws: torch.Tensor | None = None, out=None, check_info: bool = True,
        info: torch.Tensor | None = None, reuse_output: bool = False):
    """Thin SVD by direct TSQR: returns (U, S, V) or (U, S, V, Q, R) with want_qr.  precision in
    {"fp64", "fp32", "fp32_refined"} for FP64 input; FP32 input runs the FP32 path and returns
    FP32 results.  reuse_output keeps the level-0 panel factors in Q (U without want_qr)."""
    _require_gpu_matrix(A, (torch.float64, torch.float32))
    m, n = A.shape
    f32 = A.dtype == torch.float32
    if out is None:
        U = torch.empty((m, n), dtype=A.dtype, device=A.device)
        S = torch.empty((n,), dtype=A.dtype, device=A.device)
        V = torch.empty((n, n), dtype=A.dtype, device=A.device)
        Q = torch.empty((m, n), dtype=A.dtype, device=A.device) if want_qr else None
        R = torch.empty((n, n), dtype=A.dtype, device=A.device) if want_qr else None
    else:
        U, S, V, Q, R = out
    if info is None:
        info = torch.zeros(1, dtype=torch.int32, device=A.device)
    prec = "fp32" if f32 else precision
    o = make_opts(prec, panel_rows, reuse_output)
    if ws is None:
        ws = _workspace("svd", m, n, prec, panel_rows, A.device, reuse_output)
    fn = lib().tsqr_svd_f32 if f32 else lib().tsqr_svd
    check(fn(m, n, _p(A), A.stride(0), _p(U), U.stride(0), _p(S), _p(V), V.stride(0),
             _p(Q), Q.stride(0) if Q is not None else 0, _p(R),
             R.stride(0) if R is not None else 0, _p(ws), ws.numel(), _p(info),
             ctypes.byref(o), _stream(A.device)), fn.__name__)
    _info_check(info, check_info, "tsqr_svd")
    return (U, S, V, Q, R) if want_qr else (U, S, V)


def _cotangent(x, shape, A):
    if x is None:
        return None
    if tuple(x.shape) != shape:
        raise ValueError("cotangent of shape %s, expected %s" % (tuple(x.shape), shape))
    if x.device != A.device or x.dtype != torch.float64:
        raise TypeError("cotangents must be float64 tensors on A's device")
    return x if x.stride(-1) == 1 else x.contiguous()


def qr_backward(A: torch.Tensor, dQ: torch.Tensor | None, dR: torch.Tensor | None,
                ws: torch.Tensor | None = None, out: torch.Tensor | None = None,
                check_info: bool = True) -> torch.Tensor:
    """dA for the loss <dQ, Q> + <dR, R> of (Q, R) = qr(A); Q and R are recomputed from A on the
    GPU (the forward's Q1_i are not kept).  FP64 only."""
    _require_gpu_matrix(A)
    m, n = A.shape
    dQ = _cotangent(dQ, (m, n), A)
    dR = _cotangent(dR, (n, n), A)
    dA = torch.empty((m, n), dtype=A.dtype, device=A.device) if out is None else out
    info = torch.zeros(1, dtype=torch.int32, device=A.device)
    o = make_opts("fp64", 0)
    if ws is None:
        ws = _workspace("qr_backward", m, n, "fp64", 0, A.device)
    check(lib().tsqr_qr_backward(m, n, _p(A), A.stride(0), _p(dQ), dQ.stride(0) if dQ is not None
                                 else 0, _p(dR), dR.stride(0) if dR is not None else 0, _p(dA),
                                 dA.stride(0), _p(ws), ws.numel(), _p(info), ctypes.byref(o),
                                 _stream(A.device)), "tsqr_qr_backward")
    _info_check(info, check_info, "tsqr_qr_backward")
    return dA


def svd_backward(A: torch.Tensor, dU: torch.Tensor | None, dS: torch.Tensor | None,
                 dV: torch.Tensor | None, ws: torch.Tensor | None = None,
                 out: torch.Tensor | None = None, check_info: bool = True) -> torch.Tensor:
    """dA for the loss <dU, U> + <dS, S> + <dV, V> of (U, S, V) = svd(A); U, S and V are
    recomputed from A on the GPU.  FP64 only; the singular values must be distinct and nonzero."""
    _require_gpu_matrix(A)
    m, n = A.shape
    dU = _cotangent(dU, (m, n), A)
    dS = _cotangent(dS, (n,), A)
    dV = _cotangent(dV, (n, n), A)
    dA = torch.empty((m, n), dtype=A.dtype, device=A.device) if out is None else out
    info = torch.zeros(1, dtype=torch.int32, device=A.device)
    o = make_opts("fp64", 0)
    if ws is None:
        ws = _workspace("svd_backward", m, n, "fp64", 0, A.device)
    check(lib().tsqr_svd_backward(m, n, _p(A), A.stride(0), _p(dU), dU.stride(0) if dU is not None
                                  else 0, _p(dS), _p(dV), dV.stride(0) if dV is not None else 0,
                                  _p(dA), dA.stride(0), _p(ws), ws.numel(), _p(info),
                                  ctypes.byref(o), _stream(A.device)), "tsqr_svd_backward")
    _info_check(info, check_info, "tsqr_svd_backward")
    return dA


def _row_major(A):
    return A if A.stride(1) == 1 else A.contiguous()


class QRFunction(torch.autograd.Function):
    """(Q, R) = qr(A) with the adjoint of tsqr_qr_backward.  Only A is saved: Q1_i is recomputed
    in the backward rather than held in HBM between the passes."""

    @staticmethod
    def forward(ctx, A):
        A = _row_major(A)
        Q, R = qr(A)
        ctx.save_for_backward(A)
        return Q, R

    @staticmethod
    def backward(ctx, dQ, dR):
        (A,) = ctx.saved_tensors
        return qr_backward(A, dQ, dR)


class SVDFunction(torch.autograd.Function):
    """(U, S, V) = svd(A) with the adjoint of tsqr_svd_backward; only A is saved."""

    @staticmethod
    def forward(ctx, A):
        A = _row_major(A)
        U, S, V = svd(A)
        ctx.save_for_backward(A)
        return U, S, V

    @staticmethod
    def backward(ctx, dU, dS, dV):
        (A,) = ctx.saved_tensors
        return svd_backward(A, dU, dS, dV)


def qr_autograd(A: torch.Tensor):
    """Differentiable thin QR by direct TSQR (FP64)."""
    return QRFunction.apply(A)


def svd_autograd(A: torch.Tensor):
    """Differentiable thin SVD by direct TSQR (FP64)."""
    return SVDFunction.apply(A)


# ----------------------------------------------------------------------------- batched form
_DTYPES = {torch.float64: 0, torch.float32: 1}


class BatchPlan:
    """A batched-QR plan for fixed shapes (tsqr_batch_plan_create): the per-matrix trees, the
    workspace size and the device task tables.  `run` only enqueues kernels, so it can be
    captured in a CUDA/HIP graph."""

    def __init__(self, shapes, dtype=torch.float64, lda=None, ldq=None, ldr=None,
                 panel_rows: int = 0, device=None):
        from .tuning import ensure_loaded
        ensure_loaded()
        self.shapes = [(int(m), int(n)) for m, n in shapes]
        self.dtype = dtype
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        b = len(self.shapes)
        arr = lambda xs: (ctypes.c_int64 * b)(*xs)
        ms = arr([m for m, _ in self.shapes])
        ns = arr([n for _, n in self.shapes])
        self._ld = (arr(lda or [n for _, n in self.shapes]), arr(ldq or [n for _, n in self.shapes]),
                    arr(ldr or [n for _, n in self.shapes]))
        o = make_opts("fp32" if dtype == torch.float32 else "fp64", panel_rows)
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            check(lib().tsqr_batch_plan_create(b, ms, ns, *self._ld, _DTYPES[dtype], ctypes.byref(o),
                                               ctypes.byref(h)), "tsqr_batch_plan_create")
        self._h = h
        nb = ctypes.c_size_t(0)
        check(lib().tsqr_batch_workspace_bytes(h, ctypes.byref(nb)), "tsqr_batch_workspace_bytes")
        self.workspace_bytes = int(nb.value)
        nl = ctypes.c_int32(0)
        check(lib().tsqr_batch_plan_launches(h, ctypes.byref(nl)), "tsqr_batch_plan_launches")
        self.launches = int(nl.value)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            lib().tsqr_batch_plan_destroy(h)
            self._h = None

    @staticmethod
    def pointers(tensors, device):
        return torch.tensor([t.data_ptr() for t in tensors], dtype=torch.int64, device=device)

    def run(self, ptrs_a: torch.Tensor, ptrs_q: torch.Tensor, ptrs_r: torch.Tensor,
            ws: torch.Tensor, info: torch.Tensor) -> None:
        """Enqueue the batched factorization on the current stream (no checks of d_info)."""
        check(lib().tsqr_qr_batched(self._h, _p(ptrs_a), _p(ptrs_q), _p(ptrs_r), _p(ws), ws.numel(),
                                    _p(info), _stream(ws.device)), "tsqr_qr_batched")


def qr_batched(As, panel_rows: int = 0, check_info: bool = True):
    """Thin QR of every matrix in the list `As` (2-D GPU tensors, one dtype, n <= 64, row-major
    with unit column stride) in one batched launch sequence; returns a list of (Q, R)."""
    if not As:
        return []
    dtype = As[0].dtype
    dev = As[0].device
    for A in As:
        _require_gpu_matrix(A, (torch.float64, torch.float32))
        if A.dtype != dtype or A.device != dev:
            raise TypeError("all matrices of a batch must share dtype and device")
    shapes = [tuple(A.shape) for A in As]
    plan = BatchPlan(shapes, dtype, lda=[A.stride(0) for A in As], panel_rows=panel_rows,
                     device=dev)
    Qs = [torch.empty(s, dtype=dtype, device=dev) for s in shapes]
    Rs = [torch.empty((s[1], s[1]), dtype=dtype, device=dev) for s in shapes]
    ws = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device=dev)
    info = torch.zeros(len(As), dtype=torch.int32, device=dev)
    plan.run(BatchPlan.pointers(As, dev), BatchPlan.pointers(Qs, dev), BatchPlan.pointers(Rs, dev),
             ws, info)
    if check_info:
        bad = torch.nonzero(info).flatten().tolist()
        if bad:
            raise torch.linalg.LinAlgError("tsqr_qr_batched: info != 0 for matrices %s (values %s)"
                                           % (bad[:8], info[bad[:8]].tolist()))
    return list(zip(Qs, Rs))


def tune_set(dtype, n: int, variant: int) -> None:
    check(lib().tsqr_tune_set(_DTYPES[dtype], n, variant), "tsqr_tune_set")


def tune_get(dtype, n: int):
    v, b = ctypes.c_int32(0), ctypes.c_int32(0)
    check(lib().tsqr_tune_get(_DTYPES[dtype], n, ctypes.byref(v), ctypes.byref(b)), "tsqr_tune_get")
    return int(v.value), int(b.value)


def tune_variants(dtype, n: int):
    """Panel heights of the register-panel variants for width n (0 = unusable variant)."""
    buf = (ctypes.c_int32 * 8)()
    c = ctypes.c_int32(0)
    check(lib().tsqr_tune_variants(_DTYPES[dtype], n, 8, buf, ctypes.byref(c)), "tsqr_tune_variants")
    return [int(buf[i]) for i in range(c.value)]


# ----------------------------------------------------------------------------- error metrics
def metric_gram(mode: int, X: torch.Tensor, A: torch.Tensor | None = None,
                B: torch.Tensor | None = None) -> torch.Tensor:
    """Compensated n x n Gram on the GPU (tsqr_metric_gram): mode 0 X^T X - I, mode 1
    (A - X B)^T (A - X B), mode 2 X^T X.  FP64 GPU tensors; returns an n x n GPU tensor."""
    _require_gpu_matrix(X)
    m, n = X.shape
    nb = ctypes.c_size_t(0)
    check(lib().tsqr_metric_workspace_bytes(m, n, ctypes.byref(nb)), "tsqr_metric_workspace_bytes")
    ws = torch.empty(int(nb.value), dtype=torch.uint8, device=X.device)
    G = torch.empty((n, n), dtype=torch.float64, device=X.device)
    if mode == 1:
        _require_gpu_matrix(A)
        B = B if B.stride(1) == 1 else B.contiguous()
    check(lib().tsqr_metric_gram(mode, m, n, _p(X), X.stride(0), _p(A),
                                 A.stride(0) if A is not None else 0, _p(B),
                                 B.stride(0) if B is not None else 0, _p(G), _p(ws), ws.numel(),
                                 _stream(X.device)), "tsqr_metric_gram")
    return G


def _sym_norm2(G: torch.Tensor) -> float:
    import numpy as np
    return float(np.max(np.abs(np.linalg.eigvalsh(G.cpu().numpy()))))


def metric_orth(Q: torch.Tensor) -> float:
    """||Q^T Q - I||_2 (Sec. I-B), compensated Gram on the GPU."""
    return _sym_norm2(metric_gram(0, Q))


def metric_norm2(A: torch.Tensor) -> float:
    """||A||_2 = sqrt(lambda_max(A^T A))."""
    return _sym_norm2(metric_gram(2, A)) ** 0.5


def metric_residual(A: torch.Tensor, Q: torch.Tensor, B: torch.Tensor) -> float:
    """||A - Q B||_2 with compensated residual rows."""
    return _sym_norm2(metric_gram(1, Q, A, B)) ** 0.5


# ----------------------------------------------------------------------------- comparison methods
_METHODS = {"cholqr": (1, 0), "cholqr_ir": (1, 1), "indirect": (2, 0), "indirect_ir": (2, 1)}


def qr_indirect(A: torch.Tensor, method: str, out=None, ws: torch.Tensor | None = None,
                info: torch.Tensor | None = None):
    """The stability experiment's comparison methods (Sec. IV) on the GPU: "cholqr" (Sec. II-A),
    "indirect" (Sec. II-B), each with Q = A R^{-1} (Sec. II-C), and their "_ir" variants with one
    step of iterative refinement.  Returns (Q, R, info) with info the device status (-4: the
    Cholesky factorization broke down)."""
    _require_gpu_matrix(A)
    m, n = A.shape
    meth, ir = _METHODS[method]
    Q, R = out if out is not None else (torch.empty((m, n), dtype=A.dtype, device=A.device),
                                        torch.empty((n, n), dtype=A.dtype, device=A.device))
    if info is None:
        info = torch.zeros(1, dtype=torch.int32, device=A.device)
    o = make_opts("fp64", 0)
    if ws is None:
        nb = ctypes.c_size_t(0)
        check(lib().tsqr_indirect_workspace_bytes(meth, ir, m, n, ctypes.byref(o), ctypes.byref(nb)),
              "tsqr_indirect_workspace_bytes")
        ws = torch.empty(int(nb.value), dtype=torch.uint8, device=A.device)
    check(lib().tsqr_qr_indirect(meth, ir, m, n, _p(A), A.stride(0), _p(Q), Q.stride(0), _p(R),
                                 R.stride(0), _p(ws), ws.numel(), _p(info), ctypes.byref(o),
                                 _stream(A.device)), "tsqr_qr_indirect")
    return Q, R, info
