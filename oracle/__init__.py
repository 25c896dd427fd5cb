"""Reference oracle for direct TSQR -- TEST INFRASTRUCTURE ONLY.

A plain, slow FP64 CPU implementation of what the GPU library computes (Benson, Gleich & Demmel,
Sec. III-B direct TSQR, Sec. III-A Householder QR, Sec. I-B metrics), written in plain C loops in
``tsqr_oracle.c`` and wrapped here with ctypes.  Only the test-suite, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` may import this package.  It shares no code with the
GPU library (``paper_1301_1071_amd``) and never imports it.

All arrays are C-contiguous float64 numpy arrays (row-major, as the paper's row records).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "tsqr_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_lib = None


def build(force: bool = False) -> str:
    """Compile the C oracle with gcc (-O2, OpenMP) into oracle/liboracle.so."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        i64, dp, i32, dbl = ctypes.c_int64, ctypes.c_void_p, ctypes.c_int, ctypes.c_double
        lib.oracle_householder_qr.argtypes = [i64, i64, dp, i64, dp, i64, dp, i64]
        lib.oracle_householder_qr.restype = i32
        lib.oracle_partition.argtypes = [i64, i64, i64, dp]
        lib.oracle_partition.restype = i64
        lib.oracle_tsqr.argtypes = [i64, i64, dp, i64, i64, dp, i64, dp, i64, dp, i32]
        lib.oracle_tsqr.restype = i32
        lib.oracle_svd_small.argtypes = [i64, dp, i64, dp, dp, i64, dp, i64]
        lib.oracle_svd_small.restype = i32
        lib.oracle_tsqr_svd.argtypes = [i64, i64, dp, i64, i64, dp, i64, dp, dp, i64, dp, i64,
                                        dp, i64, i32]
        lib.oracle_tsqr_svd.restype = i32
        lib.oracle_qr_backward.argtypes = [i64, i64, dp, i64, dp, i64, dp, i64, dp, i64, dp, i64,
                                           i32]
        lib.oracle_qr_backward.restype = i32
        lib.oracle_svd_backward.argtypes = [i64, i64, dp, i64, dp, dp, i64, dp, i64, dp, dp, i64,
                                            dp, i64, i32]
        lib.oracle_svd_backward.restype = i32
        lib.oracle_metric_orth.argtypes = [i64, i64, dp, i64, i32]
        lib.oracle_metric_orth.restype = dbl
        lib.oracle_norm2.argtypes = [i64, i64, dp, i64, i32]
        lib.oracle_norm2.restype = dbl
        lib.oracle_residual_norm2.argtypes = [i64, i64, dp, i64, dp, i64, dp, i64, i32]
        lib.oracle_residual_norm2.restype = dbl
        lib.oracle_indirect_qr.argtypes = [i32, i32, i64, i64, dp, i64, i64, dp, i64, dp, i64,
                                           i32]
        lib.oracle_indirect_qr.restype = i32
        lib.oracle_max_threads.argtypes = [i32]
        lib.oracle_max_threads.restype = i32
        _lib = lib
    return _lib


def _c(a: np.ndarray) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a


def _p(a):
    return None if a is None else a.ctypes.data


def max_threads(nthreads: int = 0) -> int:
    return int(_load().oracle_max_threads(int(nthreads)))


def partition(m: int, n: int, block_rows: int) -> np.ndarray:
    """Row-block starts used by the oracle (a tail with < n rows merges into the previous block)."""
    lib = _load()
    nb = lib.oracle_partition(m, n, block_rows, None)
    st = np.zeros(nb + 1, dtype=np.int64)
    lib.oracle_partition(m, n, block_rows, st.ctypes.data)
    return st


def householder_qr(A: np.ndarray, want_q: bool = True):
    """Single-block Householder QR (Sec. III-A) with diag(R) > 0."""
    A = _c(A)
    m, n = A.shape
    Q = np.empty((m, n)) if want_q else None
    R = np.empty((n, n))
    st = _load().oracle_householder_qr(m, n, _p(A), n, _p(Q), n, _p(R), n)
    if st != 0:
        raise ValueError("oracle_householder_qr failed with status %d" % st)
    return (Q, R) if want_q else R


def tsqr(A: np.ndarray, block_rows: int, want_q: bool = True, want_q2: bool = False,
         nthreads: int = 0):
    """Direct TSQR (Sec. III-B): returns (Q, R) or R; with want_q2 also the step-2 Q2 blocks."""
    A = _c(A)
    m, n = A.shape
    Q = np.empty((m, n)) if want_q else None
    R = np.empty((n, n))
    nb = len(partition(m, n, block_rows)) - 1
    Q2 = np.empty((nb * n, n)) if want_q2 else None
    st = _load().oracle_tsqr(m, n, _p(A), n, block_rows, _p(Q), n, _p(R), n, _p(Q2), nthreads)
    if st != 0:
        raise ValueError("oracle_tsqr failed with status %d" % st)
    out = (Q, R) if want_q else (R,)
    if want_q2:
        out = out + (Q2,)
    return out if len(out) > 1 else out[0]


def svd_small(R: np.ndarray):
    """One-sided Jacobi SVD of a small square matrix: returns (U_R, S, V, sweeps)."""
    R = _c(R)
    n = R.shape[0]
    S = np.empty(n)
    V = np.empty((n, n))
    UR = np.empty((n, n))
    sweeps = _load().oracle_svd_small(n, _p(R), n, _p(S), _p(V), n, _p(UR), n)
    return UR, S, V, sweeps


def tsqr_svd(A: np.ndarray, block_rows: int, nthreads: int = 0, want_qr: bool = False):
    """SVD via direct TSQR (Sec. III-B): returns (U, S, V) or (U, S, V, Q, R)."""
    A = _c(A)
    m, n = A.shape
    U = np.empty((m, n))
    S = np.empty(n)
    V = np.empty((n, n))
    Q = np.empty((m, n)) if want_qr else None
    R = np.empty((n, n)) if want_qr else None
    st = _load().oracle_tsqr_svd(m, n, _p(A), n, block_rows, _p(U), n, _p(S), _p(V), n,
                                 _p(Q), n, _p(R), n, nthreads)
    if st < 0:
        raise ValueError("oracle_tsqr_svd failed with status %d" % st)
    return (U, S, V, Q, R) if want_qr else (U, S, V)


def qr_backward(Q, R, dQ=None, dR=None, nthreads: int = 0):
    """dA for the loss <dQ,Q> + <dR,R> (closed-form QR adjoint)."""
    Q, R = _c(Q), _c(R)
    m, n = Q.shape
    dQ = None if dQ is None else _c(dQ)
    dR = None if dR is None else _c(dR)
    dA = np.empty((m, n))
    st = _load().oracle_qr_backward(m, n, _p(Q), n, _p(R), n, _p(dQ), n, _p(dR), n, _p(dA), n,
                                    nthreads)
    if st != 0:
        raise ValueError("oracle_qr_backward failed with status %d" % st)
    return dA


def svd_backward(U, S, V, dU=None, dS=None, dV=None, nthreads: int = 0):
    """dA for the loss <dU,U> + <dS,S> + <dV,V> (closed-form thin-SVD adjoint)."""
    U, S, V = _c(U), _c(S), _c(V)
    m, n = U.shape
    dU = None if dU is None else _c(dU)
    dS = None if dS is None else _c(dS)
    dV = None if dV is None else _c(dV)
    dA = np.empty((m, n))
    st = _load().oracle_svd_backward(m, n, _p(U), n, _p(S), _p(V), n, _p(dU), n, _p(dS),
                                     _p(dV), n, _p(dA), n, nthreads)
    if st != 0:
        raise ValueError("oracle_svd_backward failed with status %d" % st)
    return dA


def metric_orth(Q, nthreads: int = 0) -> float:
    """||Q^T Q - I||_2 with long-double accumulation (Sec. I-B)."""
    Q = _c(Q)
    m, n = Q.shape
    return float(_load().oracle_metric_orth(m, n, _p(Q), n, nthreads))


def norm2(X, nthreads: int = 0) -> float:
    X = _c(X)
    m, n = X.shape
    return float(_load().oracle_norm2(m, n, _p(X), n, nthreads))


def residual(A, Q, B, nthreads: int = 0) -> float:
    """||A - Q B||_2 (B is n x n)."""
    A, Q, B = _c(A), _c(Q), _c(B)
    m, n = A.shape
    return float(_load().oracle_residual_norm2(m, n, _p(A), n, _p(Q), n, _p(B), n, nthreads))


def metric_backward(A, Q, R, normA=None, nthreads: int = 0) -> float:
    """||A - QR||_2 / ||A||_2 (Sec. I-B; equal to /||R||_2 in exact arithmetic)."""
    if normA is None:
        normA = norm2(A, nthreads)
    return residual(A, Q, R, nthreads) / normA


def metric_svd_backward(A, U, S, V, normA=None, nthreads: int = 0) -> float:
    """||A - U diag(S) V^T||_2 / ||A||_2."""
    if normA is None:
        normA = norm2(A, nthreads)
    B = np.asarray(S)[:, None] * np.asarray(V).T
    return residual(A, U, B, nthreads) / normA


METHODS = {"cholqr": (1, 0), "cholqr_ir": (1, 1), "indirect": (2, 0), "indirect_ir": (2, 1)}


def indirect_qr(A, method: str, block_rows: int = 1000, nthreads: int = 0):
    """The comparison methods of the stability experiment (Sec. IV): Cholesky QR (Sec. II-A) or
    indirect TSQR (Sec. II-B) with Q = A R^{-1} (Sec. II-C), and the "_ir" variants with one step
    of iterative refinement.  Returns (Q, R), or None when the Cholesky factorization breaks
    down."""
    A = _c(A)
    m, n = A.shape
    meth, ir = METHODS[method]
    Q = np.empty((m, n))
    R = np.empty((n, n))
    st = _load().oracle_indirect_qr(meth, ir, m, n, _p(A), n, block_rows, _p(Q), n, _p(R), n,
                                    nthreads)
    if st == 4:
        return None
    if st != 0:
        raise ValueError("oracle_indirect_qr failed with status %d" % st)
    return Q, R
