"""Direct TSQR (Benson, Gleich & Demmel, Sec. III-B/III-C) for one MI355X (gfx950).

The factorization runs in hand-written HIP kernels inside ``libtsqr.so`` (C ABI in
``include/tsqr.h``); this package is the thin Python binding over it.
"""
from .tsqr import (BatchPlan, QRFunction, SVDFunction, metric_gram, metric_norm2,  # noqa: F401
                   metric_orth, metric_residual, qr, qr_autograd, qr_backward, qr_batched,
                   qr_chunked, qr_chunked_workspace_bytes, qr_indirect, r, svd, svd_autograd, svd_backward, tune_get, tune_set,
                   tune_variants, workspace_bytes)
__all__ = ["qr", "r", "svd", "workspace_bytes", "qr_backward", "svd_backward", "qr_autograd",
           "svd_autograd", "QRFunction", "SVDFunction", "qr_batched", "BatchPlan", "tune_set",
           "tune_get", "tune_variants", "metric_gram", "metric_orth", "metric_norm2",
           "metric_residual", "qr_indirect", "qr_chunked", "qr_chunked_workspace_bytes"]
