"""Direct TSQR (Benson, Gleich & Demmel, Sec. III-B/III-C) for one MI355X (gfx950).

The factorization runs in hand-written HIP kernels inside ``libtsqr.so`` (C ABI in
``include/tsqr.h``); this package is the thin Python binding over it.
"""
from .tsqr import qr, r, svd, workspace_bytes  # noqa: F401

__all__ = ["qr", "r", "svd", "workspace_bytes"]
