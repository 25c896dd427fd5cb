"""Seeded synthetic inputs shaped like the paper's tall-and-skinny workloads.

This module only draws random numbers and assembles matrices from them; it holds none of the
factorization's arithmetic, so both the GPU tests and the CPU oracle can take their inputs from
it.  The paper's matrices (Sec. V, 4.0B x 4 ... 150M x 100, stored on HDFS) are not published and
their contents are never described, so the shapes are kept (column counts 4..100) and the rows
scaled to one GPU, with entries drawn as follows (numpy PCG64, fixed seeds):

  qr-small   100,000 x 10,  A_ij ~ N(0,1)                                     seed 1301107101
  svd-c50    4,000,000 x 50, A = G diag(s) V^T, G ~ N(0,1), V Haar orthogonal
             (Q factor of a 50 x 50 Gaussian with diag(R) > 0), s = logspace(0,-12,50)
                                                                               seed 1301107102
  mixed-c25  16,000,000 x 25, as svd-c50 with s = logspace(0,-4,25)           seed 1301107103
  batch512   512 matrices, m ~ U{2000..200000}, n ~ U{4,8,16,32,64}, N(0,1)    seed 1301107104
  grad-c100  1,000,000 x 100, N(0,1); cotangents N(0,1) with seed + 100 k      seed 1301107105

Paper-scale shapes (two of the paper's own, Sec. V), built on the device because the inputs
alone fill much of one GPU's HBM: A = G diag(s) V^T with V and s drawn as above (numpy) and G
drawn by torch's device generator (Philox) seeded with the same seed, chunk by chunk:
  paper-600m 600,000,000 x 25,  s = logspace(0,-8,25)                         seed 1301107106
  paper-150m 150,000,000 x 100, s = logspace(0,-8,100)                        seed 1301107107
"""
from __future__ import annotations

import numpy as np

SEEDS = {
    "qr-small": 1301107101,
    "svd-c50": 1301107102,
    "mixed-c25": 1301107103,
    "batch512": 1301107104,
    "grad-c100": 1301107105,
    "paper-600m": 1301107106,
    "paper-150m": 1301107107,
}

PAPER_SCALE = {
    "paper-600m": dict(m=600_000_000, n=25, log_cond=8.0),
    "paper-150m": dict(m=150_000_000, n=100, log_cond=8.0),
}

CONFIGS = {
    # name: (m, n, oracle block rows, spectrum exponent or None for N(0,1))
    "qr-small": dict(m=100_000, n=10, block_rows=1000, log_cond=None),
    "svd-c50": dict(m=4_000_000, n=50, block_rows=8192, log_cond=12.0),
    "mixed-c25": dict(m=16_000_000, n=25, block_rows=8192, log_cond=4.0),
    "grad-c100": dict(m=1_000_000, n=100, block_rows=8192, log_cond=None),
}


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def haar_orthogonal(n: int, g: np.random.Generator) -> np.ndarray:
    """Haar-distributed orthogonal n x n matrix: the Q factor of a Gaussian with diag(R) > 0
    (Mezzadri 2007).  LAPACK's QR is used here only to draw an input."""
    X = g.standard_normal((n, n))
    Q, R = np.linalg.qr(X)
    return Q * np.sign(np.where(np.diag(R) == 0, 1.0, np.diag(R)))[None, :]


def gaussian(m: int, n: int, seed: int, chunk_rows: int = 1 << 20) -> np.ndarray:
    """m x n matrix of i.i.d. N(0,1) entries (row-major float64), drawn row-chunk by row-chunk."""
    g = rng(seed)
    A = np.empty((m, n), dtype=np.float64)
    for r0 in range(0, m, chunk_rows):
        r1 = min(m, r0 + chunk_rows)
        A[r0:r1] = g.standard_normal((r1 - r0, n))
    return A


def spectrum_matrix(m: int, n: int, log_cond: float, seed: int,
                    chunk_rows: int = 1 << 20):
    """A = G diag(s) V^T with G ~ N(0,1), V Haar, s = logspace(0, -log_cond, n).
    Returns (A, s, V)."""
    g = rng(seed)
    V = haar_orthogonal(n, g)
    s = np.logspace(0.0, -log_cond, n)
    B = (s[:, None] * V.T)            # diag(s) V^T
    A = np.empty((m, n), dtype=np.float64)
    for r0 in range(0, m, chunk_rows):
        r1 = min(m, r0 + chunk_rows)
        A[r0:r1] = g.standard_normal((r1 - r0, n)) @ B
    return A, s, V


def config_matrix(name: str, m: int | None = None):
    """The input matrix of a named workload, optionally with fewer rows (same recipe and seed)."""
    c = CONFIGS[name]
    mm = c["m"] if m is None else m
    if c["log_cond"] is None:
        return gaussian(mm, c["n"], SEEDS[name])
    return spectrum_matrix(mm, c["n"], c["log_cond"], SEEDS[name])[0]


def cotangents(m: int, n: int, seed: int = SEEDS["grad-c100"]):
    """Cotangents dQ, dR (upper triangle), dU, dS, dV ~ N(0,1), one seed each (seed + 100 k)."""
    out = {}
    for k, (key, shape) in enumerate([("dQ", (m, n)), ("dR", (n, n)), ("dU", (m, n)),
                                      ("dS", (n,)), ("dV", (n, n))]):
        x = rng(seed + 100 * (k + 1)).standard_normal(shape)
        if key == "dR":
            x = np.triu(x)
        out[key] = x
    return out


def batch_shapes(count: int = 512, seed: int = SEEDS["batch512"], m_lo: int = 2000,
                 m_hi: int = 200_000, n_choices=(4, 8, 16, 32, 64)):
    """Ragged batch: m ~ U{m_lo..m_hi}, n ~ U(n_choices)."""
    g = rng(seed)
    ms = g.integers(m_lo, m_hi + 1, size=count)
    ns = g.choice(np.asarray(n_choices), size=count)
    return [(int(a), int(b)) for a, b in zip(ms, ns)]


def batch_matrices(shapes, seed: int = SEEDS["batch512"], dtype=np.float64):
    """One N(0,1) matrix per shape; matrix k uses seed + 1 + k.  FP32 inputs are the FP32
    rounding of the same FP64 draws."""
    mats = []
    for k, (m, n) in enumerate(shapes):
        a = rng(seed + 1 + k).standard_normal((m, n))
        mats.append(a.astype(dtype) if dtype != np.float64 else a)
    return mats


def spectrum_matrix_device(out, log_cond: float, seed: int, chunk_rows: int = 1 << 22):
    """Fill the device tensor `out` (m x n, float64, contiguous) with A = G diag(s) V^T: V Haar
    and s = logspace(0, -log_cond, n) from numpy as in spectrum_matrix, G ~ N(0,1) from torch's
    device generator seeded with `seed`, chunk_rows rows at a time.  Returns (s, V)."""
    import torch
    m, n = out.shape
    g = rng(seed)
    V = haar_orthogonal(n, g)
    s = np.logspace(0.0, -log_cond, n)
    B = torch.from_numpy(np.ascontiguousarray(s[:, None] * V.T)).to(out.device)
    gen = torch.Generator(device=out.device)
    gen.manual_seed(seed)
    for r0 in range(0, m, chunk_rows):
        r1 = min(m, r0 + chunk_rows)
        G = torch.randn((r1 - r0, n), generator=gen, dtype=torch.float64, device=out.device)
        torch.matmul(G, B, out=out[r0:r1])
        del G
    return s, V
