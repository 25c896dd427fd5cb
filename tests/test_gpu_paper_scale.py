"""Paper-scale single-GPU runs: two of the paper's own shapes (Sec. V), 600,000,000 x 25 (QR, with
the level-0 factors kept in Q so that A, Q and the workspace fit in HBM) and 150,000,000 x 100
(R only).  The oracle cannot run at this size, so the checks are properties that hold at any
size, measured with the compensated GPU metrics of Sec. I-B:
  ||Q^T Q - I||_2 <= 1e-12 and ||A - QR||_2 / ||A||_2 <= 1e-12 (backward stability of direct
  TSQR, the paper's claim of Sec. IV), diag(R) > 0, and for R alone
  ||R^T R - A^T A||_2 / ||A||_2^2 <= 1e-12 (a backward-stable R has R^T R = (A + E)^T (A + E)
  with ||E|| = O(u ||A||)).
Each test skips when the device lacks the memory for its inputs."""
import numpy as np
import pytest
import torch

import workloads

pytestmark = pytest.mark.gpu

GiB = float(1 << 30)


def _free_bytes():
    torch.cuda.empty_cache()
    free, _ = torch.cuda.mem_get_info()
    return free


def _need_or_skip(need):
    free = _free_bytes()
    if free < need:
        pytest.skip("needs %.0f GiB of free device memory, %.0f GiB available" % (need / GiB, free / GiB))


def test_qr_600m_x_25():
    import paper_1301_1071_amd as t
    c = workloads.PAPER_SCALE["paper-600m"]
    m, n = c["m"], c["n"]
    wsb = t.workspace_bytes("qr", m, n, reuse_output=True)
    _need_or_skip(2 * 8 * m * n + wsb + (2 << 30))
    print("paper-600m: generating", flush=True)
    A = torch.empty((m, n), dtype=torch.float64, device="cuda")
    workloads.spectrum_matrix_device(A, c["log_cond"], workloads.SEEDS["paper-600m"])
    Q = torch.empty_like(A)
    R = torch.empty((n, n), dtype=torch.float64, device="cuda")
    ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
    print("paper-600m: factoring", flush=True)
    t.qr(A, ws=ws, out=(Q, R), reuse_output=True)
    torch.cuda.synchronize()
    del ws
    print("paper-600m: metrics", flush=True)
    Rn = R.cpu().numpy()
    assert np.all(np.diag(Rn) > 0) and np.all(np.tril(Rn, -1) == 0)
    orth = t.metric_orth(Q)
    back = t.metric_residual(A, Q, R) / np.linalg.norm(Rn, 2)
    print("paper-600m: orth %.3e backward %.3e" % (orth, back), flush=True)
    assert orth <= 1e-12
    assert back <= 1e-12
    del A, Q
    torch.cuda.empty_cache()


def test_r_150m_x_100():
    import paper_1301_1071_amd as t
    c = workloads.PAPER_SCALE["paper-150m"]
    m, n = c["m"], c["n"]
    wsb = t.workspace_bytes("r", m, n)
    _need_or_skip(8 * m * n + wsb + (4 << 30))
    print("paper-150m: generating", flush=True)
    A = torch.empty((m, n), dtype=torch.float64, device="cuda")
    workloads.spectrum_matrix_device(A, c["log_cond"], workloads.SEEDS["paper-150m"])
    ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
    print("paper-150m: factoring", flush=True)
    R = t.r(A, ws=ws)
    torch.cuda.synchronize()
    del ws
    print("paper-150m: metrics", flush=True)
    Rn = R.cpu().numpy()
    assert np.all(np.diag(Rn) > 0) and np.all(np.tril(Rn, -1) == 0)
    G = t.metric_gram(2, A).cpu().numpy()                 # compensated A^T A
    nA2 = np.max(np.linalg.eigvalsh(G))
    err = np.max(np.abs(np.linalg.eigvalsh(Rn.T @ Rn - G))) / nA2
    print("paper-150m: |R^T R - A^T A| / |A|^2 = %.3e" % err, flush=True)
    assert err <= 1e-12
    del A
    torch.cuda.empty_cache()


def test_qr_150m_x_100_chunked():
    """The paper's widest shape as a full QR: tsqr_qr_chunked with 15,000,000-row chunks keeps the
    workspace at about one chunk's, so A, Q and the workspace fit in HBM."""
    import paper_1301_1071_amd as t
    c = workloads.PAPER_SCALE["paper-150m"]
    m, n, h = c["m"], c["n"], 15_000_000
    wsb = t.qr_chunked_workspace_bytes(m, n, h)
    _need_or_skip(2 * 8 * m * n + wsb + (2 << 30))
    print("paper-150m qr: generating", flush=True)
    A = torch.empty((m, n), dtype=torch.float64, device="cuda")
    workloads.spectrum_matrix_device(A, c["log_cond"], workloads.SEEDS["paper-150m"])
    Q = torch.empty_like(A)
    R = torch.empty((n, n), dtype=torch.float64, device="cuda")
    ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
    print("paper-150m qr: factoring", flush=True)
    t.qr_chunked(A, h, ws=ws, out=(Q, R))
    torch.cuda.synchronize()
    del ws
    print("paper-150m qr: metrics", flush=True)
    Rn = R.cpu().numpy()
    assert np.all(np.diag(Rn) > 0) and np.all(np.tril(Rn, -1) == 0)
    orth = t.metric_orth(Q)
    back = t.metric_residual(A, Q, R) / np.linalg.norm(Rn, 2)
    print("paper-150m qr: orth %.3e backward %.3e" % (orth, back), flush=True)
    assert orth <= 1e-12
    assert back <= 1e-12
    del A, Q
    torch.cuda.empty_cache()
