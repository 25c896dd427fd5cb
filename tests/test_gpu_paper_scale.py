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


def test_svd_600m_x_25():
    """The SVD variant (Sec. III-B) at 600,000,000 x 25: U comes out of step 3 in place of Q (its
    level-0 factors kept in U), S and V from the Jacobi SVD of R.  Checks: ||U^T U - I||_2,
    ||A - U S V^T||_2 / s_1 and ||V^T V - I||_2 <= 1e-12, S descending and positive, and S against
    the spectrum A was built from within the O(sqrt(n / m)) distortion of the Gaussian factor."""
    import paper_1301_1071_amd as t
    c = workloads.PAPER_SCALE["paper-600m"]
    m, n = c["m"], c["n"]
    wsb = t.workspace_bytes("svd", m, n, reuse_output=True)
    _need_or_skip(2 * 8 * m * n + wsb + (2 << 30))
    print("paper-600m svd: generating", flush=True)
    A = torch.empty((m, n), dtype=torch.float64, device="cuda")
    s_true, _ = workloads.spectrum_matrix_device(A, c["log_cond"], workloads.SEEDS["paper-600m"])
    U = torch.empty_like(A)
    S = torch.empty((n,), dtype=torch.float64, device="cuda")
    V = torch.empty((n, n), dtype=torch.float64, device="cuda")
    ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
    print("paper-600m svd: factoring", flush=True)
    t.svd(A, ws=ws, out=(U, S, V, None, None), reuse_output=True)
    torch.cuda.synchronize()
    del ws
    print("paper-600m svd: metrics", flush=True)
    Sn, Vn = S.cpu().numpy(), V.cpu().numpy()
    assert np.all(Sn > 0) and np.all(np.diff(Sn) <= 0)
    orth_u = t.metric_orth(U)
    res = t.metric_residual(A, U, (S[:, None] * V.t()).contiguous()) / Sn[0]
    orth_v = np.linalg.norm(Vn.T @ Vn - np.eye(n), 2)
    rel_s = np.max(np.abs(Sn / np.sqrt(m) - s_true) / s_true)
    print("paper-600m svd: orth U %.3e residual %.3e orth V %.3e |S/sqrt(m) - s|/s %.2e"
          % (orth_u, res, orth_v, rel_s), flush=True)
    assert orth_u <= 1e-12 and res <= 1e-12 and orth_v <= 1e-12
    assert rel_s <= 1e-2
    del A, U
    torch.cuda.empty_cache()
