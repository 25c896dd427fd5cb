"""Row-chunked QR (tsqr_qr_chunked): one more tree level above per-chunk direct TSQR, against the
oracle element by element (the factorization with diag(R) > 0 is unique, so the chunking does not
change Q or R beyond rounding)."""
import numpy as np
import pytest
import torch

import oracle

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0") if torch.cuda.is_available() else None


def gauss(m, n, seed):
    return np.random.default_rng(seed).standard_normal((m, n))


# (m, n, chunk_rows): equal chunks with a ragged last one; a last chunk shorter than n that joins
# the one before; n = 100 (explicit Q1 panels); one chunk; chunks shorter than a panel
@pytest.mark.parametrize("m,n,chunk", [(20_000, 30, 6000), (20_010, 30, 5000), (9000, 100, 4000),
                                       (7000, 50, 10_000), (5000, 8, 300)])
def test_qr_chunked_vs_oracle(m, n, chunk):
    import paper_1301_1071_amd as t
    print(f"chunked m={m} n={n} chunk={chunk}", flush=True)
    A = gauss(m, n, m + n)
    Q, R = t.qr_chunked(torch.from_numpy(A).to(DEV), chunk)
    Q, R = Q.cpu().numpy(), R.cpu().numpy()
    Qo, Ro = oracle.tsqr(A, block_rows=1000)
    assert np.all(np.tril(R, -1) == 0) and np.all(np.diag(R) > 0)
    assert np.linalg.norm(R - Ro) / np.linalg.norm(Ro) <= 1e-12
    assert np.abs(Q - Qo).max() <= 1e-12
    assert oracle.metric_orth(Q) <= 1e-12
    assert oracle.metric_backward(A, Q, R) <= 1e-12


def test_qr_chunked_rejections():
    import paper_1301_1071_amd as t
    A = torch.from_numpy(gauss(3000, 20, 1)).to(DEV)
    Qbig = torch.empty((3000, 24), dtype=torch.float64, device=DEV)
    R = torch.empty((20, 20), dtype=torch.float64, device=DEV)
    with pytest.raises(RuntimeError):                      # ldq != n
        t.qr_chunked(A, 1000, out=(Qbig[:, :20], R))
    with pytest.raises(RuntimeError):                      # wide n: no in-place level 0
        t.qr_chunked(torch.from_numpy(gauss(2000, 200, 2)).to(DEV), 1000)


def test_qr_chunked_graph_capture_replays():
    """The chunked driver only enqueues kernels: one call captured in a HIP graph replays to the
    eager result, several times, with eager work between the replays."""
    import paper_1301_1071_amd as t
    m, n, h = 12_000, 24, 5000
    A = torch.from_numpy(gauss(m, n, 3)).to(DEV)
    Q = torch.empty((m, n), dtype=torch.float64, device=DEV)
    R = torch.empty((n, n), dtype=torch.float64, device=DEV)
    info = torch.zeros(1, dtype=torch.int32, device=DEV)
    ws = torch.empty(t.qr_chunked_workspace_bytes(m, n, h), dtype=torch.uint8, device=DEV)
    t.qr_chunked(A, h, ws=ws, out=(Q, R), info=info)
    torch.cuda.synchronize()
    Q0, R0 = Q.clone(), R.clone()
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        t.qr_chunked(A, h, ws=ws, out=(Q, R), info=info, check_info=False)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    with torch.cuda.graph(g):
        t.qr_chunked(A, h, ws=ws, out=(Q, R), info=info, check_info=False)
    for _ in range(3):
        Q.zero_()
        R.zero_()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(Q, Q0) and torch.equal(R, R0)
        _ = torch.linalg.norm(A)               # eager work between replays
        torch.cuda.synchronize()
