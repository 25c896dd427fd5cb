"""Level-0 panel factors kept in the output buffer (TSQR_FLAG_REUSE_OUTPUT): the same kernels and
the same per-tile products as with the workspace copy, so Q, R (and U, S, V) agree bit for bit;
the workspace shrinks by m x n elements."""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0") if torch.cuda.is_available() else None


def gauss(m, n, seed, dtype=np.float64):
    return torch.from_numpy(np.random.default_rng(seed).standard_normal((m, n)).astype(dtype)).to(DEV)


@pytest.mark.parametrize("m,n", [(100_003, 10), (50_001, 25), (30_011, 50), (20_000, 64),
                                 (20_005, 100)])
def test_qr_reuse_output_bitwise(m, n):
    import paper_1301_1071_amd as t
    print(f"reuse qr m={m} n={n}", flush=True)
    A = gauss(m, n, 3 * n)
    Q1, R1 = t.qr(A)
    Q2, R2 = t.qr(A, reuse_output=True)
    torch.cuda.synchronize()
    assert torch.equal(Q1, Q2) and torch.equal(R1, R2)
    w0 = t.workspace_bytes("qr", m, n)
    w1 = t.workspace_bytes("qr", m, n, reuse_output=True)
    assert w0 - w1 >= 8 * m * n


@pytest.mark.parametrize("m,n,want_qr", [(40_000, 25, True), (20_000, 64, True),
                                         (20_000, 100, False)])
def test_svd_reuse_output_bitwise(m, n, want_qr):
    import paper_1301_1071_amd as t
    A = gauss(m, n, 5 * n)
    a = t.svd(A, want_qr=want_qr)
    b = t.svd(A, want_qr=want_qr, reuse_output=True)
    torch.cuda.synchronize()
    for x, y in zip(a, b):
        assert torch.equal(x, y)


def test_qr_f32_reuse_output_bitwise():
    import paper_1301_1071_amd as t
    A = gauss(70_000, 25, 11, np.float32)
    Q1, R1 = t.qr(A)
    Q2, R2 = t.qr(A, reuse_output=True)
    torch.cuda.synchronize()
    assert torch.equal(Q1, Q2) and torch.equal(R1, R2)


def test_reuse_output_rejections():
    import paper_1301_1071_amd as t
    A = gauss(5000, 20, 1)
    Qbig = torch.empty((5000, 24), dtype=torch.float64, device=DEV)
    R = torch.empty((20, 20), dtype=torch.float64, device=DEV)
    with pytest.raises(RuntimeError):                      # ldq != n
        t.qr(A, out=(Qbig[:, :20], R), reuse_output=True)
    with pytest.raises(RuntimeError):                      # 128 output columns past one LDS
        t.qr(gauss(2000, 128, 2), reuse_output=True)


def test_svd_f32_reuse_output_bitwise():
    import paper_1301_1071_amd as t
    A = gauss(30_000, 40, 13, np.float32)
    a = t.svd(A)
    b = t.svd(A, reuse_output=True)
    torch.cuda.synchronize()
    for x, y in zip(a, b):
        assert torch.equal(x, y)
