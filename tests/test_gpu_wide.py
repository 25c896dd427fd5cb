"""GPU parity of the wide path (128 < n <= 512) against the CPU oracle.

Every level of the tree factors panels of 4 n rows (or an explicit height) held in global
workspace, step 3 runs in column chunks of 128, and the SVD's Jacobi columns live in global
memory.  The bars are those of the narrow path: FP64 R relative <= 1e-12, Q elementwise
<= 1e-12 on Gaussian inputs, orthogonality and backward error <= 1e-12; FP32 <= 1e-5 against the
oracle on the FP32-rounded input.
"""
import numpy as np
import pytest
import torch

import oracle

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0") if torch.cuda.is_available() else None


def gauss(m, n, seed):
    return np.random.default_rng(seed).standard_normal((m, n))


def to_gpu(A):
    return torch.from_numpy(np.ascontiguousarray(A)).to(DEV)


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def orth(Q):
    """||Q^T Q - I||_2 with an FP64 Gram: at these m (a few thousand rows) its rounding is
    O(sqrt(m) u), far below the 1e-12 bar, so no compensated sum is needed."""
    return np.linalg.norm(Q.T @ Q - np.eye(Q.shape[1]), 2)


def backward(A, Q, R):
    return np.linalg.norm(A - Q @ R, 2) / np.linalg.norm(A, 2)


def check_qr(A, Q, R, tol_q=1e-12):
    Qo, Ro = oracle.tsqr(A, block_rows=1000)
    assert np.all(np.tril(R, -1) == 0)
    assert np.all(np.diag(R) > 0)
    assert rel(R, Ro) <= 1e-12, rel(R, Ro)
    dq = np.abs(Q - Qo).max()
    assert dq <= tol_q, dq
    assert orth(Q) <= 1e-12
    assert backward(A, Q, R) <= 1e-12


# m: several 4n-row panels and a ragged last panel, shorter than n for n = 256 (zero padded)
@pytest.mark.parametrize("m,n", [(3 * 516 + 301, 129), (3 * 1024 + 100, 256), (2048 + 600, 512)])
def test_qr_wide(m, n):
    import paper_1301_1071_amd as t
    print(f"wide qr m={m} n={n}", flush=True)
    A = gauss(m, n, 500 + n)
    Q, R = t.qr(to_gpu(A))
    check_qr(A, Q.cpu().numpy(), R.cpu().numpy())
    R2 = t.r(to_gpu(A)).cpu().numpy()
    assert np.array_equal(R2, R.cpu().numpy())        # the same factor kernels


def test_qr_wide_deep_tree():
    """An explicit level-0 panel height of 2 n (13 panels, ragged) under the default 4 n-row
    tree panels: three levels at 5,000 x 200."""
    import paper_1301_1071_amd as t
    from paper_1301_1071_amd._lib import plan_levels
    m, n = 5000, 200
    assert plan_levels("qr", m, n, panel_rows=400) == [(5000, 400), (2600, 800), (800, 800)]
    A = gauss(m, n, 77)
    Q, R = t.qr(to_gpu(A), panel_rows=400)
    check_qr(A, Q.cpu().numpy(), R.cpu().numpy())


def test_svd_wide():
    import paper_1301_1071_amd as t
    m, n = 3000, 256
    A = gauss(m, n, 91)
    U, S, V, Q, R = t.svd(to_gpu(A), want_qr=True)
    U, S, V, Q, R = (x.cpu().numpy() for x in (U, S, V, Q, R))
    Uo, So, Vo = oracle.tsqr_svd(A, block_rows=1000)
    assert np.abs(S - So).max() <= 1e-12 * So[0]
    assert np.all(np.diff(S) <= 0)
    assert orth(U) <= 1e-12
    # V = rows of the rotated R scaled to unit length: the Jacobi sweeps stop once every pair's
    # cosine is below tol = 1e-15 n, so |V^T V - I| <= tol entrywise and ||V^T V - I||_2 <= n tol
    # (the oracle, rotating the other side, has the same bound on its U: 2e-12 at this shape)
    assert orth(V) <= n * 1e-15 * n
    assert np.abs(V.T @ V - np.eye(n)).max() <= 1e-15 * n
    assert np.linalg.norm(A - (U * S) @ V.T, 2) / S[0] <= 1e-12
    assert np.abs(V - Vo).max() <= 1e-9
    assert np.abs(U - Uo).max() <= 1e-9
    check_qr(A, Q, R)


def test_qr_wide_f32():
    import paper_1301_1071_amd as t
    m, n = 4000, 256
    A32 = gauss(m, n, 65).astype(np.float32)
    A = A32.astype(np.float64)
    Q, R = t.qr(to_gpu(A32))
    Q, R = Q.cpu().numpy().astype(np.float64), R.cpu().numpy().astype(np.float64)
    _, Ro = oracle.tsqr(A, block_rows=1000)
    assert rel(R, Ro) <= 1e-5
    assert orth(Q) <= 1e-5
    assert backward(A, Q, R) <= 1e-5


def test_qr_wide_strided_input_and_output():
    """lda > n and ldq > n on the wide path: the panels read rows at lda, step 3's column chunks
    write at ldq, and the padding columns of the caller's buffers stay untouched."""
    import paper_1301_1071_amd as t
    m, n = 1900, 200
    big = gauss(m, 232, 17)
    Ad = to_gpu(big)[:, :n]
    Qbig = torch.full((m, 210), 7.0, dtype=torch.float64, device=DEV)
    Rbig = torch.full((n, 205), 7.0, dtype=torch.float64, device=DEV)
    Q, R = t.qr(Ad, out=(Qbig[:, :n], Rbig[:, :n]))
    torch.cuda.synchronize()
    assert torch.all(Qbig[:, n:] == 7.0) and torch.all(Rbig[:, n:] == 7.0)
    check_qr(big[:, :n].copy(), Q.cpu().numpy(), R.cpu().numpy())


def test_svd_wide_f32():
    """FP32 input at n = 160: FP32 wide panels, FP64 tree and global-memory Jacobi, FP32 outputs."""
    import paper_1301_1071_amd as t
    m, n = 2500, 160
    A32 = gauss(m, n, 23).astype(np.float32)
    A = A32.astype(np.float64)
    U, S, V = (x.cpu().numpy().astype(np.float64) for x in t.svd(to_gpu(A32)))
    _, So, _ = oracle.tsqr_svd(A, block_rows=1000)
    assert np.abs(S - So).max() <= 1e-5 * So[0]
    assert orth(U) <= 1e-5 and orth(V) <= 1e-5
    assert np.linalg.norm(A - (U * S) @ V.T, 2) / S[0] <= 1e-5


def test_wide_rejects_reuse_output():
    import paper_1301_1071_amd as t
    with pytest.raises(RuntimeError):
        t.qr(to_gpu(gauss(1000, 200, 3)), reuse_output=True)


def test_wide_info_rank_deficient_and_nonfinite():
    """d_info on the wide path: a zero column gives R[j][j] == 0 (info j + 1), a NaN gives -1."""
    import paper_1301_1071_amd as t
    A = gauss(1500, 200, 4)
    A[:, 150] = 0.0
    with pytest.raises(torch.linalg.LinAlgError, match="R\\[150\\]\\[150\\]"):
        t.qr(to_gpu(A))
    A = gauss(1500, 200, 4)
    A[777, 33] = np.nan
    with pytest.raises(torch.linalg.LinAlgError, match="non-finite"):
        t.qr(to_gpu(A))
