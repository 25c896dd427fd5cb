"""GPU parity: the HIP path through the C ABI against the CPU oracle, element by element.

Tolerances (FP64): R relative (Frobenius) <= 1e-12; Q elementwise <= 1e-12 where kappa(A) is
small (Gaussian inputs); ||Q^T Q - I||_2 and ||A - QR||_2/||A||_2 <= 1e-12 everywhere.  FP32
path: the same quantities <= 1e-5 against the oracle run on the FP32-rounded input promoted to
FP64; after the FP64 refinement pass: 1e-12.
"""
import numpy as np
import pytest
import torch

import oracle
import workloads

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0") if torch.cuda.is_available() else None


def tsqr_mod():
    import paper_1301_1071_amd as t
    return t


def gauss(m, n, seed):
    return np.random.default_rng(seed).standard_normal((m, n))


def to_gpu(A):
    return torch.from_numpy(np.ascontiguousarray(A)).to(DEV)


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def check_qr_fp64(A, Q, R, tol_q=1e-12, block_rows=1000):
    Qo, Ro = oracle.tsqr(A, block_rows=block_rows)
    assert np.all(np.tril(R, -1) == 0)
    assert np.all(np.diag(R) > 0)
    assert rel(R, Ro) <= 1e-12, rel(R, Ro)
    if tol_q is not None:
        dq = np.abs(Q - Qo).max()
        assert dq <= tol_q, dq
    assert oracle.metric_orth(Q) <= 1e-12
    assert oracle.metric_backward(A, Q, R) <= 1e-12


# --------------------------------------------------------------------- QR across n, ragged tails
@pytest.mark.parametrize("n", [1, 2, 3, 4, 8, 10, 16, 25, 32, 50, 64, 65, 100, 128])
def test_qr_fp64_shapes(n):
    t = tsqr_mod()
    b = 1904 if n <= 10 else 368 if n <= 50 else 512
    m = max(3 * b + 17, 4 * n + 3)
    A = gauss(m, n, 100 + n)
    Q, R = t.qr(to_gpu(A))
    check_qr_fp64(A, Q.cpu().numpy(), R.cpu().numpy())


@pytest.mark.parametrize("m,n", [(10, 10), (11, 10), (50, 50), (64, 8), (300, 7), (1, 1), (5, 1)])
def test_qr_fp64_small_and_square(m, n):
    t = tsqr_mod()
    A = gauss(m, n, 7 * m + n)
    Q, R = t.qr(to_gpu(A))
    check_qr_fp64(A, Q.cpu().numpy(), R.cpu().numpy(), tol_q=1e-11)


@pytest.mark.parametrize("n,panel_rows,m", [(8, 16, 5000), (8, 24, 777), (10, 64, 20_000),
                                             (30, 64, 9000), (4, 4, 1000)])
def test_qr_deep_trees(n, panel_rows, m):
    """Short panels force many tree levels (Sec. III-C recursion)."""
    t = tsqr_mod()
    A = gauss(m, n, 31 + n)
    Q, R = t.qr(to_gpu(A), panel_rows=panel_rows)
    check_qr_fp64(A, Q.cpu().numpy(), R.cpu().numpy())


def test_qr_strided_input_and_output():
    t = tsqr_mod()
    big = gauss(3000, 24, 5)
    Ad = to_gpu(big)[:, :17]                 # lda = 24 > n = 17
    Qbig = torch.full((3000, 20), 7.0, dtype=torch.float64, device=DEV)
    Rbig = torch.full((17, 19), 7.0, dtype=torch.float64, device=DEV)
    Q, R = t.qr(Ad, out=(Qbig[:, :17], Rbig[:, :17]))
    torch.cuda.synchronize()
    assert torch.all(Qbig[:, 17:] == 7.0) and torch.all(Rbig[:, 17:] == 7.0)
    check_qr_fp64(big[:, :17].copy(), Q.cpu().numpy(), R.cpu().numpy())


def test_r_only_matches_qr():
    t = tsqr_mod()
    A = gauss(50_000, 20, 9)
    Ad = to_gpu(A)
    R1 = t.r(Ad).cpu().numpy()
    _, R2 = t.qr(Ad)
    Ro = oracle.tsqr(A, block_rows=1000, want_q=False)
    assert rel(R1, Ro) <= 1e-12
    assert np.array_equal(R1, R2.cpu().numpy())     # the same kernels, bit for bit


def test_qr_small_config_full_size():
    """qr-small workload (100,000 x 10, N(0,1)) at full size, every element."""
    t = tsqr_mod()
    A = workloads.config_matrix("qr-small")
    Q, R = t.qr(to_gpu(A))
    check_qr_fp64(A, Q.cpu().numpy(), R.cpu().numpy(), block_rows=1000)


def test_determinism():
    t = tsqr_mod()
    A = to_gpu(gauss(40_000, 33, 11))
    Q1, R1 = t.qr(A)
    Q2, R2 = t.qr(A)
    assert torch.equal(Q1, Q2) and torch.equal(R1, R2)
    U1, S1, V1 = t.svd(A)
    U2, S2, V2 = t.svd(A)
    assert torch.equal(U1, U2) and torch.equal(S1, S2) and torch.equal(V1, V2)


# --------------------------------------------------------------------- SVD
def check_svd(A, U, S, V, tol_vec=1e-10, block_rows=1000):
    Uo, So, Vo = oracle.tsqr_svd(A, block_rows=block_rows)
    assert np.abs(S - So).max() <= 1e-12 * So[0]
    assert np.all(np.diff(S) <= 0)
    assert oracle.metric_orth(U) <= 1e-12
    assert oracle.metric_orth(V) <= 1e-12
    assert oracle.metric_svd_backward(A, U, S, V) <= 1e-12
    if tol_vec is not None:
        assert np.abs(V - Vo).max() <= tol_vec
        assert np.abs(U - Uo).max() <= tol_vec


# n = 100: Jacobi columns in LDS (the largest width whose 2 n^2 doubles fit); n = 120: in
# global scratch
@pytest.mark.parametrize("m,n", [(20_000, 10), (5000, 50), (3001, 3), (2000, 64), (4000, 100),
                                 (3000, 120)])
def test_svd_fp64(m, n):
    t = tsqr_mod()
    A = gauss(m, n, 40 + n)
    U, S, V, Q, R = t.svd(to_gpu(A), want_qr=True)
    check_svd(A, U.cpu().numpy(), S.cpu().numpy(), V.cpu().numpy(), tol_vec=1e-9)
    check_qr_fp64(A, Q.cpu().numpy(), R.cpu().numpy())
    U2, S2, V2 = t.svd(to_gpu(A))             # without Q: the same U, S, V
    assert torch.equal(U2.cpu(), U.cpu()) and torch.equal(S2.cpu(), S.cpu())


def test_svd_known_spectrum_ill_conditioned():
    """A = G diag(s) V^T with s = logspace(0, -12): backward-stable quantities at 1e-12."""
    t = tsqr_mod()
    A, s, Vt = workloads.spectrum_matrix(200_000, 50, 12.0, seed=77)
    U, S, V, Q, R = t.svd(to_gpu(A), want_qr=True)
    U, S, V, Q, R = (x.cpu().numpy() for x in (U, S, V, Q, R))
    check_svd(A, U, S, V, tol_vec=None, block_rows=8192)
    check_qr_fp64(A, Q, R, tol_q=None, block_rows=8192)


# --------------------------------------------------------------------- FP32 path and refinement
@pytest.mark.parametrize("m,n", [(100_000, 25), (30_000, 8), (9000, 64), (20_000, 100)])
def test_qr_f32_io(m, n):
    t = tsqr_mod()
    A32 = gauss(m, n, 60 + n).astype(np.float32)
    A = A32.astype(np.float64)
    Q, R = t.qr(to_gpu(A32))
    Q, R = Q.cpu().numpy().astype(np.float64), R.cpu().numpy().astype(np.float64)
    Qo, Ro = oracle.tsqr(A, block_rows=1000)
    assert rel(R, Ro) <= 1e-5
    assert oracle.metric_orth(Q) <= 1e-5
    assert oracle.metric_backward(A, Q, R) <= 1e-5


@pytest.mark.parametrize("m,n,log_cond", [(400_000, 25, 4.0), (50_000, 10, 2.0), (20_000, 64, 3.0)])
def test_precision_form(m, n, log_cond):
    t = tsqr_mod()
    A, s, _ = workloads.spectrum_matrix(m, n, log_cond, seed=90 + n)
    Ad = to_gpu(A)
    Qo, Ro = oracle.tsqr(A, block_rows=8192)
    normA = oracle.norm2(A)
    # before refinement: FP32 panels + FP32 GEMM, FP64 tree
    Qf, Rf = (x.cpu().numpy() for x in t.qr(Ad, precision="fp32"))
    assert rel(Rf, Ro) <= 1e-5
    assert oracle.metric_orth(Qf) <= 1e-5
    assert oracle.metric_backward(A, Qf, Rf, normA) <= 1e-5
    # after the FP64 refinement pass
    Qr, Rr = (x.cpu().numpy() for x in t.qr(Ad, precision="fp32_refined"))
    assert rel(Rr, Ro) <= 1e-12
    assert oracle.metric_orth(Qr) <= 1e-12
    assert oracle.metric_backward(A, Qr, Rr, normA) <= 1e-12
    assert np.all(np.diag(Rr) > 0)


# --------------------------------------------------------------------- info flag / degenerate
def test_info_rank_deficient_and_nonfinite():
    t = tsqr_mod()
    A = gauss(5000, 6, 3)
    A[:, 3] = 0.0
    with pytest.raises(torch.linalg.LinAlgError, match="R\\[3\\]\\[3\\]"):
        t.qr(to_gpu(A))
    A = gauss(5000, 6, 3)
    A[1234, 2] = np.nan
    with pytest.raises(torch.linalg.LinAlgError, match="non-finite"):
        t.qr(to_gpu(A))
    A = gauss(5000, 6, 3)
    A[:, 4] = A[:, 1]                       # exactly dependent: R[4][4] is rounding-level
    Q, R = t.qr(to_gpu(A), check_info=False)
    assert abs(float(R[4, 4])) <= 1e-12 * float(R[1, 1])


def test_zero_rows_and_padding_do_not_change_r():
    t = tsqr_mod()
    A = gauss(3000, 12, 4)
    Az = np.vstack([A, np.zeros((2000, 12))])
    R1 = t.r(to_gpu(A)).cpu().numpy()
    Q2, R2 = (x.cpu().numpy() for x in t.qr(to_gpu(Az)))
    assert rel(R2, R1) <= 1e-13
    assert np.abs(Q2[3000:]).max() == 0.0


def test_repeated_calls_reuse_workspace_and_outputs():
    """Five calls into the same workspace and output buffers (as the benchmark does): every call
    must give the same finite result (stale workspace or LDS contents must never leak in)."""
    t = tsqr_mod()
    A = workloads.spectrum_matrix(300_000, 50, 12.0, seed=5)[0]
    Ad = to_gpu(A)
    m, n = A.shape
    ws = torch.empty(t.workspace_bytes("svd", m, n), dtype=torch.uint8, device=DEV)
    outs = [torch.empty((m, n), dtype=torch.float64, device=DEV), torch.empty(n, dtype=torch.float64, device=DEV),
            torch.empty((n, n), dtype=torch.float64, device=DEV), torch.empty((m, n), dtype=torch.float64, device=DEV),
            torch.empty((n, n), dtype=torch.float64, device=DEV)]
    ref = None
    for _ in range(5):
        ws.fill_(255)                      # NaN bit patterns everywhere in the workspace
        t.svd(Ad, want_qr=True, ws=ws, out=tuple(outs))
        torch.cuda.synchronize()
        assert all(bool(torch.isfinite(o).all()) for o in outs)
        cur = [o.clone() for o in outs]
        if ref is None:
            ref = cur
        else:
            assert all(torch.equal(a, b) for a, b in zip(ref, cur))
    Q = outs[3].cpu().numpy()
    assert oracle.metric_orth(Q) <= 1e-12


# --------------------------------------------------------------------- full-size workloads
def test_svd_c50_full_size():
    """svd-c50 at its full size (4,000,000 x 50, cond 1e12) against the oracle (blocks of
    8,192 rows): R relative <= 1e-12, max |dS| / s1 <= 1e-12 and the backward-stable invariants
    <= 1e-12 (Q and U forward errors scale with kappa(A) and are not gated here)."""
    t = tsqr_mod()
    A = workloads.config_matrix("svd-c50")
    U, S, V, Q, R = (x.cpu().numpy() for x in t.svd(to_gpu(A), want_qr=True))
    Uo, So, Vo, Qo, Ro = oracle.tsqr_svd(A, block_rows=8192, want_qr=True)
    normA = So[0]
    assert rel(R, Ro) <= 1e-12, rel(R, Ro)
    assert np.abs(S - So).max() <= 1e-12 * So[0]
    assert np.all(np.diag(R) > 0) and np.all(np.tril(R, -1) == 0)
    assert oracle.metric_orth(Q) <= 1e-12
    assert oracle.metric_backward(A, Q, R, normA) <= 1e-12
    assert oracle.metric_svd_backward(A, U, S, V, normA) <= 1e-12
    assert oracle.metric_orth(U) <= 1e-12
    assert oracle.metric_orth(V) <= 1e-12


def test_mixed_c25_full_size():
    """mixed-c25 at its full size (16,000,000 x 25, cond 1e4): the FP32 form within 1e-5 of the
    FP64 oracle before refinement, the refined form within 1e-12 after."""
    t = tsqr_mod()
    A = workloads.config_matrix("mixed-c25")
    Ad = to_gpu(A)
    Ro = oracle.tsqr(A, block_rows=8192, want_q=False)
    normA = oracle.norm2(A)
    Qf, Rf = (x.cpu().numpy() for x in t.qr(Ad, precision="fp32"))
    assert rel(Rf, Ro) <= 1e-5
    assert oracle.metric_orth(Qf) <= 1e-5
    assert oracle.metric_backward(A, Qf, Rf, normA) <= 1e-5
    del Qf
    Qr, Rr = (x.cpu().numpy() for x in t.qr(Ad, precision="fp32_refined"))
    assert rel(Rr, Ro) <= 1e-12
    assert oracle.metric_orth(Qr) <= 1e-12
    assert oracle.metric_backward(A, Qr, Rr, normA) <= 1e-12


# --------------------------------------------------------------------- precision form extensions
@pytest.mark.parametrize("log_cond", [8.0, 12.0])
def test_refinement_ill_conditioned(log_cond):
    """Beyond the FP32 range of kappa(A) the refinement's second Cholesky pass keeps the FP64
    gates (R, orthogonality, backward error) at 1e-12."""
    t = tsqr_mod()
    A, s, _ = workloads.spectrum_matrix(200_000, 25, log_cond, seed=300 + int(log_cond))
    Ro = oracle.tsqr(A, block_rows=8192, want_q=False)
    Q, R = (x.cpu().numpy() for x in t.qr(to_gpu(A), precision="fp32_refined"))
    normA = oracle.norm2(A)
    assert oracle.metric_orth(Q) <= 1e-12
    assert oracle.metric_backward(A, Q, R, normA) <= 1e-12
    assert rel(R, Ro) <= 1e-12
    assert np.all(np.diag(R) > 0)


@pytest.mark.parametrize("want_qr", [False, True])
def test_svd_precision_refined(want_qr):
    t = tsqr_mod()
    A, s, _ = workloads.spectrum_matrix(150_000, 25, 4.0, seed=77)
    out = t.svd(to_gpu(A), want_qr=want_qr, precision="fp32_refined")
    U, S, V = (x.cpu().numpy() for x in out[:3])
    check_svd(A, U, S, V, tol_vec=None, block_rows=8192)
    if want_qr:
        Q, R = out[3].cpu().numpy(), out[4].cpu().numpy()
        check_qr_fp64(A, Q, R, tol_q=None, block_rows=8192)


@pytest.mark.parametrize("m,n", [(60_000, 10), (20_000, 50), (9000, 100)])
def test_svd_f32_io(m, n):
    t = tsqr_mod()
    A32 = gauss(m, n, 500 + n).astype(np.float32)
    A = A32.astype(np.float64)
    U, S, V, Q, R = (x.cpu().numpy().astype(np.float64) for x in t.svd(to_gpu(A32), want_qr=True))
    Uo, So, Vo = oracle.tsqr_svd(A, block_rows=1000)
    assert np.abs(S - So).max() <= 1e-5 * So[0]
    assert np.all(np.diff(S) <= 0)
    assert oracle.metric_orth(U) <= 1e-5
    assert oracle.metric_orth(V) <= 1e-5
    assert oracle.metric_svd_backward(A, U, S, V) <= 1e-5
    assert oracle.metric_backward(A, Q, R) <= 1e-5


def test_gpu_metrics_match_oracle_metrics():
    """The compensated GPU Gram metrics agree with the oracle's long-double metrics."""
    t = tsqr_mod()
    A = workloads.spectrum_matrix(300_000, 30, 6.0, seed=12)[0]
    Ad = to_gpu(A)
    Q, R = t.qr(Ad)
    Qh, Rh = Q.cpu().numpy(), R.cpu().numpy()
    o_gpu, o_cpu = t.metric_orth(Q), oracle.metric_orth(Qh)
    assert abs(o_gpu - o_cpu) <= 0.05 * o_cpu + 1e-18
    n_gpu, n_cpu = t.metric_norm2(Ad), oracle.norm2(A)
    assert abs(n_gpu - n_cpu) <= 1e-12 * n_cpu
    r_gpu, r_cpu = t.metric_residual(Ad, Q, R), oracle.residual(A, Qh, Rh)
    assert abs(r_gpu - r_cpu) <= 0.05 * r_cpu + 1e-30
    # a planted departure from orthogonality is seen at its size
    Qp = Q.clone()
    Qp[7, 3] += 1e-13
    assert abs(t.metric_orth(Qp) - oracle.metric_orth(Qp.cpu().numpy())) <= 1e-15
