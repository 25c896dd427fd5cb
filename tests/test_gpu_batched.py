"""GPU parity of the batched form (tsqr_qr_batched through the C ABI) against the oracle run per
matrix, the graph-captured launch sequence, and the batch512 workload at full size.

Gates: FP64 as for tsqr_qr (R relative <= 1e-12, Q elementwise <= 1e-12 on Gaussian inputs,
orthogonality and residual <= 1e-12); FP32 <= 1e-5 against the oracle on the FP32-rounded input.
"""
import numpy as np
import pytest
import torch

import oracle
import workloads

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0") if torch.cuda.is_available() else None


def t():
    import paper_1301_1071_amd as m
    return m


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def mixed_batch(seed, count, m_lo, m_hi, widths):
    g = np.random.default_rng(seed)
    shapes = [(int(g.integers(m_lo, m_hi + 1)), int(g.choice(widths))) for _ in range(count)]
    mats = [g.standard_normal((max(m, n), n)) for m, n in shapes]
    return mats


def check_fp64(A, Q, R):
    Qo, Ro = oracle.tsqr(A, block_rows=1000)
    assert np.all(np.tril(R, -1) == 0) and np.all(np.diag(R) > 0)
    assert rel(R, Ro) <= 1e-12, rel(R, Ro)
    assert np.abs(Q - Qo).max() <= 1e-12
    assert oracle.metric_orth(Q) <= 1e-12
    assert oracle.metric_backward(A, Q, R) <= 1e-12


def test_batched_fp64_mixed_widths_vs_oracle():
    widths = [1, 2, 3, 4, 5, 7, 8, 9, 12, 16, 17, 24, 31, 32, 33, 48, 63, 64]
    mats = mixed_batch(11, 60, 1, 9000, widths)
    out = t().qr_batched([torch.from_numpy(A).to(DEV) for A in mats])
    for A, (Q, R) in zip(mats, out):
        check_fp64(A, Q.cpu().numpy(), R.cpu().numpy())


@pytest.mark.parametrize("n", [4, 8, 16, 32, 64])
def test_batched_fp64_every_variant(n):
    """Each usable panel variant (the autotuner's candidates) gives the oracle's factorization."""
    mats = mixed_batch(20 + n, 12, 2000, 40_000, [n])
    As = [torch.from_numpy(A).to(DEV) for A in mats]
    heights = t().tune_variants(torch.float64, n)
    for b in heights:
        if not b:
            continue
        out = t().qr_batched(As, panel_rows=b)
        for A, (Q, R) in zip(mats[:4], out[:4]):
            check_fp64(A, Q.cpu().numpy(), R.cpu().numpy())


def test_batched_fp32_vs_oracle():
    mats = mixed_batch(12, 40, 100, 30_000, [4, 8, 16, 32, 64, 5, 50])
    mats32 = [A.astype(np.float32) for A in mats]
    out = t().qr_batched([torch.from_numpy(A).to(DEV) for A in mats32])
    for A32, (Q, R) in zip(mats32, out):
        A = A32.astype(np.float64)
        Q, R = Q.cpu().numpy().astype(np.float64), R.cpu().numpy().astype(np.float64)
        _, Ro = oracle.tsqr(A, block_rows=1000)
        assert rel(R, Ro) <= 1e-5
        assert oracle.metric_orth(Q) <= 1e-5
        assert oracle.metric_backward(A, Q, R) <= 1e-5


def test_batched_strided_inputs_and_info():
    g = np.random.default_rng(5)
    big = [g.standard_normal((3000, 40)) for _ in range(3)]
    big[1][:, 3] = 0.0                           # rank deficient: info = 4
    As = [torch.from_numpy(B).to(DEV)[:, :n] for B, n in zip(big, (10, 20, 33))]
    out = t().qr_batched([A for A in As], check_info=False)
    for k in (0, 2):
        check_fp64(big[k][:, :(10, 20, 33)[k]].copy(), out[k][0].cpu().numpy(), out[k][1].cpu().numpy())
    with pytest.raises(torch.linalg.LinAlgError, match="matrices \\[1\\]"):
        t().qr_batched(As)


def test_batched_graph_capture_replays():
    """One call captured in a graph: every replay (with eager work and syncs in between) matches
    the eager result bit for bit."""
    mats = mixed_batch(13, 24, 2000, 30_000, [4, 8, 16, 32, 64])
    As = [torch.from_numpy(A).to(DEV) for A in mats]
    plan = t().BatchPlan([tuple(A.shape) for A in As])
    Qs = [torch.empty_like(A) for A in As]
    Rs = [torch.empty((A.shape[1], A.shape[1]), dtype=A.dtype, device=DEV) for A in As]
    ws = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device=DEV)
    info = torch.zeros(len(As), dtype=torch.int32, device=DEV)
    P = t().BatchPlan.pointers
    pa, pq, pr = P(As, DEV), P(Qs, DEV), P(Rs, DEV)
    plan.run(pa, pq, pr, ws, info)
    torch.cuda.synchronize()
    refQ = [q.clone() for q in Qs]
    refR = [r.clone() for r in Rs]
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        plan.run(pa, pq, pr, ws, info)
    for rep in range(3):
        for q in Qs:
            q.fill_(float("nan"))
        ws.fill_(255)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert all(torch.equal(a, b) for a, b in zip(Qs, refQ)), rep
        assert all(torch.equal(a, b) for a, b in zip(Rs, refR)), rep
        assert int(torch.count_nonzero(info)) == 0
    check_fp64(mats[0], Qs[0].cpu().numpy(), Rs[0].cpu().numpy())


def test_batch512_full_size():
    """The 512-matrix workload (m ~ U{2,000..200,000}, n ~ U{4,...,64}) in FP64: every matrix
    checked for orthogonality and residual on the GPU, 12 sampled matrices against the oracle."""
    shapes = workloads.batch_shapes()
    mats = workloads.batch_matrices(shapes)
    As = [torch.from_numpy(A).to(DEV) for A in mats]
    out = t().qr_batched(As)
    for A, (Q, R) in zip(As, out):
        n = A.shape[1]
        # ||Q^T Q - I||_2 from the n x n Gram; ||A - QR||_F (>= the 2-norm) over ||R||_2 = ||A||_2
        G = (Q.T @ Q).cpu().numpy()
        Rh = R.cpu().numpy()
        orth = np.linalg.norm(G - np.eye(n), 2)
        res = float(torch.linalg.vector_norm(A - Q @ R)) / np.linalg.norm(Rh, 2)
        assert orth <= 1e-12 and res <= 1e-12, (orth, res)
        assert np.all(np.diag(Rh) > 0) and np.all(np.tril(Rh, -1) == 0)
    for k in np.random.default_rng(0).choice(len(mats), 12, replace=False):
        check_fp64(mats[k], out[k][0].cpu().numpy(), out[k][1].cpu().numpy())
