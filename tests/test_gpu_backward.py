"""GPU parity of the differentiation form: tsqr_qr_backward / tsqr_svd_backward through the C ABI
against the oracle's closed-form adjoints, central finite differences through the GPU forward,
and the torch.autograd.Function wrappers.

Gates: QR adjoint relative (Frobenius) <= 1e-12 against the oracle; SVD adjoint <= 1e-9 (the
1,000,000 x 100 Gaussian has singular gaps of 1e-2 at s ~ 1e3, so the 1/(s_j^2 - s_i^2) factors
amplify rounding by ~1e4 over the QR case); finite differences <= 1e-6 relative.
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


def to_gpu(x):
    return None if x is None else torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def cot(m, n, seed):
    return workloads.cotangents(m, n, seed=seed)


# --------------------------------------------------------------------- QR adjoint vs oracle
@pytest.mark.parametrize("m,n", [(2000, 8), (3001, 3), (5000, 50), (10_000, 64), (20_000, 100),
                                 (700, 1), (128, 128)])
def test_qr_backward_vs_oracle(m, n):
    A = np.random.default_rng(500 + n).standard_normal((m, n))
    c = cot(m, n, 900 + n)
    Qo, Ro = oracle.tsqr(A, block_rows=1000)
    ref = oracle.qr_backward(Qo, Ro, c["dQ"], c["dR"])
    dA = t().qr_backward(to_gpu(A), to_gpu(c["dQ"]), to_gpu(c["dR"])).cpu().numpy()
    assert rel(dA, ref) <= 1e-12, rel(dA, ref)


@pytest.mark.parametrize("which", ["dQ", "dR"])
def test_qr_backward_single_cotangent(which):
    m, n = 9000, 20
    A = np.random.default_rng(3).standard_normal((m, n))
    c = cot(m, n, 77)
    dQ = c["dQ"] if which == "dQ" else None
    dR = c["dR"] if which == "dR" else None
    Qo, Ro = oracle.tsqr(A, block_rows=1000)
    ref = oracle.qr_backward(Qo, Ro, dQ, dR)
    dA = t().qr_backward(to_gpu(A), to_gpu(dQ), to_gpu(dR)).cpu().numpy()
    assert rel(dA, ref) <= 1e-12


def test_qr_backward_ignores_lower_triangle_of_dR():
    m, n = 4000, 12
    A = np.random.default_rng(4).standard_normal((m, n))
    c = cot(m, n, 5)
    full = c["dR"] + np.tril(np.random.default_rng(6).standard_normal((n, n)), -1)
    Ad = to_gpu(A)
    d1 = t().qr_backward(Ad, to_gpu(c["dQ"]), to_gpu(c["dR"]))
    d2 = t().qr_backward(Ad, to_gpu(c["dQ"]), to_gpu(full))
    assert torch.equal(d1, d2)


def test_qr_backward_strided_cotangent_and_output():
    m, n = 6000, 10
    A = np.random.default_rng(8).standard_normal((m, n))
    c = cot(m, n, 9)
    dQbig = to_gpu(np.hstack([c["dQ"], np.full((m, 3), 5.0)]))
    out = torch.full((m, n + 2), 7.0, dtype=torch.float64, device=DEV)
    dA = t().qr_backward(to_gpu(A), dQbig[:, :n], to_gpu(c["dR"]), out=out[:, :n])
    torch.cuda.synchronize()
    assert torch.all(out[:, n:] == 7.0)
    Qo, Ro = oracle.tsqr(A, block_rows=1000)
    assert rel(dA.cpu().numpy(), oracle.qr_backward(Qo, Ro, c["dQ"], c["dR"])) <= 1e-12


# --------------------------------------------------------------------- SVD adjoint vs oracle
# n = 1 and n = 128: the narrowest and widest n x n middle steps (one work-group per row of W2)
@pytest.mark.parametrize("m,n,log_cond", [(2000, 8, 2.0), (5000, 50, 3.0), (3001, 3, 1.0),
                                          (20_000, 100, 2.0), (4000, 30, None), (700, 1, None),
                                          (3000, 128, 1.0)])
def test_svd_backward_vs_oracle(m, n, log_cond):
    if log_cond is None:
        A = np.random.default_rng(600 + n).standard_normal((m, n))
    else:
        A = workloads.spectrum_matrix(m, n, log_cond, seed=600 + n)[0]
    c = cot(m, n, 950 + n)
    Uo, So, Vo = oracle.tsqr_svd(A, block_rows=1000)
    ref = oracle.svd_backward(Uo, So, Vo, c["dU"], c["dS"], c["dV"])
    dA = t().svd_backward(to_gpu(A), to_gpu(c["dU"]), to_gpu(c["dS"]), to_gpu(c["dV"]))
    assert rel(dA.cpu().numpy(), ref) <= 1e-9, rel(dA.cpu().numpy(), ref)


@pytest.mark.parametrize("which", ["dU", "dS", "dV"])
def test_svd_backward_single_cotangent(which):
    m, n = 8000, 16
    A = workloads.spectrum_matrix(m, n, 2.0, seed=12)[0]
    c = cot(m, n, 13)
    args = {k: (c[k] if k == which else None) for k in ("dU", "dS", "dV")}
    Uo, So, Vo = oracle.tsqr_svd(A, block_rows=1000)
    ref = oracle.svd_backward(Uo, So, Vo, args["dU"], args["dS"], args["dV"])
    dA = t().svd_backward(to_gpu(A), *(to_gpu(args[k]) for k in ("dU", "dS", "dV")))
    assert rel(dA.cpu().numpy(), ref) <= 1e-10


# --------------------------------------------------------------------- finite differences
def _fd_check(loss, grad, A, seed, h=1e-5, ndir=4):
    g = np.random.default_rng(seed)
    for _ in range(ndir):
        E = g.standard_normal(A.shape)
        E /= np.linalg.norm(E)
        fd = (loss(A + h * E) - loss(A - h * E)) / (2 * h)
        an = float(np.sum(grad * E))
        assert abs(fd - an) <= 1e-6 * max(np.linalg.norm(grad), 1.0), (fd, an)


def test_qr_backward_finite_differences():
    """Central FD on the 2,000 x 8 slice of the 1,000,000 x 100 gradient workload."""
    A = workloads.config_matrix("grad-c100", m=2000)[:, :8].copy()
    c = cot(2000, 8, workloads.SEEDS["grad-c100"])
    dQd, dRd = to_gpu(c["dQ"]), to_gpu(c["dR"])

    def loss(X):
        Q, R = t().qr(to_gpu(X))
        return float(torch.sum(Q * dQd) + torch.sum(R * dRd))
    grad = t().qr_backward(to_gpu(A), dQd, dRd).cpu().numpy()
    _fd_check(loss, grad, A, 1)


def test_svd_backward_finite_differences():
    A = workloads.config_matrix("grad-c100", m=2000)[:, :8].copy()
    c = cot(2000, 8, workloads.SEEDS["grad-c100"])
    dU, dS, dV = to_gpu(c["dU"]), to_gpu(c["dS"]), to_gpu(c["dV"])

    def loss(X):
        U, S, V = t().svd(to_gpu(X))
        return float(torch.sum(U * dU) + torch.sum(S * dS) + torch.sum(V * dV))
    grad = t().svd_backward(to_gpu(A), dU, dS, dV).cpu().numpy()
    _fd_check(loss, grad, A, 2)


# --------------------------------------------------------------------- autograd wrappers
def test_autograd_qr_matches_entry_point():
    m, n = 3000, 9
    A = to_gpu(np.random.default_rng(21).standard_normal((m, n))).requires_grad_(True)
    c = cot(m, n, 22)
    Q, R = t().qr_autograd(A)
    (torch.sum(Q * to_gpu(c["dQ"])) + torch.sum(R * to_gpu(c["dR"]))).backward()
    ref = t().qr_backward(A.detach(), to_gpu(c["dQ"]), to_gpu(c["dR"]))
    assert torch.equal(A.grad, ref)


def test_autograd_svd_matches_entry_point():
    m, n = 3000, 9
    A = to_gpu(workloads.spectrum_matrix(m, n, 1.5, seed=23)[0]).requires_grad_(True)
    c = cot(m, n, 24)
    U, S, V = t().svd_autograd(A)
    (torch.sum(U * to_gpu(c["dU"])) + torch.sum(S * to_gpu(c["dS"]))
     + torch.sum(V * to_gpu(c["dV"]))).backward()
    ref = t().svd_backward(A.detach(), to_gpu(c["dU"]), to_gpu(c["dS"]), to_gpu(c["dV"]))
    assert torch.equal(A.grad, ref)


def test_autograd_gradcheck_small():
    A = to_gpu(np.random.default_rng(31).standard_normal((300, 5))).requires_grad_(True)
    assert torch.autograd.gradcheck(lambda X: t().qr_autograd(X), (A,), eps=1e-6, atol=1e-6)
    B = to_gpu(workloads.spectrum_matrix(300, 5, 1.0, seed=32)[0]).requires_grad_(True)
    assert torch.autograd.gradcheck(lambda X: t().svd_autograd(X), (B,), eps=1e-6, atol=1e-6)


def test_backward_rank_deficient_raises():
    A = np.random.default_rng(40).standard_normal((3000, 6))
    A[:, 2] = 0.0
    c = cot(3000, 6, 41)
    with pytest.raises(torch.linalg.LinAlgError):
        t().qr_backward(to_gpu(A), to_gpu(c["dQ"]), to_gpu(c["dR"]))


# --------------------------------------------------------------------- full gradient workload
@pytest.fixture(scope="module")
def c5():
    A = workloads.config_matrix("grad-c100")
    m, n = A.shape
    c = workloads.cotangents(m, n)
    U, S, V, Q, R = oracle.tsqr_svd(A, block_rows=8192, want_qr=True)
    return A, c, (U, S, V, Q, R)


def test_qr_backward_full_size(c5):
    """1,000,000 x 100 N(0,1), every element of dA against the oracle (<= 1e-12)."""
    A, c, (U, S, V, Q, R) = c5
    ref = oracle.qr_backward(Q, R, c["dQ"], c["dR"])
    dA = t().qr_backward(to_gpu(A), to_gpu(c["dQ"]), to_gpu(c["dR"])).cpu().numpy()
    assert rel(dA, ref) <= 1e-12, rel(dA, ref)


def test_svd_backward_full_size(c5):
    """The SVD adjoint on the same input (gate 1e-9: singular gaps of ~1e-2 at s ~ 1e3)."""
    A, c, (U, S, V, Q, R) = c5
    ref = oracle.svd_backward(U, S, V, c["dU"], c["dS"], c["dV"])
    dA = t().svd_backward(to_gpu(A), to_gpu(c["dU"]), to_gpu(c["dS"]), to_gpu(c["dV"]))
    assert rel(dA.cpu().numpy(), ref) <= 1e-9, rel(dA.cpu().numpy(), ref)
