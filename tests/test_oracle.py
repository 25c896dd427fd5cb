"""Pins for the CPU oracle: each check ties it to something other than itself.

* exact hand-built factorizations (tests/golden, Sec. I problem statement and Sec. III-B SVD);
* brute force on tiny inputs in 50-digit arithmetic (modified Gram-Schmidt, and the Cholesky
  factor of an exactly accumulated A^T A, which equals R by Sec. II-A's derivation);
* closed forms (n = 1, orthonormal A, A = [R0; 0]); a library special case (one block = LAPACK QR
  after the sign fix); invariances (scaling, column scaling, row permutation, block size / tree
  shape: Sec. II-B notes that the reduction tree does not change R);
* the paper's stability claim for direct TSQR (Sec. IV: ||Q^T Q - I|| around 1e-15 at every
  condition number tested) and its success metrics (Sec. I-B);
* central finite differences for the adjoints.
"""
import json
import os

import mpmath
import numpy as np
import pytest
from fractions import Fraction

import oracle
import workloads

GOLD = os.path.join(os.path.dirname(__file__), "golden", "qr_exact_small.json")
EPS = np.finfo(np.float64).eps


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


# ----------------------------------------------------------------------------- golden fixtures
def test_golden_exact_qr():
    d = json.load(open(GOLD))
    for c in d["cases"]:
        A, Q, R = (np.array(c[k], dtype=np.float64) for k in ("A", "Q", "R"))
        for br in (A.shape[1], A.shape[0]):
            Qo, Ro = oracle.tsqr(A, block_rows=br)
            assert np.abs(Ro - R).max() <= 8 * EPS * np.abs(R).max(), c["name"]
            assert np.abs(Qo - Q).max() <= 8 * EPS, c["name"]


def test_golden_exact_svd():
    d = json.load(open(GOLD))
    for c in d["svd_cases"]:
        Q0, s, V0 = (np.array(c[k], dtype=np.float64) for k in ("Q0", "s", "V0"))
        A = Q0 @ np.diag(s) @ V0.T
        U, S, V = oracle.tsqr_svd(A, block_rows=2)
        assert np.abs(S - np.array(c["S"])).max() <= 16 * EPS * s.max()
        assert np.abs(V - np.array(c["V"])).max() <= 1e-14
        assert np.abs(U - np.array(c["U"])).max() <= 1e-14


# ----------------------------------------------------------------------------- brute force
def mgs_mp(A, dps=50):
    """Modified Gram-Schmidt in 50-digit arithmetic: the unique Q, R with diag(R) > 0."""
    with mpmath.workdps(dps):
        m, n = A.shape
        V = [[mpmath.mpf(float(A[i, j])) for i in range(m)] for j in range(n)]
        R = [[mpmath.mpf(0)] * n for _ in range(n)]
        Q = []
        for j in range(n):
            v = V[j]
            for i in range(j):
                r = mpmath.fsum(Q[i][k] * v[k] for k in range(m))
                R[i][j] += r
                v = [v[k] - r * Q[i][k] for k in range(m)]
            # second pass (reorthogonalisation) keeps MGS exact to working precision
            for i in range(j):
                r = mpmath.fsum(Q[i][k] * v[k] for k in range(m))
                R[i][j] += r
                v = [v[k] - r * Q[i][k] for k in range(m)]
            nv = mpmath.sqrt(mpmath.fsum(x * x for x in v))
            R[j][j] = nv
            Q.append([x / nv for x in v])
        Qf = np.array([[float(Q[j][i]) for j in range(n)] for i in range(m)])
        Rf = np.array([[float(R[i][j]) for j in range(n)] for i in range(n)])
    return Qf, Rf


def chol_exact_gram(A, dps=50):
    """R from A^T A = R^T R (Sec. II-A): Gram accumulated exactly in rationals, then Cholesky in
    50-digit arithmetic."""
    m, n = A.shape
    F = [[Fraction(float(A[i, j])) for j in range(n)] for i in range(m)]
    G = [[sum(F[k][i] * F[k][j] for k in range(m)) for j in range(n)] for i in range(n)]
    with mpmath.workdps(dps):
        Gm = mpmath.matrix(n, n)
        for i in range(n):
            for j in range(n):
                Gm[i, j] = mpmath.mpf(G[i][j].numerator) / G[i][j].denominator
        L = mpmath.cholesky(Gm)
        return np.array([[float(L[j, i]) for j in range(n)] for i in range(n)])


@pytest.mark.parametrize("m,n,br,seed", [(12, 3, 4, 1), (40, 5, 9, 2), (64, 8, 16, 3),
                                         (33, 7, 10, 4), (9, 1, 3, 5)])
def test_brute_force_mgs(m, n, br, seed):
    A = np.random.default_rng(seed).standard_normal((m, n))
    Qb, Rb = mgs_mp(A)
    Q, R = oracle.tsqr(A, block_rows=br)
    assert rel(R, Rb) <= 1e-14
    assert np.abs(Q - Qb).max() <= 1e-14 * np.sqrt(m)


@pytest.mark.parametrize("m,n,br,seed", [(20, 4, 5, 11), (48, 6, 12, 12)])
def test_brute_force_cholesky_of_exact_gram(m, n, br, seed):
    A = np.random.default_rng(seed).standard_normal((m, n))
    R = oracle.tsqr(A, block_rows=br, want_q=False)
    assert rel(R, chol_exact_gram(A)) <= 1e-14


# ----------------------------------------------------------------------------- closed forms
def test_closed_form_single_column():
    a = np.random.default_rng(7).standard_normal((1000, 1))
    Q, R = oracle.tsqr(a, block_rows=64)
    nrm = np.sqrt(np.sum(a[:, 0] ** 2))
    assert abs(R[0, 0] - nrm) <= 4 * EPS * nrm
    assert np.abs(Q[:, 0] - a[:, 0] / nrm).max() <= 4 * EPS


def test_closed_form_orthonormal_input():
    Q0 = np.linalg.qr(np.random.default_rng(8).standard_normal((500, 6)))[0]
    Q, R = oracle.tsqr(Q0, block_rows=50)
    assert np.abs(R - np.eye(6)).max() <= 1e-14
    # columns of Q0 may carry either sign; R = I forces Q = Q0 exactly
    assert np.abs(Q - Q0).max() <= 1e-14


def test_closed_form_triangular_stack():
    rng = np.random.default_rng(9)
    R0 = np.triu(rng.standard_normal((5, 5)))
    R0[np.diag_indices(5)] = np.abs(R0[np.diag_indices(5)]) + 0.5
    A = np.vstack([R0, np.zeros((20, 5))])
    Q, R = oracle.tsqr(A, block_rows=7)
    assert rel(R, R0) <= 1e-15
    E = np.zeros((25, 5)); E[:5] = np.eye(5)
    assert np.abs(Q - E).max() <= 1e-15


def test_library_special_case_single_block():
    A = np.random.default_rng(10).standard_normal((300, 12))
    Q, R = oracle.householder_qr(A)
    Ql, Rl = np.linalg.qr(A)
    d = np.sign(np.diag(Rl))
    assert rel(R, d[:, None] * Rl) <= 1e-14
    assert np.abs(Q - Ql * d[None, :]).max() <= 1e-14


# ----------------------------------------------------------------------------- invariances
def test_invariances():
    rng = np.random.default_rng(12)
    A = rng.standard_normal((400, 9))
    Q, R = oracle.tsqr(A, block_rows=37)
    Qa, Ra = oracle.tsqr(3.5 * A, block_rows=37)
    assert rel(Ra, 3.5 * R) <= 1e-14 and np.abs(Qa - Q).max() <= 1e-14
    D = np.exp(rng.standard_normal(9))
    Qd, Rd = oracle.tsqr(A * D[None, :], block_rows=37)
    assert rel(Rd, R * D[None, :]) <= 1e-14 and np.abs(Qd - Q).max() <= 1e-13
    P = rng.permutation(400)
    Qp, Rp = oracle.tsqr(A[P], block_rows=37)
    assert rel(Rp, R) <= 1e-14 and np.abs(Qp - Q[P]).max() <= 1e-13


@pytest.mark.parametrize("blocks", [(9, 40, 400), (10, 64, 1000)])
def test_block_size_and_tree_invariance(blocks):
    """Sec. II-B: the shape of the reduction tree does not change R (and, with the sign fix, Q)."""
    A = np.random.default_rng(13).standard_normal((1000, 9))
    ref_q, ref_r = oracle.tsqr(A, block_rows=blocks[0])
    for br in blocks[1:]:
        Q, R = oracle.tsqr(A, block_rows=br)
        assert rel(R, ref_r) <= 1e-14
        assert np.abs(Q - ref_q).max() <= 1e-14


def test_partition_merges_short_tail():
    st = oracle.partition(1000, 10, 300)   # 3 blocks of 300, tail 100 >= n -> own block
    assert list(st) == [0, 300, 600, 900, 1000]
    st = oracle.partition(905, 10, 300)    # tail 5 < n -> merged
    assert list(st) == [0, 300, 600, 905]
    st = oracle.partition(50, 10, 300)
    assert list(st) == [0, 50]


def test_q2_block_layout():
    """Sec. III-B: the k-th n-row block of the step-2 Q pairs with the k-th row block: stacking
    the local factors gives [R_1; ...; R_P] = Q2 R, so Q2_k R is block k's own R factor, which
    LAPACK computes independently up to the signs of its rows."""
    A = np.random.default_rng(14).standard_normal((120, 4))
    Q, R, Q2 = oracle.tsqr(A, block_rows=30, want_q2=True)
    assert Q2.shape == (16, 4)
    assert np.abs(Q2.T @ Q2 - np.eye(4)).max() <= 1e-14
    for k in range(4):
        Rk = np.linalg.qr(A[30 * k:30 * (k + 1)], mode="r")
        got = Q2[4 * k:4 * (k + 1)] @ R
        d = np.sign(np.diag(got)) * np.sign(np.diag(Rk))      # row signs are free
        assert np.abs(got - d[:, None] * Rk).max() <= 1e-13 * np.abs(Rk).max()
        # and block k of A is reproduced by its rows of Q
        assert np.abs(A[30 * k:30 * (k + 1)] - Q[30 * k:30 * (k + 1)] @ R).max() <= 1e-13


# ----------------------------------------------------------------------------- SVD
def test_svd_known_spectrum():
    rng = np.random.default_rng(15)
    Q0 = np.linalg.qr(rng.standard_normal((600, 8)))[0]
    V0 = workloads.haar_orthogonal(8, rng)
    s = np.logspace(0, -6, 8)
    A = Q0 @ np.diag(s) @ V0.T
    U, S, V = oracle.tsqr_svd(A, block_rows=64)
    assert np.abs(S - s).max() <= 1e-14
    # align gauge of the exact factors and compare
    g = np.sign(V0[np.argmax(np.abs(V0), axis=0), np.arange(8)])
    assert np.abs(V - V0 * g).max() <= 1e-9   # gaps of 10^(6/7): singular vectors to ~eps/gap
    assert np.abs(U - Q0 * g).max() <= 1e-9
    assert oracle.metric_svd_backward(A, U, S, V) <= 1e-15 * 20


def test_svd_matches_lapack_tiny():
    A = np.random.default_rng(16).standard_normal((30, 5))
    U, S, V = oracle.tsqr_svd(A, block_rows=8)
    Ul, Sl, Vtl = np.linalg.svd(A, full_matrices=False)
    assert np.abs(S - Sl).max() <= 1e-14 * Sl[0]
    Vl = Vtl.T
    g = np.sign(Vl[np.argmax(np.abs(Vl), axis=0), np.arange(5)])
    assert np.abs(V - Vl * g).max() <= 1e-13
    assert np.abs(U - Ul * g).max() <= 1e-13


# ----------------------------------------------------------------------------- metrics / paper claims
def test_metric_orth_against_high_precision():
    rng = np.random.default_rng(17)
    Q = np.linalg.qr(rng.standard_normal((200, 4)))[0]
    Q[3, 1] += 1e-9          # a planted departure from orthonormality
    with mpmath.workdps(40):
        G = mpmath.matrix(4, 4)
        for i in range(4):
            for j in range(4):
                G[i, j] = mpmath.fsum(mpmath.mpf(float(Q[k, i])) * mpmath.mpf(float(Q[k, j]))
                                      for k in range(200)) - (1 if i == j else 0)
        ev = mpmath.eigsy(G)[0]
        ref = max(abs(float(x)) for x in ev)
    assert abs(oracle.metric_orth(Q) - ref) <= 1e-6 * ref


def test_metric_detects_planted_error():
    A = np.random.default_rng(18).standard_normal((2000, 6))
    Q, R = oracle.tsqr(A, block_rows=100)
    assert oracle.metric_backward(A, Q, R) <= 1e-15 * 10
    Rbad = R.copy(); Rbad[1, 3] *= 1 + 1e-8
    assert oracle.metric_backward(A, Q, Rbad) >= 1e-10
    Qbad = Q.copy(); Qbad[:, 2] *= 1 + 1e-9
    assert oracle.metric_orth(Qbad) >= 1e-9


@pytest.mark.parametrize("log_cond", [0, 4, 8, 12, 16])
def test_paper_stability_claim_direct_tsqr(log_cond):
    """Sec. IV: direct TSQR keeps ||Q^T Q - I||_2 around 1e-15 at every condition number, and the
    backward error is O(eps) for every algorithm (Sec. I-B)."""
    A, s, V = workloads.spectrum_matrix(20_000, 10, float(log_cond), seed=19 + log_cond)
    Q, R = oracle.tsqr(A, block_rows=1000)
    assert oracle.metric_orth(Q) <= 1e-14
    assert oracle.metric_backward(A, Q, R) <= 1e-14
    assert np.all(np.diag(R) > 0)


def test_r_is_upper_triangular_positive_diag():
    A = workloads.config_matrix("qr-small", m=5000)
    Q, R = oracle.tsqr(A, block_rows=1000)
    assert np.all(np.tril(R, -1) == 0) and np.all(np.diag(R) > 0)


# ----------------------------------------------------------------------------- adjoints vs FD
def _fd_grad(f, A, h=1e-6):
    G = np.zeros_like(A)
    for idx in np.ndindex(*A.shape):
        step = h * max(1.0, abs(A[idx]))
        Ap = A.copy(); Ap[idx] += step
        Am = A.copy(); Am[idx] -= step
        G[idx] = (f(Ap) - f(Am)) / (2 * step)
    return G


def test_qr_backward_matches_fd():
    rng = np.random.default_rng(20)
    A = rng.standard_normal((40, 5))
    dQ = rng.standard_normal((40, 5)); dR = np.triu(rng.standard_normal((5, 5)))

    def loss(X):
        Q, R = oracle.tsqr(X, block_rows=10)
        return np.sum(dQ * Q) + np.sum(dR * R)

    Q, R = oracle.tsqr(A, block_rows=10)
    g = oracle.qr_backward(Q, R, dQ, dR)
    assert rel(g, _fd_grad(loss, A)) <= 1e-7
    # each cotangent alone
    gq = oracle.qr_backward(Q, R, dQ, None)
    gr = oracle.qr_backward(Q, R, None, dR)
    assert rel(gq + gr, g) <= 1e-14


def test_svd_backward_matches_fd():
    rng = np.random.default_rng(21)
    A = rng.standard_normal((30, 4))
    dU = rng.standard_normal((30, 4)); dS = rng.standard_normal(4); dV = rng.standard_normal((4, 4))

    def loss(X):
        U, S, V = oracle.tsqr_svd(X, block_rows=10)
        return np.sum(dU * U) + np.sum(dS * S) + np.sum(dV * V)

    U, S, V = oracle.tsqr_svd(A, block_rows=10)
    g = oracle.svd_backward(U, S, V, dU, dS, dV)
    assert rel(g, _fd_grad(loss, A)) <= 1e-6
    # the S-only adjoint is U diag(dS) V^T exactly
    gs = oracle.svd_backward(U, S, V, None, dS, None)
    assert rel(gs, U @ np.diag(dS) @ V.T) <= 1e-14


def test_metrics_report_nan_for_nonfinite_input():
    Q = np.linalg.qr(np.random.default_rng(22).standard_normal((100, 3)))[0]
    Q[5, 1] = np.nan
    assert np.isnan(oracle.metric_orth(Q))
    A = np.random.default_rng(23).standard_normal((100, 3))
    assert np.isnan(oracle.metric_backward(A, Q, np.eye(3)))



# ----------------------------------------------------------------------------- comparison methods
def test_cholesky_qr_library_special_case():
    """Sec. II-A: R^T is the Cholesky factor of A^T A, and Q = A R^{-1} (Sec. II-C)."""
    A = np.random.default_rng(41).standard_normal((500, 6))
    Q, R = oracle.indirect_qr(A, "cholqr", block_rows=64)
    L = np.linalg.cholesky(A.T @ A)
    assert rel(R, L.T) <= 1e-13
    assert np.abs(Q - A @ np.linalg.inv(L.T)).max() <= 1e-13


@pytest.mark.parametrize("m,n,seed", [(20, 4, 42), (48, 6, 43)])
def test_cholesky_qr_matches_exact_gram(m, n, seed):
    A = np.random.default_rng(seed).standard_normal((m, n))
    Q, R = oracle.indirect_qr(A, "cholqr", block_rows=7)
    assert rel(R, chol_exact_gram(A)) <= 1e-13


def test_indirect_q_is_a_times_the_inverse():
    """Sec. II-B / II-C: the indirect method's R is the TSQR R, its Q is A times R^{-1}."""
    A = np.random.default_rng(44).standard_normal((400, 5))
    Q, R = oracle.indirect_qr(A, "indirect", block_rows=50)
    Rt = oracle.tsqr(A, block_rows=50, want_q=False)
    assert np.array_equal(R, Rt)
    assert np.abs(Q - A @ np.linalg.inv(R)).max() <= 1e-13


@pytest.mark.parametrize("method", ["cholqr", "indirect"])
def test_refinement_is_the_qr_repeated_on_q(method):
    """Sec. I: iterative refinement repeats the QR on the computed Q: Q1 R1 = A, Q R2 = Q1,
    R = R2 R1."""
    A = workloads.spectrum_matrix(3000, 6, 5.0, seed=45)[0]
    Q, R = oracle.indirect_qr(A, method + "_ir", block_rows=500)
    Q1, R1 = oracle.indirect_qr(A, method, block_rows=500)
    Q2, R2 = oracle.indirect_qr(Q1, method, block_rows=500)
    assert np.array_equal(Q, Q2)
    assert rel(R, R2 @ R1) <= 1e-15


@pytest.mark.parametrize("log_cond", list(range(0, 17)))
def test_stability_experiment_claims(log_cond):
    """Sec. IV on 20,000 x 10 matrices with s = logspace(0, -c, 10): direct TSQR stays at ~1e-15
    orthogonality; Q = A R^{-1} loses orthogonality in proportion to kappa (indirect TSQR) or
    kappa^2 (Cholesky QR); Cholesky QR fails from kappa = 1e8 on; one step of iterative
    refinement brings the indirect methods back to ~1e-15 where their first Q is still of full
    numerical rank; every method that completes has an O(eps) backward error (Sec. I-B)."""
    c = log_cond
    A = workloads.spectrum_matrix(20_000, 10, float(c), seed=500 + c)[0]
    normA = oracle.norm2(A)
    kappa = 10.0 ** c
    u = EPS / 2
    Qd, Rd = oracle.tsqr(A, block_rows=1000)
    assert oracle.metric_orth(Qd) <= 1e-14
    res = {m: oracle.indirect_qr(A, m) for m in ("cholqr", "cholqr_ir", "indirect", "indirect_ir")}
    orth = {m: (oracle.metric_orth(r[0]) if r is not None else np.inf) for m, r in res.items()}
    for m, r in res.items():
        if r is not None:
            assert oracle.metric_backward(A, r[0], r[1], normA) <= 1e-14, m
    if 4 <= c <= 13:
        assert 1e-2 * u * kappa <= orth["indirect"] <= 1e2 * u * kappa
    if c <= 2:
        assert orth["cholqr"] <= 1e-12
    elif c <= 6:
        assert 1e-3 * u * kappa ** 2 <= orth["cholqr"] <= 1e3 * u * kappa ** 2
    elif c >= 8:
        assert orth["cholqr"] >= 0.1          # fails: breakdown (inf) or no orthogonality left
    if c <= 7:
        assert orth["cholqr_ir"] <= 1e-14
    if c <= 15:
        assert orth["indirect_ir"] <= 1e-14
