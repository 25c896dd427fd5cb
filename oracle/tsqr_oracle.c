/*
 * Reference oracle for direct TSQR (Benson, Gleich & Demmel, "Direct QR factorizations for
 * tall-and-skinny matrices in MapReduce architectures").
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, FP64 CPU definition that the GPU
 * library is checked against.  Only the test-suite, the smoke check and the CPU-baseline leg of
 * the benchmark may load it.  It shares no code, header or constant with the GPU library.
 *
 * Everything is written as plain loops over row-major matrices (element (i,j) of X lives at
 * X[i*ldx + j]).  There is no blocking, fusion or reordering beyond what the paper's steps state;
 * OpenMP only runs independent row blocks (steps 1 and 3) and independent rows of the metrics
 * concurrently, which does not change any result.
 *
 * Paper anchors:
 *   Sec. I          problem statement: thin QR A = QR of a full-rank m x n A, m >> n.
 *   Sec. I-B        success metrics ||A - QR||_2/||R||_2 and ||Q^T Q - I||_2.
 *   Sec. III-A      textbook Householder QR; each step updates A <- A - 2 v (A^T v)^T with a unit v.
 *   Sec. III-B      direct TSQR: step 1 local QR per row block, step 2 QR of the stacked R_i
 *                   (the k-th n-row block of that Q is the block for the k-th map task), step 3
 *                   Q_i = Q1_i * Q2_i;  SVD variant: SVD of R, then U = Q U_R.
 *   Sec. II-A       Cholesky QR: A^T A summed from the row blocks' A_p^T A_p (Alg. 1), R^T = its
 *                   Cholesky factor.
 *   Sec. II-B/II-C  indirect TSQR: R from the stacked-R reduction alone, Q = A R^{-1} by the
 *                   explicit inverse of R; iterative refinement = the same QR repeated once on the
 *                   computed Q (Sec. I).  These are the comparison methods of the stability
 *                   experiment of Sec. IV.
 * The adjoints (qr/svd backward) are not in the paper; they follow the published closed forms
 * named at each function.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OK 0
#define ERR_ARG 1
#define ERR_SHAPE 2
#define ERR_NOMEM 3

static int set_threads(int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
    return omp_get_max_threads();
#else
    (void)nthreads;
    return 1;
#endif
}

int oracle_max_threads(int nthreads) { return set_threads(nthreads); }

/* ||x||_2 of a strided vector with scaling, so that squaring neither overflows nor underflows. */
static double scaled_norm(int64_t len, const double *x, int64_t stride)
{
    double scale = 0.0;
    for (int64_t i = 0; i < len; ++i) {
        double a = fabs(x[i * stride]);
        if (a > scale) scale = a;
    }
    if (scale == 0.0) return 0.0;
    double ss = 0.0;
    for (int64_t i = 0; i < len; ++i) {
        double t = x[i * stride] / scale;
        ss += t * t;
    }
    return scale * sqrt(ss);
}

/*
 * Householder QR of a b x n block W (row-major, ld = n, b >= n), in place (Sec. III-A).
 * For column k: x = W[k:,k]; v = x + s ||x|| e_1 with s = sign(x_1) and sign(0) = +1; v is
 * normalised to unit length and W[k:,k:] -= 2 v (v^T W[k:,k:]).  The unit reflectors are kept in
 * V (b x n, ld = n; column k holds v_k in rows k..b-1).  A zero x means no reflection (v = 0).
 * On exit the upper triangle of W[0:n,:] is R (diagonal of either sign).
 */
static void householder_inplace(int64_t b, int64_t n, double *W, double *V)
{
    memset(V, 0, sizeof(double) * (size_t)(b * n));
    for (int64_t k = 0; k < n; ++k) {
        double nx = scaled_norm(b - k, &W[k * n + k], n);
        if (nx == 0.0) continue;
        double s = (W[k * n + k] >= 0.0) ? 1.0 : -1.0;
        for (int64_t i = k; i < b; ++i) V[i * n + k] = W[i * n + k];
        V[k * n + k] += s * nx;
        double nv = scaled_norm(b - k, &V[k * n + k], n);
        for (int64_t i = k; i < b; ++i) V[i * n + k] /= nv;
        /* W[k:,k:] -= 2 v (v^T W[k:,k:]) */
        for (int64_t j = k; j < n; ++j) {
            double dot = 0.0;
            for (int64_t i = k; i < b; ++i) dot += V[i * n + k] * W[i * n + j];
            dot *= 2.0;
            for (int64_t i = k; i < b; ++i) W[i * n + j] -= dot * V[i * n + k];
        }
        /* the annihilated part is exactly zero in exact arithmetic */
        for (int64_t i = k + 1; i < b; ++i) W[i * n + k] = 0.0;
    }
}

/* Q1 = H_1 ... H_n [I_n; 0]  (b x n), formed by applying the reflectors in reverse order. */
static void form_q_from_reflectors(int64_t b, int64_t n, const double *V, double *Q1)
{
    memset(Q1, 0, sizeof(double) * (size_t)(b * n));
    for (int64_t i = 0; i < n; ++i) Q1[i * n + i] = 1.0;
    for (int64_t k = n - 1; k >= 0; --k) {
        for (int64_t j = 0; j < n; ++j) {
            double dot = 0.0;
            for (int64_t i = k; i < b; ++i) dot += V[i * n + k] * Q1[i * n + j];
            dot *= 2.0;
            if (dot == 0.0) continue;
            for (int64_t i = k; i < b; ++i) Q1[i * n + j] -= dot * V[i * n + k];
        }
    }
}

/*
 * Plain single-block Householder QR (Sec. III-A), with the sign of diag(R) made positive
 * (R = D R~, Q = Q~ D; D = diag(sign(R~_jj)), sign(0) = +1).  Q may be NULL.
 */
int oracle_householder_qr(int64_t m, int64_t n, const double *A, int64_t lda, double *Q,
                          int64_t ldq, double *R, int64_t ldr)
{
    if (m <= 0 || n <= 0 || !A || !R || lda < n || ldr < n || (Q && ldq < n)) return ERR_ARG;
    if (m < n) return ERR_SHAPE;
    double *W = malloc(sizeof(double) * (size_t)(m * n));
    double *V = malloc(sizeof(double) * (size_t)(m * n));
    double *Q1 = Q ? malloc(sizeof(double) * (size_t)(m * n)) : NULL;
    if (!W || !V || (Q && !Q1)) { free(W); free(V); free(Q1); return ERR_NOMEM; }
    for (int64_t i = 0; i < m; ++i)
        for (int64_t j = 0; j < n; ++j) W[i * n + j] = A[i * lda + j];
    householder_inplace(m, n, W, V);
    for (int64_t i = 0; i < n; ++i) {
        double d = (W[i * n + i] >= 0.0) ? 1.0 : -1.0;
        for (int64_t j = 0; j < n; ++j) R[i * ldr + j] = (j >= i) ? d * W[i * n + j] : 0.0;
    }
    if (Q) {
        form_q_from_reflectors(m, n, V, Q1);
        for (int64_t i = 0; i < m; ++i)
            for (int64_t j = 0; j < n; ++j) {
                double d = (W[j * n + j] >= 0.0) ? 1.0 : -1.0;
                Q[i * ldq + j] = Q1[i * n + j] * d;
            }
    }
    free(W); free(V); free(Q1);
    return OK;
}

/*
 * Row-block partition used by the oracle: blocks of `block_rows` rows; a tail with fewer than n
 * rows is merged into the previous block (the paper's examples give every map task at least n
 * rows).  Returns the number of blocks and fills start[] (nb+1 entries) when start != NULL.
 */
int64_t oracle_partition(int64_t m, int64_t n, int64_t block_rows, int64_t *start)
{
    if (block_rows < n) block_rows = n;
    int64_t nb = m / block_rows;
    int64_t tail = m - nb * block_rows;
    if (nb == 0) nb = 1;
    else if (tail >= n) nb += 1;
    if (start) {
        for (int64_t i = 0; i < nb; ++i) start[i] = i * block_rows;
        start[nb] = m;
    }
    return nb;
}

/*
 * Direct TSQR (Sec. III-B, three steps):
 *   step 1: for each row block A_i: A_i = Q1_i R_i (Householder, Sec. III-A);
 *   step 2: S = [R_1; ...; R_P] (block order = row order) = Q2 R~, then R = D R~, Q2 <- Q2 D;
 *           the k-th n-row block of Q2 belongs to the k-th row block;
 *   step 3: Q_i = Q1_i Q2_i.
 * Q may be NULL (R only: steps 1-2, the indirect-TSQR R of Sec. II-B).  The optional out-param
 * Q2 (P*n x n) returns the sign-fixed step-2 factor; it must hold oracle_partition(...)*n rows.
 */
int oracle_tsqr(int64_t m, int64_t n, const double *A, int64_t lda, int64_t block_rows,
                double *Q, int64_t ldq, double *R, int64_t ldr, double *Q2out, int nthreads)
{
    if (m <= 0 || n <= 0 || !A || !R || lda < n || ldr < n || (Q && ldq < n)) return ERR_ARG;
    if (m < n) return ERR_SHAPE;
    set_threads(nthreads);
    int64_t nb = oracle_partition(m, n, block_rows, NULL);
    int64_t *start = malloc(sizeof(int64_t) * (size_t)(nb + 1));
    double *S = malloc(sizeof(double) * (size_t)(nb * n * n));
    double **Q1 = calloc((size_t)nb, sizeof(double *));
    if (!start || !S || !Q1) { free(start); free(S); free(Q1); return ERR_NOMEM; }
    oracle_partition(m, n, block_rows, start);
    int err = 0;

    /* step 1 */
#pragma omp parallel for schedule(dynamic, 1) reduction(| : err)
    for (int64_t p = 0; p < nb; ++p) {
        int64_t b = start[p + 1] - start[p];
        double *W = malloc(sizeof(double) * (size_t)(b * n));
        double *V = malloc(sizeof(double) * (size_t)(b * n));
        if (!W || !V) { free(W); free(V); err |= 1; continue; }
        for (int64_t i = 0; i < b; ++i)
            for (int64_t j = 0; j < n; ++j) W[i * n + j] = A[(start[p] + i) * lda + j];
        householder_inplace(b, n, W, V);
        for (int64_t i = 0; i < n; ++i)
            for (int64_t j = 0; j < n; ++j) S[(p * n + i) * n + j] = (j >= i) ? W[i * n + j] : 0.0;
        if (Q) {
            Q1[p] = malloc(sizeof(double) * (size_t)(b * n));
            if (!Q1[p]) err |= 1;
            else form_q_from_reflectors(b, n, V, Q1[p]);
        }
        free(W); free(V);
    }
    if (err) goto fail;

    /* step 2: one QR of the stacked R factors */
    {
        int64_t rows = nb * n;
        double *V2 = malloc(sizeof(double) * (size_t)(rows * n));
        double *Q2 = malloc(sizeof(double) * (size_t)(rows * n));
        if (!V2 || !Q2) { free(V2); free(Q2); err = 1; goto fail; }
        householder_inplace(rows, n, S, V2);
        double *d = malloc(sizeof(double) * (size_t)n);
        for (int64_t i = 0; i < n; ++i) d[i] = (S[i * n + i] >= 0.0) ? 1.0 : -1.0;
        for (int64_t i = 0; i < n; ++i)
            for (int64_t j = 0; j < n; ++j) R[i * ldr + j] = (j >= i) ? d[i] * S[i * n + j] : 0.0;
        if (Q || Q2out) {
            form_q_from_reflectors(rows, n, V2, Q2);
            for (int64_t i = 0; i < rows; ++i)
                for (int64_t j = 0; j < n; ++j) Q2[i * n + j] *= d[j];
            if (Q2out) memcpy(Q2out, Q2, sizeof(double) * (size_t)(rows * n));
        }
        free(d);
        free(V2);

        /* step 3: Q_i = Q1_i * Q2_i */
        if (Q) {
#pragma omp parallel for schedule(dynamic, 1)
            for (int64_t p = 0; p < nb; ++p) {
                int64_t b = start[p + 1] - start[p];
                const double *Q2p = &Q2[p * n * n];
                for (int64_t i = 0; i < b; ++i)
                    for (int64_t j = 0; j < n; ++j) {
                        double acc = 0.0;
                        for (int64_t k = 0; k < n; ++k) acc += Q1[p][i * n + k] * Q2p[k * n + j];
                        Q[(start[p] + i) * ldq + j] = acc;
                    }
            }
        }
        free(Q2);
    }

fail:
    for (int64_t p = 0; p < nb; ++p) free(Q1[p]);
    free(Q1); free(S); free(start);
    return err ? ERR_NOMEM : OK;
}

/*
 * SVD of a small n x n matrix R (Sec. III-B: the second step of the SVD variant adds the SVD of the
 * n x n R; the paper does not name the method).  One-sided Jacobi (Hestenes; Demmel & Veselic 1992): columns p < q of
 * G = R V are rotated until every pair is orthogonal to |g_p^T g_q| <= tol sqrt(|g_p|^2 |g_q|^2),
 * tol = 1e-15 n, in cyclic row order, at most 60 sweeps.  Then s_k = ||g_k||, u_k = g_k / s_k
 * (u_k = 0 when s_k = 0), sorted by descending s.  Gauge: each pair (u_k, v_k) is flipped so that
 * the entry of v_k with the largest magnitude (lowest index on ties) is positive.
 * Returns the number of sweeps used, or -1 when 60 sweeps did not converge.
 */
int oracle_svd_small(int64_t n, const double *R, int64_t ldr, double *S, double *V, int64_t ldv,
                     double *UR, int64_t ldu)
{
    double *G = malloc(sizeof(double) * (size_t)(n * n));
    double *W = malloc(sizeof(double) * (size_t)(n * n));
    double *sv = malloc(sizeof(double) * (size_t)n);
    int64_t *ord = malloc(sizeof(int64_t) * (size_t)n);
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j < n; ++j) {
            G[i * n + j] = R[i * ldr + j];
            W[i * n + j] = (i == j) ? 1.0 : 0.0;
        }
    const double tol = 1e-15 * (double)n;
    int sweeps = 0, converged = 0;
    while (sweeps < 60 && !converged) {
        ++sweeps;
        int rotated = 0;
        for (int64_t p = 0; p < n - 1; ++p)
            for (int64_t q = p + 1; q < n; ++q) {
                double a = 0.0, b = 0.0, c = 0.0;
                for (int64_t i = 0; i < n; ++i) {
                    a += G[i * n + p] * G[i * n + p];
                    b += G[i * n + q] * G[i * n + q];
                    c += G[i * n + p] * G[i * n + q];
                }
                if (c == 0.0 || fabs(c) <= tol * sqrt(a * b)) continue;
                rotated = 1;
                double zeta = (b - a) / (2.0 * c);
                double t = ((zeta >= 0.0) ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                double cs = 1.0 / sqrt(1.0 + t * t);
                double sn = cs * t;
                for (int64_t i = 0; i < n; ++i) {
                    double gp = G[i * n + p], gq = G[i * n + q];
                    G[i * n + p] = cs * gp - sn * gq;
                    G[i * n + q] = sn * gp + cs * gq;
                    double wp = W[i * n + p], wq = W[i * n + q];
                    W[i * n + p] = cs * wp - sn * wq;
                    W[i * n + q] = sn * wp + cs * wq;
                }
            }
        if (!rotated) converged = 1;
    }
    for (int64_t k = 0; k < n; ++k) {
        sv[k] = scaled_norm(n, &G[k], n);
        ord[k] = k;
    }
    /* sort descending (insertion sort keeps equal values in index order) */
    for (int64_t i = 1; i < n; ++i) {
        int64_t o = ord[i];
        int64_t j = i - 1;
        while (j >= 0 && sv[ord[j]] < sv[o]) { ord[j + 1] = ord[j]; --j; }
        ord[j + 1] = o;
    }
    for (int64_t k = 0; k < n; ++k) {
        int64_t c = ord[k];
        double s = sv[c];
        int64_t imax = 0;
        double vmax = -1.0;
        for (int64_t i = 0; i < n; ++i)
            if (fabs(W[i * n + c]) > vmax) { vmax = fabs(W[i * n + c]); imax = i; }
        double g = (W[imax * n + c] < 0.0) ? -1.0 : 1.0;
        S[k] = s;
        for (int64_t i = 0; i < n; ++i) {
            V[i * ldv + k] = g * W[i * n + c];
            UR[i * ldu + k] = (s > 0.0) ? g * G[i * n + c] / s : 0.0;
        }
    }
    free(G); free(W); free(sv); free(ord);
    return converged ? sweeps : -1;
}

/*
 * SVD via direct TSQR (Sec. III-B): A = QR, R = U_R S V^T, U = Q U_R.  Q and R may be NULL.
 * Returns the Jacobi sweep count (>= 1) or a negative error.
 */
int oracle_tsqr_svd(int64_t m, int64_t n, const double *A, int64_t lda, int64_t block_rows,
                    double *U, int64_t ldu, double *S, double *V, int64_t ldv, double *Q,
                    int64_t ldq, double *R, int64_t ldr, int nthreads)
{
    if (!U || !S || !V || ldu < n || ldv < n) return -ERR_ARG;
    double *Qw = malloc(sizeof(double) * (size_t)(m * n));
    double *Rw = malloc(sizeof(double) * (size_t)(n * n));
    double *UR = malloc(sizeof(double) * (size_t)(n * n));
    if (!Qw || !Rw || !UR) { free(Qw); free(Rw); free(UR); return -ERR_NOMEM; }
    int st = oracle_tsqr(m, n, A, lda, block_rows, Qw, n, Rw, n, NULL, nthreads);
    if (st != OK) { free(Qw); free(Rw); free(UR); return -st; }
    int sweeps = oracle_svd_small(n, Rw, n, S, V, ldv, UR, n);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < m; ++i)
        for (int64_t j = 0; j < n; ++j) {
            double acc = 0.0;
            for (int64_t k = 0; k < n; ++k) acc += Qw[i * n + k] * UR[k * n + j];
            U[i * ldu + j] = acc;
        }
    if (Q)
        for (int64_t i = 0; i < m; ++i)
            for (int64_t j = 0; j < n; ++j) Q[i * ldq + j] = Qw[i * n + j];
    if (R)
        for (int64_t i = 0; i < n; ++i)
            for (int64_t j = 0; j < n; ++j) R[i * ldr + j] = Rw[i * n + j];
    free(Qw); free(Rw); free(UR);
    return sweeps;
}

/*
 * Adjoint of the thin QR (not in the paper; closed form of Walter & Lehmann 2018, Seeger et al.
 * 2017, Liao et al. 2019).  For the loss L(Q,R) with cotangents dQ (m x n) and dR (n x n; only
 * its upper triangle matters since R's strict lower part is identically zero):
 *   M = R triu(dR)^T - dQ^T Q;  copyltu(M) = tril(M) + tril(M,-1)^T;
 *   dA = (dQ + Q copyltu(M)) R^{-T}.
 * dQ or dR may be NULL (treated as zero).
 */
int oracle_qr_backward(int64_t m, int64_t n, const double *Q, int64_t ldq, const double *R,
                       int64_t ldr, const double *dQ, int64_t lddq, const double *dR,
                       int64_t lddr, double *dA, int64_t ldda, int nthreads)
{
    if (!Q || !R || !dA) return ERR_ARG;
    set_threads(nthreads);
    double *M = calloc((size_t)(n * n), sizeof(double));
    double *C = calloc((size_t)(n * n), sizeof(double));
    if (!M || !C) { free(M); free(C); return ERR_NOMEM; }
    if (dR)
        for (int64_t i = 0; i < n; ++i)
            for (int64_t j = 0; j < n; ++j) {
                double acc = 0.0;
                for (int64_t k = 0; k < n; ++k)
                    if (j <= k) acc += R[i * ldr + k] * dR[j * lddr + k];  /* triu(dR)[j][k] */
                M[i * n + j] = acc;
            }
    if (dQ) {
        /* M -= dQ^T Q, accumulated over rows in long double (threads split the rows i of the
           product; each entry still sums r = 0, 1, ... in order) */
        long double *acc = calloc((size_t)(n * n), sizeof(long double));
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i)
            for (int64_t r = 0; r < m; ++r) {
                long double a = dQ[r * lddq + i];
                for (int64_t j = 0; j < n; ++j) acc[i * n + j] += a * Q[r * ldq + j];
            }
        for (int64_t i = 0; i < n * n; ++i) M[i] -= (double)acc[i];
        free(acc);
    }
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j < n; ++j) C[i * n + j] = (j <= i) ? M[i * n + j] : M[j * n + i];
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < m; ++r) {
        double *b = malloc(sizeof(double) * (size_t)n);
        for (int64_t j = 0; j < n; ++j) {
            double acc = dQ ? dQ[r * lddq + j] : 0.0;
            for (int64_t k = 0; k < n; ++k) acc += Q[r * ldq + k] * C[k * n + j];
            b[j] = acc;
        }
        /* x R^T = b  <=>  sum_{i>=j} x_i R[j][i] = b_j : back substitution */
        for (int64_t j = n - 1; j >= 0; --j) {
            double acc = b[j];
            for (int64_t i = j + 1; i < n; ++i) acc -= R[j * ldr + i] * dA[r * ldda + i];
            dA[r * ldda + j] = acc / R[j * ldr + j];
        }
        free(b);
    }
    free(M); free(C);
    return OK;
}

/*
 * Adjoint of the thin SVD A = U diag(S) V^T with m > n (not in the paper; Townsend 2016,
 * Ionescu et al. 2015):
 *   F_ij = 1/(s_j^2 - s_i^2) (i != j), F_ii = 0;  J = F o (U^T dU - dU^T U);  K = F o (V^T dV - dV^T V);
 *   dA = U (J S + diag(dS) + S K) V^T + (dU - U (U^T dU)) S^{-1} V^T.
 * dU, dS, dV may each be NULL (zero).
 */
int oracle_svd_backward(int64_t m, int64_t n, const double *U, int64_t ldu, const double *S,
                        const double *V, int64_t ldv, const double *dU, int64_t lddu,
                        const double *dS, const double *dV, int64_t lddv, double *dA,
                        int64_t ldda, int nthreads)
{
    if (!U || !S || !V || !dA) return ERR_ARG;
    set_threads(nthreads);
    double *UtdU = calloc((size_t)(n * n), sizeof(double));
    double *Inner = calloc((size_t)(n * n), sizeof(double));
    double *B1 = calloc((size_t)(n * n), sizeof(double));
    double *B2 = calloc((size_t)(n * n), sizeof(double));
    if (!UtdU || !Inner || !B1 || !B2) { free(UtdU); free(Inner); free(B1); free(B2); return ERR_NOMEM; }
    if (dU) {
        long double *acc = calloc((size_t)(n * n), sizeof(long double));
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i)
            for (int64_t r = 0; r < m; ++r) {
                long double a = U[r * ldu + i];
                for (int64_t j = 0; j < n; ++j) acc[i * n + j] += a * dU[r * lddu + j];
            }
        for (int64_t i = 0; i < n * n; ++i) UtdU[i] = (double)acc[i];
        free(acc);
    }
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j < n; ++j) {
            double F = (i == j) ? 0.0 : 1.0 / (S[j] * S[j] - S[i] * S[i]);
            double Jij = F * (UtdU[i * n + j] - UtdU[j * n + i]);
            double VtdV_ij = 0.0, VtdV_ji = 0.0;
            if (dV)
                for (int64_t k = 0; k < n; ++k) {
                    VtdV_ij += V[k * ldv + i] * dV[k * lddv + j];
                    VtdV_ji += V[k * ldv + j] * dV[k * lddv + i];
                }
            double Kij = F * (VtdV_ij - VtdV_ji);
            double val = Jij * S[j] + S[i] * Kij;
            if (i == j && dS) val += dS[i];
            Inner[i * n + j] = val;
        }
    /* B1 = (Inner - (U^T dU) S^{-1}) V^T ; B2 = S^{-1} V^T */
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j < n; ++j) {
            double a1 = 0.0, a2 = 0.0;
            for (int64_t k = 0; k < n; ++k) {
                a1 += (Inner[i * n + k] - UtdU[i * n + k] / S[k]) * V[j * ldv + k];
            }
            a2 = V[j * ldv + i] / S[i];
            B1[i * n + j] = a1;
            B2[i * n + j] = a2;
        }
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < m; ++r)
        for (int64_t j = 0; j < n; ++j) {
            double acc = 0.0;
            for (int64_t k = 0; k < n; ++k) {
                acc += U[r * ldu + k] * B1[k * n + j];
                if (dU) acc += dU[r * lddu + k] * B2[k * n + j];
            }
            dA[r * ldda + j] = acc;
        }
    free(UtdU); free(Inner); free(B1); free(B2);
    return OK;
}

/* ---------------------------------------------------------------------------------------------
 * Metrics (Sec. I-B).  Sums over the m rows are accumulated in long double (64-bit mantissa):
 * plain FP64 summation over millions of rows overstates ||Q^T Q - I|| by orders of magnitude.
 * The 2-norm of an n x n symmetric matrix is its largest |eigenvalue|, found by cyclic Jacobi.
 * ------------------------------------------------------------------------------------------- */

/* largest |eigenvalue| of a symmetric n x n matrix (destroyed), cyclic Jacobi in long double;
 * NaN if any entry is not finite */
static double sym_norm2(int64_t n, long double *Mx)
{
    for (int64_t i = 0; i < n * n; ++i)
        if (!isfinite(Mx[i])) return NAN;
    for (int sweep = 0; sweep < 100; ++sweep) {
        long double off = 0.0L, tot = 0.0L;
        for (int64_t i = 0; i < n; ++i)
            for (int64_t j = 0; j < n; ++j) {
                long double v = Mx[i * n + j] * Mx[i * n + j];
                tot += v;
                if (i != j) off += v;
            }
        if (off <= 1e-36L * tot || off == 0.0L) break;
        for (int64_t p = 0; p < n - 1; ++p)
            for (int64_t q = p + 1; q < n; ++q) {
                long double apq = Mx[p * n + q];
                if (apq == 0.0L) continue;
                long double app = Mx[p * n + p], aqq = Mx[q * n + q];
                long double theta = (aqq - app) / (2.0L * apq);
                long double t = ((theta >= 0.0L) ? 1.0L : -1.0L) /
                                (fabsl(theta) + sqrtl(1.0L + theta * theta));
                long double c = 1.0L / sqrtl(1.0L + t * t), s = t * c;
                for (int64_t k = 0; k < n; ++k) {
                    long double akp = Mx[k * n + p], akq = Mx[k * n + q];
                    Mx[k * n + p] = c * akp - s * akq;
                    Mx[k * n + q] = s * akp + c * akq;
                }
                for (int64_t k = 0; k < n; ++k) {
                    long double apk = Mx[p * n + k], aqk = Mx[q * n + k];
                    Mx[p * n + k] = c * apk - s * aqk;
                    Mx[q * n + k] = s * apk + c * aqk;
                }
            }
    }
    long double mx = 0.0L;
    for (int64_t i = 0; i < n; ++i)
        if (fabsl(Mx[i * n + i]) > mx) mx = fabsl(Mx[i * n + i]);
    return (double)mx;
}

/* X^T X of an m x n matrix in long double, rows split across threads then summed in fixed order */
static void gram_ld(int64_t m, int64_t n, const double *X, int64_t ldx, long double *out)
{
    int nt = 1;
#ifdef _OPENMP
    nt = omp_get_max_threads();
#endif
    long double *part = calloc((size_t)(nt * n * n), sizeof(long double));
#pragma omp parallel num_threads(nt)
    {
        int t = 0, T = 1;
#ifdef _OPENMP
        t = omp_get_thread_num();
        T = omp_get_num_threads();
#endif
        long double *g = &part[(int64_t)t * n * n];
        int64_t r0 = m * t / T, r1 = m * (t + 1) / T;
        for (int64_t r = r0; r < r1; ++r)
            for (int64_t i = 0; i < n; ++i) {
                long double a = X[r * ldx + i];
                for (int64_t j = i; j < n; ++j) g[i * n + j] += a * X[r * ldx + j];
            }
    }
    for (int64_t i = 0; i < n * n; ++i) out[i] = 0.0L;
    for (int t = 0; t < nt; ++t)
        for (int64_t i = 0; i < n; ++i)
            for (int64_t j = i; j < n; ++j) out[i * n + j] += part[(int64_t)t * n * n + i * n + j];
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j < i; ++j) out[i * n + j] = out[j * n + i];
    free(part);
}

/* ||Q^T Q - I||_2 */
double oracle_metric_orth(int64_t m, int64_t n, const double *Q, int64_t ldq, int nthreads)
{
    set_threads(nthreads);
    long double *G = malloc(sizeof(long double) * (size_t)(n * n));
    gram_ld(m, n, Q, ldq, G);
    for (int64_t i = 0; i < n; ++i) G[i * n + i] -= 1.0L;
    double r = sym_norm2(n, G);
    free(G);
    return r;
}

/* ||X||_2 of an m x n matrix: sqrt(lambda_max(X^T X)) */
double oracle_norm2(int64_t m, int64_t n, const double *X, int64_t ldx, int nthreads)
{
    set_threads(nthreads);
    long double *G = malloc(sizeof(long double) * (size_t)(n * n));
    gram_ld(m, n, X, ldx, G);
    double r = sqrt(sym_norm2(n, G));
    free(G);
    return r;
}

/*
 * ||A - Q B||_2 where B is n x n (B = R for the QR residual, B = diag(S) V^T for the SVD residual).
 * E = A - Q B is formed row by row in long double, then ||E||_2 = sqrt(lambda_max(E^T E)).
 */
double oracle_residual_norm2(int64_t m, int64_t n, const double *A, int64_t lda, const double *Q,
                             int64_t ldq, const double *B, int64_t ldb, int nthreads)
{
    set_threads(nthreads);
    double *E = malloc(sizeof(double) * (size_t)(m * n));
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < m; ++r)
        for (int64_t j = 0; j < n; ++j) {
            long double acc = A[r * lda + j];
            for (int64_t k = 0; k < n; ++k) acc -= (long double)Q[r * ldq + k] * B[k * ldb + j];
            E[r * n + j] = (double)acc;
        }
    double res = oracle_norm2(m, n, E, n, nthreads);
    free(E);
    return res;
}


/* ---------------------------------------------------------------------------------------------
 * Comparison methods of the stability experiment (Sec. IV): Cholesky QR (Sec. II-A) and indirect
 * TSQR (Sec. II-B), each with Q = A R^{-1} (Sec. II-C) and optionally one step of iterative
 * refinement (the same QR repeated on the computed Q, Sec. I): Q1 R1 = A, Q R2 = Q1, R = R2 R1.
 * ------------------------------------------------------------------------------------------- */
#define ORACLE_CHOLQR 1
#define ORACLE_INDIRECT 2
#define ERR_BREAKDOWN 4

/* R^{-1} of an upper-triangular n x n R (ld n), column by column: R x = e_j by back substitution. */
static void upper_inverse(int64_t n, const double *R, double *X)
{
    for (int64_t j = 0; j < n; ++j) {
        for (int64_t i = n - 1; i >= 0; --i) {
            double acc = (i == j) ? 1.0 : 0.0;
            for (int64_t t = i + 1; t < n; ++t) acc -= R[i * n + t] * X[t * n + j];
            X[i * n + j] = (i <= j) ? acc / R[i * n + i] : 0.0;
        }
    }
}

/* Q = A X for an m x n A and an n x n X (plain triple loop, rows in parallel). */
static void times_small(int64_t m, int64_t n, const double *A, int64_t lda, const double *X,
                        double *Q, int64_t ldq)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < m; ++i)
        for (int64_t j = 0; j < n; ++j) {
            double acc = 0.0;
            for (int64_t k = 0; k < n; ++k) acc += A[i * lda + k] * X[k * n + j];
            Q[i * ldq + j] = acc;
        }
}

/* One QR of A by `method`: R (n x n, ld n) and Q = A R^{-1} (ld ldq).  Cholesky QR: the Gram
 * matrix is summed block by block as the map tasks of Alg. 1 produce it (blocks of block_rows
 * rows, each A_p^T A_p accumulated over its rows, then the blocks added in order); G = L L^T by
 * the column-by-column Cholesky algorithm, R = L^T.  Returns ERR_BREAKDOWN when a pivot is not
 * positive (G not numerically positive definite). */
static int one_qr(int method, int64_t m, int64_t n, const double *A, int64_t lda,
                  int64_t block_rows, double *Q, int64_t ldq, double *R)
{
    if (method == ORACLE_INDIRECT) {
        int st = oracle_tsqr(m, n, A, lda, block_rows, NULL, 0, R, n, NULL, 0);
        if (st != OK) return st;
    } else {
        double *G = calloc((size_t)(n * n), sizeof(double));
        double *Gp = malloc(sizeof(double) * (size_t)(n * n));
        if (!G || !Gp) { free(G); free(Gp); return ERR_NOMEM; }
        for (int64_t r0 = 0; r0 < m; r0 += block_rows) {
            int64_t r1 = (r0 + block_rows < m) ? r0 + block_rows : m;
            for (int64_t e = 0; e < n * n; ++e) Gp[e] = 0.0;
            for (int64_t i = r0; i < r1; ++i)
                for (int64_t a = 0; a < n; ++a)
                    for (int64_t b = 0; b < n; ++b) Gp[a * n + b] += A[i * lda + a] * A[i * lda + b];
            for (int64_t e = 0; e < n * n; ++e) G[e] += Gp[e];
        }
        free(Gp);
        /* G = L L^T; L stored transposed into R (R = L^T) */
        for (int64_t e = 0; e < n * n; ++e) R[e] = 0.0;
        int bad = 0;
        for (int64_t j = 0; j < n && !bad; ++j) {
            double d = G[j * n + j];
            for (int64_t k = 0; k < j; ++k) d -= R[k * n + j] * R[k * n + j];
            if (!(d > 0.0)) { bad = 1; break; }
            double ljj = sqrt(d);
            R[j * n + j] = ljj;
            for (int64_t i = j + 1; i < n; ++i) {
                double x = G[i * n + j];
                for (int64_t k = 0; k < j; ++k) x -= R[k * n + i] * R[k * n + j];
                R[j * n + i] = x / ljj;
            }
        }
        free(G);
        if (bad) return ERR_BREAKDOWN;
    }
    double *X = malloc(sizeof(double) * (size_t)(n * n));
    if (!X) return ERR_NOMEM;
    upper_inverse(n, R, X);
    times_small(m, n, A, lda, X, Q, ldq);
    free(X);
    return OK;
}

/*
 * Cholesky QR (method 1) or indirect TSQR (method 2), with `refine` steps of iterative refinement
 * (0 or 1).  Q: m x n (ldq), R: n x n (ldr).  Returns 0, or ERR_BREAKDOWN (Cholesky of a Gram
 * matrix that is not numerically positive definite; Q and R are then not written).
 */
int oracle_indirect_qr(int method, int refine, int64_t m, int64_t n, const double *A, int64_t lda,
                       int64_t block_rows, double *Q, int64_t ldq, double *R, int64_t ldr,
                       int nthreads)
{
    if (m <= 0 || n <= 0 || !A || !Q || !R || lda < n || ldq < n || ldr < n) return ERR_ARG;
    if (method != ORACLE_CHOLQR && method != ORACLE_INDIRECT) return ERR_ARG;
    if (m < n) return ERR_SHAPE;
    set_threads(nthreads);
    double *R1 = malloc(sizeof(double) * (size_t)(n * n));
    double *Q1 = refine ? malloc(sizeof(double) * (size_t)(m * n)) : NULL;
    if (!R1 || (refine && !Q1)) { free(R1); free(Q1); return ERR_NOMEM; }
    int st = one_qr(method, m, n, A, lda, block_rows, refine ? Q1 : Q, refine ? n : ldq, R1);
    if (st == OK && refine) {
        double *R2 = malloc(sizeof(double) * (size_t)(n * n));
        if (!R2) st = ERR_NOMEM;
        else {
            st = one_qr(method, m, n, Q1, n, block_rows, Q, ldq, R2);
            if (st == OK) { /* R = R2 R1 */
                double *T = malloc(sizeof(double) * (size_t)(n * n));
                for (int64_t i = 0; i < n; ++i)
                    for (int64_t j = 0; j < n; ++j) {
                        double acc = 0.0;
                        for (int64_t k = 0; k < n; ++k) acc += R2[i * n + k] * R1[k * n + j];
                        T[i * n + j] = acc;
                    }
                memcpy(R1, T, sizeof(double) * (size_t)(n * n));
                free(T);
            }
            free(R2);
        }
    }
    if (st == OK)
        for (int64_t i = 0; i < n; ++i)
            for (int64_t j = 0; j < n; ++j) R[i * ldr + j] = R1[i * n + j];
    free(R1);
    free(Q1);
    return st;
}
