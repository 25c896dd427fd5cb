/*
 * tsqr.h -- C ABI of the MI355X (gfx950) direct-TSQR library.
 *
 * Method: direct TSQR of Benson, Gleich & Demmel, "Direct QR factorizations for tall-and-skinny
 * matrices in MapReduce architectures", Sec. III-B (three steps: Householder QR of every row
 * block, QR of the stacked R factors, reconstruction Q_i = Q1_i Q2_i; SVD variant: SVD of R and
 * U = Q U_R) with the recursive extension of Sec. III-C (Alg. 2: when the stacked R is too large
 * for one task it is itself factored by direct TSQR).
 *
 * Conventions for every entry point
 *   - Matrices are ROW-MAJOR: element (i,j) of X is X[i*ldx + j], ldx >= number of columns.
 *     A row of A is one record of the paper's key-value layout (Sec. I-A).
 *   - Every matrix/vector pointer is a DEVICE pointer; the caller owns all buffers.  The library
 *     never allocates, frees or synchronises on the call path; all work is enqueued on `stream`
 *     (a hipStream_t; NULL = default stream).  Calls are safe to capture in a HIP graph.
 *   - `ws` is a device workspace of at least tsqr_workspace_bytes(...) bytes; its contents on
 *     entry are ignored.
 *   - Argument errors are returned synchronously, before anything is enqueued.
 *   - Numerical conditions are reported through `d_info` (one device int32, written by the
 *     kernels of the call; read it after synchronising the stream):
 *         0  success;
 *         j  (j > 0) R[j-1][j-1] == 0: A is rank deficient (the paper assumes full rank, Sec. I);
 *        -1  a non-finite value reached R (non-finite input);
 *        -2  (TSQR_FP32_REFINED only) a Cholesky step of the refinement broke down: the FP32
 *            R-hat does not precondition A (kappa(A) beyond about 1e14, or an R-hat that is
 *            numerically singular in FP32); Q and R are then not valid;
 *        -3  (adjoints only) the adjoint is undefined (zero pivot, repeated singular value);
 *        -4  (Cholesky QR only) A^T A is not numerically positive definite.
 *   - The factorization is the unique thin QR with diag(R) > 0 (A full rank).  Q is m x n with
 *     orthonormal columns, R is n x n upper triangular (strict lower triangle written as 0).
 *   - Supported: 1 <= n <= TSQR_NMAX, m >= n.  Values must be well inside the floating-point
 *     range (|a_ij| < 1e150 in FP64, < 1e17 in FP32): column norms are formed without scaling.
 *     Widths 128 < n <= TSQR_NMAX run the wide path: every level of the tree factors panels of
 *     4 n rows held in global workspace (a quarter of the rows per level, Sec. III-C), and step 3
 *     runs in column chunks of 128.  The adjoints, the comparison methods and the metrics keep
 *     n <= TSQR_NMAX_SMALL (their n x n work runs in one work-group's LDS); the refined
 *     precision form and the batched form keep n <= 64.
 */
#ifndef TSQR_H
#define TSQR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TSQR_ABI_VERSION 1
#define TSQR_NMAX 512
#define TSQR_NMAX_SMALL 128

typedef enum {
    TSQR_OK = 0,
    TSQR_ERR_INVALID_ARG = 1, /* NULL pointer, ld < n, m <= 0, n <= 0, bad enum */
    TSQR_ERR_SHAPE = 2,       /* m < n, or n above the entry point's limit */
    TSQR_ERR_WORKSPACE = 3,   /* ws == NULL or ws_bytes too small */
    TSQR_ERR_UNSUPPORTED = 4, /* option combination not implemented */
    TSQR_ERR_HIP = 5          /* a HIP launch/runtime error */
} tsqr_status;

/* Arithmetic of the per-panel work (steps 1 and 3).  The stacked-R tree and the SVD of R are
 * always FP64. */
typedef enum {
    TSQR_FP64 = 0,         /* everything FP64 */
    TSQR_FP32_REFINED = 1, /* FP64 in/out: R-hat from FP32 panels and the FP64 tree, then an FP64
                              refinement against A that returns FP64 Q and R (see tsqr_qr) */
    TSQR_FP32 = 2          /* FP32 panels and GEMM, FP64 tree, no refinement */
} tsqr_precision;

typedef struct {
    int32_t struct_size; /* sizeof(tsqr_opts) */
    int32_t precision;   /* tsqr_precision */
    int32_t panel_rows;  /* 0 = library default for (n, precision); otherwise a supported height */
    int32_t flags;       /* 0 or TSQR_FLAG_REUSE_OUTPUT */
} tsqr_opts;

/* Keep the level-0 panel factors (Q1_i, or their reflectors) in the output buffer that step 3
 * overwrites (Q; U for tsqr_svd without Q) instead of in the workspace, which then shrinks by
 * m x n elements: A, Q and the workspace of a 600,000,000 x 25 QR fit in one GPU's HBM.  Step 3
 * then covers all output columns of a row block in one work-group, which reads the block's
 * factors before it writes the block.  Needs that output contiguous (ldq == n, or ldu == n;
 * TSQR_ERR_INVALID_ARG otherwise) and supports n <= 128 with at most 128 output columns (n for
 * tsqr_qr; n for tsqr_svd without Q, 2 n with Q) when the level-0 arithmetic has the input's
 * element type (not TSQR_FP32 on FP64 input); other cases return TSQR_ERR_UNSUPPORTED, from the
 * call and from the workspace query (which for TSQR_FP32 with this flag assumes FP32 input and,
 * for TSQR_OP_SVD, sizes the layouts the flag supports).  Ignored where no Q is formed (tsqr_r,
 * the refined precision form) and by the adjoints. */
#define TSQR_FLAG_REUSE_OUTPUT 1

/* Operation codes for tsqr_workspace_bytes. */
typedef enum {
    TSQR_OP_R = 0,
    TSQR_OP_QR = 1,
    TSQR_OP_SVD = 2,
    TSQR_OP_QR_BACKWARD = 3,
    TSQR_OP_SVD_BACKWARD = 4
} tsqr_op;

/* Default options: FP64, default panel height. */
void tsqr_default_opts(tsqr_opts *opts);

/* Workspace (bytes) needed by `op` on an m x n input with the given options (opts may be NULL). */
tsqr_status tsqr_workspace_bytes(int32_t op, int64_t m, int64_t n, const tsqr_opts *opts,
                                 size_t *bytes);

/*
 * R factor only (steps 1-2 of Sec. III-B; the indirect TSQR of Sec. II-B computes the same R,
 * whatever the shape of the reduction tree).  A: m x n (lda); R: n x n (ldr), diag(R) > 0.
 */
tsqr_status tsqr_r(int64_t m, int64_t n, const double *A, int64_t lda, double *R, int64_t ldr,
                   void *ws, size_t ws_bytes, int32_t *d_info, const tsqr_opts *opts,
                   void *stream);

/*
 * tsqr_r without a caller workspace, for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).  The same kernels as
 * tsqr_r (bit-identical R); the workspace is a fixed device array inside the library of
 * TSQR_NOALLOC_SCRATCH_BYTES bytes per GPU, held from the first call on that GPU until the process
 * ends.  The call itself allocates nothing.  Inputs whose tsqr_r workspace
 * (tsqr_workspace_bytes(TSQR_OP_R, ...)) exceeds that size return TSQR_ERR_WORKSPACE before
 * anything is enqueued (e.g. n = 50 up to about 3.4M rows, n = 10 up to about 60M rows).  Every
 * call on one GPU shares the array: calls that overlap in time on one GPU (other streams, other
 * host threads) race and must be serialised by the caller.  Nothing in it needs clearing.
 */
#define TSQR_NOALLOC_SCRATCH_BYTES (128ull << 20)
tsqr_status tsqr_r_noalloc(int64_t m, int64_t n, const double *A, int64_t lda, double *R,
                           int64_t ldr, int32_t *d_info, const tsqr_opts *opts, void *stream);

/*
 * Thin QR by direct TSQR (Sec. III-B steps 1-3): A (m x n, lda) = Q (m x n, ldq) R (n x n, ldr).
 * TSQR_FP32 runs steps 1 and 3 (panels and the Q1*Q2 GEMM) in FP32 and returns that result in
 * FP64 storage.  TSQR_FP32_REFINED (n <= 64) takes R-hat from the FP32 panels and FP64 tree and
 * refines against A in FP64 (the indirect Q = A R^{-1} of Sec. II-B with the refinement of
 * Sec. II-C): Y = A R-hat^{-1} by row-wise triangular solves, Y^T Y = Rc1^T Rc1,
 * Q = Y Rc1^{-1}, R = Rc1 R-hat, with a second Cholesky pass (Rc2) decided on the device when
 * ||Y^T Y - I||_F > 1/2.  A is read two or three times; no m x n intermediate is stored.  The
 * backward error stays O(u) for any kappa(A); orthogonality holds to O(u) up to kappa(A) about
 * 1e14, beyond which d_info may report -2.
 */
tsqr_status tsqr_qr(int64_t m, int64_t n, const double *A, int64_t lda, double *Q, int64_t ldq,
                    double *R, int64_t ldr, void *ws, size_t ws_bytes, int32_t *d_info,
                    const tsqr_opts *opts, void *stream);

/*
 * Thin SVD by direct TSQR (Sec. III-B): A = Q R, R = U_R diag(S) V^T, U = Q U_R, with U computed
 * in the same pass as Q (U_R is passed to step 3).  U: m x n (ldu); S: n values, descending;
 * V: n x n (ldv).  Gauge: each (u_k, v_k) pair is signed so that the largest-magnitude entry of
 * v_k (lowest index on ties) is positive.  Q (ldq) and R (ldr) are optional (NULL = not wanted).
 * TSQR_FP32 runs the FP32 panels and product; TSQR_FP32_REFINED refines Q and R as tsqr_qr does,
 * then takes the SVD of the refined R and U = Q U_R (one more product).  The workspace query
 * (TSQR_OP_SVD) covers both the call with and without Q.
 */
tsqr_status tsqr_svd(int64_t m, int64_t n, const double *A, int64_t lda, double *U, int64_t ldu,
                     double *S, double *V, int64_t ldv, double *Q, int64_t ldq, double *R,
                     int64_t ldr, void *ws, size_t ws_bytes, int32_t *d_info,
                     const tsqr_opts *opts, void *stream);

/*
 * Row-chunked thin QR, for inputs whose tsqr_qr workspace would not fit beside A and Q (the
 * paper's 150,000,000 x 100, Sec. V): one more level of the Sec. III-C recursion above direct
 * TSQR.  Rows are cut into chunks of chunk_rows (a last chunk shorter than n joins the one
 * before); each chunk is factored by tsqr_qr with its level-0 factors kept in its rows of Q
 * (TSQR_FLAG_REUSE_OUTPUT), A_c = Q_c R_c; the stacked R_c are factored by tsqr_qr,
 * [R_1; ...; R_C] = [Q2_1; ...; Q2_C] R; then Q_c <- Q_c Q2_c in place.  The result is the same
 * unique factorization (diag(R) > 0) as tsqr_qr's.  FP64 only (opts->precision TSQR_FP64, flags
 * 0), n <= 128, Q contiguous (ldq == n).  A chunk's own rank deficiency is not reported; d_info
 * is that of the stacked factorization (the R of A).  Workspace:
 * tsqr_qr_chunked_workspace_bytes, about one chunk's tsqr_qr workspace.
 */
tsqr_status tsqr_qr_chunked_workspace_bytes(int64_t m, int64_t n, int64_t chunk_rows,
                                            const tsqr_opts *opts, size_t *bytes);
tsqr_status tsqr_qr_chunked(int64_t m, int64_t n, int64_t chunk_rows, const double *A,
                            int64_t lda, double *Q, int64_t ldq, double *R, int64_t ldr,
                            void *ws, size_t ws_bytes, int32_t *d_info, const tsqr_opts *opts,
                            void *stream);

/* FP32 input/output twins: FP32 panels and GEMM, FP64 tree and SVD of R.  opts->precision
 * may be TSQR_FP64 or TSQR_FP32 (both run this path; the workspace query with TSQR_FP32 gives the
 * size); TSQR_FP32_REFINED returns TSQR_ERR_UNSUPPORTED (the refinement needs FP64 input). */
tsqr_status tsqr_r_f32(int64_t m, int64_t n, const float *A, int64_t lda, float *R, int64_t ldr,
                       void *ws, size_t ws_bytes, int32_t *d_info, const tsqr_opts *opts,
                       void *stream);
tsqr_status tsqr_qr_f32(int64_t m, int64_t n, const float *A, int64_t lda, float *Q, int64_t ldq,
                        float *R, int64_t ldr, void *ws, size_t ws_bytes, int32_t *d_info,
                        const tsqr_opts *opts, void *stream);
/* SVD variant of Sec. III-B on FP32 data: FP32 panels and step-3 product (Q and U = Q U_R in one
 * pass), FP64 tree and FP64 one-sided Jacobi SVD of R; S, V (and the optional Q, R) are written in
 * FP32 with the conventions of tsqr_svd. */
tsqr_status tsqr_svd_f32(int64_t m, int64_t n, const float *A, int64_t lda, float *U, int64_t ldu,
                         float *S, float *V, int64_t ldv, float *Q, int64_t ldq, float *R,
                         int64_t ldr, void *ws, size_t ws_bytes, int32_t *d_info,
                         const tsqr_opts *opts, void *stream);

/*
 * Differentiation form: adjoint of tsqr_qr.  For the loss <dQ, Q> + <dR, R> with cotangents dQ
 * (m x n, lddq; NULL = zero) and dR (n x n, lddr; NULL = zero; only its upper triangle matters,
 * R's strict lower part being identically zero) writes dA (m x n, ldda).  Q and R are recomputed
 * from A by the forward kernels, so nothing from a forward call (in particular no Q1_i) needs to
 * be kept.  Closed form (not in the paper; Walter & Lehmann 2018, Seeger et al. 2017):
 *     M = R triu(dR)^T - dQ^T Q,   dA = (dQ + Q copyltu(M)) R^{-T},
 *     copyltu(M) = tril(M) + tril(M, -1)^T.
 * FP64 only (opts->precision must be TSQR_FP64), n <= TSQR_NMAX_SMALL.  Workspace:
 * tsqr_workspace_bytes with TSQR_OP_QR_BACKWARD.  d_info as for tsqr_qr, or -3 if R has a zero
 * diagonal entry.
 */
tsqr_status tsqr_qr_backward(int64_t m, int64_t n, const double *A, int64_t lda,
                             const double *dQ, int64_t lddq, const double *dR, int64_t lddr,
                             double *dA, int64_t ldda, void *ws, size_t ws_bytes,
                             int32_t *d_info, const tsqr_opts *opts, void *stream);

/*
 * Adjoint of tsqr_svd (m > n, distinct nonzero singular values): for the loss
 * <dU, U> + <dS, S> + <dV, V> (each cotangent NULL = zero; dS has n entries) writes dA.  U, S, V
 * are recomputed from A.  Closed form (Townsend 2016, Ionescu et al. 2015):
 *     F_ij = 1/(s_j^2 - s_i^2) (i != j), F_ii = 0, J = F o (U^T dU - dU^T U),
 *     K = F o (V^T dV - dV^T V),
 *     dA = U (J S + diag(dS) + S K) V^T + (dU - U (U^T dU)) S^{-1} V^T.
 * The result follows the gauge of tsqr_svd.  d_info as for tsqr_svd, or -3 if two singular
 * values coincide or one is zero.  n <= TSQR_NMAX_SMALL.  Workspace: TSQR_OP_SVD_BACKWARD.
 */
tsqr_status tsqr_svd_backward(int64_t m, int64_t n, const double *A, int64_t lda,
                              const double *dU, int64_t lddu, const double *dS,
                              const double *dV, int64_t lddv, double *dA, int64_t ldda,
                              void *ws, size_t ws_bytes, int32_t *d_info,
                              const tsqr_opts *opts, void *stream);

/* ------------------------------------------------------------------------------------------
 * Batched form: many independent tall-skinny QRs (each by direct TSQR, Sec. III-B/III-C) in one
 * fixed launch sequence.  Not in the paper: its map tasks factor row blocks of ONE matrix; here
 * the panels of every matrix of the batch share the same launches.
 *
 * A plan is built once on the host for the shapes (m_i, n_i, 1 <= n_i <= 64, m_i >= n_i) and
 * leading dimensions of the batch; creating it allocates and fills a small device table (the
 * only allocation and host-device copy of the batched form), so create plans outside any graph
 * capture.  tsqr_qr_batched then only enqueues kernels (no allocation, memset or host
 * synchronisation): capturing one call in a HIP graph gives one graph launch for the batch.
 * ------------------------------------------------------------------------------------------ */
typedef struct tsqr_batch_plan_t *tsqr_batch_plan;

typedef enum { TSQR_DTYPE_F64 = 0, TSQR_DTYPE_F32 = 1 } tsqr_dtype;

/*
 * m, n, lda, ldq, ldr: HOST arrays of `batch` entries (row-major leading dimensions of A_i, Q_i,
 * R_i).  dtype: element type of A, Q and R (TSQR_DTYPE_F32 runs FP32 panels and GEMM with the
 * FP64 tree of TSQR_FP32).  opts may be NULL; opts->precision must match dtype (TSQR_FP64 or
 * TSQR_FP32); opts->panel_rows = 0 takes each width's panel height from the tune table
 * (tsqr_tune_set), otherwise it must equal one of the heights tsqr_tune_variants lists for
 * every width in the batch; opts->flags must be 0 (TSQR_ERR_INVALID_ARG otherwise).  The plan
 * belongs to the device current at creation.
 */
tsqr_status tsqr_batch_plan_create(int32_t batch, const int64_t *m, const int64_t *n,
                                   const int64_t *lda, const int64_t *ldq, const int64_t *ldr,
                                   int32_t dtype, const tsqr_opts *opts, tsqr_batch_plan *plan);
tsqr_status tsqr_batch_plan_destroy(tsqr_batch_plan plan);
/* Workspace the plan needs (about the bytes of all A_i plus the stacked-R trees). */
tsqr_status tsqr_batch_workspace_bytes(tsqr_batch_plan plan, size_t *bytes);
/* Number of kernel launches one tsqr_qr_batched call enqueues. */
tsqr_status tsqr_batch_plan_launches(tsqr_batch_plan plan, int32_t *nlaunches);

/*
 * Factor every A_i = Q_i R_i.  d_A, d_Q, d_R: DEVICE arrays of `batch` device pointers (element
 * type per the plan).  d_info: DEVICE array of `batch` int32, entry i as d_info of tsqr_qr.
 * Matrices must not overlap their outputs.
 */
tsqr_status tsqr_qr_batched(tsqr_batch_plan plan, const void *const *d_A, void *const *d_Q,
                            void *const *d_R, void *ws, size_t ws_bytes, int32_t *d_info,
                            void *stream);

/*
 * Panel-height table used by batched plans, one entry per (dtype, width class n <= 4, 8, 16,
 * 32, 64).  Each class has up to three variants of the blocked panel kernel, the same heights
 * for FP64 and FP32: 0 = default (384 rows for n <= 32, 256 above), 1 = half the row tiles per
 * wave (half height), 2 = 512 rows (n <= 16 only).  tsqr_tune_variants lists their heights for
 * width n (0 = not usable: a panel must hold at least 3n rows, or the variant repeats the
 * default).  The autotuner (paper_1301_1071_amd/autotune.py) times them and records its choice
 * with tsqr_tune_set.  Set the table before creating plans; it is process-wide.
 */
tsqr_status tsqr_tune_set(int32_t dtype, int64_t n, int32_t variant);
tsqr_status tsqr_tune_get(int32_t dtype, int64_t n, int32_t *variant, int32_t *panel_rows);
tsqr_status tsqr_tune_variants(int32_t dtype, int64_t n, int32_t max, int32_t *panel_rows,
                               int32_t *count);

/*
 * The recursive tree the library runs for `op` on an m x n input (Sec. III-C): level 0 factors A,
 * level L >= 1 the stacked R factors of level L-1.  Writes the number of levels to *nlevels and,
 * for the first max_levels levels, the rows of the level matrix and its panel height (host
 * arrays).  Same argument errors as tsqr_workspace_bytes.
 */
tsqr_status tsqr_plan_levels(int32_t op, int64_t m, int64_t n, const tsqr_opts *opts,
                             int32_t max_levels, int32_t *nlevels, int64_t *rows,
                             int32_t *panel_rows);

/*
 * Kernel timing for benchmarks.  While enabled, every kernel launch the library makes is
 * bracketed by a pair of HIP events recorded on the launch stream (events are created on first
 * use and reused).  Not for use under graph capture.  tsqr_profile_collect waits for the recorded
 * events, writes the summed milliseconds and launch counts of each kernel class c < nclasses
 * into ms[c] / launches[c] (host arrays), and clears the record.
 */
tsqr_status tsqr_profile_enable(int32_t on);
/* Record only the kernel classes whose bit is set in `mask` (bit c = class c; default: all), so
 * that a timed region can be measured with events around one class only. */
tsqr_status tsqr_profile_set_mask(uint32_t mask);
tsqr_status tsqr_profile_collect(double *ms, int64_t *launches, int32_t nclasses);
int32_t tsqr_profile_num_classes(void);
const char *tsqr_profile_class_name(int32_t c);

/* ------------------------------------------------------------------------------------------
 * Comparison methods of the stability experiment (Sec. IV), not direct TSQR: they exist so that
 * the experiment can run beside tsqr_qr on the same GPU.
 *   TSQR_METHOD_CHOLQR    Cholesky QR (Sec. II-A): R^T R = A^T A, the Gram summed over row blocks
 *                         (Alg. 1) and factored by Cholesky; fails when A^T A is not numerically
 *                         positive definite (d_info = -4; Q and R are then not valid).
 *   TSQR_METHOD_INDIRECT  indirect TSQR (Sec. II-B): R from the stacked-R reduction alone.
 * Both form Q = A R^{-1} with the explicit inverse of R (Sec. II-C), which is not backward
 * stable: ||Q^T Q - I|| grows with kappa(A) (Cholesky QR: with kappa(A)^2).  refine = 1 repeats
 * the same QR once on the computed Q (iterative refinement, Sec. I): Q = Q1 R2^{-1}, R = R2 R1.
 * FP64 only (opts->precision must be TSQR_FP64), n <= TSQR_NMAX_SMALL.  A, Q: m x n; R: n x n
 * upper triangular.
 * ------------------------------------------------------------------------------------------ */
typedef enum { TSQR_METHOD_CHOLQR = 1, TSQR_METHOD_INDIRECT = 2 } tsqr_method;
tsqr_status tsqr_indirect_workspace_bytes(int32_t method, int32_t refine, int64_t m, int64_t n,
                                          const tsqr_opts *opts, size_t *bytes);
tsqr_status tsqr_qr_indirect(int32_t method, int32_t refine, int64_t m, int64_t n, const double *A,
                             int64_t lda, double *Q, int64_t ldq, double *R, int64_t ldr, void *ws,
                             size_t ws_bytes, int32_t *d_info, const tsqr_opts *opts,
                             void *stream);

/* ------------------------------------------------------------------------------------------
 * Error metrics of Sec. I-B (measurement, not part of the factorization).  Compensated Gram
 * matrices over the m rows, accumulated in double-double (TwoProd by FMA and TwoSum, Ogita, Rump
 * & Oishi 2005), so that ||Q^T Q - I|| is not swamped by the O(m u) rounding of an FP64 sum:
 *   mode 0: G = X^T X - I;  mode 1: G = E^T E with E = A - X B (B n x n, each entry of E a
 *   compensated dot product);  mode 2: G = X^T X.
 * X, A: m x n device matrices (row-major, ldx, lda); G: n x n device (ld n, symmetric).  The
 * caller takes the 2-norm of the small G (||Q^T Q - I||_2 = ||G||_2 for mode 0,
 * ||A - QR||_2 = sqrt(lambda_max(G)) for mode 1).  n <= TSQR_NMAX_SMALL.
 * ws: tsqr_metric_workspace_bytes.
 * ------------------------------------------------------------------------------------------ */
tsqr_status tsqr_metric_workspace_bytes(int64_t m, int64_t n, size_t *bytes);
tsqr_status tsqr_metric_gram(int32_t mode, int64_t m, int64_t n, const double *X, int64_t ldx,
                             const double *A, int64_t lda, const double *B, int64_t ldb,
                             double *G, void *ws, size_t ws_bytes, void *stream);

/* Human-readable status name (static string). */
const char *tsqr_status_string(tsqr_status status);
/* Description of the calling thread's most recent TSQR_ERR_HIP (HIP error text and the failing
 * library call); "" if none. */
const char *tsqr_last_error(void);
/* TSQR_ABI_VERSION of the loaded library. */
int32_t tsqr_abi_version(void);

#ifdef __cplusplus
}
#endif

#endif /* TSQR_H */
