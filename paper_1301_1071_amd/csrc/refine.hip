// The FP64 refinement pass of the precision form (FP32 panels and step-3 product, FP64 tree).
//
// The paper's iterative refinement (Sec. I-B and Sec. II-C) repeats the QR factorization on a
// computed Q.  Re-factoring the FP32 direct-TSQR Q-hat restores its orthogonality but cannot bring
// ||A - QR|| below the FP32 level, because Q-hat R-hat differs from A by O(u_32 ||A||).  The pass
// therefore refines against A itself, with the FP32-path R-hat as a preconditioner (the indirect
// Q = A R^{-1} of Sec. II-B followed by the refinement of Sec. II-C, with a Cholesky QR of the
// well-conditioned Y as the repeated factorization; Yamazaki, Tomov & Dongarra 2015):
//     pass 1   Y = A R-hat^{-1}            G1 = Y^T Y = Rc1^T Rc1
//     pass 1b  Y2 = Y Rc1^{-1}             G2 = Y2^T Y2 = Rc2^T Rc2   (only if ||G1 - I||_F > 1/2)
//     pass 2   Q = Y Rc1^{-1} [Rc2^{-1}],  R = [Rc2] Rc1 R-hat.
// Every product with an inverse is a row-by-row triangular solve (each row of A is one lane's
// forward substitution), which is backward stable row by row: ||A - QR|| stays O(u ||A||) for
// any conditioning, while an explicit inverse would leave an error of O(u kappa(A) ||A||).  Y
// is recomputed from A in each pass instead of being stored (A is read three times at most, Q
// written once).  kappa(Y) ~ 1 + u_32 kappa(A), so one Cholesky pass keeps Q^T Q = I to
// rounding up to kappa(A) ~ 1e9 and the second pass (skipped on the device when G1 is within
// 1/2 of I in Frobenius norm) to ~1e14.  Beyond that, or when the FP32 factorization reaches a
// numerically singular R-hat, a Cholesky step breaks down and the call reports -2.
#include "tsqr_internal.h"

namespace tsqr {
namespace {

typedef double d4_t __attribute__((ext_vector_type(4)));

constexpr int kRefThreads = 256;     // one row per thread and chunk
constexpr int kRefMaxBlocks = 512;   // work-groups (and Gram partials) of a pass: two per CU

// Workspace of the pass, for padded width NP (NP = 16, 32 or 64):
//   tri   3 x NP x NP  R-hat, Rc1, Rc2 (upper triangular), each stored transposed with the
//                      reciprocal of its diagonal on the diagonal, zero padded
//   diag  3 x NP       their diagonals
//   G     NP x NP      the summed Gram
//   flag  1 int        second pass needed
//   part  nblk x NP x NP  per-work-group partial Grams
struct RefLayout {
    int np = 0, nblk = 0;
    size_t tri = 0, diag = 0, g = 0, flag = 0, part = 0, total = 0;
};

int pad_width(int64_t n) { return n <= 16 ? 16 : (n <= 32 ? 32 : 64); }

RefLayout ref_layout(int64_t m, int64_t n)
{
    RefLayout L;
    L.np = pad_width(n);
    const int64_t chunks = ceil_div(m, kRefThreads);
    L.nblk = (int)std::min<int64_t>(chunks, kRefMaxBlocks);
    const size_t nn = (size_t)L.np * L.np;
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t at = off; off = align_up(off + bytes); return at; };
    L.tri = take(3 * nn * sizeof(double));
    L.diag = take(3 * (size_t)L.np * sizeof(double));
    L.g = take(nn * sizeof(double));
    L.flag = take(sizeof(int));
    L.part = take((size_t)L.nblk * nn * sizeof(double));
    L.total = off;
    return L;
}

template <int I, int N, typename F> __device__ __forceinline__ void static_for(F &&f)
{
    if constexpr (I < N) {
        f(std::integral_constant<int, I>{});
        static_for<I + 1, N>(f);
    }
}

// A triangular factor is stored TRANSPOSED with its reciprocal diagonal: column j of the
// upper-triangular Tm occupies TmT[j * NP + 0 .. j], entries i < j holding Tm[i][j] and entry j
// holding 1 / Tm[j][j].  A solve reads these values with scalar loads, whole columns at a time,
// in batches of consecutive columns holding at most kBatchVals values.  Scalar loads return out
// of order, so every wait on them waits for all of them: one wait per batch is the cost, and the
// batches are made as large as the scalar registers allow.
constexpr int kBatchVals = 32;
constexpr int batch_end(int j0, int np)
{
    int j = j0, v = 0;
    while (j < np && (v + j + 1 <= kBatchVals || j == j0)) { v += j + 1; ++j; }
    return j;
}
template <int NP> constexpr int batch_count()
{
    int b = 0;
    for (int j = 0; j < NP; j = batch_end(j, NP)) ++b;
    return b;
}
template <int NP> constexpr int batch_start(int b)
{
    int j = 0;
    for (int k = 0; k < b; ++k) j = batch_end(j, NP);
    return j;
}

// y <- y Tm^{-1} (forward substitution along the row: y_j = (y_j - sum_{i<j} y_i Tm[i][j]) /
// Tm[j][j], the division a product with the stored reciprocal).  Each batch of columns is one
// region between scheduling barriers: its scalar loads, one wait, its FMAs (the barriers keep the
// compiler from hoisting later batches' loads, which would exhaust the scalar registers).
// Columns j >= n (padding) are skipped.
template <int NP>
__device__ __forceinline__ void solve_row(double (&y)[NP], const double *__restrict__ TmT, int n)
{
    // `j < n` is evaluated where it is used: an opaque copy of n keeps the compiler from
    // hoisting one predicate per column out of the row loop (which spilled scalar registers)
    auto live = [&](int j) {
        int nv = n;
        asm volatile("" : "+s"(nv));
        return j < nv;
    };
    static_for<0, batch_count<NP>()>([&](auto B) {
        constexpr int j0 = batch_start<NP>(decltype(B)::value);
        constexpr int j1 = batch_end(j0, NP);
        if (live(j0)) {
            static_for<j0, j1>([&](auto J) {
                constexpr int j = decltype(J)::value;
                if (j == j0 || live(j)) {
                    double a0 = y[j], a1 = 0.0;
#pragma unroll
                    for (int i = 0; i < j; ++i) {
                        if (i & 1) a1 = fma(-y[i], TmT[j * NP + i], a1);
                        else a0 = fma(-y[i], TmT[j * NP + i], a0);
                    }
                    y[j] = (a0 + a1) * TmT[j * NP + j];
                }
            });
        }
        __builtin_amdgcn_sched_barrier(0);
    });
}

// One pass over the rows of A.  Every chunk of 256 rows is staged through LDS with coalesced
// loads; each thread takes one row into registers and applies `ns` triangular solves (factors
// 0..ns-1 of `tri`, and with flag3 a third one only if *flag3 != 0).  GRAM: the solved rows go
// back to LDS and Y^T Y is accumulated on the matrix cores, every wave taking the k-steps
// k = w (mod 4) of every upper tile (independent accumulators), the waves' sums added through LDS
// at the end; one partial per work-group.  Otherwise the rows are written to Q through LDS.  With
// skip_flag the whole pass is skipped unless *skip_flag != 0.
template <int NP, bool GRAM>
__global__ void __launch_bounds__(kRefThreads)
k_ref_rows(int64_t m, int n, const double *__restrict__ A, int64_t lda,
           const double *__restrict__ tri, int ns, const int *__restrict__ flag3,
           const int *__restrict__ skip_flag, double *__restrict__ part, double *__restrict__ Q,
           int64_t ldq)
{
    constexpr int LD = NP + 1;
    constexpr int T = NP / 16, NTILE = T * (T + 1) / 2;
    extern __shared__ double ys[];                 // kRefThreads x LD
    if (skip_flag && *skip_flag == 0) return;
    const int tid = threadIdx.x, lane = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int nsolve = ns + ((flag3 && *flag3 != 0) ? 1 : 0);
    const int64_t nchunks = (m + kRefThreads - 1) / kRefThreads;

    d4_t acc[NTILE];
#pragma unroll
    for (int t = 0; t < NTILE; ++t) acc[t] = d4_t{0, 0, 0, 0};

    // Staging: thread tid always holds column c = tid % NP of rows tid / NP + q (256 / NP), q <
    // NP, of a chunk.  Every load is unconditional at a clamped in-bounds address, so a chunk's
    // NP loads are in flight together; the next chunk is fetched while the current one is
    // solved.  The padding (rows past m, columns past n) is zeroed only when the values are
    // staged: a select right after the loads would wait for them there.
    constexpr int RSTEP = kRefThreads / NP;
    const int cc = tid % NP, rr0 = tid / NP;
    const int ccl = min(cc, n - 1);
    double pre[NP];
    auto fetch = [&](int64_t chk) {
        const int64_t rb = chk * kRefThreads;
        const int last = (int)min((int64_t)kRefThreads, m - rb) - 1;
#pragma unroll
        for (int q = 0; q < NP; ++q) pre[q] = A[(rb + min(rr0 + RSTEP * q, last)) * lda + ccl];
    };
    if (blockIdx.x < nchunks) fetch(blockIdx.x);
    for (int64_t ch = blockIdx.x; ch < nchunks; ch += gridDim.x) {
        const int64_t r0 = ch * kRefThreads;
        const int nr = (int)min((int64_t)kRefThreads, m - r0);
#pragma unroll
        for (int q = 0; q < NP; ++q) {
            const int r = rr0 + RSTEP * q;
            ys[r * LD + cc] = (r < nr && cc < n) ? pre[q] : 0.0;
        }
        __syncthreads();
        if (ch + gridDim.x < nchunks) fetch(ch + gridDim.x);
        double y[NP];
#pragma unroll
        for (int c = 0; c < NP; ++c) y[c] = ys[tid * LD + c];
        for (int s = 0; s < nsolve; ++s) solve_row<NP>(y, tri + (size_t)s * NP * NP, n);
#pragma unroll
        for (int c = 0; c < NP; ++c) ys[tid * LD + c] = y[c];
        __syncthreads();
        if constexpr (GRAM) {
            // A = Y^T (lane l: Y[4k + l/16][16a + l%16]), B = Y (lane l: Y[4k + l/16][16b + l%16])
            for (int k = w; k < kRefThreads / 4; k += 4) {
                const int r = 4 * k + (lane >> 4);
                double yv[T];
#pragma unroll
                for (int a = 0; a < T; ++a) yv[a] = ys[r * LD + 16 * a + (lane & 15)];
                int t = 0;
#pragma unroll
                for (int a = 0; a < T; ++a)
#pragma unroll
                    for (int b = a; b < T; ++b, ++t)
                        acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(yv[a], yv[b], acc[t], 0, 0, 0);
            }
        } else {
            double outv[NP];
#pragma unroll
            for (int q = 0; q < NP; ++q) outv[q] = ys[(rr0 + RSTEP * q) * LD + cc];
#pragma unroll
            for (int q = 0; q < NP; ++q) {
                const int r = rr0 + RSTEP * q;
                if (r < nr && cc < n) Q[(r0 + r) * ldq + cc] = outv[q];
            }
        }
        __syncthreads();
    }
    if constexpr (GRAM) {
        // the four waves' accumulators, summed in a fixed order
        double *red = ys;                          // [4][NTILE][256]
#pragma unroll
        for (int t = 0; t < NTILE; ++t)
#pragma unroll
            for (int i = 0; i < 4; ++i) red[(w * NTILE + t) * 256 + i * 64 + lane] = acc[t][i];
        __syncthreads();
        double *out = part + (size_t)blockIdx.x * NP * NP;
        for (int e = tid; e < NTILE * 256; e += kRefThreads) {
            const int t = e >> 8, i = (e >> 6) & 3, l = e & 63;
            const double v = red[(0 * NTILE + t) * 256 + (e & 255)] + red[(1 * NTILE + t) * 256 + (e & 255)] +
                             red[(2 * NTILE + t) * 256 + (e & 255)] + red[(3 * NTILE + t) * 256 + (e & 255)];
            int a = 0, tt = t;
            while (tt >= T - a) { tt -= T - a; ++a; }
            const int b = a + tt;
            const int row = 16 * a + (l >> 4) + 4 * i, col = 16 * b + (l & 15);   // f64 layout
            out[row * NP + col] = v;
        }
    }
}

// G (upper triangle, np-padded) = sum of the work-groups' partials: one wave per entry, lane l
// summing the partials l, l + 64, ..., the lanes' sums added by a fixed butterfly (deterministic).
// With skip_flag, nothing is done unless *skip_flag != 0 (the second pass did not run).
__global__ void __launch_bounds__(256)
k_ref_gsum(int n, int np, int nblk, const double *__restrict__ part, double *__restrict__ G,
           const int *__restrict__ skip_flag)
{
    if (skip_flag && *skip_flag == 0) return;
    const int nent = n * (n + 1) / 2;
    const int e0 = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (e0 >= nent) return;                        // whole waves
    int r = 0, e = e0;
    while (e >= n - r) { e -= n - r; ++r; }
    const int c = r + e;
    double a0 = 0.0, a1 = 0.0;
    int b = lane;
    for (; b + 64 < nblk; b += 128) {
        a0 += part[(size_t)b * np * np + r * np + c];
        a1 += part[(size_t)(b + 64) * np * np + r * np + c];
    }
    if (b < nblk) a0 += part[(size_t)b * np * np + r * np + c];
    double v = a0 + a1;
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    if (lane == 0) G[r * np + c] = v;
}

// Cholesky G = Rc^T Rc of the upper triangle of G (n x n in an np-padded array, in place in LDS
// `Gs`); returns false if a pivot is not positive.  Called by every thread of the work-group.
__device__ bool chol_lds(int n, int np, double *Gs)
{
    __shared__ int s_fail;
    if (threadIdx.x == 0) s_fail = 0;
    __syncthreads();
    for (int k = 0; k < n; ++k) {
        const double d = Gs[k * np + k];
        if (!(d > 0.0)) {
            if (threadIdx.x == 0) s_fail = 1;
            break;
        }
        const double rkk = sqrt(d);
        __syncthreads();
        for (int j = k + threadIdx.x; j < n; j += blockDim.x)
            Gs[k * np + j] = (j == k) ? rkk : Gs[k * np + j] / rkk;
        __syncthreads();
        const int wd = n - k - 1;
        for (int e = threadIdx.x; e < wd * wd; e += blockDim.x) {
            const int i = k + 1 + e / wd, j = k + 1 + e % wd;
            if (j >= i) Gs[i * np + j] -= Gs[k * np + i] * Gs[k * np + j];
        }
        __syncthreads();
    }
    __syncthreads();
    return s_fail == 0;
}

// Stores the upper-triangular X (element (r, c) from get(r, c), r, c < n) as factor `slot`:
// transposed with the reciprocal diagonal in tri, its true diagonal in diag.
template <typename F>
__device__ void store_factor(int n, int np, int slot, F get, double *tri, double *diag)
{
    double *XT = tri + (size_t)slot * np * np;
    for (int e = threadIdx.x; e < np * np; e += blockDim.x) {
        const int r = e / np, c = e - r * np;        // element (r, c) of X goes to XT[c][r]
        double v = 0.0;
        if (r < n && c < n && c >= r) v = (r == c) ? 1.0 / get(r, c) : get(r, c);
        XT[c * np + r] = v;
    }
    for (int j = threadIdx.x; j < np; j += blockDim.x) diag[slot * np + j] = (j < n) ? get(j, j) : 0.0;
}

// Factor 0 = R-hat.
__global__ void __launch_bounds__(256)
k_ref_setup(int n, int np, const double *__restrict__ Rhat, double *__restrict__ tri,
            double *__restrict__ diag)
{
    store_factor(n, np, 0, [&](int r, int c) { return Rhat[r * n + c]; }, tri, diag);
}

// After a Gram pass (G summed by k_ref_gsum): Cholesky into factor `slot` (identity on breakdown,
// with info = -2).  slot 1 also decides the second pass: flag = ||G - I||_F > 1/2.  slot 2 (always
// launched; it only factors when flag is set, otherwise factor 2 = I) writes R = Rc2 Rc1 R-hat to
// R (ldr).
__global__ void __launch_bounds__(256)
k_ref_chol(int n, int np, int slot, const double *__restrict__ G, double *__restrict__ tri,
           double *__restrict__ diag, int *flag, double *R, int64_t ldr, int32_t *info)
{
    extern __shared__ double Gs[];          // np x np
    __shared__ double s_dev;
    const int tid = threadIdx.x, nth = blockDim.x;
    const bool second = (slot == 2);
    if (second && *flag == 0) {
        store_factor(n, np, 2, [&](int r, int c) { return r == c ? 1.0 : 0.0; }, tri, diag);
    } else {
        for (int e = tid; e < np * np; e += nth) {
            const int r = e / np, c = e - r * np;
            Gs[e] = (r < n && c < n && c >= r) ? G[r * np + c] : 0.0;
        }
        if (tid == 0) s_dev = 0.0;
        __syncthreads();
        if (!second && tid == 0) {
            double d = 0.0;
            for (int r = 0; r < n; ++r)
                for (int c = r; c < n; ++c) {
                    const double x = Gs[r * np + c] - (r == c ? 1.0 : 0.0);
                    d += (r == c ? 1.0 : 2.0) * x * x;
                }
            s_dev = d;
        }
        __syncthreads();
        const bool ok = chol_lds(n, np, Gs);
        if (ok) store_factor(n, np, slot, [&](int r, int c) { return Gs[r * np + c]; }, tri, diag);
        else store_factor(n, np, slot, [&](int r, int c) { return r == c ? 1.0 : 0.0; }, tri, diag);
        if (!second && tid == 0) *flag = (s_dev > 0.25) ? 1 : 0;   // ||G - I||_F > 1/2
        if (!ok && tid == 0) *info = -2;
    }
    if (!second) return;
    __syncthreads();
    // R = Rc2 (Rc1 R-hat): upper-triangular products of the stored (transposed) factors
    auto el = [&](int s, int r, int c) {
        return r == c ? diag[s * np + r] : tri[(size_t)s * np * np + c * np + r];
    };
    double *M = Gs;                          // Rc1 R-hat, np x np
    for (int e = tid; e < np * np; e += nth) {
        const int i = e / np, j = e - i * np;
        double a = 0.0;
        if (j >= i && j < n)
            for (int t = i; t <= j; ++t) a = fma(el(1, i, t), el(0, t, j), a);
        M[e] = a;
    }
    __syncthreads();
    for (int e = tid; e < n * n; e += nth) {
        const int i = e / n, j = e - i * n;
        double a = 0.0;
        if (j >= i)
            for (int t = i; t <= j; ++t) a = fma(el(2, i, t), M[t * np + j], a);
        R[(int64_t)i * ldr + j] = a;
    }
}

int grid_of(int64_t m) { return (int)std::min<int64_t>(ceil_div(m, kRefThreads), kRefMaxBlocks); }

template <int NP, bool GRAM>
hipError_t launch_rows_t(int64_t m, int64_t n, const double *A, int64_t lda, const double *tri,
                         int ns, const int *flag3, const int *skip, double *part, double *Q,
                         int64_t ldq, hipStream_t st)
{
    const size_t lds = sizeof(double) * kRefThreads * (NP + 1);
    auto kern = k_ref_rows<NP, GRAM>;
    hipError_t e = ensure_dynamic_lds((const void *)kern, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3(grid_of(m)), dim3(kRefThreads), lds, st, m, (int)n, A, lda,
                       tri, ns, flag3, skip, part, Q, ldq);
    return hipGetLastError();
}

hipError_t rows_pass(int np, bool gram, int64_t m, int64_t n, const double *A, int64_t lda,
                     const double *tri, int ns, const int *flag3, const int *skip, double *part,
                     double *Q, int64_t ldq, hipStream_t st)
{
#define TSQR_ROWS(NP)                                                                          \
    return gram ? launch_rows_t<NP, true>(m, n, A, lda, tri, ns, flag3, skip, part, Q, ldq, st) \
                : launch_rows_t<NP, false>(m, n, A, lda, tri, ns, flag3, skip, part, Q, ldq, st)
    switch (np) {
    case 16: TSQR_ROWS(16);
    case 32: TSQR_ROWS(32);
    default: TSQR_ROWS(64);
    }
#undef TSQR_ROWS
}

}  // namespace

size_t refine_scratch_bytes(int64_t m, int64_t n) { return ref_layout(m, n).total; }

hipError_t launch_refine(int64_t m, int64_t n, const double *A, int64_t lda, const double *Rhat,
                         double *Q, int64_t ldq, double *R, int64_t ldr, void *scratch,
                         int32_t *info, hipStream_t st)
{
    if (n > 64) return hipErrorInvalidValue;
    const RefLayout L = ref_layout(m, n);
    char *base = (char *)scratch;
    double *tri = (double *)(base + L.tri), *diag = (double *)(base + L.diag);
    double *G = (double *)(base + L.g), *part = (double *)(base + L.part);
    int *flag = (int *)(base + L.flag);
    const int np = L.np;
    const size_t lds = sizeof(double) * (size_t)np * np;
    const int nent = (int)(n * (n + 1) / 2);
    hipError_t e;
    hipLaunchKernelGGL(k_ref_setup, dim3(1), dim3(256), 0, st, (int)n, np, Rhat, tri, diag);
    // pass 1: Y = A Rhat^{-1}, G1 = Y^T Y -> Rc1, flag
    if ((e = rows_pass(np, true, m, n, A, lda, tri, 1, nullptr, nullptr, part, nullptr, 0, st)) !=
        hipSuccess)
        return e;
    hipLaunchKernelGGL(k_ref_gsum, dim3((nent + 3) / 4), dim3(256), 0, st, (int)n, np, L.nblk,
                       part, G, nullptr);
    hipLaunchKernelGGL(k_ref_chol, dim3(1), dim3(256), lds, st, (int)n, np, 1, G, tri, diag, flag,
                       R, ldr, info);
    // pass 1b (skipped on the device unless flag): Y Rc1^{-1}, G2 -> Rc2; then R
    if ((e = rows_pass(np, true, m, n, A, lda, tri, 2, nullptr, flag, part, nullptr, 0, st)) !=
        hipSuccess)
        return e;
    hipLaunchKernelGGL(k_ref_gsum, dim3((nent + 3) / 4), dim3(256), 0, st, (int)n, np, L.nblk,
                       part, G, flag);
    hipLaunchKernelGGL(k_ref_chol, dim3(1), dim3(256), lds, st, (int)n, np, 2, G, tri, diag, flag,
                       R, ldr, info);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    // pass 2: Q = A Rhat^{-1} Rc1^{-1} [Rc2^{-1}]
    return rows_pass(np, false, m, n, A, lda, tri, 2, flag, nullptr, nullptr, Q, ldq, st);
}

}  // namespace tsqr
