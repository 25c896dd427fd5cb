// One FP64 refinement pass for the precision form (FP32 panels, FP64 tree).
//
// The paper's iterative refinement (Sec. I and Sec. II-C) repeats the QR on the computed Q; that
// restores orthogonality but cannot lift the backward error ||A - QR|| above the FP32 level, so
// the pass below refines against A itself (preconditioned Cholesky QR, Yamazaki, Tomov & Dongarra
// 2015): with Rhat the FP64-promoted R of the FP32 factorization,
//     Y = A Rhat^{-1}   (row-wise forward substitution, FP64),
//     G = Y^T Y = Rc^T Rc (Cholesky, FP64),
//     R = Rc Rhat,  Q = Y Rc^{-1}.
// Y has condition number 1 + O(u_32 kappa(A)), so the Cholesky step is well conditioned.
#include "tsqr_internal.h"

namespace tsqr {
namespace {

constexpr int kRefineRows = 64;     // rows staged per step
constexpr int kRefineBlocks = 512;  // work-groups of the Gram pass

// y = a Rhat^{-1} for one row (a row vector; Rhat upper triangular, ld n, held in LDS)
template <int NPM>
__device__ __forceinline__ void row_solve(int n, const double *__restrict__ Rs, double (&y)[NPM])
{
#pragma unroll
    for (int j = 0; j < NPM; ++j) {
        if (j < n) {
            double acc = y[j];
#pragma unroll
            for (int i = 0; i < NPM; ++i)
                if (i < j) acc = fma(-y[i], Rs[i * n + j], acc);
            y[j] = acc / Rs[j * n + j];
        }
    }
}

template <int NPM>
__global__ void __launch_bounds__(kThreads)
k_refine_gram(int64_t m, int n, const double *__restrict__ A, int64_t lda,
              const double *__restrict__ Rhat, double *__restrict__ Gpart)
{
    __shared__ double Rs[NPM * NPM];
    __shared__ double Ys[kRefineRows][NPM + 1];
    const int tid = threadIdx.x;
    for (int e = tid; e < n * n; e += kThreads) Rs[e] = Rhat[e];
    constexpr int kSlots = (NPM * NPM + kThreads - 1) / kThreads;
    double acc[kSlots];
#pragma unroll
    for (int s = 0; s < kSlots; ++s) acc[s] = 0.0;
    __syncthreads();
    for (int64_t r0 = (int64_t)blockIdx.x * kRefineRows; r0 < m;
         r0 += (int64_t)gridDim.x * kRefineRows) {
        const int nr = (int)min((int64_t)kRefineRows, m - r0);
        if (tid < kRefineRows) {
            double y[NPM];
#pragma unroll
            for (int j = 0; j < NPM; ++j)
                y[j] = (tid < nr && j < n) ? A[(r0 + tid) * lda + j] : 0.0;
            if (tid < nr) row_solve<NPM>(n, Rs, y);
#pragma unroll
            for (int j = 0; j < NPM; ++j) Ys[tid][j] = (tid < nr) ? y[j] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int s = 0; s < kSlots; ++s) {
            const int e = tid + s * kThreads;
            if (e < n * n) {
                const int i = e / n, j = e - i * n;
                double a = acc[s];
                for (int r = 0; r < nr; ++r) a = fma(Ys[r][i], Ys[r][j], a);
                acc[s] = a;
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int s = 0; s < kSlots; ++s) {
        const int e = tid + s * kThreads;
        if (e < n * n) Gpart[(int64_t)blockIdx.x * n * n + e] = acc[s];
    }
}

// G = sum of the partial Grams (fixed order), G = Rc^T Rc, R = Rc Rhat; Rc kept for the Q pass.
__global__ void __launch_bounds__(kThreads)
k_refine_chol(int n, int nblocks, const double *__restrict__ Gpart, const double *__restrict__ Rhat,
              double *__restrict__ Rc, double *__restrict__ R, int64_t ldr, int32_t *info)
{
    extern __shared__ double Gs[];   // n x n
    __shared__ int s_fail;
    const int tid = threadIdx.x;
    if (tid == 0) s_fail = 0;
    for (int e = tid; e < n * n; e += kThreads) {
        double a = 0.0;
        for (int b = 0; b < nblocks; ++b) a += Gpart[(int64_t)b * n * n + e];
        Gs[e] = a;
    }
    __syncthreads();
    // right-looking Cholesky, upper factor in the upper triangle of Gs
    for (int k = 0; k < n; ++k) {
        const double d = Gs[k * n + k];
        if (!(d > 0.0)) {
            if (tid == 0) s_fail = 1;
            break;
        }
        const double rkk = sqrt(d);
        __syncthreads();
        for (int j = k + tid; j < n; j += kThreads) Gs[k * n + j] = (j == k) ? rkk : Gs[k * n + j] / rkk;
        __syncthreads();
        for (int e = tid; e < (n - k - 1) * (n - k - 1); e += kThreads) {
            const int i = k + 1 + e / (n - k - 1), j = k + 1 + e % (n - k - 1);
            if (j >= i) Gs[i * n + j] -= Gs[k * n + i] * Gs[k * n + j];
        }
        __syncthreads();
    }
    __syncthreads();
    for (int e = tid; e < n * n; e += kThreads) {
        const int i = e / n, j = e - i * n;
        const double rc = (j >= i) ? Gs[e] : 0.0;
        Rc[e] = rc;
    }
    __syncthreads();
    for (int e = tid; e < n * n; e += kThreads) {
        const int i = e / n, j = e - i * n;
        double a = 0.0;
        if (j >= i)
            for (int t = i; t <= j; ++t) a = fma(Rc[i * n + t], Rhat[t * n + j], a);
        R[(int64_t)i * ldr + j] = a;
    }
    if (tid == 0 && s_fail) *info = -2;
}

template <int NPM>
__global__ void __launch_bounds__(kThreads)
k_refine_q(int64_t m, int n, const double *__restrict__ A, int64_t lda,
           const double *__restrict__ Rhat, const double *__restrict__ Rc, double *__restrict__ Q,
           int64_t ldq)
{
    __shared__ double Rs[NPM * NPM];
    __shared__ double Cs[NPM * NPM];
    const int tid = threadIdx.x;
    for (int e = tid; e < n * n; e += kThreads) { Rs[e] = Rhat[e]; Cs[e] = Rc[e]; }
    __syncthreads();
    for (int64_t r = (int64_t)blockIdx.x * kThreads + tid; r < m; r += (int64_t)gridDim.x * kThreads) {
        double y[NPM];
#pragma unroll
        for (int j = 0; j < NPM; ++j) y[j] = (j < n) ? A[r * lda + j] : 0.0;
        row_solve<NPM>(n, Rs, y);
        row_solve<NPM>(n, Cs, y);
#pragma unroll
        for (int j = 0; j < NPM; ++j)
            if (j < n) Q[r * ldq + j] = y[j];
    }
}

}  // namespace

int refine_blocks(int64_t m, int64_t n)
{
    (void)n;
    int64_t b = ceil_div(m, kRefineRows);
    return (int)(b < kRefineBlocks ? b : kRefineBlocks);
}

size_t refine_scratch_bytes(int64_t m, int64_t n)
{
    // partial Grams + Rc
    return sizeof(double) * ((size_t)refine_blocks(m, n) * n * n + (size_t)n * n);
}

hipError_t launch_refine(int64_t m, int64_t n, const double *A, int64_t lda, double *Rhat,
                         double *Q, int64_t ldq, double *R, int64_t ldr, void *scratch,
                         int32_t *info, hipStream_t st)
{
    const int nb = refine_blocks(m, n);
    double *Gpart = (double *)scratch;
    double *Rc = Gpart + (size_t)nb * n * n;
    const int qblocks = (int)((m + kThreads - 1) / kThreads < 2048 ? (m + kThreads - 1) / kThreads : 2048);
#define TSQR_REFINE_CASE(NPM)                                                                   \
    do {                                                                                        \
        hipLaunchKernelGGL((k_refine_gram<NPM>), dim3(nb), dim3(kThreads), 0, st, m, (int)n, A,   \
                           lda, Rhat, Gpart);                                                   \
        hipLaunchKernelGGL(k_refine_chol, dim3(1), dim3(kThreads), sizeof(double) * n * n, st,   \
                           (int)n, nb, Gpart, Rhat, Rc, R, ldr, info);                          \
        hipLaunchKernelGGL((k_refine_q<NPM>), dim3(qblocks), dim3(kThreads), 0, st, m, (int)n, A, \
                           lda, Rhat, Rc, Q, ldq);                                              \
    } while (0)
    if (n <= 16) TSQR_REFINE_CASE(16);
    else if (n <= 32) TSQR_REFINE_CASE(32);
    else if (n <= 64) TSQR_REFINE_CASE(64);
    else return hipErrorInvalidValue;
#undef TSQR_REFINE_CASE
    return hipGetLastError();
}

}  // namespace tsqr
