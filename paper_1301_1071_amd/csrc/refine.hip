// One FP64 refinement pass for the precision form (FP32 panels, FP64 tree).
//
// The paper's iterative refinement (Sec. I and Sec. II-C) repeats the QR on the computed Q; that
// restores orthogonality but cannot lift the backward error ||A - QR|| above the FP32 level, so
// the pass below refines against A itself (preconditioned Cholesky QR, Yamazaki, Tomov & Dongarra
// 2015): with Rhat the FP64-promoted R of the FP32 factorization,
//     Y = A Rhat^{-1}      (one MFMA product with the explicit inverse, stored),
//     G = Y^T Y = Rc^T Rc  (MFMA Gram, Cholesky in FP64),
//     R = Rc Rhat,  Q = Y Rc^{-1}  (a second MFMA product).
// Y has condition number 1 + O(u_32 kappa(A)), so the Cholesky step is well conditioned, and
// Q is formed from the same Y whose Gram gave Rc, which keeps Q^T Q = I to rounding.
#include "tsqr_internal.h"

namespace tsqr {
namespace {

// Xinv = X^{-1} for an upper-triangular n x n X (ld ldx): thread j solves column j by back
// substitution.  Skipped (left as garbage) when a diagonal entry is not positive; the caller's
// info reports it.
__device__ void tri_inv(int n, const double *__restrict__ X, int64_t ldx, double *__restrict__ Xinv)
{
    for (int j = threadIdx.x; j < n; j += blockDim.x) {
        for (int i = n - 1; i > j; --i) Xinv[i * n + j] = 0.0;
        for (int i = j; i >= 0; --i) {
            double acc = (i == j) ? 1.0 : 0.0;
            for (int t = i + 1; t <= j; ++t) acc = fma(-X[i * ldx + t], Xinv[t * n + j], acc);
            Xinv[i * n + j] = acc / X[i * ldx + i];
        }
    }
}

__global__ void __launch_bounds__(256)
k_refine_rinv(int n, const double *__restrict__ Rhat, double *__restrict__ Rinv)
{
    tri_inv(n, Rhat, n, Rinv);
}

// G = Rc^T Rc (right-looking Cholesky in LDS), R = Rc Rhat, Rcinv = Rc^{-1}; info = -2 when G
// is not positive definite.
__global__ void __launch_bounds__(256)
k_refine_chol(int n, const double *__restrict__ G, const double *__restrict__ Rhat,
              double *__restrict__ Rc, double *__restrict__ Rcinv, double *__restrict__ R,
              int64_t ldr, int32_t *info)
{
    extern __shared__ double Gs[];   // n x n
    __shared__ int s_fail;
    const int tid = threadIdx.x, nth = blockDim.x;
    if (tid == 0) s_fail = 0;
    for (int e = tid; e < n * n; e += nth) Gs[e] = G[e];
    __syncthreads();
    for (int k = 0; k < n; ++k) {
        const double d = Gs[k * n + k];
        if (!(d > 0.0)) {
            if (tid == 0) s_fail = 1;
            break;
        }
        const double rkk = sqrt(d);
        __syncthreads();
        for (int j = k + tid; j < n; j += nth) Gs[k * n + j] = (j == k) ? rkk : Gs[k * n + j] / rkk;
        __syncthreads();
        const int w = n - k - 1;
        for (int e = tid; e < w * w; e += nth) {
            const int i = k + 1 + e / w, j = k + 1 + e % w;
            if (j >= i) Gs[i * n + j] -= Gs[k * n + i] * Gs[k * n + j];
        }
        __syncthreads();
    }
    __syncthreads();
    for (int e = tid; e < n * n; e += nth) {
        const int i = e / n, j = e - i * n;
        Rc[e] = (j >= i) ? Gs[e] : 0.0;
    }
    __syncthreads();
    tri_inv(n, Rc, n, Rcinv);
    for (int e = tid; e < n * n; e += nth) {
        const int i = e / n, j = e - i * n;
        double a = 0.0;
        if (j >= i)
            for (int t = i; t <= j; ++t) a = fma(Rc[i * n + t], Rhat[t * n + j], a);
        R[(int64_t)i * ldr + j] = a;
    }
    if (tid == 0 && s_fail) *info = -2;
}

constexpr int kRefPanel = 256;   // rows per work-group of the two products

}  // namespace

int refine_blocks(int64_t m, int64_t n)
{
    (void)n;
    return gram_blocks(m);
}

size_t refine_scratch_bytes(int64_t m, int64_t n)
{
    // Y (m x n), Gram partials, G, Rinv, Rc, Rcinv (n x n each)
    const size_t nn = (size_t)n * n;
    return sizeof(double) * ((size_t)m * n + (size_t)refine_blocks(m, n) * nn + 4 * nn) + 1024;
}

hipError_t launch_refine(int64_t m, int64_t n, const double *A, int64_t lda, double *Rhat,
                         double *Q, int64_t ldq, double *R, int64_t ldr, void *scratch,
                         int32_t *info, hipStream_t st)
{
    if (n > 64) return hipErrorInvalidValue;
    const size_t nn = (size_t)n * n;
    double *Y = (double *)scratch;
    double *part = Y + (size_t)m * n;
    double *G = part + (size_t)refine_blocks(m, n) * nn;
    double *Rinv = G + nn, *Rc = Rinv + nn, *Rcinv = Rc + nn;
    hipLaunchKernelGGL(k_refine_rinv, dim3(1), dim3(256), 0, st, (int)n, Rhat, Rinv);
    hipError_t e = launch_gemm_mfma(F64, F64, m, n, kRefPanel, A, lda, Rinv, n, 0, (int)n, Y, n,
                                    (int)n, nullptr, 0, 0, st);
    if (e != hipSuccess) return e;
    if ((e = launch_gram(m, n, Y, n, Y, n, part, G, st)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_refine_chol, dim3(1), dim3(256), sizeof(double) * nn, st, (int)n, G, Rhat,
                       Rc, Rcinv, R, ldr, info);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    return launch_gemm_mfma(F64, F64, m, n, kRefPanel, Y, n, Rcinv, n, 0, (int)n, Q, ldq, (int)n,
                            nullptr, 0, 0, st);
}

}  // namespace tsqr
