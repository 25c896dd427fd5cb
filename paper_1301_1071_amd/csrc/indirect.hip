// The comparison methods of the stability experiment (Sec. IV), on the GPU:
//   Cholesky QR (Sec. II-A)   R^T R = A^T A (the Gram summed over row blocks, then a Cholesky
//                              factorization of the n x n sum), Q = A R^{-1};
//   indirect TSQR (Sec. II-B) R from the stacked-R reduction alone (steps 1-2 of direct TSQR),
//                              Q = A R^{-1};
// with Q = A R^{-1} formed as the paper describes it (Sec. II-C): the explicit inverse of the
// triangular R, then one product with A.  Iterative refinement (Sec. I: the QR repeated once on
// the computed Q) gives Q = Q1 R2^{-1}, R = R2 R1.  Not part of direct TSQR; they exist so that
// the stability experiment can run beside it on the same GPU.
#include "tsqr_internal.h"

namespace tsqr {
namespace {

constexpr int kSmallThreads = 256;

// R^{-1} of an upper-triangular n x n R (ld n) by back substitution, one column per thread
// (R X = e_j), into X (ld n).
__device__ void upper_inverse(int n, const double *__restrict__ R, double *__restrict__ X)
{
    for (int j = threadIdx.x; j < n; j += blockDim.x) {
        for (int i = n - 1; i >= 0; --i) {
            double acc = (i == j) ? 1.0 : 0.0;
            for (int t = i + 1; t <= j; ++t) acc = fma(-R[i * n + t], X[t * n + j], acc);
            X[i * n + j] = (i <= j) ? acc / R[i * n + i] : 0.0;
        }
    }
}

// Cholesky QR's small step: G = L L^T (column by column, in LDS), R = L^T, Rinv = R^{-1}.  A pivot
// that is not positive (G not numerically positive definite) sets info = -4 and leaves R = Rinv =
// I so that nothing non-finite follows.
__global__ void __launch_bounds__(kSmallThreads)
k_cholqr_small(int n, const double *__restrict__ G, double *__restrict__ R,
               double *__restrict__ Rinv, int32_t *info, int keep_info)
{
    extern __shared__ double Ls[];          // n x n, Ls[i*n + j] = R[j][i] = L[i][j]
    __shared__ int s_fail;
    const int tid = threadIdx.x;
    if (tid == 0) s_fail = 0;
    for (int e = tid; e < n * n; e += blockDim.x) Ls[e] = G[e];
    __syncthreads();
    for (int j = 0; j < n; ++j) {
        // L[j][j] = sqrt(G[j][j] - sum_k L[j][k]^2); L[i][j] = (G[i][j] - sum_k L[i][k] L[j][k]) / L[j][j]
        __shared__ double s_ljj;
        if (tid == 0) {
            double d = Ls[j * n + j];
            for (int k = 0; k < j; ++k) d -= Ls[j * n + k] * Ls[j * n + k];
            if (!(d > 0.0)) s_fail = 1;
            s_ljj = (d > 0.0) ? sqrt(d) : 1.0;
            Ls[j * n + j] = s_ljj;
        }
        __syncthreads();
        if (s_fail) break;
        for (int i = j + 1 + tid; i < n; i += blockDim.x) {
            double x = Ls[i * n + j];
            for (int k = 0; k < j; ++k) x -= Ls[i * n + k] * Ls[j * n + k];
            Ls[i * n + j] = x / s_ljj;
        }
        __syncthreads();
    }
    const bool ok = (s_fail == 0);
    for (int e = tid; e < n * n; e += blockDim.x) {
        const int i = e / n, j = e - i * n;
        R[e] = ok ? ((j >= i) ? Ls[j * n + i] : 0.0) : (i == j ? 1.0 : 0.0);
    }
    __syncthreads();
    upper_inverse(n, R, Rinv);
    // keep_info: the refinement's second QR keeps a condition the first one reported
    if (tid == 0 && (!keep_info || *info == 0)) *info = ok ? 0 : -4;
}

// Rinv = R^{-1} (indirect TSQR's R from the finalize step, diag > 0).
__global__ void __launch_bounds__(kSmallThreads)
k_rinv_small(int n, const double *__restrict__ R, double *__restrict__ Rinv)
{
    upper_inverse(n, R, Rinv);
}

// Rout (ldr) = R2 R1 (upper-triangular n x n products, ld n); R2 == nullptr copies R1.
__global__ void __launch_bounds__(kSmallThreads)
k_trmul_small(int n, const double *__restrict__ R2, const double *__restrict__ R1,
              double *__restrict__ Rout, int64_t ldr)
{
    for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
        const int i = e / n, j = e - i * n;
        double a = 0.0;
        if (j >= i) {
            if (R2)
                for (int t = i; t <= j; ++t) a = fma(R2[i * n + t], R1[t * n + j], a);
            else
                a = R1[i * n + j];
        }
        Rout[(int64_t)i * ldr + j] = a;
    }
}

}  // namespace

hipError_t launch_cholqr_small(int64_t n, const double *G, double *R, double *Rinv, int32_t *info,
                               int keep_info, hipStream_t st)
{
    const size_t lds = sizeof(double) * (size_t)n * n;
    hipError_t e = ensure_dynamic_lds((const void *)k_cholqr_small, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_cholqr_small, dim3(1), dim3(kSmallThreads), lds, st, (int)n, G, R, Rinv,
                       info, keep_info);
    return hipGetLastError();
}

hipError_t launch_rinv_small(int64_t n, const double *R, double *Rinv, hipStream_t st)
{
    hipLaunchKernelGGL(k_rinv_small, dim3(1), dim3(kSmallThreads), 0, st, (int)n, R, Rinv);
    return hipGetLastError();
}

hipError_t launch_trmul_small(int64_t n, const double *R2, const double *R1, double *Rout,
                              int64_t ldr, hipStream_t st)
{
    hipLaunchKernelGGL(k_trmul_small, dim3(1), dim3(kSmallThreads), 0, st, (int)n, R2, R1, Rout,
                       ldr);
    return hipGetLastError();
}

}  // namespace tsqr
