// Error metrics of Sec. I-B on the GPU: ||Q^T Q - I||_2 and ||A - QR||_2 / ||A||_2 need Gram
// matrices summed over all m rows.  At m in the millions an FP64 sum of Q^T Q overstates the
// departure from I by orders of magnitude (the entries are 1 + O(u) and the rounding of the sum
// is O(m u)), so the sums here are double-double: TwoProd by FMA and TwoSum (Ogita, Rump & Oishi,
// "Accurate sum and dot product", 2005), as accurate as a sum in twice the working precision.
// The residual rows e = a - x B are formed with the same compensated dot product.  The n x n
// result goes to the caller, which takes its 2-norm.  Not part of the factorization.
#include "tsqr_internal.h"

namespace tsqr {
namespace {

constexpr int kMetThreads = 256;
constexpr int kMetRows = 32;         // rows staged per chunk
constexpr int kMetMaxBlocks = 1024;

__device__ __forceinline__ void two_sum(double a, double b, double &s, double &t)
{
    s = a + b;
    const double bb = s - a;
    t = (a - (s - bb)) + (b - bb);
}

// (hi, lo) += x y
__device__ __forceinline__ void dd_fma(double x, double y, double &hi, double &lo)
{
    const double p = x * y;
    const double ep = fma(x, y, -p);
    double s, t;
    two_sum(hi, p, s, t);
    hi = s;
    lo += t + ep;
}

// mode 0: X^T X - I; mode 1: E^T E with E = A - X B; mode 2: X^T X.  Upper triangle entries
// e = 0 .. n(n+1)/2 - 1 in row order, NE per thread; one double-double partial per work-group.
template <int NE>
__global__ void __launch_bounds__(kMetThreads)
k_metric(int mode, int64_t m, int n, const double *__restrict__ X, int64_t ldx,
         const double *__restrict__ A, int64_t lda, const double *__restrict__ B, int64_t ldb,
         double *__restrict__ part)
{
    extern __shared__ double cs[];          // kMetRows x (n + 1)
    const int tid = threadIdx.x;
    const int ld = n + 1;
    const int nent = n * (n + 1) / 2;
    int ei[NE], ej[NE];
#pragma unroll
    for (int q = 0; q < NE; ++q) {
        int e = tid + q * kMetThreads, i = 0;
        if (e < nent) {
            while (e >= n - i) { e -= n - i; ++i; }
            ei[q] = i;
            ej[q] = i + e;
        } else {
            ei[q] = -1;
            ej[q] = 0;
        }
    }
    double hi[NE], lo[NE];
#pragma unroll
    for (int q = 0; q < NE; ++q) { hi[q] = 0.0; lo[q] = 0.0; }
    const int64_t nchunks = (m + kMetRows - 1) / kMetRows;
    for (int64_t ch = blockIdx.x; ch < nchunks; ch += gridDim.x) {
        const int64_t r0 = ch * kMetRows;
        const int nr = (int)min((int64_t)kMetRows, m - r0);
        for (int e = tid; e < kMetRows * n; e += kMetThreads) {
            const int r = e / n, c = e - r * n;
            double v = 0.0;
            if (r < nr) {
                const double *xr = X + (r0 + r) * ldx;
                if (mode == 1) {
                    double s = A[(r0 + r) * lda + c], cc = 0.0;
                    for (int k = 0; k < n; ++k) dd_fma(-xr[k], B[(int64_t)k * ldb + c], s, cc);
                    v = s + cc;
                } else {
                    v = xr[c];
                }
            }
            cs[r * ld + c] = v;
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < NE; ++q) {
            if (ei[q] < 0) continue;
            for (int r = 0; r < nr; ++r) dd_fma(cs[r * ld + ei[q]], cs[r * ld + ej[q]], hi[q], lo[q]);
        }
        __syncthreads();
    }
    double *out = part + (size_t)blockIdx.x * 2 * nent;
#pragma unroll
    for (int q = 0; q < NE; ++q) {
        const int e = tid + q * kMetThreads;
        if (e < nent) {
            out[e] = hi[q];
            out[nent + e] = lo[q];
        }
    }
}

// Double-double sum of the partials; G (n x n, symmetric, ld n) = hi - [I] + lo.
__global__ void __launch_bounds__(256)
k_metric_sum(int mode, int n, int nblk, const double *__restrict__ part, double *__restrict__ G)
{
    const int nent = n * (n + 1) / 2;
    const int e0 = blockIdx.x * blockDim.x + threadIdx.x;
    if (e0 >= nent) return;
    double hi = 0.0, lo = 0.0;
    for (int b = 0; b < nblk; ++b) {
        const double *p = part + (size_t)b * 2 * nent;
        double s, t;
        two_sum(hi, p[e0], s, t);
        hi = s;
        lo += t + p[nent + e0];
    }
    int e = e0, i = 0;
    while (e >= n - i) { e -= n - i; ++i; }
    const int j = i + e;
    if (mode == 0 && i == j) hi -= 1.0;     // exact for hi near 1
    const double v = hi + lo;
    G[(int64_t)i * n + j] = v;
    G[(int64_t)j * n + i] = v;
}

int metric_blocks(int64_t m)
{
    return (int)std::min<int64_t>((m + kMetRows - 1) / kMetRows, kMetMaxBlocks);
}

template <int NE>
hipError_t launch_metric_t(int mode, int64_t m, int64_t n, const double *X, int64_t ldx,
                           const double *A, int64_t lda, const double *B, int64_t ldb,
                           double *part, hipStream_t st)
{
    const size_t lds = sizeof(double) * kMetRows * (n + 1);
    hipLaunchKernelGGL(k_metric<NE>, dim3(metric_blocks(m)), dim3(kMetThreads), lds, st, mode, m,
                       (int)n, X, ldx, A, lda, B, ldb, part);
    return hipGetLastError();
}

}  // namespace
}  // namespace tsqr

using namespace tsqr;

extern "C" {

tsqr_status tsqr_metric_workspace_bytes(int64_t m, int64_t n, size_t *bytes)
{
    if (!bytes || m <= 0 || n <= 0) return TSQR_ERR_INVALID_ARG;
    if (n > TSQR_NMAX_SMALL) return TSQR_ERR_SHAPE;
    *bytes = sizeof(double) * 2 * (size_t)metric_blocks(m) * (size_t)(n * (n + 1) / 2);
    return TSQR_OK;
}

tsqr_status tsqr_metric_gram(int32_t mode, int64_t m, int64_t n, const double *X, int64_t ldx,
                             const double *A, int64_t lda, const double *B, int64_t ldb,
                             double *G, void *ws, size_t ws_bytes, void *stream)
{
    if (mode < 0 || mode > 2 || !X || !G || m <= 0 || n <= 0 || ldx < n)
        return TSQR_ERR_INVALID_ARG;
    if (mode == 1 && (!A || !B || lda < n || ldb < n)) return TSQR_ERR_INVALID_ARG;
    if (n > TSQR_NMAX_SMALL) return TSQR_ERR_SHAPE;
    size_t need = 0;
    tsqr_metric_workspace_bytes(m, n, &need);
    if (!ws || ws_bytes < need) return TSQR_ERR_WORKSPACE;
    hipStream_t st = (hipStream_t)stream;
    double *part = (double *)ws;
    const int nent = (int)(n * (n + 1) / 2);
    const int ne = (nent + kMetThreads - 1) / kMetThreads;
    hipError_t e;
    if (ne <= 4) e = launch_metric_t<4>(mode, m, n, X, ldx, A, lda, B, ldb, part, st);
    else if (ne <= 8) e = launch_metric_t<8>(mode, m, n, X, ldx, A, lda, B, ldb, part, st);
    else if (ne <= 16) e = launch_metric_t<16>(mode, m, n, X, ldx, A, lda, B, ldb, part, st);
    else e = launch_metric_t<33>(mode, m, n, X, ldx, A, lda, B, ldb, part, st);
    if (e != hipSuccess) {
        set_last_error(e, "k_metric", __LINE__);
        return TSQR_ERR_HIP;
    }
    hipLaunchKernelGGL(k_metric_sum, dim3((nent + 255) / 256), dim3(256), 0, st, (int)mode, (int)n,
                       metric_blocks(m), part, G);
    e = hipGetLastError();
    if (e != hipSuccess) {
        set_last_error(e, "k_metric_sum", __LINE__);
        return TSQR_ERR_HIP;
    }
    return TSQR_OK;
}

}  // extern "C"
