// Panel kernels with the row panel resident in LDS or, for panels too tall or too wide for LDS, in
// a global scratch panel (general n <= TSQR_NMAX, FP64 or FP32).
//
// Step 1 of direct TSQR (Sec. III-B): one work-group factors one row panel A_p = Q1_p R_p with
// Householder reflections (Sec. III-A), writes R_p into the stacked-R buffer (block p = rows
// [p n, p n + n), the ordering the step-2 reduce task relies on) and, when Q is wanted, forms
// Q1_p = H_1 ... H_n [I; 0] explicitly so that step 3 is a plain product Q1_p * Q2_p.  Used for
// explicitly requested panel heights (tsqr_opts.panel_rows), short FP32 stacks and every level
// of the wide path (n > 128), whose panels live in global scratch.
//
// Householder convention: for column k, x = A[k:, k], alpha = x_0, s2 = ||x_{1:}||^2;
// beta = -sign(alpha) sqrt(alpha^2 + s2) (sign(0) = +1), tau = (beta - alpha) / beta and
// v = [1; x_{1:} / (alpha - beta)], so that (I - tau v v^T) x = beta e_1.  s2 == 0 means no
// reflection (tau = 0).  The below-diagonal part of x is kept unscaled in the panel and the scale
// 1 / (alpha - beta) is folded into the update coefficients.
#include "tsqr_internal.h"

namespace tsqr {
namespace {

constexpr int kLdsBudget = 150 * 1024;   // bytes of LDS used by one panel work-group

template <typename T>
__device__ __forceinline__ T shfl_xor(T v, int mask) { return __shfl_xor(v, mask, 64); }

// NPAD: column capacity of the small per-column LDS arrays (128, or 512 for the wide path).
// GP: the panel lives in the global scratch gpanel (known at compile time, so that LDS panels
// are addressed with LDS instructions).
template <typename Tin, typename T, int NPAD, bool GP>
__global__ void __launch_bounds__(kThreads)
k_factor_lds(int64_t rows, int n, int b, int ldp, int nc_log2, const Tin *__restrict__ X,
             int64_t ldx, T *__restrict__ q1, double *__restrict__ S, T *gpanel)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ T red[4 * NPAD];                   // per-wave partial dots
    __shared__ T rowk[NPAD];                      // row k of the panel, published per step
    __shared__ T s_tau[NPAD];
    __shared__ T s_umk[NPAD];                     // alpha - beta
    __shared__ T s_beta[NPAD];                    // R_kk
    // the panel: in LDS n columns of ldp rows (column-major, odd stride: lanes walking down
    // different columns hit different banks); for panels too tall or wide for LDS, a global
    // scratch panel (one per work-group) in row-major order, so that the lanes of a wave, which
    // own consecutive columns, read consecutive addresses of a row
    T *P = GP ? gpanel + (size_t)blockIdx.x * n * ldp : reinterpret_cast<T *>(smem_raw);
    const size_t sr = GP ? (size_t)n : 1, sc = GP ? 1 : (size_t)ldp;
    auto at = [&](int i, int c) -> T & { return P[(size_t)i * sr + (size_t)c * sc]; };

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int NC = 1 << nc_log2;                   // columns per pass
    const int G = 64 >> nc_log2;                   // row sub-groups per wave
    const int cl = lane & (NC - 1);
    const int g = lane >> nc_log2;
    const int npass = (n + NC - 1) / NC;

    const int64_t p = blockIdx.x;
    const int64_t prow0 = p * (int64_t)b;
    const int bp = (int)min((int64_t)b, rows - prow0);   // rows of A in this panel
    const int re = max(bp, n);                            // rows processed (zero padded)

    for (int64_t e = tid; e < (int64_t)re * n; e += kThreads) {
        const int i = (int)(e / n), c = (int)(e - (int64_t)i * n);
        at(i, c) = (i < bp) ? (T)X[(prow0 + i) * ldx + c] : T(0);
    }
    __syncthreads();

    const int rs = (re + 3) / 4;
    const int r0 = w * rs, r1 = min(re, r0 + rs);

    // ---------------- factorization ------------------------------------------------------
    for (int k = 0; k < n; ++k) {
        const int i0 = max(r0, k + 1);
        for (int ps = 0; ps < npass; ++ps) {
            const int c = cl + ps * NC;
            T d = T(0);
            if (c >= k && c < n)
                for (int i = i0 + g; i < r1; i += G) d = fma(at(i, k), at(i, c), d);
            for (int off = NC; off < 64; off <<= 1) d += shfl_xor(d, off);
            if (g == 0 && c < n) {
                red[w * NPAD + c] = d;
                if (w == 0) rowk[c] = at(k, c);
            }
        }
        __syncthreads();
        const T alpha = rowk[k];
        const T s2 = red[k] + red[NPAD + k] + red[2 * NPAD + k] + red[3 * NPAD + k];
        T tau = T(0), umk = T(0), beta = alpha;
        if (s2 != T(0)) {
            const T nrm = sqrt(alpha * alpha + s2);
            beta = (alpha >= T(0)) ? -nrm : nrm;
            tau = (beta - alpha) / beta;
            umk = alpha - beta;
        }
        if (tid == 0) { s_tau[k] = tau; s_umk[k] = umk; s_beta[k] = beta; }
        if (tau != T(0)) {
            const T inv = T(1) / umk;
            for (int ps = 0; ps < npass; ++ps) {
                const int c = cl + ps * NC;
                if (c > k && c < n) {
                    const T pcs = red[c] + red[NPAD + c] + red[2 * NPAD + c] + red[3 * NPAD + c];
                    const T wc = rowk[c] + inv * pcs;          // v^T A[k:, c]
                    const T coef = tau * wc * inv;
                    for (int i = i0 + g; i < r1; i += G) at(i, c) = fma(-coef, at(i, k), at(i, c));
                    if (w == 0 && g == 0) at(k, c) = rowk[c] - tau * wc;
                }
            }
        }
        __syncthreads();
    }

    // R_p into the stacked buffer: upper triangle of the top n rows, diagonal = beta
    for (int e = tid; e < n * n; e += kThreads) {
        const int r = e / n, c = e - r * n;
        const double v = (c > r) ? (double)at(r, c) : ((c == r) ? (double)s_beta[r] : 0.0);
        S[(p * n + r) * n + c] = v;
    }
    if (q1 == nullptr) return;

    // ---------------- explicit Q1 = H_1 ... H_n [I; 0], in place (backward accumulation) ---
    for (int k = n - 1; k >= 0; --k) {
        const T tau = s_tau[k];
        const T umk = s_umk[k];
        const T inv = (umk != T(0)) ? T(1) / umk : T(0);
        const int i0 = max(r0, k + 1);
        for (int ps = 0; ps < npass; ++ps) {
            const int c = cl + ps * NC;
            T d = T(0);
            if (c > k && c < n && tau != T(0))
                for (int i = i0 + g; i < r1; i += G) d = fma(at(i, k), at(i, c), d);
            for (int off = NC; off < 64; off <<= 1) d += shfl_xor(d, off);
            if (g == 0 && c < n) red[w * NPAD + c] = d;
        }
        __syncthreads();
        if (tau != T(0)) {
            for (int ps = 0; ps < npass; ++ps) {
                const int c = cl + ps * NC;
                if (c > k && c < n) {
                    // row k of column c is zero here (cleared when column c was formed)
                    const T wc = inv * (red[c] + red[NPAD + c] + red[2 * NPAD + c] + red[3 * NPAD + c]);
                    const T coef = tau * wc * inv;
                    for (int i = i0 + g; i < r1; i += G) at(i, c) = fma(-coef, at(i, k), at(i, c));
                    if (w == 0 && g == 0) at(k, c) = -tau * wc;
                }
            }
        }
        __syncthreads();
        const T sk = -tau * inv;
        for (int i = tid; i < re; i += kThreads) {
            const T v = (i > k) ? sk * at(i, k) : ((i == k) ? T(1) - tau : T(0));
            at(i, k) = v;
        }
        __syncthreads();
    }
    for (int64_t e = tid; e < (int64_t)bp * n; e += kThreads) {
        const int i = (int)(e / n), c = (int)(e - (int64_t)i * n);
        q1[(prow0 + i) * n + c] = at(i, c);
    }
}

template <typename T>
size_t lds_bytes(int n, int b) { return sizeof(T) * (size_t)n * (b + 1); }

int nc_log2_for(int64_t n)
{
    int l = 0;
    while ((1 << l) < n && l < 6) ++l;
    return l;
}

template <typename Tin, typename T>
hipError_t factor_impl(int64_t rows, int64_t n, int b, const void *X, int64_t ldx, void *q1,
                       double *S, void *gpanel, hipStream_t st)
{
    const size_t lds = gpanel ? 0 : lds_bytes<T>((int)n, b);
    if (n > kNmaxWide || (n > kNmaxPad && !gpanel)) return hipErrorInvalidValue;
    auto kern = (n > kNmaxPad) ? k_factor_lds<Tin, T, kNmaxWide, true>
                : gpanel ? k_factor_lds<Tin, T, kNmaxPad, true> : k_factor_lds<Tin, T, kNmaxPad, false>;
    hipError_t e = ensure_dynamic_lds((const void *)kern, lds);
    if (e != hipSuccess) return e;
    const int64_t panels = ceil_div(rows, b);
    hipLaunchKernelGGL(kern, dim3((unsigned)panels), dim3(kThreads), lds, st, rows, (int)n, b,
                       b + 1, nc_log2_for(n), (const Tin *)X, ldx, (T *)q1, S, (T *)gpanel);
    return hipGetLastError();
}

}  // namespace

int lds_panel_rows_max(int64_t n, int dtype)
{
    const size_t es = (dtype == F32) ? 4 : 8;
    const int64_t elems = (int64_t)(kLdsBudget / es);
    int64_t b = elems / n - 1;
    b = b / 16 * 16;
    if (b > 4096) b = 4096;
    return (int)b;
}

int lds_panel_rows(int64_t n, int dtype)
{
    int64_t b = lds_panel_rows_max(n, dtype);
    if (b > 2048) b = 2048;
    return (int)b;
}

hipError_t launch_factor(int in_dtype, int dtype, int64_t rows, int64_t n, int b, const void *X,
                         int64_t ldx, void *q1, double *S, void *gpanel, hipStream_t st)
{
    if (dtype == F64) {
        if (in_dtype == F64)
            return factor_impl<double, double>(rows, n, b, X, ldx, q1, S, gpanel, st);
        return factor_impl<float, double>(rows, n, b, X, ldx, q1, S, gpanel, st);
    }
    if (in_dtype == F64) return factor_impl<double, float>(rows, n, b, X, ldx, q1, S, gpanel, st);
    return factor_impl<float, float>(rows, n, b, X, ldx, q1, S, gpanel, st);
}

}  // namespace tsqr
