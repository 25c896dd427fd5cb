// Register-resident panel kernels (the fast path for every tree level).
//
// Step 1 of direct TSQR (Sec. III-B) for one row panel per work-group, with the panel held in
// VGPRs: lane l owns column c = l % NC (plus c + 64 for n > 64) of row sub-group g = l / NC, and
// each lane holds RW rows of that column.  Householder column k (Sec. III-A) then needs
//   * the pivot column x = A[k:, k] of the lane's own rows: the lane owning column k copies its
//     rows into a per-wave LDS buffer and every lane reads them back as broadcasts;
//   * the dot products x^T A[:, c] for all columns: in-lane FMAs, a shuffle over the G row
//     sub-groups and one cross-wave sum through LDS (the only barrier of the step);
//   * a rank-1 update in registers.
// The explicit Q1 = H_1 ... H_n [I; 0] is then formed in a second register array by applying the
// reflectors backwards, with the same broadcast/reduce/update step, so step 3 is a plain product.
//
// Householder convention as in the LDS kernel: beta = -sign(alpha) sqrt(alpha^2 + s2),
// tau = (beta - alpha)/beta, v = [1; x_{1:}/(alpha - beta)]; the below-diagonal x is stored
// unscaled and the scale is folded into the coefficients.  Rows <= k of the broadcast buffer are
// zeroed by the writer, and row k is set to (alpha - beta) before the update, so the same FMA
// loop updates row k (by tau w_c) and rows > k (by tau w_c x_i / (alpha - beta)).
#include "tsqr_internal.h"

namespace tsqr {
namespace {

template <typename T>
__device__ __forceinline__ T shfl_xor_t(T v, int mask) { return __shfl_xor(v, mask, 64); }

// Panel geometry.  NC: lanes per row sub-group (power of two, >= n unless CPL == 2);
// CPL: columns per lane (1, or 2 for 64 < n <= 128); RW: rows per lane; NW: waves per group.
template <typename Tin, typename T, int NC, int CPL, int RW, int NW>
__global__ void __launch_bounds__(NW * 64)
k_factor_reg(int64_t rows, int n, const Tin *__restrict__ X, int64_t ldx, T *__restrict__ q1,
             double *__restrict__ S)
{
    constexpr int G = 64 / NC;              // row sub-groups per wave
    constexpr int GR = G * RW;              // rows per wave
    constexpr int B = NW * GR;              // panel rows
    constexpr int XS = RW + 2;              // padded stride of a sub-group's broadcast buffer
    __shared__ T xb[NW][G][XS];             // per-wave pivot-column broadcast buffers
    __shared__ T part[2][NW][64 * CPL];     // per-wave partial dots (double-buffered by step)
    __shared__ T rowk[2][64 * CPL];         // row k of the panel
    __shared__ T s_tau[kNmaxPad], s_umk[kNmaxPad], s_beta[kNmaxPad];

    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int cl = lane & (NC - 1);
    const int g = lane / NC;
    const int64_t p = blockIdx.x;
    const int64_t prow0 = p * (int64_t)B;
    const int nrow = (int)min((int64_t)B, rows - prow0);   // rows of X in this panel

    T a[RW][CPL];
    T q[RW][CPL];
#pragma unroll
    for (int i = 0; i < RW; ++i) {
        const int r = w * GR + i * G + g;               // panel row of register i
#pragma unroll
        for (int s = 0; s < CPL; ++s) {
            const int c = cl + 64 * s;
            a[i][s] = (r < nrow && c < n) ? (T)X[(prow0 + r) * ldx + c] : T(0);
            q[i][s] = (r == c) ? T(1) : T(0);           // [I; 0]
        }
    }

    // publish panel row `rr` (all columns) into rowk[buf]
    auto publish_row = [&](int rr, int buf) {
        const int wr = rr / GR, rem = rr - wr * GR;
        const int ir = rem / G, gr = rem - ir * G;
        if (w == wr && g == gr) {
#pragma unroll
            for (int i = 0; i < RW; ++i)
                if (i == ir) {
#pragma unroll
                    for (int s = 0; s < CPL; ++s) rowk[buf][cl + 64 * s] = a[i][s];
                }
        }
    };

    const int wmin = w * GR, wmax = w * GR + GR - 1;   // panel rows held by this wave

    // the lanes owning column k copy their rows of column k into the broadcast buffer; rows <= k
    // are written as zero (only the wave that straddles row k needs the mask)
    auto write_pivot = [&](int k, const T (&src)[RW][CPL]) {
        if (wmax < k) return;                         // every row of this wave is above k
        if (cl == (k & 63)) {
            const int s = k >> 6;
            if (wmin > k) {
#pragma unroll
                for (int i = 0; i < RW; ++i) xb[w][g][i] = (s == 0) ? src[i][0] : src[i][CPL - 1];
            } else {
                const int first = wmin + g;               // panel row of register 0
#pragma unroll
                for (int i = 0; i < RW; ++i) {
                    const T v = (s == 0) ? src[i][0] : src[i][CPL - 1];
                    xb[w][g][i] = (first + i * G > k) ? v : T(0);
                }
            }
        }
    };
    // partial dots x^T M[:, c] over this wave's rows (rows <= k contribute zero)
    auto pivot_dots = [&](int k, const T (&M)[RW][CPL], T (&d)[CPL]) {
#pragma unroll
        for (int s = 0; s < CPL; ++s) d[s] = T(0);
        if (wmax > k) {
#pragma unroll
            for (int s = 0; s < CPL; ++s) {
                T d0 = T(0), d1 = T(0);
#pragma unroll
                for (int i = 0; i < RW; i += 2) {
                    d0 = fma(xb[w][g][i], M[i][s], d0);
                    if (i + 1 < RW) d1 = fma(xb[w][g][i + 1], M[i + 1][s], d1);
                }
                d[s] = d0 + d1;
            }
        }
#pragma unroll
        for (int s = 0; s < CPL; ++s)
#pragma unroll
            for (int off = NC; off < 64; off <<= 1) d[s] += shfl_xor_t(d[s], off);
    };
    // M[i][c] -= coef_c * x_i with x_k = (alpha - beta): row k gets tau w_c, rows > k the rest
    auto pivot_update = [&](int k, T umk, const T (&coef)[CPL], T (&M)[RW][CPL]) {
        if (wmax < k) return;
        if (wmin <= k) {
            const int rem = k - wmin;
            const int ir = rem / G, gr = rem - ir * G;
            if (g == gr && cl == (k & 63)) xb[w][g][ir] = umk;
        }
#pragma unroll
        for (int i = 0; i < RW; ++i) {
            const T x = xb[w][g][i];
#pragma unroll
            for (int s = 0; s < CPL; ++s) M[i][s] = fma(-coef[s], x, M[i][s]);
        }
    };

    if (nrow > 0) publish_row(0, 0);
    __syncthreads();

    // ---------------- factorization ------------------------------------------------------
    // One barrier per step: partial dots and the published row are double-buffered by step
    // parity, and every wave finishes reading step k-1's buffers before it reaches step k's
    // barrier.
    for (int k = 0; k < n; ++k) {
        const int par = k & 1;
        write_pivot(k, a);
        T d[CPL];
        pivot_dots(k, a, d);
        if (g == 0) {
#pragma unroll
            for (int s = 0; s < CPL; ++s) part[par][w][cl + 64 * s] = d[s];
        }
        __syncthreads();
        const T alpha = rowk[par][k];
        T s2 = T(0);
#pragma unroll
        for (int ww = 0; ww < NW; ++ww) s2 += part[par][ww][k];
        T tau = T(0), umk = T(0), beta = alpha;
        if (s2 != T(0)) {
            const T nrm = sqrt(alpha * alpha + s2);
            beta = (alpha >= T(0)) ? -nrm : nrm;
            tau = (beta - alpha) / beta;
            umk = alpha - beta;
        }
        if (threadIdx.x == 0) { s_tau[k] = tau; s_umk[k] = umk; s_beta[k] = beta; }
        if (tau != T(0)) {
            const T inv = T(1) / umk;
            T coef[CPL];
#pragma unroll
            for (int s = 0; s < CPL; ++s) {
                const int c = cl + 64 * s;
                T pc = T(0);
#pragma unroll
                for (int ww = 0; ww < NW; ++ww) pc += part[par][ww][c];
                coef[s] = (c > k && c < n) ? tau * (rowk[par][c] + inv * pc) * inv : T(0);
            }
            pivot_update(k, umk, coef, a);
        }
        if (k + 1 < n) publish_row(k + 1, par ^ 1);
    }
    __syncthreads();

    // R_p: rows 0..n-1 of the panel, strict upper part from the registers, diagonal = beta
#pragma unroll
    for (int i = 0; i < RW; ++i) {
        const int r = w * GR + i * G + g;
        if (r < n) {
#pragma unroll
            for (int s = 0; s < CPL; ++s) {
                const int c = cl + 64 * s;
                if (c < n)
                    S[(p * n + r) * n + c] =
                        (c > r) ? (double)a[i][s] : ((c == r) ? (double)s_beta[r] : 0.0);
            }
        }
    }
    if (q1 == nullptr) return;

    // ---------------- explicit Q1 = H_1 ... H_n [I; 0] -----------------------------------
    // (buffer parity follows the executed steps, so skipped steps keep the one-barrier scheme)
    int nstep = 0;
    for (int k = n - 1; k >= 0; --k) {
        const T tau = s_tau[k];
        if (tau == T(0)) continue;                     // uniform: H_k = I
        const int par = (nstep++) & 1;
        const T umk = s_umk[k];
        const T inv = T(1) / umk;
        write_pivot(k, a);
        T d[CPL];
        pivot_dots(k, q, d);
        if (g == 0) {
#pragma unroll
            for (int s = 0; s < CPL; ++s) part[par][w][cl + 64 * s] = d[s];
        }
        __syncthreads();
        T coef[CPL];
#pragma unroll
        for (int s = 0; s < CPL; ++s) {
            const int c = cl + 64 * s;
            T pc = T(0);
#pragma unroll
            for (int ww = 0; ww < NW; ++ww) pc += part[par][ww][c];
            // row k of Q1 is still e_k^T here, so v^T Q1[:, c] = delta_kc + inv * pc
            const T wc = ((c == k) ? T(1) : T(0)) + inv * pc;
            coef[s] = (c < n) ? tau * wc * inv : T(0);
        }
        pivot_update(k, umk, coef, q);
    }
#pragma unroll
    for (int i = 0; i < RW; ++i) {
        const int r = w * GR + i * G + g;
        if (r < nrow) {
#pragma unroll
            for (int s = 0; s < CPL; ++s) {
                const int c = cl + 64 * s;
                if (c < n) q1[(prow0 + r) * n + c] = q[i][s];
            }
        }
    }
}

// out rows of panel p = Q1_p (b x n) * W_p (n x k).  Q1 rows are staged through LDS in chunks
// of 64 rows (coalesced loads, broadcast reads); each lane owns JPL output columns whose W
// entries live in registers.
template <typename Tq, typename To, int NPM, int JPL>
__global__ void __launch_bounds__(256)
k_apply_staged(int64_t rows, int n, int b, const Tq *__restrict__ q1, const double *__restrict__ W,
               int64_t ldw, int64_t wstride, int k, To *__restrict__ out0, int64_t ld0, int k0,
               To *__restrict__ out1, int64_t ld1)
{
    constexpr int CH = (NPM * sizeof(Tq) <= 512) ? 64 : 32;   // rows per staged chunk
    constexpr int LDQ = NPM + 2;
    __shared__ Tq qs[2][CH][LDQ];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int64_t p = blockIdx.x;
    const int jbase = blockIdx.y * 64 * JPL;
    const double *Wp = W + p * wstride * ldw;
    Tq wr[NPM][JPL];
#pragma unroll
    for (int c = 0; c < NPM; ++c)
#pragma unroll
        for (int s = 0; s < JPL; ++s) {
            const int j = jbase + lane + 64 * s;
            wr[c][s] = (c < n && j < k) ? (Tq)Wp[(int64_t)c * ldw + j] : Tq(0);
        }
    const int64_t rb = p * (int64_t)b;
    const int nr = (int)min((int64_t)b, rows - rb);
    const int nchunks = (nr + CH - 1) / CH;
    auto stage = [&](int ch, int buf) {
        const int r0 = ch * CH;
        const int cnt = min(CH, nr - r0) * n;
        const Tq *src = q1 + (rb + r0) * n;
        for (int e = tid; e < cnt; e += 256) {
            const int r = e / n, c = e - r * n;
            qs[buf][r][c] = src[e];
        }
    };
    // the padding columns [n, NPM) of both buffers are read by the FMA loop: zero them once
    if (n < NPM)
        for (int e = tid; e < 2 * CH * (NPM - n); e += 256) {
            const int bufr = e / (NPM - n), c = n + e % (NPM - n);
            qs[bufr / CH][bufr % CH][c] = Tq(0);
        }
    if (nchunks > 0) stage(0, 0);
    __syncthreads();
    for (int ch = 0; ch < nchunks; ++ch) {
        const int buf = ch & 1;
        if (ch + 1 < nchunks) stage(ch + 1, buf ^ 1);
        const int r0 = ch * CH;
        const int rcnt = min(CH, nr - r0);
        for (int rr = w; rr < rcnt; rr += 4) {
            Tq acc[JPL];
#pragma unroll
            for (int s = 0; s < JPL; ++s) acc[s] = Tq(0);
#pragma unroll
            for (int c = 0; c < NPM; ++c) {
                const Tq qv = qs[buf][rr][c];
#pragma unroll
                for (int s = 0; s < JPL; ++s) acc[s] = fma(qv, wr[c][s], acc[s]);
            }
            const int64_t r = rb + r0 + rr;
#pragma unroll
            for (int s = 0; s < JPL; ++s) {
                const int j = jbase + lane + 64 * s;
                if (j < k0) out0[r * ld0 + j] = (To)acc[s];
                else if (j < k) out1[r * ld1 + (j - k0)] = (To)acc[s];
            }
        }
        __syncthreads();
    }
}

template <typename Tin, typename T, int NC, int CPL, int RW, int NW>
hipError_t factor_reg_launch(int64_t rows, int64_t n, const void *X, int64_t ldx, void *q1,
                             double *S, hipStream_t st)
{
    constexpr int B = NW * (64 / NC) * RW;
    const int64_t panels = ceil_div(rows, B);
    hipLaunchKernelGGL((k_factor_reg<Tin, T, NC, CPL, RW, NW>), dim3((unsigned)panels),
                       dim3(NW * 64), 0, st, rows, (int)n, (const Tin *)X, ldx, (T *)q1, S);
    return hipGetLastError();
}

// Register budget: a and q hold 2 * RW * CPL elements per lane.  FP64: 64 doubles (128 VGPRs)
// with 2 waves per SIMD; FP32 doubles RW for the same footprint.
template <typename T> struct RegCfg { static constexpr int RW = 32; };
template <> struct RegCfg<float> { static constexpr int RW = 64; };

template <typename Tin, typename T>
hipError_t factor_reg_dispatch(int64_t rows, int64_t n, const void *X, int64_t ldx, void *q1,
                               double *S, hipStream_t st)
{
    constexpr int RW = RegCfg<T>::RW;
    if (n <= 16) return factor_reg_launch<Tin, T, 16, 1, RW, 8>(rows, n, X, ldx, q1, S, st);
    if (n <= 32) return factor_reg_launch<Tin, T, 32, 1, RW, 8>(rows, n, X, ldx, q1, S, st);
    if (n <= 64) return factor_reg_launch<Tin, T, 64, 1, RW, 8>(rows, n, X, ldx, q1, S, st);
    return factor_reg_launch<Tin, T, 64, 2, RW / 2, 12>(rows, n, X, ldx, q1, S, st);
}

template <typename Tq, typename To, int NPM>
hipError_t apply_staged_np(int64_t rows, int64_t n, int b, const void *q1, const double *W,
                           int64_t ldw, int64_t wstride, int k, void *out0, int64_t ld0, int k0,
                           void *out1, int64_t ld1, hipStream_t st)
{
    const int64_t panels = ceil_div(rows, b);
    if (k > 64 && NPM <= 64) {
        dim3 grid((unsigned)panels, (unsigned)ceil_div(k, 128));
        hipLaunchKernelGGL((k_apply_staged<Tq, To, NPM, 2>), grid, dim3(256), 0, st, rows, (int)n,
                           b, (const Tq *)q1, W, ldw, wstride, k, (To *)out0, ld0, k0,
                           (To *)out1, ld1);
    } else {
        dim3 grid((unsigned)panels, (unsigned)ceil_div(k, 64));
        hipLaunchKernelGGL((k_apply_staged<Tq, To, NPM, 1>), grid, dim3(256), 0, st, rows, (int)n,
                           b, (const Tq *)q1, W, ldw, wstride, k, (To *)out0, ld0, k0,
                           (To *)out1, ld1);
    }
    return hipGetLastError();
}

template <typename Tq, typename To>
hipError_t apply_staged_dispatch(int64_t rows, int64_t n, int b, const void *q1, const double *W,
                                 int64_t ldw, int64_t wstride, int k, void *out0, int64_t ld0,
                                 int k0, void *out1, int64_t ld1, hipStream_t st)
{
#define TSQR_NP_CASE(NP)                                                                       \
    if (n <= NP)                                                                               \
        return apply_staged_np<Tq, To, NP>(rows, n, b, q1, W, ldw, wstride, k, out0, ld0, k0,  \
                                           out1, ld1, st);
    TSQR_NP_CASE(4) TSQR_NP_CASE(8) TSQR_NP_CASE(16) TSQR_NP_CASE(24) TSQR_NP_CASE(32)
    TSQR_NP_CASE(40) TSQR_NP_CASE(48) TSQR_NP_CASE(56) TSQR_NP_CASE(64) TSQR_NP_CASE(80)
    TSQR_NP_CASE(96) TSQR_NP_CASE(112) TSQR_NP_CASE(128)
#undef TSQR_NP_CASE
    return hipErrorInvalidValue;
}

}  // namespace

int reg_panel_rows(int64_t n, int dtype)
{
    const int rw = (dtype == F32) ? RegCfg<float>::RW : RegCfg<double>::RW;
    if (n <= 16) return 8 * 4 * rw;
    if (n <= 32) return 8 * 2 * rw;
    if (n <= 64) return 8 * 1 * rw;
    return 12 * 1 * (rw / 2);
}

hipError_t launch_factor_reg(int in_dtype, int dtype, int64_t rows, int64_t n, const void *X,
                             int64_t ldx, void *q1, double *S, hipStream_t st)
{
    if (dtype == F64) {
        if (in_dtype == F64) return factor_reg_dispatch<double, double>(rows, n, X, ldx, q1, S, st);
        return factor_reg_dispatch<float, double>(rows, n, X, ldx, q1, S, st);
    }
    if (in_dtype == F64) return factor_reg_dispatch<double, float>(rows, n, X, ldx, q1, S, st);
    return factor_reg_dispatch<float, float>(rows, n, X, ldx, q1, S, st);
}

hipError_t launch_apply_staged(int q_dtype, int out_dtype, int64_t rows, int64_t n, int b,
                               const void *q1, const double *W, int64_t ldw, int64_t wstride,
                               int k, void *out0, int64_t ld0, int k0, void *out1, int64_t ld1,
                               hipStream_t st)
{
    if (q_dtype == F64) {
        if (out_dtype == F64)
            return apply_staged_dispatch<double, double>(rows, n, b, q1, W, ldw, wstride, k, out0,
                                                         ld0, k0, out1, ld1, st);
        return apply_staged_dispatch<double, float>(rows, n, b, q1, W, ldw, wstride, k, out0, ld0,
                                                    k0, out1, ld1, st);
    }
    if (out_dtype == F64)
        return apply_staged_dispatch<float, double>(rows, n, b, q1, W, ldw, wstride, k, out0, ld0,
                                                    k0, out1, ld1, st);
    return apply_staged_dispatch<float, float>(rows, n, b, q1, W, ldw, wstride, k, out0, ld0, k0,
                                               out1, ld1, st);
}

}  // namespace tsqr
