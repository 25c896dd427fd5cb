// Register-resident Householder panel factorization: the device body shared by the
// single-matrix kernels (panel_reg.hip) and the batched ones (batched.hip).
//
// Step 1 of direct TSQR (Sec. III-B) for one row panel per work-group, with the panel held in
// VGPRs: lane l owns column c = l % NC (plus c + 64 for n > 64) of row sub-group g = l / NC, and
// each lane holds RW rows of that column.  Householder column k (Sec. III-A) then needs
//   * the pivot column x = A[k:, k] of the lane's own rows: the lane owning column k copies its
//     rows into a per-wave LDS buffer (or, with one sub-group, hands them out by v_readlane);
//   * the dot products x^T A[:, c] for all columns: in-lane FMAs, a shuffle over the G row
//     sub-groups and one cross-wave sum through LDS (the only barrier of the step);
//   * a rank-1 update in registers.
// The explicit Q1 = H_1 ... H_n [I; 0] is then formed in place by applying the reflectors
// backwards, with the same broadcast/reduce/update step, so step 3 is a plain product.
//
// Householder convention: beta = -sign(alpha) sqrt(alpha^2 + s2), tau = (beta - alpha)/beta,
// v = [1; x_{1:}/(alpha - beta)]; the below-diagonal x is stored unscaled and the scale is folded
// into the coefficients.  Rows <= k of the broadcast buffer are zeroed by the writer, and row k is
// set to (alpha - beta) before the update, so the same FMA loop updates row k (by tau w_c) and
// rows > k (by tau w_c x_i / (alpha - beta)).
#pragma once

#include "tsqr_internal.h"

namespace tsqr {
namespace regpanel {

template <typename T>
__device__ __forceinline__ T shfl_xor_t(T v, int mask) { return __shfl_xor(v, mask, 64); }

// Refined reciprocal: v_rcp plus one Newton step (relative error a few ulp), used for the two
// divisions of each Householder step, whose latency sits on the critical path of every column.
__device__ __forceinline__ double fast_rcp(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    r = fma(r, fma(-x, r, 1.0), r);
    return fma(r, fma(-x, r, 1.0), r);
}
__device__ __forceinline__ float fast_rcp(float x)
{
    float r = __builtin_amdgcn_rcpf(x);
    return fmaf(r, fmaf(-x, r, 1.0f), r);
}

// Broadcast lane `src` (wave-uniform) of v to the whole wave through v_readlane (scalar result).
__device__ __forceinline__ double readlane_t(double v, int src)
{
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), src);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), src);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ float readlane_t(float v, int src)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), src));
}

// Panel geometry.  NC: lanes per row sub-group (power of two, >= n unless CPL == 2);
// CPL: columns per lane (1, or 2 for 64 < n <= 128); RW: rows per lane; NW: waves per group.
// Lane l holds rows  w*G*RW + i*G + g  (i < RW, g = l / NC) of column  l % NC (+ 64 s).
template <typename Tin, typename T, int NC, int CPL, int RW, int NW>
__device__ __forceinline__ void factor_reg_panel(int64_t rows, int n, const Tin *__restrict__ X,
                                                 int64_t ldx, T *__restrict__ q1,
                                                 double *__restrict__ S, int64_t p)
{
    constexpr int G = 64 / NC;              // row sub-groups per wave
    constexpr int GR = G * RW;              // rows per wave
    constexpr int B = NW * GR;              // panel rows
    constexpr int XS = RW + 2;              // padded stride of a sub-group's broadcast buffer
    __shared__ T xb[2][NW][G][XS];          // pivot-column broadcast buffers, by step parity
    __shared__ T part[2][NW][64 * CPL];     // per-wave partial dots, by step parity
    __shared__ T rowk[2][64 * CPL];         // row k of the panel, by step parity
    __shared__ T s_tau[kNmaxPad], s_umk[kNmaxPad], s_beta[kNmaxPad];

    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int cl = lane & (NC - 1);
    const int g = lane / NC;
    const int64_t prow0 = p * (int64_t)B;
    const int nrow = (int)min((int64_t)B, rows - prow0);   // rows of X in this panel
    const int wmin = w * GR, wmax = w * GR + GR - 1;      // panel rows held by this wave
    const int row0 = wmin + g;                             // panel row of register 0

    T a[RW][CPL];
#pragma unroll
    for (int i = 0; i < RW; ++i) {
        const int r = row0 + i * G;
#pragma unroll
        for (int s = 0; s < CPL; ++s) {
            const int c = cl + 64 * s;
            a[i][s] = (r < nrow && c < n) ? (T)X[(prow0 + r) * ldx + c] : T(0);
        }
    }
    auto colv = [&](int i, int slot) -> T { return (CPL == 1 || slot == 0) ? a[i][0] : a[i][CPL - 1]; };

    // The lanes owning column kk copy their rows of it into xb[buf]; rows <= kk are zeroed.
    // With one row sub-group (G == 1) a row's pivot value sits in lane (k & 63) of the same
    // wave, so it is broadcast with v_readlane straight into scalar registers (kept in xs for
    // the update) and the LDS pivot buffers are not used.
    T xs[RW];
#pragma unroll
    for (int i = 0; i < RW; ++i) xs[i] = T(0);

    // (a wave whose last row is kk still writes its zeros: its row kk receives alpha - beta)
    auto write_pivot = [&](int kk, int buf) {
        if (G == 1) return;
        if (wmax < kk || cl != (kk & 63)) return;
        const int slot = kk >> 6;
        if (wmin > kk) {
#pragma unroll
            for (int i = 0; i < RW; ++i) xb[buf][w][g][i] = colv(i, slot);
        } else {
#pragma unroll
            for (int i = 0; i < RW; ++i) xb[buf][w][g][i] = (row0 + i * G > kk) ? colv(i, slot) : T(0);
        }
    };
    // partial dots x^T a[:, c] over this wave's rows > k, reduced over the row sub-groups
    auto pivot_dots = [&](int k, int buf, T (&d)[CPL]) {
#pragma unroll
        for (int s = 0; s < CPL; ++s) d[s] = T(0);
        if (G == 1) {
            if (wmax > k) {
                const int src = k & 63, slot = k >> 6;
                T d0[CPL], d1[CPL];
#pragma unroll
                for (int s = 0; s < CPL; ++s) { d0[s] = T(0); d1[s] = T(0); }
#pragma unroll
                for (int i = 0; i < RW; ++i) {
                    T x = readlane_t((CPL == 1 || slot == 0) ? a[i][0] : a[i][CPL - 1], src);
                    x = (wmin + i > k) ? x : T(0);
                    xs[i] = x;
#pragma unroll
                    for (int s = 0; s < CPL; ++s) {
                        if (i & 1) d1[s] = fma(x, a[i][s], d1[s]);
                        else d0[s] = fma(x, a[i][s], d0[s]);
                    }
                }
#pragma unroll
                for (int s = 0; s < CPL; ++s) d[s] = d0[s] + d1[s];
            } else {
#pragma unroll
                for (int i = 0; i < RW; ++i) xs[i] = T(0);
            }
            return;
        }
        if (wmax > k) {
#pragma unroll
            for (int s = 0; s < CPL; ++s) {
                T d0 = T(0), d1 = T(0);
#pragma unroll
                for (int i = 0; i < RW; i += 2) {
                    d0 = fma(xb[buf][w][g][i], a[i][s], d0);
                    if (i + 1 < RW) d1 = fma(xb[buf][w][g][i + 1], a[i + 1][s], d1);
                }
                d[s] = d0 + d1;
            }
        }
#pragma unroll
        for (int s = 0; s < CPL; ++s)
#pragma unroll
            for (int off = NC; off < 64; off <<= 1) d[s] += shfl_xor_t(d[s], off);
    };
    // a[i][c] -= coef_c x_i over rows >= k, with x_k = (alpha - beta) so that row k moves by
    // tau w_c.  Fused: the lanes owning column kn copy their updated rows into xb[nbuf] (the
    // next pivot, rows <= kn zeroed), and row kn is published into rowk[nbuf] when pub is set.
    auto pivot_update = [&](int k, int buf, T umk, const T (&coef)[CPL], int kn, int nbuf,
                            bool pub) {
        if (G == 1) {
            if (wmax >= k) {
#pragma unroll
                for (int i = 0; i < RW; ++i) {
                    const T x = (wmin + i == k) ? umk : xs[i];
#pragma unroll
                    for (int s = 0; s < CPL; ++s) a[i][s] = fma(-coef[s], x, a[i][s]);
                }
            }
            const bool pubw1 = pub && kn < n && wmin <= kn && wmax >= kn;
            if (pubw1) {
#pragma unroll
                for (int i = 0; i < RW; ++i)
                    if (wmin + i == kn) {
#pragma unroll
                        for (int s = 0; s < CPL; ++s) rowk[nbuf][cl + 64 * s] = a[i][s];
                    }
            }
            return;
        }
        if (wmax < k) {
            // nothing to update here, but in the backward sweep (kn = k - 1) this wave may hold
            // row kn and needs its pivot buffer for the next step
            if (kn >= 0 && kn < n) write_pivot(kn, nbuf);
            return;
        }
        if (wmin <= k) {
            const int rem = k - wmin, ir = rem / G, gr = rem - ir * G;
            if (g == gr && cl == (k & 63)) xb[buf][w][g][ir] = umk;
        }
        const bool own = (kn >= 0 && kn < n) && wmax >= kn && cl == (kn & 63);
        const int nslot = kn >> 6;
        const bool pubw = pub && kn < n && wmin <= kn && wmax >= kn;
        const int remn = kn - wmin, irn = pubw ? remn / G : -1, grn = pubw ? remn - (remn / G) * G : -1;
        // reads and FMAs first (no stores in between, so the LDS reads stay pipelined) ...
#pragma unroll
        for (int i = 0; i < RW; ++i) {
            const T x = xb[buf][w][g][i];
#pragma unroll
            for (int s = 0; s < CPL; ++s) a[i][s] = fma(-coef[s], x, a[i][s]);
        }
        // ... then the next pivot and the published row
        if (own) {
            if (wmin > kn) {
#pragma unroll
                for (int i = 0; i < RW; ++i) xb[nbuf][w][g][i] = colv(i, nslot);
            } else {
#pragma unroll
                for (int i = 0; i < RW; ++i)
                    xb[nbuf][w][g][i] = (row0 + i * G > kn) ? colv(i, nslot) : T(0);
            }
        }
        if (pubw && g == grn) {
#pragma unroll
            for (int i = 0; i < RW; ++i)
                if (i == irn) {
#pragma unroll
                    for (int s = 0; s < CPL; ++s) rowk[nbuf][cl + 64 * s] = a[i][s];
                }
        }
    };

    // row 0 and pivot 0 for the first step
    if (w == 0 && g == 0) {
#pragma unroll
        for (int s = 0; s < CPL; ++s) rowk[0][cl + 64 * s] = a[0][s];
    }
    write_pivot(0, 0);
    __syncthreads();

    // ---------------- factorization ------------------------------------------------------
    // One barrier per step: pivots, partial dots and the published row are double-buffered by
    // step parity, and every wave finishes reading step k-1's buffers before step k's barrier.
    for (int k = 0; k < n; ++k) {
        const int par = k & 1;
        T d[CPL];
        pivot_dots(k, par, d);
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
            tau = T(1) - alpha * fast_rcp(beta);      // (beta - alpha) / beta
            umk = alpha - beta;
        }
        if (threadIdx.x == 0) { s_tau[k] = tau; s_umk[k] = umk; s_beta[k] = beta; }
        T coef[CPL];
        if (tau != T(0)) {
            const T inv = fast_rcp(umk);
#pragma unroll
            for (int s = 0; s < CPL; ++s) {
                const int c = cl + 64 * s;
                T pc = T(0);
#pragma unroll
                for (int ww = 0; ww < NW; ++ww) pc += part[par][ww][c];
                coef[s] = (c > k && c < n) ? tau * (rowk[par][c] + inv * pc) * inv : T(0);
            }
        } else {
#pragma unroll
            for (int s = 0; s < CPL; ++s) coef[s] = T(0);
        }
        pivot_update(k, par, umk, coef, k + 1, par ^ 1, true);
    }
    __syncthreads();

    // R_p: rows 0..n-1 of the panel, strict upper part from the registers, diagonal = beta
#pragma unroll
    for (int i = 0; i < RW; ++i) {
        const int r = row0 + i * G;
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

    // ---------------- explicit Q1 = H_1 ... H_n [I; 0], in place ----------------------------
    // Backward accumulation as in LAPACK's orgqr: step k updates the already formed columns
    // c > k and then turns column k into e_k - tau v_k.  Column c is kept as sig_c * a[:, c]
    // (a per-lane scale), so forming column k only rescales it (sig_k = -tau/(alpha - beta),
    // the stored x is kept) and writes row k and the zeros above it.  The dot/update of the
    // formed columns are unaffected by the scale: their coefficient is tau inv^2 x^T a[:, c].
    T sig[CPL];
#pragma unroll
    for (int s = 0; s < CPL; ++s) sig[s] = T(1);
    auto form_column = [&](int k, T sk, T diag) {
        if (cl != (k & 63)) return;
        const int slot = k >> 6;
#pragma unroll
        for (int s = 0; s < CPL; ++s)
            if (s == slot) sig[s] = sk;                 // every wave's copy of column k
        if (wmin > k) return;                          // no rows <= k here
#pragma unroll
        for (int i = 0; i < RW; ++i) {
            const int r = row0 + i * G;
#pragma unroll
            for (int s = 0; s < CPL; ++s)
                if (s == slot) a[i][s] = (r < k) ? T(0) : ((r == k) ? diag : a[i][s]);
        }
    };
    int nstep = 0;
    write_pivot(n - 1, 0);
    __syncthreads();
    for (int k = n - 1; k >= 0; --k) {
        const T tau = s_tau[k];
        if (tau == T(0)) {
            // H_k = I: column k is e_k (its x is zero), and the next pivot replaces this one
            form_column(k, T(1), T(1));
            if (k > 0) write_pivot(k - 1, nstep & 1);
            continue;
        }
        const int par = (nstep++) & 1;
        const T umk = s_umk[k];
        const T inv = fast_rcp(umk);
        T d[CPL];
        pivot_dots(k, par, d);
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
            // row k of a formed column is zero, so v^T Q1[:, c] = inv * sig_c * pc
            coef[s] = (c > k && c < n) ? tau * inv * inv * pc : T(0);
        }
        pivot_update(k, par, umk, coef, k - 1, par ^ 1, false);
        const T sk = -tau * inv;
        form_column(k, sk, (T(1) - tau) * fast_rcp(sk));
    }
#pragma unroll
    for (int i = 0; i < RW; ++i) {
        const int r = row0 + i * G;
        if (r < nrow) {
#pragma unroll
            for (int s = 0; s < CPL; ++s) {
                const int c = cl + 64 * s;
                if (c < n) q1[(prow0 + r) * n + c] = sig[s] * a[i][s];
            }
        }
    }
}


// Panel shapes.  Variant 0 is the default; variants 1 and 2 halve the panel height (half the
// rows per lane, or half the waves) for the autotuner to choose from.  RW is chosen so that the
// kernel fits 128 VGPRs without spills; FP32 packs more rows into the same registers.
template <typename T, int NC, int CPL, int V = 0> struct RegCfg {
    static constexpr int RW0 = (sizeof(T) == 8) ? (CPL == 2 ? 16 : (NC == 64 ? 24 : 16))
                                                : (CPL == 2 ? 24 : (NC == 64 ? 32 : 24));
    static constexpr int NW0 = (CPL == 2) ? 12 : 8;
    static constexpr int RW = (V == 1) ? RW0 / 2 : RW0;
    static constexpr int NW = (V == 2) ? NW0 / 2 : NW0;
    static constexpr int B = NW * (64 / NC) * RW;
};

// Panel height of variant v for (n, dtype): the class is the smallest NC in {4, 8, 16, 32, 64}
// with n <= NC, or NC = 64 with two columns per lane for 64 < n <= 128.
template <int V> inline int reg_rows_v(int64_t n, int dtype)
{
    if (dtype == F32) {
        if (n <= 4) return RegCfg<float, 4, 1, V>::B;
        if (n <= 8) return RegCfg<float, 8, 1, V>::B;
        if (n <= 16) return RegCfg<float, 16, 1, V>::B;
        if (n <= 32) return RegCfg<float, 32, 1, V>::B;
        if (n <= 64) return RegCfg<float, 64, 1, V>::B;
        return RegCfg<float, 64, 2, V>::B;
    }
    if (n <= 4) return RegCfg<double, 4, 1, V>::B;
    if (n <= 8) return RegCfg<double, 8, 1, V>::B;
    if (n <= 16) return RegCfg<double, 16, 1, V>::B;
    if (n <= 32) return RegCfg<double, 32, 1, V>::B;
    if (n <= 64) return RegCfg<double, 64, 1, V>::B;
    return RegCfg<double, 64, 2, V>::B;
}

}  // namespace regpanel

inline int reg_panel_rows_variant(int64_t n, int dtype, int v)
{
    return v == 1 ? regpanel::reg_rows_v<1>(n, dtype)
                  : (v == 2 ? regpanel::reg_rows_v<2>(n, dtype) : regpanel::reg_rows_v<0>(n, dtype));
}

}  // namespace tsqr
