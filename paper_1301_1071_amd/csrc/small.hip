// Top of the tree (one work-group): sign normalisation of R~, the info flag, and the SVD of R.
//
// Sec. III-B: the single reduce task ends with R~; the factorization with a positive diagonal is
// unique for full-rank A (Sec. I), so R = D R~ with D = diag(sign(R~_jj)), sign(0) = +1, and the
// step-3 blocks become Q2_p D.  For the SVD variant the reduce task also computes R = U_R S V^T
// (the paper treats this n x n SVD as negligible and names no method): one-sided Jacobi
// (Hestenes) on R^T, columns rotated until pairwise orthogonal, in parallel round-robin order.
// U_R is passed down the tree so that U = Q U_R comes out of step 3 in the same pass as Q.
#include "tsqr_internal.h"

namespace tsqr {
namespace {

constexpr size_t kLdsPerWorkgroup = 160 * 1024;   // LDS one work-group may hold on gfx950

// player at position `pos` of round `r` in the round-robin tournament of np players
// (0 <= pos < np, 0 <= r < np - 1): player 0 stays, the others rotate by one place per round.
// pos - 1 + r < 2 (np - 1), so one conditional subtraction is the reduction modulo np - 1.
__device__ __forceinline__ int rr_player(int pos, int r, int np)
{
    int x = pos - 1 + r;
    if (x >= np - 1) x -= np - 1;
    return pos == 0 ? 0 : 1 + x;
}

// reciprocal and reciprocal square root: hardware estimate plus two Newton steps (a few ulp)
__device__ __forceinline__ double rcp_nr(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    r = fma(r, fma(-x, r, 1.0), r);
    return fma(r, fma(-x, r, 1.0), r);
}
__device__ __forceinline__ double rsqrt_nr(double x)
{
    double y = __builtin_amdgcn_rsq(x);
    y = y * fma(-0.5 * x * y, y, 1.5);
    return y * fma(-0.5 * x * y, y, 1.5);
}

constexpr int kSvdThreads = 1024;   // 16 waves: 64 groups of 16 lanes, one column pair each

// DPP lane move; the patterns used here (quad_perm, row_ror, row_newbcast) read a valid lane for
// every lane, so the old value is never used and needs no zeroing (bound_ctrl)
template <int CTRL> __device__ __forceinline__ double dpp_d(double v)
{
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xf, 0xf, true);
    return __hiloint2double(hi, lo);
}

// Sum over the 16 lanes of a group (one DPP row): butterflies within quads, rotations by 4 and 8
// across the quads, then lane 0's sum broadcast to the row so every lane of the group takes the
// same rotation decision.
__device__ __forceinline__ double group16_sum(double v)
{
    v += dpp_d<0xB1>(v);          // quad_perm [1,0,3,2]
    v += dpp_d<0x4E>(v);          // quad_perm [2,3,0,1]
    v += dpp_d<0x124>(v);         // row_ror:4
    v += dpp_d<0x128>(v);         // row_ror:8
    return dpp_d<0x150>(v);       // row_newbcast:0
}

// NPAD: column capacity (64, 128, or 512 for the wide path, whose Jacobi columns are re-read from
// memory for the rotation instead of being kept in registers).  LDSM: the Jacobi columns live in
// LDS (known at compile time, so that their accesses are LDS instructions, not flat ones that
// could reach either memory) or in the global scratch G, Vw.
template <int NPAD, bool LDSM>
__global__ void __launch_bounds__(kSvdThreads)
k_finalize(int n, const double *__restrict__ Rt, double *__restrict__ R, float *__restrict__ Rf,
           int64_t ldr, double *__restrict__ Wtop, int k, int want_q, int want_u,
           double *__restrict__ S, float *__restrict__ Sf, double *__restrict__ V,
           float *__restrict__ Vf, int64_t ldv, double *G, double *Vw,
           int32_t *__restrict__ info, int keep_info)
{
    extern __shared__ __align__(16) double sm[];
    constexpr int NJ = NPAD / 16;                 // 16-row chunks of a column
    constexpr bool kCache = NJ <= 8;              // columns held in registers between the passes
    __shared__ double d_s[NPAD];
    __shared__ double s_sv[NPAD];
    __shared__ double s_sg[NPAD];
    __shared__ int perm[NPAD];
    __shared__ int s_zero, s_nonfinite, s_rot;

    const int tid = threadIdx.x;
    const int nth = blockDim.x;

    if (tid == 0) { s_zero = 0x7fffffff; s_nonfinite = 0; }
    __syncthreads();
    for (int i = tid; i < n; i += nth) {
        const double rii = Rt[(int64_t)i * n + i];
        d_s[i] = (rii >= 0.0) ? 1.0 : -1.0;
        if (rii == 0.0) atomicMin(&s_zero, i);
    }
    for (int e = tid; e < n * n; e += nth) {
        const int r = e / n, c = e - r * n;
        if (c >= r && !isfinite(Rt[e])) s_nonfinite = 1;
    }
    __syncthreads();
    for (int e = tid; e < n * n; e += nth) {
        const int r = e / n, c = e - r * n;
        const double v = (c >= r) ? d_s[r] * Rt[e] : 0.0;
        if (R) R[(int64_t)r * ldr + c] = v;
        if (Rf) Rf[(int64_t)r * ldr + c] = (float)v;
        if (want_q) Wtop[(int64_t)r * k + c] = (r == c) ? d_s[r] : 0.0;
    }
    const int kq = want_q ? n : 0;

    if (want_u || S != nullptr || Sf != nullptr) {
        double *gG = LDSM ? sm : G;                        // column-major n x n
        double *gV = LDSM ? sm + (size_t)n * n : Vw;
        // one-sided Jacobi on R^T (column r of R^T is row r of R): R^T J = G with orthogonal
        // columns, so R = J diag(|g|) (G diag(|g|)^{-1})^T, i.e. U_R = J and V = G / |g|.
        // Rotating the rows of the triangular R converges in far fewer sweeps than rotating its
        // columns when R is ill conditioned.
        for (int e = tid; e < n * n; e += nth) {
            const int r = e / n, c = e - r * n;
            gG[(int64_t)r * n + c] = (c >= r) ? d_s[r] * Rt[e] : 0.0;
            gV[(int64_t)c * n + r] = (r == c) ? 1.0 : 0.0;
        }
        const int np = n + (n & 1);                    // players of the round-robin tournament
        const int npairs = np / 2;
        const int grp = tid >> 4, gl = tid & 15;       // 16-lane group and lane within it
        const int ngrp = nth >> 4;
        const int nj = (n + 15) >> 4;                  // 16-row chunks of a column
        const double tol = 1e-15 * (double)n;
        const double tol2 = tol * tol;
        for (int sweep = 0; sweep < 60; ++sweep) {
            __syncthreads();
            if (tid == 0) s_rot = 0;
            __syncthreads();
            for (int round = 0; round < np - 1; ++round) {
                for (int t = grp; t < npairs; t += ngrp) {      // uniform within each group
                    const int a = rr_player(t, round, np), bq = rr_player(np - 1 - t, round, np);
                    const int p = min(a, bq), q = max(a, bq);
                    if (q >= n) continue;
                    double *gp = gG + (int64_t)p * n, *gq = gG + (int64_t)q * n;
                    double *vp = gV + (int64_t)p * n, *vq = gV + (int64_t)q * n;
                    double xp[kCache ? NJ : 1], xq[kCache ? NJ : 1];
                    double al = 0.0, be = 0.0, ga = 0.0;
                    if constexpr (kCache) {
                        // all chunks (NJ = 16-row chunks of the padded width) loaded at once from
                        // clamped in-bounds rows, so the loads are in flight together
#pragma unroll
                        for (int j = 0; j < NJ; ++j) {
                            const int i = gl + 16 * j, ic = min(i, n - 1);
                            xp[j] = gp[ic];
                            xq[j] = gq[ic];
                        }
#pragma unroll
                        for (int j = 0; j < NJ; ++j) {
                            const bool in = gl + 16 * j < n;
                            xp[j] = in ? xp[j] : 0.0;
                            xq[j] = in ? xq[j] : 0.0;
                            al = fma(xp[j], xp[j], al);
                            be = fma(xq[j], xq[j], be);
                            ga = fma(xp[j], xq[j], ga);
                        }
                    } else {
                        for (int j = 0; j < nj; ++j) {
                            const int i = gl + 16 * j;
                            const double a = (i < n) ? gp[i] : 0.0;
                            const double c = (i < n) ? gq[i] : 0.0;
                            al = fma(a, a, al);
                            be = fma(c, c, be);
                            ga = fma(a, c, ga);
                        }
                    }
                    al = group16_sum(al);
                    be = group16_sum(be);
                    ga = group16_sum(ga);
                    if (ga != 0.0 && ga * ga > tol2 * (al * be)) {
                        // t = sign(zeta) / (|zeta| + sqrt(1 + zeta^2)); |zeta| < 1 / (2 tol) here,
                        // so 1 + zeta^2 neither overflows nor needs a correctly rounded root
                        // (cs and sn are formed from the same t, cs^2 + sn^2 = 1 to rounding)
                        const double zeta = 0.5 * (be - al) * rcp_nr(ga);
                        const double z2 = fma(zeta, zeta, 1.0);
                        const double tt = ((zeta >= 0.0) ? 1.0 : -1.0) *
                                          rcp_nr(fabs(zeta) + z2 * rsqrt_nr(z2));
                        const double cs = rsqrt_nr(fma(tt, tt, 1.0));
                        const double sn = cs * tt;
                        if constexpr (kCache) {
                            double yp[NJ], yq[NJ];
#pragma unroll
                            for (int j = 0; j < NJ; ++j) {
                                const int ic = min(gl + 16 * j, n - 1);
                                yp[j] = vp[ic];
                                yq[j] = vq[ic];
                            }
#pragma unroll
                            for (int j = 0; j < NJ; ++j) {
                                const int i = gl + 16 * j;
                                if (i < n) {
                                    gp[i] = cs * xp[j] - sn * xq[j];
                                    gq[i] = sn * xp[j] + cs * xq[j];
                                    vp[i] = cs * yp[j] - sn * yq[j];
                                    vq[i] = sn * yp[j] + cs * yq[j];
                                }
                            }
                        } else {
                            for (int j = 0; j < nj; ++j) {
                                const int i = gl + 16 * j;
                                if (i < n) {
                                    const double a = gp[i], c = gq[i];
                                    gp[i] = cs * a - sn * c;
                                    gq[i] = sn * a + cs * c;
                                    const double y1 = vp[i], y2 = vq[i];
                                    vp[i] = cs * y1 - sn * y2;
                                    vq[i] = sn * y1 + cs * y2;
                                }
                            }
                        }
                        if (gl == 0) s_rot = 1;        // every writer stores the same value
                    }
                }
                __syncthreads();
            }
            if (s_rot == 0) break;
        }
        __syncthreads();
        for (int c = tid; c < n; c += nth) {
            double ss = 0.0;
            for (int r = 0; r < n; ++r) ss += gG[(int64_t)c * n + r] * gG[(int64_t)c * n + r];
            s_sv[c] = sqrt(ss);
        }
        __syncthreads();
        for (int c = tid; c < n; c += nth) {
            int rank = 0;
            for (int j = 0; j < n; ++j)
                rank += (s_sv[j] > s_sv[c]) || (s_sv[j] == s_sv[c] && j < c);
            perm[rank] = c;
        }
        __syncthreads();
        // gauge: the largest-magnitude entry of each v_k = g_c / |g_c| is positive
        for (int o = tid; o < n; o += nth) {
            const int c = perm[o];
            int imax = 0;
            double vmax = -1.0;
            for (int i = 0; i < n; ++i) {
                const double a = fabs(gG[(int64_t)c * n + i]);
                if (a > vmax) { vmax = a; imax = i; }
            }
            s_sg[o] = (gG[(int64_t)c * n + imax] < 0.0) ? -1.0 : 1.0;
            if (S) S[o] = s_sv[c];
            if (Sf) Sf[o] = (float)s_sv[c];
        }
        __syncthreads();
        for (int e = tid; e < n * n; e += nth) {
            const int i = e / n, o = e - i * n;
            const int c = perm[o];
            const double s = s_sv[c];
            const double vio = (s > 0.0) ? s_sg[o] * gG[(int64_t)c * n + i] / s : 0.0;
            if (V) V[(int64_t)i * ldv + o] = vio;
            if (Vf) Vf[(int64_t)i * ldv + o] = (float)vio;
            if (want_u) Wtop[(int64_t)i * k + kq + o] = d_s[i] * s_sg[o] * gV[(int64_t)c * n + i];
        }
    }
    if (tid == 0) {
        const int32_t code = s_nonfinite ? -1 : (s_zero == 0x7fffffff ? 0 : s_zero + 1);
        // keep_info: an earlier kernel of the call may already have reported a condition
        if (!keep_info || *info == 0) *info = code;
    }
}

}  // namespace

hipError_t launch_finalize(int64_t n, const double *Rt, double *R, float *Rf, int64_t ldr,
                           double *Wtop, int k, int want_q, int want_u, double *S, float *Sf,
                           double *V, float *Vf, int64_t ldv, double *G, double *Vw,
                           int32_t *info, hipStream_t st, int keep_info)
{
    const bool svd = want_u || S != nullptr || Sf != nullptr;
    if (n > kNmaxWide) return hipErrorInvalidValue;
    // the Jacobi columns (G and V, 2 n^2 doubles) go to LDS when they fit beside the kernel's
    // static arrays (up to n = 100 with the 128-column instantiation), else to global scratch
    const size_t need = svd ? 2 * sizeof(double) * (size_t)n * n : 0;
    bool use_lds = false;
    if (svd && n <= kNmaxPad) {
        const void *lk = (n > 64) ? (const void *)k_finalize<kNmaxPad, true>
                                  : (const void *)k_finalize<64, true>;
        hipFuncAttributes fa;
        hipError_t e = hipFuncGetAttributes(&fa, lk);
        if (e != hipSuccess) return e;
        use_lds = need + align_up(fa.sharedSizeBytes, 16) <= kLdsPerWorkgroup;
    }
    const size_t lds = use_lds ? need : 0;
    auto kern = (n > kNmaxPad) ? k_finalize<kNmaxWide, false>
                : (n > 64) ? (use_lds ? k_finalize<kNmaxPad, true> : k_finalize<kNmaxPad, false>)
                           : (use_lds ? k_finalize<64, true> : k_finalize<64, false>);
    hipError_t e = ensure_dynamic_lds((const void *)kern, lds);
    if (e != hipSuccess) return e;
    // one 16-lane group per column pair of a Jacobi round, whole waves, so that each round's
    // barrier waits only for waves that have work
    const int64_t pairs = (n + (n & 1)) / 2;
    const int threads = (int)std::min<int64_t>(kSvdThreads, std::max<int64_t>(64, (16 * pairs + 63) / 64 * 64));
    hipLaunchKernelGGL(kern, dim3(1), dim3(threads), lds, st, (int)n, Rt, R,
                       Rf, ldr, Wtop, k, want_q, want_u, S, Sf, V, Vf, ldv, G, Vw, info,
                       keep_info);
    return hipGetLastError();
}

}  // namespace tsqr
