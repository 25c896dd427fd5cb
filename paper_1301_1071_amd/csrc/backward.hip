// Differentiation form: the closed-form adjoints of the thin QR and thin SVD (not in the paper;
// Walter & Lehmann 2018 / Seeger et al. 2017 for QR, Townsend 2016 / Ionescu et al. 2015 for the
// SVD), evaluated with the forward kernels recomputing Q (or U) from A.
//   QR:  M = R triu(dR)^T - dQ^T Q,  dA = (dQ + Q copyltu(M)) R^{-T}
//        = [dQ, Q] [R^{-T}; copyltu(M) R^{-T}]
//   SVD: F_ij = 1/(s_j^2 - s_i^2) (i != j), J = F o (U^T dU - dU^T U), K = F o (V^T dV - dV^T V),
//        dA = U (J S + diag(dS) + S K) V^T + (dU - U U^T dU) S^{-1} V^T
//           = [U, dU] [(J S + diag(dS) + S K - (U^T dU) S^{-1}) V^T; S^{-1} V^T]
// The tall products run on the MFMA GEMM; this file holds the n x n middle steps and the Gram
// reduction dQ^T Q (U^T dU) over the m rows.
#include "tsqr_internal.h"

namespace tsqr {
namespace {

typedef double d4_t __attribute__((ext_vector_type(4)));

constexpr int kGramMaxBlocks = 1024;
constexpr int kGramThreads = 256;
// rows per staged chunk (the X and Y chunks stay within 36 KiB of LDS)
template <int NP> constexpr int gram_rows() { return NP <= 64 ? 32 : 16; }

// Partial Gram of one row range on the matrix cores: C_b = X_b^T Y_b.  Chunks of 32 (or 16) rows of X
// and Y are loaded with coalesced reads one chunk ahead (registers), staged through LDS, and
// every wave accumulates its share of the T x T output tiles (T = ceil(n/16)) with
// v_mfma_f64_16x16x4 over the chunk: A = X^T (lane l: X[r + l/16][16 a + l%16]), B = Y (lane l:
// Y[r + l/16][16 b + l%16]).
template <int NP>
__global__ void __launch_bounds__(kGramThreads)
k_gram(int64_t m, int n, const double *__restrict__ X, int64_t ldx, const double *__restrict__ Y,
       int64_t ldy, int64_t rows_per_block, double *__restrict__ part)
{
    constexpr int kGramRows = gram_rows<NP>();
    constexpr int T = NP / 16, NTILE = T * T, TPW = (NTILE + 3) / 4;   // tiles per wave
    constexpr int LDS_LD = NP + 1;
    constexpr int PER = kGramRows * NP / kGramThreads;                 // prefetched values
    static_assert(kGramRows * NP % kGramThreads == 0, "whole prefetch rounds");
    __shared__ double xs[kGramRows * LDS_LD], ys[kGramRows * LDS_LD];
    const int tid = threadIdx.x, lane = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int64_t r_begin = (int64_t)blockIdx.x * rows_per_block;
    const int64_t r_end = min(m, r_begin + rows_per_block);
    d4_t acc[TPW];
#pragma unroll
    for (int t = 0; t < TPW; ++t) acc[t] = d4_t{0, 0, 0, 0};
    double px[PER], py[PER];
    auto fetch = [&](int64_t r0) {
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int e = tid + q * kGramThreads;
            const int r = e / NP, c = e - r * NP;
            const bool ok = (r0 + r < r_end) && c < n;
            px[q] = ok ? X[(r0 + r) * ldx + c] : 0.0;
            py[q] = ok ? Y[(r0 + r) * ldy + c] : 0.0;
        }
    };
    if (r_begin < r_end) fetch(r_begin);
    for (int64_t r0 = r_begin; r0 < r_end; r0 += kGramRows) {
        __syncthreads();                       // previous chunk fully consumed
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int e = tid + q * kGramThreads;
            const int r = e / NP, c = e - r * NP;
            xs[r * LDS_LD + c] = px[q];
            ys[r * LDS_LD + c] = py[q];
        }
        __syncthreads();
        if (r0 + kGramRows < r_end) fetch(r0 + kGramRows);
#pragma unroll
        for (int k = 0; k < kGramRows / 4; ++k) {
            const int r = 4 * k + (lane >> 4);
#pragma unroll
            for (int t = 0; t < TPW; ++t) {
                const int tile = w * TPW + t;
                if (tile < NTILE) {
                    const int a = tile / T, b = tile - a * T;
                    acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(xs[r * LDS_LD + 16 * a + (lane & 15)],
                                                                  ys[r * LDS_LD + 16 * b + (lane & 15)],
                                                                  acc[t], 0, 0, 0);
                }
            }
        }
    }
    double *out = part + (int64_t)blockIdx.x * n * n;
#pragma unroll
    for (int t = 0; t < TPW; ++t) {
        const int tile = w * TPW + t;
        if (tile < NTILE) {
            const int a = tile / T, b = tile - a * T;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int row = 16 * a + (lane >> 4) + 4 * i, col = 16 * b + (lane & 15);   // f64 layout
                if (row < n && col < n) out[(int64_t)row * n + col] = acc[t][i];
            }
        }
    }
}

// G = sum of the partial Grams (one thread per entry), blocks y, y + S, y + 2S, ... of split
// y = blockIdx.y summed in block order; with S > 1 the sum of split y goes to slot y of part
// (slot y is read only by split y, first) and a second launch with S = 1 adds the S slots.
__global__ void __launch_bounds__(256)
k_gram_sum(int64_t nn, double *part, int nblk, double *__restrict__ G)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nn) return;
    const int y = blockIdx.y, S = gridDim.y;
    double a = 0.0;
    for (int b = y; b < nblk; b += S) a += part[(int64_t)b * nn + e];
    if (S > 1) part[(int64_t)y * nn + e] = a;
    else G[e] = a;
}

// v summed over the 64 lanes of the wave (every lane gets the sum)
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Row j of R^{-T} (column j of R^{-1}, R upper triangular, n <= 128) into W2[j][:]: one wave
// per work-group solves R x = e_j by back substitution; lane t keeps x_t and x_{t+64} in
// registers, so each step is two FMAs, a wave sum and one division, with the next row of R
// fetched while the current step reduces.  Work-group 0 also flags a zero diagonal (info = -3).
__global__ void __launch_bounds__(64)
k_qr_bwd_rinv(int n, const double *__restrict__ R, double *__restrict__ W2,
              int32_t *__restrict__ info)
{
    const int lane = threadIdx.x;
    const int j = blockIdx.x;
    double x0 = 0.0, x1 = 0.0;                       // x_lane, x_{lane+64}
    double r0 = (lane <= j) ? R[j * n + lane] : 0.0;
    double r1 = (lane + 64 <= j) ? R[j * n + lane + 64] : 0.0;
    for (int i = j; i >= 0; --i) {
        // prefetch row i - 1 (columns up to j)
        double n0 = 0.0, n1 = 0.0;
        if (i > 0) {
            n0 = (lane <= j) ? R[(i - 1) * n + lane] : 0.0;
            n1 = (lane + 64 <= j) ? R[(i - 1) * n + lane + 64] : 0.0;
        }
        // sum_{t > i} R[i][t] x_t (x_t = 0 for t > j or not yet computed)
        double part = 0.0;
        if (lane > i) part = fma(r0, x0, part);
        if (lane + 64 > i) part = fma(r1, x1, part);
        const double s = wave_sum(part);
        const double rii = __shfl(i < 64 ? r0 : r1, i & 63, 64);
        const double xi = (((i == j) ? 1.0 : 0.0) - s) / rii;
        if (lane == i) x0 = xi;
        if (lane + 64 == i) x1 = xi;
        r0 = n0;
        r1 = n1;
    }
    if (lane < n) W2[(int64_t)j * n + lane] = (lane <= j) ? x0 : 0.0;
    if (lane + 64 < n) W2[(int64_t)j * n + lane + 64] = (lane + 64 <= j) ? x1 : 0.0;
    if (j == 0 && lane == 0) {
        int bad = 0;
        for (int i = 0; i < n; ++i) bad |= !(R[i * n + i] != 0.0);
        if (bad) *info = -3;
    }
}

// Row i of C = copyltu(M), M = R triu(dR)^T - G (lower triangle), into LDS, then row i of the
// lower block of W2 = C R^{-T}, with R^{-T} from the top block of W2 (lower triangular, read
// along rows so that the lanes load consecutive entries).  One work-group of 128 threads per
// row; thread j forms entry j.  G == nullptr: dQ = 0.
__global__ void __launch_bounds__(128)
k_qr_bwd_rows(int n, const double *__restrict__ R, const double *__restrict__ dR, int64_t lddr,
              const double *__restrict__ G, double *__restrict__ W2)
{
    __shared__ double c_row[128];
    const int i = blockIdx.x, j = threadIdx.x;
    if (j < n) {
        // M[a][b], b <= a: sum_{k >= b} R[a][k] dR[b][k] - G[a][b]
        const int a = (j <= i) ? i : j, b = (j <= i) ? j : i;
        double m = 0.0;
        if (dR)
            for (int k = b; k < n; ++k) m = fma(R[a * n + k], dR[(int64_t)b * lddr + k], m);
        if (G) m -= G[a * n + b];
        c_row[j] = m;
    }
    __syncthreads();
    if (j < n) {
        double acc = 0.0;
        for (int t = j; t < n; ++t) acc = fma(c_row[t], W2[(int64_t)t * n + j], acc);
        W2[(int64_t)(n + i) * n + j] = acc;
    }
}

// Row i of T1 = J S + diag(dS) + S K - (U^T dU) S^{-1} (J, K from U^T dU and V^T dV, whose
// entries (i, j) and (j, i) thread j forms with the lanes reading consecutive columns), then row
// i of W2 = [T1 V^T; S^{-1} V^T] with V^T staged in LDS.  One work-group of 128 threads per row.
// Work-group 0 flags singular values that are not positive and distinct (info = -3).
__global__ void __launch_bounds__(128)
k_svd_bwd_rows(int n, const double *__restrict__ S, const double *__restrict__ V,
               const double *__restrict__ dS, const double *__restrict__ dV, int64_t lddv,
               const double *__restrict__ UtdU, double *__restrict__ W2,
               int32_t *__restrict__ info)
{
    extern __shared__ double vt[];                   // vt[t * n + j] = V[j][t]
    __shared__ double t1_row[128];
    const int i = blockIdx.x, j = threadIdx.x;
    for (int e = j; e < n * n; e += blockDim.x) {
        const int r = e / n, c = e - r * n;
        vt[c * n + r] = V[e];
    }
    if (j < n) {
        double vij = 0.0, vji = 0.0;                 // (V^T dV)[i][j], (V^T dV)[j][i]
        if (dV)
            for (int k = 0; k < n; ++k) {
                vij = fma(V[k * n + i], dV[(int64_t)k * lddv + j], vij);
                vji = fma(V[k * n + j], dV[(int64_t)k * lddv + i], vji);
            }
        const double F = (i == j) ? 0.0 : 1.0 / (S[j] * S[j] - S[i] * S[i]);
        const double uij = UtdU ? UtdU[i * n + j] : 0.0, uji = UtdU ? UtdU[j * n + i] : 0.0;
        const double Jij = F * (uij - uji);
        const double Kij = F * (vij - vji);
        double v = Jij * S[j] + S[i] * Kij - uij / S[j];
        if (i == j && dS) v += dS[i];
        t1_row[j] = v;
    }
    __syncthreads();
    if (j < n) {
        double acc = 0.0;
        for (int t = 0; t < n; ++t) acc = fma(t1_row[t], vt[t * n + j], acc);
        W2[(int64_t)i * n + j] = acc;
        W2[(int64_t)(n + i) * n + j] = vt[i * n + j] / S[i];
    }
    if (i == 0 && j == 0) {
        int bad = 0;
        for (int k = 0; k < n; ++k) {
            bad |= !(S[k] > 0.0);
            if (k > 0) bad |= !(S[k - 1] != S[k]);
        }
        if (bad) *info = -3;
    }
}

}  // namespace

int gram_blocks(int64_t m)
{
    // about 2,048 rows per work-group: two work-groups per CU at a million rows
    int64_t b = ceil_div(m, 2048);
    return (int)(b < 1 ? 1 : (b > kGramMaxBlocks ? kGramMaxBlocks : b));
}

hipError_t launch_gram(int64_t m, int64_t n, const double *X, int64_t ldx, const double *Y,
                       int64_t ldy, double *part, double *G, hipStream_t st)
{
    const int nb = gram_blocks(m);
    const int64_t rpb = ceil_div(ceil_div(m, nb), 32) * 32;
#define TSQR_GRAM(NP)                                                                          \
    hipLaunchKernelGGL(k_gram<NP>, dim3(nb), dim3(kGramThreads), 0, st, m, (int)n, X, ldx, Y,  \
                       ldy, rpb, part)
    // the tile grid padded to the next multiple of 16 columns only
    switch ((n + 15) / 16) {
    case 1: TSQR_GRAM(16); break;
    case 2: TSQR_GRAM(32); break;
    case 3: TSQR_GRAM(48); break;
    case 4: TSQR_GRAM(64); break;
    case 5: TSQR_GRAM(80); break;
    case 6: TSQR_GRAM(96); break;
    case 7: TSQR_GRAM(112); break;
    case 8: TSQR_GRAM(128); break;
    default: return hipErrorInvalidValue;
    }
#undef TSQR_GRAM
    const int64_t nn = n * n;
    // the partials summed in 16 interleaved splits first when there are many of them
    const int splits = nb >= 64 ? 16 : 1;
    if (splits > 1)
        hipLaunchKernelGGL(k_gram_sum, dim3((unsigned)ceil_div(nn, 256), splits), dim3(256), 0, st,
                           nn, part, nb, G);
    hipLaunchKernelGGL(k_gram_sum, dim3((unsigned)ceil_div(nn, 256)), dim3(256), 0, st, nn, part,
                       splits > 1 ? splits : nb, G);
    return hipGetLastError();
}

hipError_t launch_qr_bwd_small(int64_t n, const double *R, const double *dR, int64_t lddr,
                               const double *G, double *W2, double *scratch, int32_t *info,
                               hipStream_t st)
{
    (void)scratch;
    if (n < 1 || n > 128) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_qr_bwd_rinv, dim3((unsigned)n), dim3(64), 0, st, (int)n, R, W2, info);
    hipLaunchKernelGGL(k_qr_bwd_rows, dim3((unsigned)n), dim3(128), 0, st, (int)n, R, dR, lddr, G,
                       W2);
    return hipGetLastError();
}

hipError_t launch_svd_bwd_small(int64_t n, const double *S, const double *V, const double *dS,
                                const double *dV, int64_t lddv, const double *UtdU, double *W2,
                                double *scratch, int32_t *info, hipStream_t st)
{
    (void)scratch;
    if (n < 1 || n > 128) return hipErrorInvalidValue;
    const size_t lds = sizeof(double) * (size_t)n * n;
    hipError_t e = ensure_dynamic_lds((const void *)k_svd_bwd_rows, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_svd_bwd_rows, dim3((unsigned)n), dim3(128), lds, st, (int)n, S, V, dS, dV,
                       lddv, UtdU, W2, info);
    return hipGetLastError();
}

}  // namespace tsqr
