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

// G = sum of the partial Grams, in block order (one thread per entry)
__global__ void __launch_bounds__(256)
k_gram_sum(int64_t nn, const double *__restrict__ part, int nblk, double *__restrict__ G)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nn) return;
    double a = 0.0;
    for (int b = 0; b < nblk; ++b) a += part[(int64_t)b * nn + e];
    G[e] = a;
}

// v summed over the 64 lanes of the wave (every lane gets the sum)
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Rinv = R^{-1} (R upper triangular, n x n, n <= 128): one wave per column j solves R x = e_j by
// back substitution; lane t keeps x_t and x_{t+64} in registers, so each step is two FMAs, a
// wave sum and one division, with the next row of R fetched while the current step reduces.
__device__ void tri_inverse(int n, const double *R, double *Rinv)
{
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6, nwaves = blockDim.x >> 6;
    for (int j = wave; j < n; j += nwaves) {
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
        if (lane < n) Rinv[lane * n + j] = (lane <= j) ? x0 : 0.0;
        if (lane + 64 < n) Rinv[(lane + 64) * n + j] = (lane + 64 <= j) ? x1 : 0.0;
    }
}

// G = dQ^T Q (NULL: dQ = 0); scratch (2 n^2): Rinv, C
__global__ void __launch_bounds__(1024)
k_qr_bwd_small(int n, const double *__restrict__ R, const double *__restrict__ dR, int64_t lddr,
               const double *__restrict__ G, double *__restrict__ W2,
               double *__restrict__ scratch, int32_t *__restrict__ info)
{
    double *Rinv = scratch, *C = scratch + (size_t)n * n;
    const int tid = threadIdx.x;
    tri_inverse(n, R, Rinv);
    __syncthreads();
    // M = R triu(dR)^T - G, then C = copyltu(M) (lower triangle mirrored up)
    for (int e = tid; e < n * n; e += blockDim.x) {
        const int i = e / n, j = e - i * n;
        if (j > i) continue;
        double mij = 0.0, mji = 0.0;
        if (dR) {
            for (int k = j; k < n; ++k) mij = fma(R[i * n + k], dR[(int64_t)j * lddr + k], mij);
            (void)mji;
        }
        if (G) mij -= G[i * n + j];
        C[i * n + j] = mij;
        C[j * n + i] = mij;
    }
    __syncthreads();
    // W2 = [R^{-T}; C R^{-T}]
    for (int e = tid; e < n * n; e += blockDim.x) {
        const int i = e / n, j = e - i * n;
        W2[(int64_t)i * n + j] = Rinv[j * n + i];
        double acc = 0.0;
        for (int t = j; t < n; ++t) acc = fma(C[i * n + t], Rinv[j * n + t], acc);
        W2[(int64_t)(n + i) * n + j] = acc;
    }
    if (tid == 0) {
        int bad = 0;
        for (int i = 0; i < n; ++i) bad |= !(R[i * n + i] != 0.0);
        if (bad) *info = -3;
    }
}

// UtdU = U^T dU (NULL: dU = 0); scratch (2 n^2): VtdV, T1
__global__ void __launch_bounds__(1024)
k_svd_bwd_small(int n, const double *__restrict__ S, const double *__restrict__ V,
                const double *__restrict__ dS, const double *__restrict__ dV, int64_t lddv,
                const double *__restrict__ UtdU, double *__restrict__ W2,
                double *__restrict__ scratch, int32_t *__restrict__ info)
{
    double *VtdV = scratch, *T1 = scratch + (size_t)n * n;
    const int tid = threadIdx.x;
    for (int e = tid; e < n * n; e += blockDim.x) {
        const int i = e / n, j = e - i * n;
        double acc = 0.0;
        if (dV)
            for (int k = 0; k < n; ++k) acc = fma(V[k * n + i], dV[(int64_t)k * lddv + j], acc);
        VtdV[e] = acc;
    }
    __syncthreads();
    // T1 = J S + diag(dS) + S K - (U^T dU) S^{-1}
    for (int e = tid; e < n * n; e += blockDim.x) {
        const int i = e / n, j = e - i * n;
        const double F = (i == j) ? 0.0 : 1.0 / (S[j] * S[j] - S[i] * S[i]);
        const double uij = UtdU ? UtdU[i * n + j] : 0.0, uji = UtdU ? UtdU[j * n + i] : 0.0;
        const double Jij = F * (uij - uji);
        const double Kij = F * (VtdV[i * n + j] - VtdV[j * n + i]);
        double v = Jij * S[j] + S[i] * Kij - uij / S[j];
        if (i == j && dS) v += dS[i];
        T1[e] = v;
    }
    __syncthreads();
    // W2 = [T1 V^T; S^{-1} V^T]
    for (int e = tid; e < n * n; e += blockDim.x) {
        const int i = e / n, j = e - i * n;
        double acc = 0.0;
        for (int t = 0; t < n; ++t) acc = fma(T1[i * n + t], V[j * n + t], acc);
        W2[(int64_t)i * n + j] = acc;
        W2[(int64_t)(n + i) * n + j] = V[j * n + i] / S[i];
    }
    if (tid == 0) {
        int bad = 0;
        for (int i = 0; i < n; ++i) {
            bad |= !(S[i] > 0.0);
            if (i > 0) bad |= !(S[i - 1] != S[i]);
        }
        if (bad) *info = -3;
    }
}

}  // namespace

int gram_blocks(int64_t m)
{
    int64_t b = ceil_div(m, 4096);
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
    if (n <= 16) TSQR_GRAM(16);
    else if (n <= 32) TSQR_GRAM(32);
    else if (n <= 64) TSQR_GRAM(64);
    else if (n <= 128) TSQR_GRAM(128);
    else return hipErrorInvalidValue;
#undef TSQR_GRAM
    const int64_t nn = n * n;
    hipLaunchKernelGGL(k_gram_sum, dim3((unsigned)ceil_div(nn, 256)), dim3(256), 0, st, nn, part,
                       nb, G);
    return hipGetLastError();
}

hipError_t launch_qr_bwd_small(int64_t n, const double *R, const double *dR, int64_t lddr,
                               const double *G, double *W2, double *scratch, int32_t *info,
                               hipStream_t st)
{
    hipLaunchKernelGGL(k_qr_bwd_small, dim3(1), dim3(1024), 0, st, (int)n, R, dR, lddr, G, W2,
                       scratch, info);
    return hipGetLastError();
}

hipError_t launch_svd_bwd_small(int64_t n, const double *S, const double *V, const double *dS,
                                const double *dV, int64_t lddv, const double *UtdU, double *W2,
                                double *scratch, int32_t *info, hipStream_t st)
{
    hipLaunchKernelGGL(k_svd_bwd_small, dim3(1), dim3(1024), 0, st, (int)n, S, V, dS, dV, lddv,
                       UtdU, W2, scratch, info);
    return hipGetLastError();
}

}  // namespace tsqr
