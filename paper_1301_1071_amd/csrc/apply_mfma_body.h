// Step 3 of direct TSQR on the matrix cores: out_p = Q1_p * W_p for one row panel p
// (Sec. III-B: Q_i = Q1_i Q2_i; with the SVD, W_p = [Q2_p, Q2_p U_R] so Q and U come out of the
// same pass).  Device body shared by the single-matrix launches (apply_mfma.hip) and the batched
// ones (batched.hip).  One work-group per panel; each wave walks 16-row blocks of the panel:
//   * the 16 x n block of Q1 is staged through LDS with coalesced loads,
//   * W_p sits in LDS in MFMA B-operand order (one 64-value record per 4 x 16 tile),
//   * v_mfma_{f64,f32}_16x16x4 accumulates 16 x 16 output tiles over K = n in steps of 4.
// Operand layouts of the 16x16x4 instructions (lane l): A[l % 16][l / 16], B[l / 16][l % 16];
// result element i of lane l is D[l/16 + 4 i][l % 16] for f64 and D[4 (l/16) + i][l % 16] for
// f32.
#pragma once

#include "tsqr_internal.h"

namespace tsqr {
namespace mfmaapply {

typedef double d4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));

template <typename T> struct Mfma;
template <> struct Mfma<double> {
    typedef d4_t acc_t;
    static __device__ __forceinline__ acc_t run(double a, double b, acc_t c)
    {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lane, int i) { return (lane >> 4) + 4 * i; }
};
template <> struct Mfma<float> {
    typedef f4_t acc_t;
    static __device__ __forceinline__ acc_t run(float a, float b, acc_t c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lane, int i) { return 4 * (lane >> 4) + i; }
};

constexpr int kMaxKC = 32;      // n <= 128
constexpr int kWaves = 4;

template <typename T, typename To, int NT>
__device__ __forceinline__ void apply_mfma_panel(int64_t rows, int n, int b,
                                                 const T *__restrict__ q1, int64_t ldq,
                                                 const double *__restrict__ W, int64_t ldw,
                                                 int64_t wstride, int k, To *__restrict__ out0,
                                                 int64_t ld0, int k0, To *__restrict__ out1,
                                                 int64_t ld1, int accumulate, int64_t p, int j0)
{
    typedef typename Mfma<T>::acc_t acc_t;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int KC = (n + 3) >> 2;            // K chunks of 4
    const int LDA = 4 * KC + 1;             // odd row stride of the staged A block
    T *wl = reinterpret_cast<T *>(smem_raw);                  // [KC][NT][64]
    T *as_all = wl + (size_t)KC * NT * 64;                     // [kWaves][16][LDA]
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    T *as = as_all + (size_t)w * 16 * LDA;
    const double *Wp = W + p * wstride * ldw;

    for (int e = tid; e < KC * NT * 64; e += kWaves * 64) {
        const int l = e & 63, t = e >> 6;
        const int nt = t % NT, kc = t / NT;
        const int kk = 4 * kc + (l >> 4), j = j0 + 16 * nt + (l & 15);
        wl[e] = (kk < n && j < k) ? (T)Wp[(int64_t)kk * ldw + j] : T(0);
    }
    // zero this wave's staging block once: columns [n, 4 KC) stay zero
    for (int e = lane; e < 16 * LDA; e += 64) as[e] = T(0);
    __syncthreads();

    const int64_t rb = p * (int64_t)b;
    const int nr = (int)min((int64_t)b, rows - rb);
    const int nblk = (nr + 15) >> 4;
    const int jl = j0 + (lane & 15);
    // The 16 x n blocks of Q1 are fetched one block ahead into registers (lane owns columns
    // lane and lane + 64 of every row), so the next block's loads are in flight during this
    // block's products; each block is then staged through this wave's LDS rows.
    T pre[16], pre2[16];
    auto fetch = [&](int blk) {
        const int r0 = blk * 16;
        const int cnt = min(16, nr - r0);
        const T *src = q1 + (rb + r0) * ldq;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            pre[r] = (r < cnt && lane < n) ? src[(int64_t)r * ldq + lane] : T(0);
            pre2[r] = (r < cnt && lane + 64 < n) ? src[(int64_t)r * ldq + lane + 64] : T(0);
        }
    };
    if (w < nblk) fetch(w);
    for (int blk = w; blk < nblk; blk += kWaves) {
        const int r0 = blk * 16;
        const int cnt = min(16, nr - r0);
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            if (lane < n) as[r * LDA + lane] = pre[r];
            if (lane + 64 < n) as[r * LDA + lane + 64] = pre2[r];
        }
        if (blk + kWaves < nblk) fetch(blk + kWaves);
        // the wave reads back what its own lanes wrote: LDS operations of a wave are ordered
        acc_t acc[NT];
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[t] = acc_t{0, 0, 0, 0};
        for (int kc = 0; kc < KC; ++kc) {
            const T a = as[(lane & 15) * LDA + 4 * kc + (lane >> 4)];
            const T *wk = wl + (size_t)kc * NT * 64 + lane;
#pragma unroll
            for (int t = 0; t < NT; ++t) acc[t] = Mfma<T>::run(a, wk[t * 64], acc[t]);
        }
        // results: row pointers once per block, then a column offset per tile
        To *o0[4], *o1[4];
        bool rok[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int r = Mfma<T>::row(lane, i);
            rok[i] = r < cnt;
            const int64_t gr = rb + r0 + (rok[i] ? r : 0);
            o0[i] = out0 + gr * ld0;
            o1[i] = out1 ? out1 + gr * ld1 - k0 : nullptr;
        }
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const int j = jl + 16 * t;
            if (j >= k) continue;
            const bool first = j < k0;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                if (!rok[i]) continue;
                To *o = (first ? o0[i] : o1[i]) + j;
                *o = accumulate ? (To)(acc[t][i] + (T)*o) : (To)acc[t][i];
            }
        }
    }
}

// Dynamic LDS of one work-group for n columns and NT output tiles.
template <typename T, int NT> inline size_t apply_lds_bytes(int64_t n)
{
    const int KC = (int)((n + 3) / 4);
    return sizeof(T) * ((size_t)KC * NT * 64 + (size_t)kWaves * 16 * (4 * KC + 1));
}

}  // namespace mfmaapply
}  // namespace tsqr
