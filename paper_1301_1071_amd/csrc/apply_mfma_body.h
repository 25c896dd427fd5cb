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
    for (int blk = w; blk < nblk; blk += kWaves) {
        const int r0 = blk * 16;
        const int cnt = min(16, nr - r0);
        const T *src = q1 + (rb + r0) * ldq;
        for (int e = lane; e < 16 * n; e += 64) {
            const int r = e / n, c = e - r * n;
            as[r * LDA + c] = (r < cnt) ? src[(int64_t)r * ldq + c] : T(0);
        }
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
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const int j = j0 + 16 * t + (lane & 15);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int r = Mfma<T>::row(lane, i);
                if (r < cnt) {
                    const int64_t gr = rb + r0 + r;
                    if (j < k0) {
                        To *o = out0 + gr * ld0 + j;
                        *o = accumulate ? (To)(acc[t][i] + (T)*o) : (To)acc[t][i];
                    } else if (j < k) {
                        To *o = out1 + gr * ld1 + (j - k0);
                        *o = accumulate ? (To)(acc[t][i] + (T)*o) : (To)acc[t][i];
                    }
                }
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
