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

// One panel.  ACC: add to the output instead of overwriting it; WIDE: n > 64 (lane l also holds
// column l + 64 of a row).  VK: q1 holds the panel's reflectors V and kmat its n x n K
// (Q1 = [I; 0] - V K), and the product is Q1 W = [W; 0] - V (K W): the staged operand is -K W
// instead of W, and W is added to the panel's top n rows.
template <typename T, typename To, int NT, bool ACC, bool WIDE, bool VK>
__device__ __forceinline__ void apply_panel_impl(int64_t rows, int n, int b,
                                                 const T *__restrict__ q1, int64_t ldq,
                                                 const double *__restrict__ W, int64_t ldw,
                                                 int64_t wstride, int k, To *__restrict__ out0,
                                                 int64_t ld0, int k0, To *__restrict__ out1,
                                                 int64_t ld1, int64_t p, int j0, int rc, int nrc,
                                                 const T *__restrict__ kmat)
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

    const int64_t rb = p * (int64_t)b;
    const int nr = (int)min((int64_t)b, rows - rb);
    const int nblk = (nr + 15) >> 4;
    // The 16 x n blocks of Q1 are fetched one block ahead into registers (lane l holds columns
    // l and, if WIDE, l + 64 of every row), so the next block's loads are in flight during this
    // block's products; each block is then staged through this wave's LDS rows.  Every load is
    // in bounds: a lane past column n reads column n - 1 and rows past the panel read its last
    // row; neither reaches LDS or an output row.
    const bool ok0 = lane < n, ok1 = WIDE && lane + 64 < n;
    const uint32_t c0 = ok0 ? lane : n - 1, c1 = ok1 ? lane + 64 : n - 1;
    T pre[16], pre2[WIDE ? 16 : 1];
    auto fetch = [&](int blk) {
        const int last = min(16, nr - blk * 16) - 1;
        const T *src = q1 + (rb + blk * 16) * ldq;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const T *row = src + (int64_t)min(r, last) * ldq;      // uniform
            pre[r] = row[c0];
            if constexpr (WIDE) pre2[r] = row[c1];
        }
    };
    if constexpr (VK) {
        // K_p (row-major, ld n) is staged into this work-group's A-block area and W into wl as
        // usual (below); after a barrier the waves form the tiles (a, t) of M = K W on the matrix
        // cores from LDS (K upper triangular: K-chunks q >= 4 a only), hold them in registers
        // across a second barrier, and overwrite wl with -M in the same B-operand order.
        static_assert(!WIDE, "the V + K form is for n <= 64");
        const T *Kp = kmat + p * (int64_t)n * n;
        T *ks = as_all;                                   // n x n, ld n (fits the A-block area)
        // all of a thread's loads first (n <= 64: at most 16 per thread), then the stores, so
        // the loads are in flight together instead of one memory round trip each
        constexpr int KPT = 64 * 64 / (kWaves * 64);
        T kv[KPT];
        const int nn = n * n;
#pragma unroll
        for (int u = 0; u < KPT; ++u) kv[u] = Kp[min(tid + u * kWaves * 64, nn - 1)];
#pragma unroll
        for (int u = 0; u < KPT; ++u)
            if (tid + u * kWaves * 64 < nn) ks[tid + u * kWaves * 64] = kv[u];
    }
    // W's loads go out eight at a time, so staging it waits for a few memory round trips rather
    // than one per value; the first block's loads are issued right after, before the barrier
    {
        constexpr int U = 8;
        const int total = KC * NT * 64;
        for (int e0 = tid; e0 < total; e0 += U * kWaves * 64) {
            T v[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int e = e0 + u * kWaves * 64;
                const int l = e & 63, t = e >> 6;
                const int nt = t % NT, kc = t / NT;
                const int kk = 4 * kc + (l >> 4), j = j0 + 16 * nt + (l & 15);
                // unconditional load at a clamped (in-bounds) index, then a select: no branch
                // around the load, so the eight loads stay in flight together
                const double x = Wp[(int64_t)min(kk, n - 1) * ldw + min(j, k - 1)];
                v[u] = (e < total && kk < n && j < k) ? (T)x : T(0);
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int e = e0 + u * kWaves * 64;
                if (e < total) wl[e] = v[u];
            }
        }
    }
    if constexpr (VK) {
        constexpr int MT = 4 * NT;                        // at most (64 / 16) x NT tiles
        constexpr int TPW = (MT + kWaves - 1) / kWaves;
        const T *ks = as_all;
        const int KT = (n + 15) >> 4;
        const int l16 = lane & 15, lhi = lane >> 4;
        __syncthreads();
        acc_t macc[TPW];
#pragma unroll
        for (int u = 0; u < TPW; ++u) {
            macc[u] = acc_t{0, 0, 0, 0};
            const int tile = w + kWaves * u;
            if (tile >= KT * NT) continue;
            const int a = tile / NT, t = tile - a * NT;
            const int ar = min(16 * a + l16, n - 1);
            const bool arok = 16 * a + l16 < n;
            for (int q = 4 * a; q < KC; ++q) {
                const int kr = 4 * q + lhi;
                const T av = (arok && kr < n) ? ks[ar * n + min(kr, n - 1)] : T(0);
                macc[u] = Mfma<T>::run(av, wl[(q * NT + t) * 64 + lane], macc[u]);
            }
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < TPW; ++u) {
            const int tile = w + kWaves * u;
            if (tile >= KT * NT) continue;
            const int a = tile / NT, t = tile - a * NT;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int r = 16 * a + Mfma<T>::row(lane, i);
                if (r < 4 * KC) wl[((r >> 2) * NT + t) * 64 + (r & 3) * 16 + l16] = -macc[u][i];
            }
        }
        // rows of -M past 4 KC do not exist; rows in [n, 4 KC) hold zeros (K's rows past n)
    }
    // this work-group's share of the panel's 16-row blocks: chunk rc of nrc, blocks dealt to the
    // waves in turn
    const int b0 = w + kWaves * rc, bstep = kWaves * nrc;
    if (b0 < nblk) fetch(b0);
    // zero this wave's staging block once: columns [n, 4 KC) stay zero
    for (int e = lane; e < 16 * LDA; e += 64) as[e] = T(0);
    __syncthreads();
    const int jl = j0 + (lane & 15);
    const T *ap = as + (lane & 15) * LDA + (lane >> 4);
    const T *wk = wl + lane;
    // output element i of a tile: row Mfma::row(lane, i) of the block, column jl + 16 t; the
    // lane's offsets from the block's first row are fixed, the block base is uniform
    int64_t off0[4], off1[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int r = Mfma<T>::row(lane, i);
        off0[i] = r * ld0 + jl;
        off1[i] = r * ld1 + jl - k0;
    }
    for (int blk = b0; blk < nblk; blk += bstep) {
        const int r0 = blk * 16;
        const int cnt = min(16, nr - r0);
        if (ok0) {
#pragma unroll
            for (int r = 0; r < 16; ++r) as[r * LDA + lane] = pre[r];
        }
        if constexpr (WIDE) {
            if (ok1) {
#pragma unroll
                for (int r = 0; r < 16; ++r) as[r * LDA + lane + 64] = pre2[r];
            }
        }
        if (blk + bstep < nblk) fetch(blk + bstep);
        // the wave reads back what its own lanes wrote: LDS operations of a wave are ordered
        acc_t acc[NT];
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[t] = acc_t{0, 0, 0, 0};
        for (int kc = 0; kc < KC; ++kc) {
            const T a = ap[4 * kc];
#pragma unroll
            for (int t = 0; t < NT; ++t) acc[t] = Mfma<T>::run(a, wk[(kc * NT + t) * 64], acc[t]);
        }
        // columns below k0 go to out0, the rest to out1 (shifted by k0); a tile lies on one
        // side of k0 except at most one, which selects per lane
        To *const b0 = out0 + (rb + r0) * ld0;
        To *const b1 = out1 ? out1 + (rb + r0) * ld1 : b0;
        auto put = [&](To *o, T v) {
            if constexpr (ACC) *o = (To)(v + (T)*o);
            else *o = (To)v;
        };
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const int jt = j0 + 16 * t;                 // uniform first column of the tile
            if (jt >= k) break;
            const bool jok = jl + 16 * t < k;
            if constexpr (VK) {
                // the [W; 0] term on the panel's top n rows
                if (r0 < n) {
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const int rr = r0 + Mfma<T>::row(lane, i);
                        if (jok && rr < n && Mfma<T>::row(lane, i) < cnt)
                            acc[t][i] += (T)Wp[(int64_t)rr * ldw + jl + 16 * t];
                    }
                }
            }
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                if (!(jok && Mfma<T>::row(lane, i) < cnt)) continue;
                if (jt + 16 <= k0) put(b0 + off0[i] + 16 * t, acc[t][i]);
                else if (jt >= k0) put(b1 + off1[i] + 16 * t, acc[t][i]);
                else put(jl + 16 * t < k0 ? b0 + off0[i] + 16 * t : b1 + off1[i] + 16 * t,
                         acc[t][i]);
            }
        }
    }
}

template <typename T, typename To, int NT>
__device__ __forceinline__ void apply_mfma_panel(int64_t rows, int n, int b,
                                                 const T *__restrict__ q1, int64_t ldq,
                                                 const double *__restrict__ W, int64_t ldw,
                                                 int64_t wstride, int k, To *__restrict__ out0,
                                                 int64_t ld0, int k0, To *__restrict__ out1,
                                                 int64_t ld1, int accumulate, int64_t p, int j0,
                                                 int rc = 0, int nrc = 1,
                                                 const T *__restrict__ kmat = nullptr)
{
#define TSQR_APPLY(ACC, WIDE)                                                                   \
    apply_panel_impl<T, To, NT, ACC, WIDE, false>(rows, n, b, q1, ldq, W, ldw, wstride, k, out0, \
                                                  ld0, k0, out1, ld1, p, j0, rc, nrc, nullptr)
    if (kmat != nullptr && n <= 64) {
        apply_panel_impl<T, To, NT, false, false, true>(rows, n, b, q1, ldq, W, ldw, wstride, k,
                                                        out0, ld0, k0, out1, ld1, p, j0, rc, nrc,
                                                        kmat);
        return;
    }
    if (n > 64) {
        if (accumulate) TSQR_APPLY(true, true);
        else TSQR_APPLY(false, true);
    } else {
        if (accumulate) TSQR_APPLY(true, false);
        else TSQR_APPLY(false, false);
    }
#undef TSQR_APPLY
}

inline size_t apply_lds_bytes_nt(size_t elem, int64_t n, int nt)
{
    const int KC = (int)((n + 3) / 4);
    return elem * ((size_t)KC * nt * 64 + (size_t)kWaves * 16 * (4 * KC + 1));
}
template <typename T, int NT> inline size_t apply_lds_bytes(int64_t n)
{
    return apply_lds_bytes_nt(sizeof(T), n, NT);
}

}  // namespace mfmaapply
}  // namespace tsqr
