// Blocked Householder panel factorization on the matrix cores (FP64, n <= 64): the device body
// shared by the single-matrix and batched launches.
//
// Step 1 of direct TSQR (Sec. III-B) for one row panel of B = NW * RT * 16 rows per work-group.
// The panel lives in registers in the accumulator layout of v_mfma_f64_16x16x4: it is cut into
// 16 x 16 tiles; wave w owns row tiles w*RT .. w*RT+RT-1 of every column tile, and lane l holds
// element (l/16 + 4i, l%16) of a tile in value i.  Columns are factored in blocks of 16 (one
// column tile):
//   * inside a block, Householder column k (Sec. III-A) is one barrier-separated step: the pivot
//     column is broadcast within each 16-lane row group, the dot products with the block's 16
//     columns are reduced over the lanes, the waves (through LDS) and the rows, and the block's
//     columns get the rank-1 update;
//   * the block's reflectors are then gathered as V (unit lower trapezoidal) with the compact
//     WY factor T (upper triangular, from V^T V by the column recurrence), and the trailing column
//     tiles receive A <- (I - V T^T V^T) A through two products on the matrix cores:
//     W = V^T A (the accumulator layout of V is directly the A operand of V^T) and A -= V (T^T W)
//     (V re-laid out through LDS as the A operand);
//   * then either (FORM_Q1) the explicit Q1 = H_1 ... H_n [I; 0] is formed in place, block by
//     block from the last, with the same two products and T in place of T^T, so that step 3 is a
//     plain GEMM; or (STORE_VK, n <= 64) the reflectors V are stored with the n x n matrix
//     K = T_p V1^T, T_p the compact-WY factor of the whole panel and V1 the top n rows of V, so
//     that Q1 = [I; 0] - V K and step 3 forms Q1 W = [W; 0] - V (K W) without Q1 ever existing.
//     T_p is assembled from the blocks' T and the cross products V_l^T V_j of the blocks:
//     T_p[i][j] = -(sum_{l=i..j-1} T_p[i][l] V_l^T V_j) T_jj (tiles of 16).  This costs far fewer
//     matrix-core operations than forming Q1 (no product over the panel's rows per block).
//
// Householder convention (as in the other panel kernels): beta = -sign(alpha) sqrt(alpha^2 + s2),
// tau = (beta - alpha)/beta, v = [1; x/(alpha - beta)], tau = 0 when the column below the
// diagonal is already zero.  The x below the diagonal is kept unscaled until V is gathered.
#pragma once

#include <type_traits>

#include "tsqr_internal.h"

namespace tsqr {
namespace blkpanel {

typedef double d4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));

// Element-type specifics of the 16x16x4 matrix-core tiles.  The A and B operand layouts are
// the same for FP64 and FP32 (lane l: A[l % 16][l / 16], B[l / 16][l % 16]); the accumulator
// holds row rit(l / 16, i) of column l % 16 in value i, with rit = l/16 + 4i (FP64) or
// 4 (l/16) + i (FP32).
template <typename T> struct BlkT;
template <> struct BlkT<double> {
    typedef d4_t acc_t;
    static __device__ __forceinline__ acc_t mfma(double a, double b, acc_t c)
    {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static constexpr __host__ __device__ int rit(int lr, int i) { return lr + 4 * i; }
    static constexpr __host__ __device__ int kk_lr(int kk) { return kk & 3; }
    static constexpr __host__ __device__ int kk_i(int kk) { return kk >> 2; }
    // value of lane KK of this lane's 16-lane row (DPP row_newbcast). Every lane reads a valid
    // source lane, so the old value is never used: bound_ctrl lets the compiler skip zeroing it.
    template <int KK> static __device__ __forceinline__ double bcast16(double v)
    {
        const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), 0x150 + KK, 0xf, 0xf, true);
        const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), 0x150 + KK, 0xf, 0xf, true);
        return __hiloint2double(hi, lo);
    }
    // v[l] + v[l ^ 16] and v[l] + v[l ^ 32] through the gfx950 lane-swap instructions (the two
    // partners end up in the two outputs, so each pair of lanes forms the same sum)
    static __device__ __forceinline__ double sum_xor16(double v)
    {
        const auto lo = __builtin_amdgcn_permlane16_swap(__double2loint(v), __double2loint(v), false, false);
        const auto hi = __builtin_amdgcn_permlane16_swap(__double2hiint(v), __double2hiint(v), false, false);
        return __hiloint2double(hi[0], lo[0]) + __hiloint2double(hi[1], lo[1]);
    }
    static __device__ __forceinline__ double sum_xor32(double v)
    {
        const auto lo = __builtin_amdgcn_permlane32_swap(__double2loint(v), __double2loint(v), false, false);
        const auto hi = __builtin_amdgcn_permlane32_swap(__double2hiint(v), __double2hiint(v), false, false);
        return __hiloint2double(hi[0], lo[0]) + __hiloint2double(hi[1], lo[1]);
    }
    // reciprocal: hardware estimate and two Newton steps
    static __device__ __forceinline__ double rcp(double x)
    {
        double r = __builtin_amdgcn_rcp(x);
        r = fma(r, fma(-x, r, 1.0), r);
        return fma(r, fma(-x, r, 1.0), r);
    }
    // square root of x > 0 inside the normal range (column norms are formed unscaled, as the
    // contract requires): the hardware reciprocal square root y, then coupled Newton iterations
    // for g = x y ~ sqrt(x) and h = y / 2, and two residual corrections g += (x - g^2) h.  Without
    // the range scaling of the general routine.  (x = 0 gives a NaN the caller discards.)
    static __device__ __forceinline__ double sqrt_pos(double x)
    {
        const double y = __builtin_amdgcn_rsq(x);
        double g = x * y, h = 0.5 * y;
        const double r = fma(-g, h, 0.5);
        g = fma(g, r, g);
        h = fma(h, r, h);
        g = fma(fma(-g, g, x), h, g);
        return fma(fma(-g, g, x), h, g);
    }
};
template <> struct BlkT<float> {
    typedef f4_t acc_t;
    static __device__ __forceinline__ acc_t mfma(float a, float b, acc_t c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static constexpr __host__ __device__ int rit(int lr, int i) { return 4 * lr + i; }
    static constexpr __host__ __device__ int kk_lr(int kk) { return kk >> 2; }
    static constexpr __host__ __device__ int kk_i(int kk) { return kk & 3; }
    template <int KK> static __device__ __forceinline__ float bcast16(float v)
    {
        return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x150 + KK, 0xf, 0xf, true));
    }
    static __device__ __forceinline__ float sum_xor16(float v)
    {
        const auto x = __builtin_amdgcn_permlane16_swap(__float_as_int(v), __float_as_int(v), false, false);
        return __int_as_float(x[0]) + __int_as_float(x[1]);
    }
    static __device__ __forceinline__ float sum_xor32(float v)
    {
        const auto x = __builtin_amdgcn_permlane32_swap(__float_as_int(v), __float_as_int(v), false, false);
        return __int_as_float(x[0]) + __int_as_float(x[1]);
    }
    static __device__ __forceinline__ float rcp(float x)
    {
        float r = __builtin_amdgcn_rcpf(x);
        return fmaf(r, fmaf(-x, r, 1.0f), r);
    }
    static __device__ __forceinline__ float sqrt_pos(float x)
    {
        const float y = __builtin_amdgcn_rsqf(x);
        float g = x * y, h = 0.5f * y;
        const float r = fmaf(-g, h, 0.5f);
        g = fmaf(g, r, g);
        h = fmaf(h, r, h);
        return fmaf(fmaf(-g, g, x), h, g);
    }
};

template <int I, int N, typename F> __device__ __forceinline__ void static_for(F &&f)
{
    if constexpr (I < N) {
        f(std::integral_constant<int, I>{});
        static_for<I + 1, N>(f);
    }
}

// LDS of one work-group (dynamic: more than 64 KiB for the widest panels).  TC = column tiles
// whose per-wave products are reduced at a time.
// LDS behind BlkSmem for the STORE_VK tail: the cross products gx[l][j] = V_l^T V_j (l < j) of
// the blocks' reflectors, later reused for the top row tiles v1[j][l] of V (j >= l); every tile
// 16 x 16 row-major.  (The tiles of T_p overlay BlkSmem::red, free by then.)
template <typename T, int NCT> struct BlkTail {
    T tiles[NCT][NCT][256];
};

template <typename T, int NCT, int RT, int NW, int TC> struct BlkSmem {
    T part[2][NW][16];               // per-step partial dots of the block's columns
    T rowk[2][16];                   // pivot row k restricted to the block
    T tau[NCT * 16], u[NCT * 16], beta[NCT * 16];
    union {
        T red[NW][TC][256];          // per-wave partial products (G, W) before the wave sum
        T vt[NW][16][17];            // one row tile of V per wave, row-major (A operand of V Y)
    };
    T wsum[NCT][256];                // summed products: slot kt = G = V^T V, slot t = W of tile t
    T tstore[NCT][16][17];           // T of every block (kept for the Q1 formation)
    T ybuf[16][NCT * 16 + 1];        // Y = T^T W (or T W) for the trailing tiles
};

// q1 == nullptr: R only.  Otherwise VK: q1 receives V (rows x n, ld n) and kout the panel's K
// (n x n, ld n, at p n n); !VK: q1 receives the explicit Q1.
template <typename Tin, typename T, int NCT, int RT, int NW, int TC, bool VK = false>
__device__ __forceinline__ void factor_blk_panel(int64_t rows, int n, const Tin *__restrict__ X,
                                                 int64_t ldx, T *__restrict__ q1,
                                                 double *__restrict__ S, int64_t p,
                                                 T *__restrict__ kout = nullptr)
{
    using K = BlkT<T>;
    typedef typename K::acc_t acc_t;
    constexpr int B = NW * RT * 16;
    constexpr int NT = NW * 64;
    extern __shared__ __align__(16) unsigned char blk_smem_raw[];
    BlkSmem<T, NCT, RT, NW, TC> &sm = *reinterpret_cast<BlkSmem<T, NCT, RT, NW, TC> *>(blk_smem_raw);

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lc = lane & 15, lr = lane >> 4;
    const int64_t prow0 = p * (int64_t)B;
    const int nrow = (int)min((int64_t)B, rows - prow0);
    // row tiles are dealt out to the waves in turn (tile g belongs to wave g % NW), so the
    // finished top rows and the pivot tile of every block are spread over the waves
    auto row_of = [&](int rt, int i) { return 16 * (rt * NW + w) + K::rit(lr, i); };

    // ---- load the panel (zero rows past the end and columns past n) -------------------------
    acc_t P[RT][NCT];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int ct = 0; ct < NCT; ++ct)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int r = row_of(rt, i), c = 16 * ct + lc;
                P[rt][ct][i] = (r < nrow && c < n) ? (T)X[(prow0 + r) * ldx + c] : T(0);
            }

    // V of block KT from the stored x's: unit diagonal, zero above, x / (alpha - beta) below;
    // zero for a skipped reflector (tau = 0) or a padding column
    auto gather_v = [&](auto KT, T (&V)[RT][4]) {
        constexpr int kt = decltype(KT)::value;
        const int c = 16 * kt + lc;
        const T tc = (c < n) ? sm.tau[c] : T(0);
        const T inv = (tc != T(0)) ? K::rcp(sm.u[c]) : T(0);
#pragma unroll
        for (int rt = 0; rt < RT; ++rt)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int r = row_of(rt, i);
                T v = T(0);
                if (tc != T(0)) v = (r > c) ? P[rt][kt][i] * inv : ((r == c) ? T(1) : T(0));
                V[rt][i] = v;
            }
    };

    // W_t = V^T A[:, tile t] for tiles t >= T0 into wsum[t], and with WITH_G also G = V^T V into
    // wsum[KT] (then T0 > KT); summed over the waves in a fixed order, TC products at a time.
    // Ends with a barrier.
    auto block_products = [&](auto KT, auto T0, auto WITH_G, const T (&V)[RT][4]) {
        constexpr int kt = decltype(KT)::value, t0 = decltype(T0)::value;
        constexpr bool with_g = decltype(WITH_G)::value;
        constexpr int L = (with_g ? 1 : 0) + (NCT - t0);          // products: [G,] tiles t0..
        constexpr int NCH = (L + TC - 1) / TC;
        static_for<0, NCH>([&](auto CH) {
            constexpr int c0 = decltype(CH)::value * TC;
            // product e of the list: G for e == 0 with_g, else tile t0 + e - with_g
            acc_t acc[TC];
#pragma unroll
            for (int s = 0; s < TC; ++s) acc[s] = acc_t{0, 0, 0, 0};
#pragma unroll
            for (int rt = 0; rt < RT; ++rt)
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int s = 0; s < TC; ++s) {
                        const int e = c0 + s;
                        if (e >= L) continue;
                        if (with_g && e == 0) acc[s] = K::mfma(V[rt][i], V[rt][i], acc[s]);
                        else acc[s] = K::mfma(V[rt][i], P[rt][t0 + e - (with_g ? 1 : 0)][i], acc[s]);
                    }
#pragma unroll
            for (int s = 0; s < TC; ++s)
                if (c0 + s < L)
#pragma unroll
                    for (int i = 0; i < 4; ++i) sm.red[w][s][K::rit(lr, i) * 16 + lc] = acc[s][i];
            __syncthreads();
            for (int e2 = tid; e2 < TC * 256; e2 += NT) {
                const int s = e2 >> 8, e = c0 + s;
                if (e >= L) continue;
                const int slot = (with_g && e == 0) ? kt : t0 + e - (with_g ? 1 : 0);
                T sum = T(0);
#pragma unroll
                for (int ww = 0; ww < NW; ++ww) sum += sm.red[ww][s][e2 & 255];
                sm.wsum[slot][e2 & 255] = sum;
            }
            __syncthreads();
        });
    };

    // T of block KT (Q_blk = H_1 ... H_16 = I - V T V^T) from G = wsum[KT] = V^T V by the
    // column recurrence T[0:j, j] = -tau_j T[0:j, 0:j] G[0:j, j], T[j][j] = tau_j.  Row i of T
    // needs only earlier entries of row i, so wave 0 computes all rows at once: lane (i, q) =
    // i + 16 q holds T[i][l] for the columns l = q mod 4 in registers (zero until computed, and
    // zero below the diagonal), forms its share of the sum over l < j, and the four shares of a
    // row are added with the lane swaps.  Ends with a barrier.
    auto block_t = [&](auto KT) {
        constexpr int kt = decltype(KT)::value;
        if (w == 0) {
            const int i = lane & 15, q = lane >> 4;
            const T *gq = &sm.wsum[kt][q * 16];             // row q of G; row 4m + q at +64 m
            T tr[4] = {T(0), T(0), T(0), T(0)};
            static_for<0, 16>([&](auto J) {
                constexpr int j = decltype(J)::value;
                const int cj = 16 * kt + j;
                const T tj = (cj < n) ? sm.tau[cj] : T(0);
                T part = T(0);
#pragma unroll
                for (int m = 0; m < 4; ++m) part = fma(tr[m], gq[64 * m + j], part);
                const T sum = K::sum_xor32(K::sum_xor16(part));
                const T tij = (i < j) ? -tj * sum : ((i == j) ? tj : T(0));
                if (q == (j & 3)) tr[j >> 2] = tij;
            });
#pragma unroll
            for (int m = 0; m < 4; ++m) sm.tstore[kt][i][4 * m + q] = tr[m];
        }
        __syncthreads();
    };

    // Y_t = T^T W_t (TRANS) or T W_t for tiles t >= T0 into sm.ybuf, one 16 x 16 tile per wave
    // on the matrix cores.  Ends with a barrier.
    auto block_y = [&](auto KT, auto T0, auto TRANS) {
        constexpr int kt = decltype(KT)::value, t0 = decltype(T0)::value;
        constexpr bool trans = decltype(TRANS)::value;
        for (int t = t0 + w; t < NCT; t += NW) {
            acc_t acc = acc_t{0, 0, 0, 0};
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const T a = trans ? sm.tstore[kt][4 * q + lr][lc] : sm.tstore[kt][lc][4 * q + lr];
                const T b = sm.wsum[t][(4 * q + lr) * 16 + lc];
                acc = K::mfma(a, b, acc);
            }
#pragma unroll
            for (int i = 0; i < 4; ++i) sm.ybuf[K::rit(lr, i)][16 * t + lc] = acc[i];
        }
        __syncthreads();
    };

    // A[:, tiles t >= T0] -= V * Y[:, tiles], Y in sm.ybuf; V re-laid out row tile by row tile
    // through this wave's sm.vt as the row-major A operand
    auto block_update = [&](auto T0, const T (&V)[RT][4]) {
        constexpr int t0 = decltype(T0)::value;
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) {
#pragma unroll
            for (int i = 0; i < 4; ++i) sm.vt[w][K::rit(lr, i)][lc] = V[rt][i];
            // (the wave reads back what its own lanes wrote: LDS operations of a wave are ordered)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const T a = sm.vt[w][lc][4 * q + lr];
#pragma unroll
                for (int t = t0; t < NCT; ++t)
                    P[rt][t] = K::mfma(a, -sm.ybuf[4 * q + lr][16 * t + lc], P[rt][t]);
            }
        }
    };

    // ---- factorization, block by block ---------------------------------------------------
    static_for<0, NCT>([&](auto KT) {
        constexpr int kt = decltype(KT)::value;
        if (16 * kt >= n) return;
        // the 16 Householder steps of the block, unrolled: row k = 16 kt + kk lives in row tile
        // kt, i.e. in wave kt % NW, tile slot kt / NW, at row kk of that tile
        static_for<0, 16>([&](auto KK) {
            constexpr int kk = decltype(KK)::value;
            constexpr int par = kk & 1;
            constexpr int rtk = kt / NW, ik = K::kk_i(kk);
            const int k = 16 * kt + kk;
            if (k >= n) return;
            const bool own = (w == kt % NW);                  // this wave holds row tile kt
            if (own && lr == K::kk_lr(kk)) sm.rowk[par][lc] = P[rtk][kt][ik];
            // pivot column x (rows > k) and the partial dots with the block's columns; tiles
            // above tile kt hold finished rows (x = 0, no update)
            T xm[RT][4];
            T dacc[4] = {T(0), T(0), T(0), T(0)};      // four independent FMA chains
#pragma unroll
            for (int rt = 0; rt < RT; ++rt) {
                const int gt = rt * NW + w;
                if (gt > kt) {
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        xm[rt][i] = K::template bcast16<kk>(P[rt][kt][i]);
                        dacc[i] = fma(xm[rt][i], P[rt][kt][i], dacc[i]);
                    }
                } else if (gt == kt) {
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const T xv = K::template bcast16<kk>(P[rt][kt][i]);
                        xm[rt][i] = (K::rit(lr, i) > kk) ? xv : T(0);
                        dacc[i] = fma(xm[rt][i], P[rt][kt][i], dacc[i]);
                    }
                } else {
#pragma unroll
                    for (int i = 0; i < 4; ++i) xm[rt][i] = T(0);
                }
            }
            const T d = K::sum_xor32(K::sum_xor16((dacc[0] + dacc[1]) + (dacc[2] + dacc[3])));
            if (lr == 0) sm.part[par][w][lc] = d;
            __syncthreads();
            // the waves' partials and the pivot row, read together and added pairwise (NW is a
            // power of two)
            T ps[NW], pp[NW];
#pragma unroll
            for (int ww = 0; ww < NW; ++ww) {
                ps[ww] = sm.part[par][ww][kk];
                pp[ww] = sm.part[par][ww][lc];
            }
            const T alpha = sm.rowk[par][kk];
            T rowc = sm.rowk[par][lc];
#pragma unroll
            for (int h = NW / 2; h >= 1; h /= 2)
#pragma unroll
                for (int ww = 0; ww < h; ++ww) {
                    ps[ww] += ps[ww + h];
                    pp[ww] += pp[ww + h];
                }
            const T s2 = ps[0];
            T pc = pp[0];
            // an empty use of pc and rowc here: without it the compiler sinks their reads into
            // the branch that needs them, after the square root, and pays a second LDS round trip
            asm volatile("" : "+v"(pc), "+v"(rowc));
            // one reciprocal per step: with r = 1 / (u beta), tau = (beta - alpha)/beta = -u^2 r
            // and the coefficient tau (a_kc + pc/u)/u of column c is -(a_kc u + pc) r
            // Computed without a branch and then selected (s2 = 0: no reflection, tau = 0), so
            // the sum for pc can overlap the square root; the discarded values of that case
            // (a reciprocal of zero) never reach a result.
            const bool live = s2 != T(0);
            const T nrm = K::sqrt_pos(fma(alpha, alpha, s2));
            const T bl = (alpha >= T(0)) ? -nrm : nrm;
            const T ul = alpha - bl;
            const T rl = K::rcp(ul * bl);
            const T beta = live ? bl : alpha;
            const T u = live ? ul : T(0);
            const T r = live ? rl : T(0);
            const T tau = live ? -ul * ul * rl : T(0);
            const T cl = -fma(rowc, u, pc) * r;
            const T coef = (live && lc > kk && 16 * kt + lc < n) ? cl : T(0);
#pragma unroll
            for (int rt = 0; rt < RT; ++rt) {
                const int gt = rt * NW + w;
                if (gt > kt) {
#pragma unroll
                    for (int i = 0; i < 4; ++i) P[rt][kt][i] = fma(-coef, xm[rt][i], P[rt][kt][i]);
                } else if (gt == kt) {
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const T x = (K::rit(lr, i) == kk) ? u : xm[rt][i];
                        P[rt][kt][i] = fma(-coef, x, P[rt][kt][i]);
                    }
                }
            }
            // read only after the barrier that ends the block (each step writes its own slot)
            if (tid == 0) { sm.tau[k] = tau; sm.u[k] = u; sm.beta[k] = beta; }
        });
        __syncthreads();      // tau, u of the block visible to every wave
        if constexpr (kt + 1 < NCT) {
            if (16 * (kt + 1) < n) {
                T V[RT][4];
                gather_v(KT, V);
                block_products(KT, std::integral_constant<int, kt + 1>{}, std::true_type{}, V);
                block_t(KT);
                block_y(KT, std::integral_constant<int, kt + 1>{}, std::true_type{});
                block_update(std::integral_constant<int, kt + 1>{}, V);
            }
        }
    });
    __syncthreads();

    // ---- R_p: rows 0..n-1, strict upper part from the registers, diagonal = beta -----------
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int ct = 0; ct < NCT; ++ct)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int r = row_of(rt, i), c = 16 * ct + lc;
                if (r < n && c < n)
                    S[(p * n + r) * n + c] = (c > r) ? (double)P[rt][ct][i] : ((c == r) ? (double)sm.beta[r] : T(0) /*keep*/);
            }
    if (q1 == nullptr) return;
    const int nblk = (n + 15) >> 4;

    if constexpr (VK) {
        static_assert(NCT * NCT <= NW * TC, "the tiles of T_p overlay BlkSmem::red");
        BlkTail<T, NCT> &tl = *reinterpret_cast<BlkTail<T, NCT> *>(blk_smem_raw + sizeof(sm));
        T(*tf)[256] = reinterpret_cast<T(*)[256]>(&sm.red[0][0][0]);     // tile (i, j) at tf[i * NCT + j]
        // acc += A B for 16 x 16 tiles in LDS: A row-major (ld lda); B row-major (ld ldb), or
        // transposed when BT (element (k, c) of B at b[c * ldb + k])
        auto tile_mma = [&](acc_t acc, const T *a, int lda, const T *b, int ldb, bool bt) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int kq = 4 * q + lr;
                const T av = a[lc * lda + kq];
                const T bv = bt ? b[lc * ldb + kq] : b[kq * ldb + lc];
                acc = K::mfma(av, bv, acc);
            }
            return acc;
        };
        // the last block's T (its trailing step did not run)
        static_for<0, NCT>([&](auto I) {
            constexpr int kt = decltype(I)::value;
            if (kt != nblk - 1) return;
            T V[RT][4];
            gather_v(I, V);
            block_products(I, std::integral_constant<int, NCT>{}, std::true_type{}, V);
            block_t(I);
        });
        // V of every block, in place in P (zero in the tiles past n), and stored
        static_for<0, NCT>([&](auto I) {
            constexpr int kt = decltype(I)::value;
            T V[RT][4];
            if (kt < nblk) {
                gather_v(I, V);
            } else {
#pragma unroll
                for (int rt = 0; rt < RT; ++rt)
#pragma unroll
                    for (int i = 0; i < 4; ++i) V[rt][i] = T(0);
            }
#pragma unroll
            for (int rt = 0; rt < RT; ++rt)
#pragma unroll
                for (int i = 0; i < 4; ++i) P[rt][kt][i] = V[rt][i];
        });
#pragma unroll
        for (int rt = 0; rt < RT; ++rt)
#pragma unroll
            for (int ct = 0; ct < NCT; ++ct)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int r = row_of(rt, i), c = 16 * ct + lc;
                    if (r < nrow && c < n) q1[(prow0 + r) * n + c] = P[rt][ct][i];
                }
        // cross products V_l^T V_j, l < j (over the panel's rows, summed over the waves)
        static_for<0, NCT - 1>([&](auto L) {
            constexpr int l = decltype(L)::value;
            if (l + 1 >= nblk) return;
            T V[RT][4];
#pragma unroll
            for (int rt = 0; rt < RT; ++rt)
#pragma unroll
                for (int i = 0; i < 4; ++i) V[rt][i] = P[rt][l][i];
            block_products(L, std::integral_constant<int, l + 1>{}, std::false_type{}, V);
            for (int e = tid; e < (NCT - 1 - l) * 256; e += NT) tl.tiles[l][l + 1 + (e >> 8)][e & 255] = sm.wsum[l + 1 + (e >> 8)][e & 255];
            __syncthreads();
        });
        // T_p tile rows: wave i computes row i (T_p[i][j], j > i, from its own earlier tiles)
        for (int e = tid; e < nblk * 256; e += NT) {
            const int i = e >> 8, r = (e >> 4) & 15, c = e & 15;
            tf[i * NCT + i][e & 255] = sm.tstore[i][r][c];
        }
        __syncthreads();
        if (w < nblk) {
            const int i = w;
            for (int j = i + 1; j < nblk; ++j) {
                acc_t y = acc_t{0, 0, 0, 0};
                for (int l = i; l < j; ++l) y = tile_mma(y, tf[i * NCT + l], 16, tl.tiles[l][j], 16, false);
#pragma unroll
                for (int q = 0; q < 4; ++q) tf[i * NCT + j][K::rit(lr, q) * 16 + lc] = y[q];
                // (the wave reads back what its own lanes wrote: LDS operations of a wave are ordered)
                acc_t t = acc_t{0, 0, 0, 0};
                t = tile_mma(t, tf[i * NCT + j], 16, &sm.tstore[j][0][0], 17, false);
#pragma unroll
                for (int q = 0; q < 4; ++q) tf[i * NCT + j][K::rit(lr, q) * 16 + lc] = -t[q];
            }
        }
        __syncthreads();
        // the top row tiles of V (row tile g holds blocks l <= g), in place of the cross products
        static_for<0, RT>([&](auto RTI) {
            constexpr int rt = decltype(RTI)::value;
            const int g = rt * NW + w;
            if (g < nblk) {
#pragma unroll
                for (int l = 0; l < NCT; ++l)
                    if (l <= g)
#pragma unroll
                        for (int q = 0; q < 4; ++q) tl.tiles[g][l][K::rit(lr, q) * 16 + lc] = P[rt][l][q];
            }
        });
        __syncthreads();
        // K = T_p V1^T: tile (i, j) = sum_{l=i..j} T_p[i][l] (V1^T)[l][j], (V1^T)[l][j] = v1[j][l]^T
        T *kp = kout + p * (int64_t)n * n;
        for (int tt = w; tt < NCT * NCT; tt += NW) {
            const int i = tt / NCT, j = tt - i * NCT;
            if (i >= nblk || j >= nblk) continue;
            acc_t acc = acc_t{0, 0, 0, 0};
            if (i <= j)
                for (int l = i; l <= j; ++l) acc = tile_mma(acc, tf[i * NCT + l], 16, tl.tiles[j][l], 16, true);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int r = 16 * i + K::rit(lr, q), c = 16 * j + lc;
                if (r < n && c < n) kp[(int64_t)r * n + c] = acc[q];
            }
        }
        return;
    }

    // ---- explicit Q1 = H_1 ... H_n [I; 0], in place, block by block from the last -----------
    static_for<0, NCT>([&](auto I) {
        constexpr int kt = NCT - 1 - decltype(I)::value;
        if (kt >= nblk) return;
        using KT = std::integral_constant<int, kt>;
        T V[RT][4];
        gather_v(KT{}, V);
        if (kt == nblk - 1) {
            // the last block's T (its trailing step did not run)
            block_products(KT{}, std::integral_constant<int, NCT>{}, std::true_type{}, V);
            block_t(KT{});
        }
        // the block's own columns are still identity columns of [I; 0]
#pragma unroll
        for (int rt = 0; rt < RT; ++rt)
#pragma unroll
            for (int i = 0; i < 4; ++i)
                P[rt][kt][i] = (row_of(rt, i) == 16 * kt + lc) ? T(1) : T(0);
        block_products(KT{}, KT{}, std::false_type{}, V);
        block_y(KT{}, KT{}, std::false_type{});
        block_update(KT{}, V);
        __syncthreads();
    });
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int ct = 0; ct < NCT; ++ct)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int r = row_of(rt, i), c = 16 * ct + lc;
                if (r < nrow && c < n) q1[(prow0 + r) * n + c] = P[rt][ct][i];
            }
}

}  // namespace blkpanel
}  // namespace tsqr
