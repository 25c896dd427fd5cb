// Register-resident panel kernels of the single-matrix path: the panel factorization (device
// body in panel_reg_body.h) and the LDS-staged vector apply.
#include "panel_blk_body.h"
#include "panel_reg_body.h"


namespace tsqr {
namespace {

using namespace regpanel;

template <typename Tin, typename T, int NC, int CPL, int RW, int NW>
__global__ void __launch_bounds__(NW * 64, (NW <= 8) ? 4 : 3)
k_factor_reg(int64_t rows, int n, const Tin *__restrict__ X, int64_t ldx, T *__restrict__ q1,
             double *__restrict__ S)
{
    factor_reg_panel<Tin, T, NC, CPL, RW, NW>(rows, n, X, ldx, q1, S, blockIdx.x);
}

// Panel shapes of the blocked FP64 kernel (no spills, two work-groups per CU up to n = 64):
// 4 waves with 256 rows for 32 < n <= 64, 384 rows for n <= 32; 8 waves with 256 rows for
// 64 < n <= 128 (one work-group per CU).
template <int NCT> struct BlkShape {
    static constexpr int NW = (NCT <= 4) ? 4 : 8;
    static constexpr int RT = (NCT <= 2) ? 6 : ((NCT <= 4) ? 4 : 2);
    static constexpr int TC = (NCT <= 4) ? NCT : 2;
    static constexpr int B = NW * RT * 16;
    static constexpr size_t LDS = sizeof(blkpanel::BlkSmem<NCT, RT, NW, TC>);
};

template <int NCT>
__global__ void __launch_bounds__(BlkShape<NCT>::NW * 64, (NCT <= 4) ? 2 : 1)
k_factor_blk(int64_t rows, int n, const double *__restrict__ X, int64_t ldx,
             double *__restrict__ q1, double *__restrict__ S)
{
    using C = BlkShape<NCT>;
    blkpanel::factor_blk_panel<NCT, C::RT, C::NW, C::TC>(rows, n, X, ldx, q1, S, blockIdx.x);
}

template <int NCT>
hipError_t factor_blk_launch(int64_t rows, int64_t n, const void *X, int64_t ldx, void *q1,
                             double *S, hipStream_t st)
{
    using C = BlkShape<NCT>;
    const int64_t panels = ceil_div(rows, C::B);
    static bool attr_set = false;
    if (C::LDS > 64 * 1024 && !attr_set) {
        hipError_t e = hipFuncSetAttribute((const void *)k_factor_blk<NCT>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)C::LDS);
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    hipLaunchKernelGGL((k_factor_blk<NCT>), dim3((unsigned)panels), dim3(C::NW * 64), C::LDS, st,
                       rows, (int)n, (const double *)X, ldx, (double *)q1, S);
    return hipGetLastError();
}

hipError_t factor_blk_dispatch(int64_t rows, int64_t n, const void *X, int64_t ldx, void *q1,
                               double *S, hipStream_t st)
{
    switch ((n + 15) / 16) {
    case 1: return factor_blk_launch<1>(rows, n, X, ldx, q1, S, st);
    case 2: return factor_blk_launch<2>(rows, n, X, ldx, q1, S, st);
    case 3: return factor_blk_launch<3>(rows, n, X, ldx, q1, S, st);
    case 4: return factor_blk_launch<4>(rows, n, X, ldx, q1, S, st);
    case 5: return factor_blk_launch<5>(rows, n, X, ldx, q1, S, st);
    case 6: return factor_blk_launch<6>(rows, n, X, ldx, q1, S, st);
    case 7: return factor_blk_launch<7>(rows, n, X, ldx, q1, S, st);
    default: return factor_blk_launch<8>(rows, n, X, ldx, q1, S, st);
    }
}

int blk_panel_rows(int64_t n)
{
    switch ((n + 15) / 16) {
    case 1: return BlkShape<1>::B;
    case 2: return BlkShape<2>::B;
    case 3: return BlkShape<3>::B;
    case 4: return BlkShape<4>::B;
    case 5: return BlkShape<5>::B;
    case 6: return BlkShape<6>::B;
    case 7: return BlkShape<7>::B;
    default: return BlkShape<8>::B;
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

template <typename Tin, typename T, int NC, int CPL>
hipError_t factor_reg_cfg(int64_t rows, int64_t n, const void *X, int64_t ldx, void *q1,
                          double *S, hipStream_t st)
{
    using C = RegCfg<T, NC, CPL>;
    return factor_reg_launch<Tin, T, NC, CPL, C::RW, C::NW>(rows, n, X, ldx, q1, S, st);
}

template <typename Tin, typename T>
hipError_t factor_reg_dispatch(int64_t rows, int64_t n, const void *X, int64_t ldx, void *q1,
                               double *S, hipStream_t st)
{
    if (n <= 4) return factor_reg_cfg<Tin, T, 4, 1>(rows, n, X, ldx, q1, S, st);
    if (n <= 8) return factor_reg_cfg<Tin, T, 8, 1>(rows, n, X, ldx, q1, S, st);
    if (n <= 16) return factor_reg_cfg<Tin, T, 16, 1>(rows, n, X, ldx, q1, S, st);
    if (n <= 32) return factor_reg_cfg<Tin, T, 32, 1>(rows, n, X, ldx, q1, S, st);
    if (n <= 64) return factor_reg_cfg<Tin, T, 64, 1>(rows, n, X, ldx, q1, S, st);
    return factor_reg_cfg<Tin, T, 64, 2>(rows, n, X, ldx, q1, S, st);
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
    if (dtype == F64) return blk_panel_rows(n);
    return reg_panel_rows_variant(n, dtype, 0);
}

hipError_t launch_factor_reg(int in_dtype, int dtype, int64_t rows, int64_t n, const void *X,
                             int64_t ldx, void *q1, double *S, hipStream_t st)
{
    if (dtype == F64) {
        if (in_dtype == F64) return factor_blk_dispatch(rows, n, X, ldx, q1, S, st);
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
