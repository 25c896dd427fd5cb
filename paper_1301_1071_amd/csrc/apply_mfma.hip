// Single-matrix launches of the MFMA apply (device body in apply_mfma_body.h).
#include "apply_mfma_body.h"

namespace tsqr {
namespace {

using namespace mfmaapply;

// One work-group per (panel, 16 NT-column slice, row chunk).  The 1-D grid keeps the ny * nrc
// slices of one panel on the same XCD (work-group b runs on XCD b % 8): b = 8 S g + 8 s + x with
// S = ny nrc covers panel 8 g + x, column slice s % ny and row chunk s / ny, so a panel's Q1 rows
// are read from HBM once and served from that XCD's L2 to the other column slices.  Row chunks
// (nrc > 1) only for launches with few panels, where one work-group per panel would leave most of
// the chip idle and walk all of a panel's row blocks in turn.
template <typename T, typename To, int NT>
__global__ void __launch_bounds__(kWaves * 64)
k_apply_mfma(int64_t rows, int n, int b, const T *__restrict__ q1, int64_t ldq,
             const double *__restrict__ W, int64_t ldw, int64_t wstride, int k,
             To *__restrict__ out0, int64_t ld0, int k0, To *__restrict__ out1, int64_t ld1,
             int accumulate, int64_t panels, int ny, int nrc, const T *__restrict__ kmat)
{
    const int64_t bid = blockIdx.x;
    const int S = ny * nrc;
    const int64_t grp = bid / (8 * S);
    const int rem = (int)(bid - grp * 8 * S);
    const int sl = rem >> 3;
    const int y = sl % ny, rc = sl / ny;
    const int64_t p = grp * 8 + (rem & 7);
    if (p >= panels) return;
    apply_mfma_panel<T, To, NT>(rows, n, b, q1, ldq, W, ldw, wstride, k, out0, ld0, k0, out1,
                                ld1, accumulate, p, y * 16 * NT, rc, nrc, kmat);
}

template <typename T, typename To, int NT>
hipError_t apply_mfma_nt(int64_t rows, int64_t n, int b, const void *q1, int64_t ldq,
                         const double *W, int64_t ldw, int64_t wstride, int k, void *out0,
                         int64_t ld0, int k0, void *out1, int64_t ld1, int acc, const void *kmat,
                         hipStream_t st)
{
    const size_t lds = apply_lds_bytes<T, NT>(n);
    auto kern = k_apply_mfma<T, To, NT>;
    hipError_t e = ensure_dynamic_lds((const void *)kern, lds);
    if (e != hipSuccess) return e;
    const int64_t panels = ceil_div(rows, b);
    const int ny = (int)ceil_div(k, 16 * NT);
    // row chunks: about 1024 work-groups (four per CU), at most one 16-row block per wave and
    // chunk round.  A launch with hundreds of panels (the first tree level of a tall matrix)
    // then keeps one work-group per panel, which measured faster than splitting its rows
    const int max_chunks = (int)ceil_div(ceil_div(b, 16), kWaves);
    const int64_t want = 1024 / (panels * ny);
    const int nrc = (int)std::max<int64_t>(1, std::min<int64_t>(max_chunks, want));
    const int64_t blocks = ceil_div(panels, 8) * 8 * ny * nrc;
    hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(kWaves * 64), lds, st, rows, (int)n, b,
                       (const T *)q1, ldq, W, ldw, wstride, k, (To *)out0, ld0, k0, (To *)out1,
                       ld1, acc, panels, ny, nrc, (const T *)kmat);
    return hipGetLastError();
}

constexpr size_t kMaxLds = 160 * 1024;

template <typename T, typename To>
hipError_t apply_mfma_t(int64_t rows, int64_t n, int b, const void *q1, int64_t ldq,
                        const double *W, int64_t ldw, int64_t wstride, int k, void *out0,
                        int64_t ld0, int k0, void *out1, int64_t ld1, int acc, const void *kmat,
                        hipStream_t st, int one_slice)
{
    // Column slices per panel: as few as keep a work-group within 8 output tiles and 80 KB of
    // LDS (the W image plus the staged Q1 blocks), so that two work-groups share a CU.  Every
    // slice stages the panel's Q1 rows again (from the XCD's L2), so fewer slices read less.
    const int tiles = (int)ceil_div(k, 16);
    int ny = 1;
    auto nt_of = [&](int y) { return (int)ceil_div(tiles, y); };
    if (one_slice) {
        if (nt_of(1) > 8 || apply_lds_bytes_nt(sizeof(T), n, nt_of(1)) > kMaxLds)
            return hipErrorInvalidValue;
    } else {
        while (ny < tiles &&
               (nt_of(ny) > 8 || apply_lds_bytes_nt(sizeof(T), n, nt_of(ny)) > 80 * 1024))
            ++ny;
    }
#define TSQR_NT(NT)                                                                           \
    case NT:                                                                                  \
        return apply_mfma_nt<T, To, NT>(rows, n, b, q1, ldq, W, ldw, wstride, k, out0, ld0, k0, \
                                        out1, ld1, acc, kmat, st)
    switch (nt_of(ny)) {
        TSQR_NT(1);
        TSQR_NT(2);
        TSQR_NT(3);
        TSQR_NT(4);
        TSQR_NT(5);
        TSQR_NT(6);
        TSQR_NT(7);
        TSQR_NT(8);
    default: return hipErrorInvalidValue;
    }
#undef TSQR_NT
}

}  // namespace

hipError_t launch_apply_vk(int q_dtype, int out_dtype, int64_t rows, int64_t n, int b,
                          const void *q1, int64_t ldq, const double *W, int64_t ldw,
                          int64_t wstride, int k, void *out0, int64_t ld0, int k0, void *out1,
                          int64_t ld1, int accumulate, const void *kmat, hipStream_t st,
                          int one_slice = 0)
{
    if (n > 4 * kMaxKC) {
        // wide n: the product runs in K chunks of 4 kMaxKC columns of Q1 (rows of W), the
        // first overwriting the output and the others adding to it
        if (kmat || one_slice || n > kNmaxWide) return hipErrorInvalidValue;
        const size_t es = (q_dtype == F64) ? sizeof(double) : sizeof(float);
        for (int64_t c0 = 0; c0 < n; c0 += 4 * kMaxKC) {
            const int64_t nc = std::min<int64_t>(4 * kMaxKC, n - c0);
            hipError_t e = launch_apply_vk(q_dtype, out_dtype, rows, nc, b,
                                           (const char *)q1 + es * c0, ldq, W + c0 * ldw, ldw,
                                           wstride, k, out0, ld0, k0, out1, ld1,
                                           (accumulate || c0 > 0) ? 1 : 0, nullptr, st);
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    }
    if (kmat && (n > 64 || accumulate)) return hipErrorInvalidValue;
    if (q_dtype == F64) {
        if (out_dtype == F64)
            return apply_mfma_t<double, double>(rows, n, b, q1, ldq, W, ldw, wstride, k, out0, ld0,
                                                k0, out1, ld1, accumulate, kmat, st, one_slice);
        return apply_mfma_t<double, float>(rows, n, b, q1, ldq, W, ldw, wstride, k, out0, ld0, k0,
                                           out1, ld1, accumulate, kmat, st, one_slice);
    }
    if (out_dtype == F64)
        return apply_mfma_t<float, double>(rows, n, b, q1, ldq, W, ldw, wstride, k, out0, ld0, k0,
                                           out1, ld1, accumulate, kmat, st, one_slice);
    return apply_mfma_t<float, float>(rows, n, b, q1, ldq, W, ldw, wstride, k, out0, ld0, k0, out1,
                                      ld1, accumulate, kmat, st, one_slice);
}

hipError_t launch_gemm_mfma(int q_dtype, int out_dtype, int64_t rows, int64_t n, int b,
                            const void *q1, int64_t ldq, const double *W, int64_t ldw,
                            int64_t wstride, int k, void *out0, int64_t ld0, int k0, void *out1,
                            int64_t ld1, int accumulate, hipStream_t st, int one_slice)
{
    return launch_apply_vk(q_dtype, out_dtype, rows, n, b, q1, ldq, W, ldw, wstride, k, out0, ld0,
                           k0, out1, ld1, accumulate, nullptr, st, one_slice);
}

hipError_t launch_apply_mfma(int q_dtype, int out_dtype, int64_t rows, int64_t n, int b,
                             const void *q1, const double *W, int64_t ldw, int64_t wstride, int k,
                             void *out0, int64_t ld0, int k0, void *out1, int64_t ld1,
                             const void *kmat, hipStream_t st, int one_slice)
{
    return launch_apply_vk(q_dtype, out_dtype, rows, n, b, q1, n, W, ldw, wstride, k, out0, ld0, k0,
                           out1, ld1, 0, kmat, st, one_slice);
}

bool apply_one_slice_ok(int q_dtype, int out_dtype, int64_t n, int k)
{
    (void)out_dtype;
    if (n < 1 || n > 4 * kMaxKC || k < 1) return false;
    const int64_t tiles = ceil_div(k, 16);
    const size_t es = (q_dtype == F64) ? sizeof(double) : sizeof(float);
    return tiles <= 8 && apply_lds_bytes_nt(es, n, (int)tiles) <= kMaxLds;
}

}  // namespace tsqr
