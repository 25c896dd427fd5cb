// Shapes, kernel and launcher of the blocked panel kernel for the single-matrix path (device
// body in panel_blk_body.h); included by panel_blk.hip and the per-width panel_blk_wide*.hip.
#pragma once

#include "panel_blk_body.h"

namespace tsqr {
namespace blklaunch {

using blkpanel::BlkSmem;

// Panel shapes (no register spills): 4 waves with 384 rows for n <= 32 (two work-groups per
// CU); 8 waves with 512 rows for 32 < n <= 64 and 256 rows for 64 < n <= 128 (one work-group per
// CU).  FP32 uses the same shapes.
template <typename T, int NCT> struct BlkShape {
    static constexpr int NW = (NCT <= 2) ? 4 : 8;
    static constexpr int RT = (NCT <= 2) ? 6 : ((NCT <= 4) ? 4 : 2);
    static constexpr int TC = (NCT <= 2) ? NCT : 4;
    static constexpr int B = NW * RT * 16;
    static constexpr size_t LDS = sizeof(BlkSmem<T, NCT, RT, NW, TC>);
    // with the STORE_VK tail (n <= 64)
    static constexpr size_t LDS_VK = LDS + sizeof(blkpanel::BlkTail<T, NCT>);
};

// VK: kout != nullptr selects the STORE_VK tail (q1 receives V, kout the panels' K); otherwise
// q1 receives the explicit Q1 (or nothing when null).
template <typename Tin, typename T, int NCT, bool VK>
__global__ void __launch_bounds__((NCT <= 2) ? 256 : 512, (NCT <= 2) ? 2 : 1)
k_factor_blk(int64_t rows, int n, const Tin *__restrict__ X, int64_t ldx, T *__restrict__ q1,
             double *__restrict__ S, T *__restrict__ kout)
{
    using C = BlkShape<T, NCT>;
    blkpanel::factor_blk_panel<Tin, T, NCT, C::RT, C::NW, C::TC, VK>(rows, n, X, ldx, q1, S,
                                                                    blockIdx.x, kout);
}

template <typename Tin, typename T, int NCT>
hipError_t factor_blk_launch(int64_t rows, int64_t n, const void *X, int64_t ldx, void *q1,
                             double *S, hipStream_t st, void *kout = nullptr)
{
    using C = BlkShape<T, NCT>;
    const int64_t panels = ceil_div(rows, C::B);
    if constexpr (NCT <= 4) {
        if (kout) {
            hipError_t e = ensure_dynamic_lds((const void *)k_factor_blk<Tin, T, NCT, true>, C::LDS_VK);
            if (e != hipSuccess) return e;
            hipLaunchKernelGGL((k_factor_blk<Tin, T, NCT, true>), dim3((unsigned)panels),
                               dim3(C::NW * 64), C::LDS_VK, st, rows, (int)n, (const Tin *)X, ldx,
                               (T *)q1, S, (T *)kout);
            return hipGetLastError();
        }
    }
    if (kout) return hipErrorInvalidValue;
    hipError_t e = ensure_dynamic_lds((const void *)k_factor_blk<Tin, T, NCT, false>, C::LDS);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_factor_blk<Tin, T, NCT, false>), dim3((unsigned)panels), dim3(C::NW * 64),
                       C::LDS, st, rows, (int)n, (const Tin *)X, ldx, (T *)q1, S, (T *)nullptr);
    return hipGetLastError();
}

}  // namespace blklaunch
}  // namespace tsqr
