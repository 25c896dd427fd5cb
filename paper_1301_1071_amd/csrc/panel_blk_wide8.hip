// FP64 blocked panels for 113 <= n <= 128 (one width class per translation unit).
#include "panel_blk_launch.h"

namespace tsqr {

hipError_t factor_blk_wide8(int64_t rows, int64_t n, const void *X, int64_t ldx, void *q1,
                            double *S, hipStream_t st)
{
    return blklaunch::factor_blk_launch<double, double, 8>(rows, n, X, ldx, q1, S, st);
}

}  // namespace tsqr
