// Blocked panels for 97 <= n <= 112 (one width class per translation unit, so that the
// build compiles the wide classes in parallel): FP64 panels, and FP32 panels on FP64 or FP32 input.
#include "panel_blk_launch.h"

namespace tsqr {

hipError_t factor_blk_wide7(int in_dtype, int dtype, int64_t rows, int64_t n, const void *X,
                            int64_t ldx, void *q1, double *S, hipStream_t st)
{
    using namespace blklaunch;
    if (dtype == F64) return factor_blk_launch<double, double, 7>(rows, n, X, ldx, q1, S, st);
    if (in_dtype == F64) return factor_blk_launch<double, float, 7>(rows, n, X, ldx, q1, S, st);
    return factor_blk_launch<float, float, 7>(rows, n, X, ldx, q1, S, st);
}

}  // namespace tsqr
