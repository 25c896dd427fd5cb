// Launchers of the blocked panel kernel for the single-matrix path (device body in
// panel_blk_body.h): every register-panel level of the tree, FP64 or FP32 arithmetic.
#include "panel_blk_launch.h"

namespace tsqr {
namespace {
using namespace blklaunch;

template <typename T> struct BlkShapeRows {
    static int rows(int64_t n)
    {
        switch ((n + 15) / 16) {
        case 1: return BlkShape<T, 1>::B;
        case 2: return BlkShape<T, 2>::B;
        case 3: return BlkShape<T, 3>::B;
        default: return BlkShape<T, 4>::B;
        }
    }
};

}  // namespace

// Panels wider than 64 columns (panel_blk_wide*.hip, one translation unit per width class so
// that the build compiles them in parallel)
hipError_t factor_blk_wide(int nct, int in_dtype, int dtype, int64_t rows, int64_t n,
                           const void *X, int64_t ldx, void *q1, double *S, hipStream_t st);

namespace {
using namespace blklaunch;

template <typename Tin, typename T>
hipError_t factor_blk_dispatch(int64_t rows, int64_t n, const void *X, int64_t ldx, void *q1,
                               double *S, void *kout, hipStream_t st)
{
    switch ((n + 15) / 16) {
    case 1: return factor_blk_launch<Tin, T, 1>(rows, n, X, ldx, q1, S, st, kout);
    case 2: return factor_blk_launch<Tin, T, 2>(rows, n, X, ldx, q1, S, st, kout);
    case 3: return factor_blk_launch<Tin, T, 3>(rows, n, X, ldx, q1, S, st, kout);
    default: return factor_blk_launch<Tin, T, 4>(rows, n, X, ldx, q1, S, st, kout);
    }
}

}  // namespace

int reg_panel_rows(int64_t n, int dtype)
{
    if (n > 64) return blklaunch::BlkShape<double, 5>::B;   // every class above 64 columns
    if (dtype == F32) return BlkShapeRows<float>::rows(n);
    return BlkShapeRows<double>::rows(n);
}

hipError_t launch_factor_reg(int in_dtype, int dtype, int64_t rows, int64_t n, const void *X,
                             int64_t ldx, void *q1, double *S, void *kout, hipStream_t st)
{
    if (n < 1 || n > 128) return hipErrorInvalidValue;
    if (dtype == F64 && in_dtype != F64) return hipErrorInvalidValue;
    if (n > 64) {
        if (kout) return hipErrorInvalidValue;     // V + K form only for n <= 64
        return factor_blk_wide((int)((n + 15) / 16), in_dtype, dtype, rows, n, X, ldx, q1, S, st);
    }
    if (dtype == F64) return factor_blk_dispatch<double, double>(rows, n, X, ldx, q1, S, kout, st);
    if (in_dtype == F64) return factor_blk_dispatch<double, float>(rows, n, X, ldx, q1, S, kout, st);
    return factor_blk_dispatch<float, float>(rows, n, X, ldx, q1, S, kout, st);
}

}  // namespace tsqr
