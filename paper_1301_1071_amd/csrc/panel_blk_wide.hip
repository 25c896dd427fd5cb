// Dispatch of the FP64 blocked panels wider than 64 columns (panel_blk_wide5..8.hip).
#include "tsqr_internal.h"

namespace tsqr {

hipError_t factor_blk_wide5(int64_t, int64_t, const void *, int64_t, void *, double *, hipStream_t);
hipError_t factor_blk_wide6(int64_t, int64_t, const void *, int64_t, void *, double *, hipStream_t);
hipError_t factor_blk_wide7(int64_t, int64_t, const void *, int64_t, void *, double *, hipStream_t);
hipError_t factor_blk_wide8(int64_t, int64_t, const void *, int64_t, void *, double *, hipStream_t);

hipError_t factor_blk_wide(int nct, int64_t rows, int64_t n, const void *X, int64_t ldx, void *q1,
                           double *S, hipStream_t st)
{
    switch (nct) {
    case 5: return factor_blk_wide5(rows, n, X, ldx, q1, S, st);
    case 6: return factor_blk_wide6(rows, n, X, ldx, q1, S, st);
    case 7: return factor_blk_wide7(rows, n, X, ldx, q1, S, st);
    case 8: return factor_blk_wide8(rows, n, X, ldx, q1, S, st);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace tsqr
