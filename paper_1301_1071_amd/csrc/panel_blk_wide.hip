// Dispatch of the blocked panels wider than 64 columns (panel_blk_wide5..8.hip).
#include "tsqr_internal.h"

namespace tsqr {

#define TSQR_WIDE_DECL(I)                                                                      \
    hipError_t factor_blk_wide##I(int in_dtype, int dtype, int64_t rows, int64_t n,          \
                                  const void *X, int64_t ldx, void *q1, double *S,           \
                                  hipStream_t st);
TSQR_WIDE_DECL(5)
TSQR_WIDE_DECL(6)
TSQR_WIDE_DECL(7)
TSQR_WIDE_DECL(8)
#undef TSQR_WIDE_DECL

hipError_t factor_blk_wide(int nct, int in_dtype, int dtype, int64_t rows, int64_t n,
                           const void *X, int64_t ldx, void *q1, double *S, hipStream_t st)
{
    switch (nct) {
    case 5: return factor_blk_wide5(in_dtype, dtype, rows, n, X, ldx, q1, S, st);
    case 6: return factor_blk_wide6(in_dtype, dtype, rows, n, X, ldx, q1, S, st);
    case 7: return factor_blk_wide7(in_dtype, dtype, rows, n, X, ldx, q1, S, st);
    case 8: return factor_blk_wide8(in_dtype, dtype, rows, n, X, ldx, q1, S, st);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace tsqr
