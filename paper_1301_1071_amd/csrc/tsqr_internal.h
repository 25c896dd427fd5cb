// Internal declarations shared by the HIP translation units of libtsqr.so (not installed).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/tsqr.h"

namespace tsqr {

constexpr int kThreads = 256;          // work-group size of the panel kernels (4 waves of 64)
constexpr int kMaxLevels = 48;         // recursion depth limit of the in-HBM tree
constexpr size_t kAlign = 256;         // workspace sub-buffer alignment
constexpr int kNmaxPad = 128;          // column capacity of per-column LDS arrays, n <= 128
constexpr int kNmaxWide = 512;         // the same for the wide path (128 < n <= TSQR_NMAX)

// ---- optional per-launch timing (benchmarks): HIP event pairs on the launch stream (api.hip)
enum ProfClass {
    PC_FACTOR0 = 0, PC_FACTOR_TREE, PC_FINALIZE, PC_APPLY_TREE, PC_APPLY0, PC_REFINE,
    PC_BWD_GRAM, PC_BWD_SMALL, PC_BWD_GEMM, PC_COUNT
};
extern const char *kProfNames[PC_COUNT];
struct ProfScope {
    int cls;
    hipStream_t st;
    hipEvent_t a = nullptr;
    ProfScope(int c, hipStream_t s);
    ~ProfScope();
};

// Record the text of a failed HIP call for tsqr_last_error().
void set_last_error(hipError_t e, const char *what, int line);
#define TSQR_HIP_CHECK(expr)                                                                \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess) {                                                             \
            ::tsqr::set_last_error(e_, #expr, __LINE__);                                    \
            return TSQR_ERR_HIP;                                                            \
        }                                                                                   \
    } while (0)

// Raise `kernel`'s dynamic-LDS limit to at least `bytes` on the current device.  The attribute
// is set once per (kernel, device, larger size) under a lock, so concurrent host threads and
// several devices are safe.  A no-op at or below the 64 KiB default.
hipError_t ensure_dynamic_lds(const void *kernel, size_t bytes);

inline size_t align_up(size_t x, size_t a = kAlign) { return (x + a - 1) / a * a; }
inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Which element type a buffer holds.
enum Dtype : int { F64 = 0, F32 = 1 };

// One level of the recursive direct TSQR (Sec. III-C, Alg. 2).  Level 0 factors A; level L >= 1
// factors the stacked R factors of level L-1 (P_{L-1} * n rows, FP64).
struct Level {
    int64_t rows = 0;     // rows of the matrix factored at this level
    int64_t panels = 0;   // number of row panels (map tasks)
    int b = 0;            // panel height
    int dtype = F64;      // arithmetic of the panel work at this level
    size_t q1 = 0;        // offset of explicit Q1 panels (rows x n, ld n), 0 if not kept; with
                          // kv != 0 the panels' reflectors V instead
    size_t kv = 0;        // offset of the panels' K (panels x n x n): Q1_p = [I; 0] - V_p K_p
    size_t s = 0;         // offset of the stacked R output (panels*n x n, FP64)
    size_t x = 0;         // offset of this level's Q (rows x k, FP64), levels >= 1 only
    size_t gpanel = 0;    // offset of global scratch panels (panels tall for LDS), 0 if unused
    bool global = false;  // panel held in global scratch instead of LDS
    bool reg = true;      // register-resident panel kernel (else the LDS/global one)
};

struct Plan {
    int op = 0;
    int64_t m = 0, n = 0;
    int precision = TSQR_FP64;
    int in_dtype = F64;   // element type of A
    int nlev = 0;
    Level lev[kMaxLevels];
    int k = 0;            // columns carried down the tree (n for Q or U, 2n for Q and U)
    size_t wtop = 0;      // n x k FP64: [D | D U_R]
    size_t svd_g = 0, svd_v = 0;   // n x n FP64 scratch for the Jacobi SVD
    size_t refine = 0;    // refinement scratch (padded triangles, Gram partials)
    size_t qtmp = 0;      // m x n FP64 Q for an SVD of the precision form without a Q output
    size_t rhat = 0;      // n x n FP64 R-hat of the FP32 path (precision form with refinement)
    size_t rref = 0;      // n x n FP64 refined R (SVD of the precision form)
    bool reuse_output = false;   // level-0 panel factors kept in the Q (or U) output
    size_t total = 0;
};

// ---- launchers (panel_lds.hip) ------------------------------------------------------------
// Default panel height for (n, dtype) of the LDS-resident panel kernel.
int lds_panel_rows(int64_t n, int dtype);
// Largest panel height the LDS-resident kernel supports for (n, dtype).
int lds_panel_rows_max(int64_t n, int dtype);

// Factor every panel of a rows x n matrix X (element type in_dtype, ld ldx) in `dtype`
// arithmetic: write R_p (FP64) into S (panels*n x n) and, if q1 != nullptr, the explicit
// Q1_p (rows x n, ld n, element type dtype).  gpanel != nullptr holds the panels in global
// scratch (panels * n * (b + 1) elements) instead of LDS.
hipError_t launch_factor(int in_dtype, int dtype, int64_t rows, int64_t n, int b,
                         const void *X, int64_t ldx, void *q1, double *S, void *gpanel,
                         hipStream_t st);

// ---- launchers (panel_blk.hip): blocked register panels, the default for every level --------
// Panel height of the blocked kernel for (n, dtype): 384 rows for n <= 32, 512 for n <= 64, 256
// above.  q1 == nullptr: R only; kout != nullptr (n <= 64): q1 receives V and kout the panels' K
// (element type dtype, panels x n x n); otherwise q1 receives the explicit Q1.
int reg_panel_rows(int64_t n, int dtype);
hipError_t launch_factor_reg(int in_dtype, int dtype, int64_t rows, int64_t n, const void *X,
                             int64_t ldx, void *q1, double *S, void *kout, hipStream_t st);

// ---- launchers (apply_mfma.hip): step 3 on the matrix cores --------------------------------
// out = Q1 * W per panel: panel p (rows [p b, p b + b)) uses W rows [p*wstride, p*wstride + n).
// Columns [0, k0) of the product go to out0 (ld0), columns [k0, k) to out1 (ld1).  With kmat
// (n <= 64) q1 holds the reflectors V and kmat the panels' K (Q1 = [I; 0] - V K).
// one_slice: one work-group covers all k output columns of its rows (no column slices), so the
// output may be the buffer q1 itself (each row block is read before it is written).
hipError_t launch_apply_mfma(int q_dtype, int out_dtype, int64_t rows, int64_t n, int b,
                             const void *q1, const double *W, int64_t ldw, int64_t wstride, int k,
                             void *out0, int64_t ld0, int k0, void *out1, int64_t ld1,
                             const void *kmat, hipStream_t st, int one_slice = 0);
// Whether launch_apply_mfma supports one_slice for (q_dtype, n, k): n <= 128, k <= 128 and the
// W image plus the staged blocks within one work-group's LDS.
bool apply_one_slice_ok(int q_dtype, int out_dtype, int64_t n, int k);

// General tall product on the same kernel: out = X * W (X: rows x n, row stride ldq) panel by
// panel (panel p of b rows uses W rows [p*wstride, +n)); accumulate != 0 adds to out.
hipError_t launch_gemm_mfma(int q_dtype, int out_dtype, int64_t rows, int64_t n, int b,
                            const void *q1, int64_t ldq, const double *W, int64_t ldw,
                            int64_t wstride, int k, void *out0, int64_t ld0, int k0, void *out1,
                            int64_t ld1, int accumulate, hipStream_t st, int one_slice = 0);

// ---- launchers (backward.hip) ----------------------------------------------------------------
// Partial Grams C_b = X_b^T Y_b of row blocks (X, Y: m x n FP64) into part (nblk x n x n).
int gram_blocks(int64_t m);
hipError_t launch_gram(int64_t m, int64_t n, const double *X, int64_t ldx, const double *Y,
                       int64_t ldy, double *part, double *G, hipStream_t st);
// The n x n middle steps (n <= 128) as row-parallel launches, one work-group per row of W2;
// `scratch` is not used.
hipError_t launch_qr_bwd_small(int64_t n, const double *R, const double *dR, int64_t lddr,
                               const double *G, double *W2, double *scratch, int32_t *info,
                               hipStream_t st);
hipError_t launch_svd_bwd_small(int64_t n, const double *S, const double *V, const double *dS,
                                const double *dV, int64_t lddv, const double *UtdU, double *W2,
                                double *scratch, int32_t *info, hipStream_t st);

// ---- launchers (small.hip) -----------------------------------------------------------------
// Top of the tree: R = D Rt (D = diag(sign(Rt_jj)), sign(0) = +1) written to R (FP64, ldr) or Rf
// (FP32, ldr); W_top (n x k) = [D | D U_R] (Q columns first if want_q, then U columns if want_u);
// the SVD of R (one-sided Jacobi) when want_u or S != nullptr.  Sets *info.
// S / V (FP64) or Sf / Vf (FP32) receive the singular values and right singular vectors.
// keep_info != 0 leaves a nonzero *info from an earlier kernel of the call in place.
hipError_t launch_finalize(int64_t n, const double *Rt, double *R, float *Rf, int64_t ldr,
                           double *Wtop, int k, int want_q, int want_u, double *S, float *Sf,
                           double *V, float *Vf, int64_t ldv, double *G, double *Vw,
                           int32_t *info, hipStream_t st, int keep_info = 0);

// ---- launchers (refine.hip) ----------------------------------------------------------------
// One FP64 refinement of the precision form (n <= 64): Q (FP64, ldq) and R (FP64, ldr) from A
// and the FP32-path R-hat (n x n, ld n, diag > 0); info = -2 when a Cholesky step breaks down.
size_t refine_scratch_bytes(int64_t m, int64_t n);
hipError_t launch_refine(int64_t m, int64_t n, const double *A, int64_t lda, const double *Rhat,
                         double *Q, int64_t ldq, double *R, int64_t ldr, void *scratch,
                         int32_t *info, hipStream_t st);

// ---- launchers (indirect.hip): comparison methods of the stability experiment --------------
// Cholesky of the Gram G (n x n): R = L^T and Rinv = R^{-1} (info = -4 on breakdown).
hipError_t launch_cholqr_small(int64_t n, const double *G, double *R, double *Rinv, int32_t *info,
                               int keep_info, hipStream_t st);
hipError_t launch_rinv_small(int64_t n, const double *R, double *Rinv, hipStream_t st);
// Rout (ldr) = R2 R1 for upper-triangular n x n factors (ld n).
hipError_t launch_trmul_small(int64_t n, const double *R2, const double *R1, double *Rout,
                              int64_t ldr, hipStream_t st);

}  // namespace tsqr
