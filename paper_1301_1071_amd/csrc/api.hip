// C ABI of libtsqr.so: argument checks, the level plan of the recursive tree, workspace layout
// and the launch sequence.  See include/tsqr.h for the contract of every entry point.
//
// Launch sequence of tsqr_qr / tsqr_svd (all on the caller's stream, no host synchronisation):
//   level 0 .. T   factor:  panels of the level matrix -> explicit Q1 panels + stacked R
//                  (level 0 factors A; level L factors the stacked R of level L-1, Sec. III-C);
//   finalize       R = D R~ (+ SVD of R), W_top = [D | D U_R], info;
//   level T .. 0   apply:   Q1_p * W_p, W_p = rows [p n, p n + n) of the level above (the
//                  reduce task's k-th key <-> rows (k-1)n+1..kn of its Q, Sec. III-B).
#include <algorithm>
#include <map>
#include <mutex>
#include <stdio.h>
#include <string.h>
#include <utility>
#include <vector>

#include "tsqr_internal.h"

namespace tsqr {

const char *kProfNames[PC_COUNT] = {"factor_level0", "factor_tree", "finalize_svd",
                                    "apply_tree", "apply_level0", "refine",
                                    "bwd_gram", "bwd_small", "bwd_gemm"};

struct ProfRec { int cls; hipEvent_t a, b; };
struct Profiler {
    std::mutex mu;
    bool on = false;
    uint32_t mask = 0xffffffffu;    // kernel classes recorded while on
    std::vector<hipEvent_t> pool;
    std::vector<ProfRec> recs;
    size_t next = 0;
};

// text of the most recent HIP failure (per thread), for tsqr_last_error()
thread_local char g_last_error[512] = "";

void set_last_error(hipError_t e, const char *what, int line)
{
    snprintf(g_last_error, sizeof(g_last_error), "%s (%d) in %.300s [line %d]",
             hipGetErrorString(e), (int)e, what, line);
}

hipError_t ensure_dynamic_lds(const void *kernel, size_t bytes)
{
    if (bytes <= 64 * 1024) return hipSuccess;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    static std::mutex mu;
    static std::map<std::pair<const void *, int>, size_t> granted;
    std::lock_guard<std::mutex> lk(mu);
    size_t &cur = granted[std::make_pair(kernel, dev)];
    if (cur >= bytes) return hipSuccess;
    e = hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (e == hipSuccess) cur = bytes;
    return e;
}

namespace {

Profiler g_prof;

hipEvent_t prof_event()
{
    if (g_prof.next < g_prof.pool.size()) return g_prof.pool[g_prof.next++];
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    g_prof.pool.push_back(e);
    g_prof.next = g_prof.pool.size();
    return e;
}

enum Op { OP_R = TSQR_OP_R, OP_QR = TSQR_OP_QR, OP_SVD = TSQR_OP_SVD };

size_t elem_size(int dt) { return dt == F32 ? 4 : 8; }

tsqr_status validate_opts(const tsqr_opts *o, int64_t n)
{
    if (!o) return TSQR_OK;
    if (o->struct_size != (int32_t)sizeof(tsqr_opts)) return TSQR_ERR_INVALID_ARG;
    if (o->precision < TSQR_FP64 || o->precision > TSQR_FP32) return TSQR_ERR_INVALID_ARG;
    if ((o->flags & ~TSQR_FLAG_REUSE_OUTPUT) != 0) return TSQR_ERR_INVALID_ARG;
    if (o->panel_rows < 0) return TSQR_ERR_INVALID_ARG;
    if (o->panel_rows > 0 && (o->panel_rows < n || o->panel_rows > (1 << 16)))
        return TSQR_ERR_INVALID_ARG;
    return TSQR_OK;
}

// Build the level plan and workspace layout.  want_q / want_u select the columns carried down.
tsqr_status build_plan(int op, int64_t m, int64_t n, int in_dtype, const tsqr_opts *o,
                       bool want_q, bool want_u, Plan &pl)
{
    if (m <= 0 || n <= 0) return TSQR_ERR_INVALID_ARG;
    if (n > TSQR_NMAX || m < n) return TSQR_ERR_SHAPE;
    tsqr_status vs = validate_opts(o, n);
    if (vs != TSQR_OK) return vs;
    pl = Plan();
    pl.op = op;
    pl.m = m;
    pl.n = n;
    pl.in_dtype = in_dtype;
    pl.precision = o ? o->precision : TSQR_FP64;
    if (in_dtype == F32) {
        // FP32 input always runs the FP32 path; a refinement needs FP64 input
        if (pl.precision == TSQR_FP32_REFINED) return TSQR_ERR_UNSUPPORTED;
        pl.precision = TSQR_FP32;
    }
    if (pl.precision == TSQR_FP32_REFINED && n > 64) return TSQR_ERR_UNSUPPORTED;
    const int dtype0 = (pl.precision == TSQR_FP64) ? F64 : F32;
    // the refined precision form keeps only R-hat from the FP32 tree (steps 1-2), then refines
    // against A; the SVD variant adds the SVD of the refined R and U = Q U_R
    const bool refined = (pl.precision == TSQR_FP32_REFINED) && op != OP_R;
    const bool need_q = (op != OP_R) && !refined;
    pl.k = need_q ? (int)((want_q ? n : 0) + (want_u ? n : 0)) : (refined && op == OP_SVD ? (int)n : 0);
    if (need_q && o && (o->flags & TSQR_FLAG_REUSE_OUTPUT)) {
        // the output is rewritten row block by row block while step 3 reads the same rows, so
        // one work-group must cover all of a panel's columns, in one chunk of K, in a buffer of
        // the level-0 element size
        if (n > kNmaxPad || elem_size(dtype0) != elem_size(in_dtype) ||
            !apply_one_slice_ok(dtype0, in_dtype, n, pl.k))
            return TSQR_ERR_UNSUPPORTED;
        pl.reuse_output = true;
    }

    size_t off = kAlign;   // offset 0 is reserved so that 0 means "not allocated"
    auto take = [&](size_t bytes) {
        size_t at = off;
        off = align_up(off + (bytes ? bytes : 1));
        return at;
    };
    int64_t rows = m;
    for (int L = 0;; ++L) {
        if (L >= kMaxLevels) return TSQR_ERR_UNSUPPORTED;
        Level &lv = pl.lev[L];
        lv.rows = rows;
        lv.dtype = (L == 0) ? dtype0 : F64;
        const int req = (L == 0 && o) ? o->panel_rows : 0;
        const int bl = lds_panel_rows_max(n, lv.dtype);
        const int breg = reg_panel_rows(n, lv.dtype);
        // levels run the blocked kernel, whose panels always shrink a stack of more than one
        // panel (b >= 2n); a short FP32 stack that they would not shrink uses one LDS (or
        // global-memory) panel instead
        const bool shrinks = ceil_div(rows, breg) * n < rows;
        if (n > kNmaxPad) {
            // the wide path: global-scratch panels of 4 n rows (explicit heights allowed), each
            // level a quarter of the one below
            lv.reg = false;
            const int64_t want = req ? req : 4 * n;
            lv.b = (int)(want < rows ? want : rows);
            lv.global = true;
        } else if (req == 0 && (rows <= breg || (shrinks && (lv.dtype == F64 || rows > 8 * n)))) {
            // default: register-resident panels of the register kernel's height
            lv.reg = true;
            lv.global = false;
            lv.b = (int)(rows < breg ? rows : breg);
        } else if (req == 0) {
            // a short stack that register panels would not shrink: one LDS (or global) panel
            lv.reg = false;
            lv.b = (int)rows;
            lv.global = lv.b > bl;
        } else {
            // an explicit panel height runs the LDS-resident kernel (global scratch if too tall)
            lv.reg = false;
            lv.b = (int)(req < rows ? req : rows);
            lv.global = lv.b > bl;
        }
        lv.panels = ceil_div(rows, lv.b);
        const size_t es = elem_size(lv.dtype);
        if (need_q && !(L == 0 && pl.reuse_output)) lv.q1 = take(es * (size_t)rows * n);
        // register panels with n <= 64 keep V and K (Q1 = [I; 0] - V K) instead of forming Q1
        if (need_q && lv.reg && n <= 64) lv.kv = take(es * (size_t)lv.panels * n * n);
        lv.s = take(sizeof(double) * (size_t)lv.panels * n * n);
        if (need_q && L >= 1) lv.x = take(sizeof(double) * (size_t)rows * pl.k);
        if (lv.global) lv.gpanel = take(es * (size_t)lv.panels * n * (lv.b + 1));
        pl.nlev = L + 1;
        if (lv.panels == 1) break;
        rows = lv.panels * n;
    }
    if (pl.k) pl.wtop = take(sizeof(double) * (size_t)n * pl.k);
    if (op == OP_SVD) {
        pl.svd_g = take(sizeof(double) * (size_t)n * n);
        pl.svd_v = take(sizeof(double) * (size_t)n * n);
    }
    if (refined) {
        pl.refine = take(refine_scratch_bytes(m, n));
        pl.rhat = take(sizeof(double) * (size_t)n * n);
        pl.rref = take(sizeof(double) * (size_t)n * n);
        if (op == OP_SVD && !want_q) pl.qtmp = take(sizeof(double) * (size_t)m * n);
    }
    pl.total = off;
    return TSQR_OK;
}

inline char *wsp(void *ws, size_t off) { return off ? (char *)ws + off : nullptr; }


// Steps 1-2 (+ finalize): every level's factor launch, then the top.
// q1_out: the output buffer that holds level 0's panel factors when pl.reuse_output.
tsqr_status run_factor_levels(const Plan &pl, const void *A, int64_t lda, void *ws,
                              hipStream_t st, void *q1_out = nullptr)
{
    for (int L = 0; L < pl.nlev; ++L) {
        const Level &lv = pl.lev[L];
        void *q1 = (L == 0 && pl.reuse_output) ? q1_out : (void *)wsp(ws, lv.q1);
        const void *X = (L == 0) ? A : (const void *)wsp(ws, pl.lev[L - 1].s);
        const int64_t ldx = (L == 0) ? lda : pl.n;
        const int in_dt = (L == 0) ? pl.in_dtype : F64;
        ProfScope ps(L == 0 ? PC_FACTOR0 : PC_FACTOR_TREE, st);
        if (lv.reg)
            TSQR_HIP_CHECK(launch_factor_reg(in_dt, lv.dtype, lv.rows, pl.n, X, ldx, q1,
                                             (double *)wsp(ws, lv.s), wsp(ws, lv.kv), st));
        else
            TSQR_HIP_CHECK(launch_factor(in_dt, lv.dtype, lv.rows, pl.n, lv.b, X, ldx, q1,
                                         (double *)wsp(ws, lv.s),
                                         lv.global ? wsp(ws, lv.gpanel) : nullptr, st));
    }
    return TSQR_OK;
}

// Step 3 down the tree.  Level 0 writes columns [0, k0) to out0 and [k0, k) to out1.
tsqr_status run_apply_levels(const Plan &pl, void *ws, int out_dtype, void *out0, int64_t ld0,
                             int k0, void *out1, int64_t ld1, hipStream_t st,
                             void *q1_out = nullptr)
{
    const double *W = (const double *)wsp(ws, pl.wtop);
    int64_t ldw = pl.k, wstride = 0;
    for (int L = pl.nlev - 1; L >= 0; --L) {
        const Level &lv = pl.lev[L];
        ProfScope ps(L == 0 ? PC_APPLY0 : PC_APPLY_TREE, st);
        if (L > 0) {
            double *X = (double *)wsp(ws, lv.x);
            TSQR_HIP_CHECK(launch_apply_mfma(F64, F64, lv.rows, pl.n, lv.b, wsp(ws, lv.q1), W,
                                             ldw, wstride, pl.k, X, pl.k, pl.k, nullptr, 0,
                                             wsp(ws, lv.kv), st));
            W = X;
            ldw = pl.k;
            wstride = pl.n;
        } else {
            const void *q1 = pl.reuse_output ? q1_out : (const void *)wsp(ws, lv.q1);
            TSQR_HIP_CHECK(launch_apply_mfma(lv.dtype, out_dtype, lv.rows, pl.n, lv.b, q1, W, ldw,
                                             wstride, pl.k, out0, ld0, k0, out1, ld1,
                                             wsp(ws, lv.kv), st, pl.reuse_output ? 1 : 0));
        }
    }
    return TSQR_OK;
}

const tsqr_opts *opts_or_default(const tsqr_opts *o, tsqr_opts &tmp)
{
    if (o) return o;
    tsqr_default_opts(&tmp);
    return &tmp;
}

tsqr_status check_ws(const Plan &pl, void *ws, size_t ws_bytes)
{
    if (!ws || ws_bytes < pl.total) return TSQR_ERR_WORKSPACE;
    return TSQR_OK;
}

tsqr_status do_r(int in_dtype, int64_t m, int64_t n, const void *A, int64_t lda, double *R,
                 float *Rf, int64_t ldr, void *ws, size_t ws_bytes, int32_t *d_info,
                 const tsqr_opts *opts, void *stream)
{
    if (!A || (!R && !Rf) || !d_info) return TSQR_ERR_INVALID_ARG;
    if (lda < n || ldr < n) return TSQR_ERR_INVALID_ARG;
    tsqr_opts tmp;
    Plan pl;
    tsqr_status s = build_plan(OP_R, m, n, in_dtype, opts_or_default(opts, tmp), false, false, pl);
    if (s != TSQR_OK) return s;
    if ((s = check_ws(pl, ws, ws_bytes)) != TSQR_OK) return s;
    hipStream_t st = (hipStream_t)stream;
    if ((s = run_factor_levels(pl, A, lda, ws, st)) != TSQR_OK) return s;
    const Level &top = pl.lev[pl.nlev - 1];
    ProfScope ps(PC_FINALIZE, st);
    TSQR_HIP_CHECK(launch_finalize(n, (const double *)wsp(ws, top.s), R, Rf, ldr, nullptr, 0, 0,
                                   0, nullptr, nullptr, nullptr, nullptr, 0, nullptr, nullptr,
                                   d_info, st));
    return TSQR_OK;
}

// The precision form's refinement (after the FP32 steps 1-2): R-hat = D R~ from the FP64 tree,
// then the FP64 refinement writing Q (ldq) and R (ldr).
tsqr_status run_refined(const Plan &pl, const double *A, int64_t lda, double *Q, int64_t ldq,
                        double *R, int64_t ldr, void *ws, int32_t *d_info, hipStream_t st)
{
    const Level &top = pl.lev[pl.nlev - 1];
    double *Rhat = (double *)wsp(ws, pl.rhat);
    {
        ProfScope ps(PC_FINALIZE, st);
        TSQR_HIP_CHECK(launch_finalize(pl.n, (const double *)wsp(ws, top.s), Rhat, nullptr, pl.n,
                                       nullptr, 0, 0, 0, nullptr, nullptr, nullptr, nullptr, 0,
                                       nullptr, nullptr, d_info, st));
    }
    ProfScope ps(PC_REFINE, st);
    TSQR_HIP_CHECK(launch_refine(pl.m, pl.n, A, lda, Rhat, Q, ldq, R, ldr, wsp(ws, pl.refine),
                                 d_info, st));
    return TSQR_OK;
}

tsqr_status do_qr(int in_dtype, int64_t m, int64_t n, const void *A, int64_t lda, void *Q,
                  int64_t ldq, double *R, float *Rf, int64_t ldr, void *ws, size_t ws_bytes,
                  int32_t *d_info, const tsqr_opts *opts, void *stream)
{
    if (!A || !Q || (!R && !Rf) || !d_info) return TSQR_ERR_INVALID_ARG;
    if (lda < n || ldq < n || ldr < n) return TSQR_ERR_INVALID_ARG;
    tsqr_opts tmp;
    const tsqr_opts *o = opts_or_default(opts, tmp);
    Plan pl;
    tsqr_status s = build_plan(OP_QR, m, n, in_dtype, o, true, false, pl);
    if (s != TSQR_OK) return s;
    if (pl.reuse_output && ldq != n) return TSQR_ERR_INVALID_ARG;
    if ((s = check_ws(pl, ws, ws_bytes)) != TSQR_OK) return s;
    hipStream_t st = (hipStream_t)stream;
    if ((s = run_factor_levels(pl, A, lda, ws, st, Q)) != TSQR_OK) return s;
    const Level &top = pl.lev[pl.nlev - 1];
    if (pl.rhat)   // precision form with refinement
        return run_refined(pl, (const double *)A, lda, (double *)Q, ldq, R, ldr, ws, d_info, st);
    {
        ProfScope ps(PC_FINALIZE, st);
        TSQR_HIP_CHECK(launch_finalize(n, (const double *)wsp(ws, top.s), R, Rf, ldr,
                                       (double *)wsp(ws, pl.wtop), pl.k, 1, 0, nullptr, nullptr,
                                       nullptr, nullptr, 0, nullptr, nullptr, d_info, st));
    }
    return run_apply_levels(pl, ws, in_dtype, Q, ldq, (int)n, nullptr, 0, st, Q);
}

// Thin SVD (Sec. III-B, SVD paragraph): R = U_R S V^T at the top of the tree, U_R carried down
// so that U = Q1 Q2 U_R comes out of step 3 with Q.  The refined precision form refines Q and R
// first, then takes the SVD of the refined R and forms U = Q U_R with one more product.
tsqr_status do_svd(int in_dtype, int64_t m, int64_t n, const void *A, int64_t lda, void *U,
                   int64_t ldu, void *S, void *V, int64_t ldv, void *Q, int64_t ldq, void *R,
                   int64_t ldr, void *ws, size_t ws_bytes, int32_t *d_info, const tsqr_opts *opts,
                   void *stream)
{
    if (!A || !U || !S || !V || !d_info) return TSQR_ERR_INVALID_ARG;
    if (lda < n || ldu < n || ldv < n || (Q && ldq < n) || (R && ldr < n))
        return TSQR_ERR_INVALID_ARG;
    tsqr_opts tmp;
    const tsqr_opts *o = opts_or_default(opts, tmp);
    Plan pl;
    const bool want_q = Q != nullptr;
    tsqr_status s = build_plan(OP_SVD, m, n, in_dtype, o, want_q, true, pl);
    if (s != TSQR_OK) return s;
    // with reuse, level 0's panel factors sit in Q when it is wanted, else in U
    void *q1_out = want_q ? Q : U;
    if (pl.reuse_output && (want_q ? ldq : ldu) != n) return TSQR_ERR_INVALID_ARG;
    if ((s = check_ws(pl, ws, ws_bytes)) != TSQR_OK) return s;
    hipStream_t st = (hipStream_t)stream;
    const bool f32 = in_dtype == F32;
    if ((s = run_factor_levels(pl, A, lda, ws, st, q1_out)) != TSQR_OK) return s;
    if (pl.rhat) {
        // refined: Q (caller's or workspace) and R in FP64, then the SVD of R and U = Q U_R
        double *Qd = want_q ? (double *)Q : (double *)wsp(ws, pl.qtmp);
        const int64_t ldqd = want_q ? ldq : n;
        double *Rr = (double *)wsp(ws, pl.rref);
        if ((s = run_refined(pl, (const double *)A, lda, Qd, ldqd, Rr, n, ws, d_info, st)) != TSQR_OK)
            return s;
        {
            ProfScope ps(PC_FINALIZE, st);
            TSQR_HIP_CHECK(launch_finalize(n, Rr, (double *)R, nullptr, ldr,
                                           (double *)wsp(ws, pl.wtop), pl.k, 0, 1, (double *)S,
                                           nullptr, (double *)V, nullptr, ldv,
                                           (double *)wsp(ws, pl.svd_g), (double *)wsp(ws, pl.svd_v),
                                           d_info, st, 1));
        }
        ProfScope ps(PC_APPLY0, st);
        TSQR_HIP_CHECK(launch_gemm_mfma(F64, F64, m, n, 256, Qd, ldqd, (const double *)wsp(ws, pl.wtop),
                                        n, 0, (int)n, U, ldu, (int)n, nullptr, 0, 0, st));
        return TSQR_OK;
    }
    const Level &top = pl.lev[pl.nlev - 1];
    {
        ProfScope ps(PC_FINALIZE, st);
        TSQR_HIP_CHECK(launch_finalize(n, (const double *)wsp(ws, top.s),
                                       f32 ? nullptr : (double *)R, f32 ? (float *)R : nullptr, ldr,
                                       (double *)wsp(ws, pl.wtop), pl.k, want_q ? 1 : 0, 1,
                                       f32 ? nullptr : (double *)S, f32 ? (float *)S : nullptr,
                                       f32 ? nullptr : (double *)V, f32 ? (float *)V : nullptr, ldv,
                                       (double *)wsp(ws, pl.svd_g), (double *)wsp(ws, pl.svd_v),
                                       d_info, st));
    }
    if (want_q) return run_apply_levels(pl, ws, in_dtype, Q, ldq, (int)n, U, ldu, st, q1_out);
    return run_apply_levels(pl, ws, in_dtype, U, ldu, (int)n, nullptr, 0, st, q1_out);
}

// Comparison methods of the stability experiment (Sec. IV): workspace = the R-only plan of
// indirect TSQR, then R1, Rinv, R2 (n x n), the Gram G and its row-block partials, and Q1 (m x n)
// when refining.
struct IndirLayout {
    Plan pr;
    size_t r1 = 0, rinv = 0, r2 = 0, g = 0, part = 0, q1 = 0, total = 0;
};

tsqr_status build_indirect_layout(int method, int refine, int64_t m, int64_t n, const tsqr_opts *o,
                                  IndirLayout &L)
{
    if (method != TSQR_METHOD_CHOLQR && method != TSQR_METHOD_INDIRECT) return TSQR_ERR_INVALID_ARG;
    if (refine != 0 && refine != 1) return TSQR_ERR_INVALID_ARG;
    if (o && o->precision != TSQR_FP64) return TSQR_ERR_UNSUPPORTED;
    if (n > TSQR_NMAX_SMALL) return TSQR_ERR_SHAPE;     // Cholesky and inverse in LDS
    tsqr_status s = build_plan(OP_R, m, n, F64, o, false, false, L.pr);
    if (s != TSQR_OK) return s;
    size_t off = align_up(L.pr.total);
    auto take = [&](size_t bytes) {
        size_t at = off;
        off = align_up(off + (bytes ? bytes : 1));
        return at;
    };
    const size_t nn = sizeof(double) * (size_t)n * n;
    L.r1 = take(nn);
    L.rinv = take(nn);
    L.r2 = take(nn);
    L.g = take(nn);
    L.part = take(nn * (size_t)gram_blocks(m));
    if (refine) L.q1 = take(sizeof(double) * (size_t)m * n);
    L.total = off;
    return TSQR_OK;
}

// One QR by `method` of X (m x n, ldx): R (n x n, ld n) and Qout = X R^{-1} (ldq).
tsqr_status one_indirect_qr(int method, const IndirLayout &L, int64_t m, int64_t n, const double *X,
                            int64_t ldx, double *Qout, int64_t ldq, double *R, void *ws,
                            int32_t *d_info, int keep_info, hipStream_t st)
{
    double *Rinv = (double *)wsp(ws, L.rinv);
    if (method == TSQR_METHOD_CHOLQR) {
        ProfScope ps(PC_BWD_GRAM, st);
        TSQR_HIP_CHECK(launch_gram(m, n, X, ldx, X, ldx, (double *)wsp(ws, L.part),
                                   (double *)wsp(ws, L.g), st));
        TSQR_HIP_CHECK(launch_cholqr_small(n, (const double *)wsp(ws, L.g), R, Rinv, d_info,
                                           keep_info, st));
    } else {
        tsqr_status s = run_factor_levels(L.pr, X, ldx, ws, st);
        if (s != TSQR_OK) return s;
        ProfScope ps(PC_FINALIZE, st);
        TSQR_HIP_CHECK(launch_finalize(n, (const double *)wsp(ws, L.pr.lev[L.pr.nlev - 1].s), R,
                                       nullptr, n, nullptr, 0, 0, 0, nullptr, nullptr, nullptr,
                                       nullptr, 0, nullptr, nullptr, d_info, st, keep_info));
        TSQR_HIP_CHECK(launch_rinv_small(n, R, Rinv, st));
    }
    ProfScope ps(PC_BWD_GEMM, st);
    TSQR_HIP_CHECK(launch_gemm_mfma(F64, F64, m, n, 256, X, ldx, Rinv, n, 0, (int)n, Qout, ldq,
                                    (int)n, nullptr, 0, 0, st));
    return TSQR_OK;
}

// Backward workspace: the forward plan's workspace, then the recomputed factor and the adjoint
// scratch.
struct BwdLayout {
    Plan fwd;
    size_t q = 0, r = 0, s = 0, v = 0, part = 0, g = 0, w2 = 0, scratch = 0, total = 0;
    int nblk = 0;
};

tsqr_status build_bwd_layout(bool svd, int64_t m, int64_t n, const tsqr_opts *o, BwdLayout &bl)
{
    if (o && o->precision != TSQR_FP64) return TSQR_ERR_UNSUPPORTED;
    if (n > TSQR_NMAX_SMALL) return TSQR_ERR_SHAPE;     // the n x n adjoint work in LDS
    tsqr_opts fo;                                       // the recomputed forward keeps its Q1
    if (o) {
        fo = *o;
        fo.flags &= ~TSQR_FLAG_REUSE_OUTPUT;
        o = &fo;
    }
    tsqr_status s = svd ? build_plan(OP_SVD, m, n, F64, o, false, true, bl.fwd)
                        : build_plan(OP_QR, m, n, F64, o, true, false, bl.fwd);
    if (s != TSQR_OK) return s;
    size_t off = align_up(bl.fwd.total);
    auto take = [&](size_t bytes) {
        size_t at = off;
        off = align_up(off + (bytes ? bytes : 1));
        return at;
    };
    bl.q = take(sizeof(double) * (size_t)m * n);
    bl.r = take(sizeof(double) * (size_t)n * n);
    bl.s = take(sizeof(double) * (size_t)n);
    bl.v = take(sizeof(double) * (size_t)n * n);
    bl.nblk = gram_blocks(m);
    bl.part = take(sizeof(double) * (size_t)bl.nblk * n * n);
    bl.g = take(sizeof(double) * (size_t)n * n);
    bl.w2 = take(sizeof(double) * 2 * (size_t)n * n);
    bl.scratch = take(sizeof(double) * 2 * (size_t)n * n);
    bl.total = off;
    return TSQR_OK;
}

constexpr int kBwdPanel = 256;   // rows per work-group of the backward's tall products

// Workspace of tsqr_r_noalloc: a fixed device array (each GPU that runs the library holds its
// own copy until the process ends).  Host code never uses the array's name as an address: the
// device address is taken once per device with hipGetSymbolAddress, with that device current.
constexpr size_t kNoallocScratchBytes = (size_t)TSQR_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];
constexpr int kMaxDevices = 64;
std::once_flag g_scratch_once[kMaxDevices];
void *g_scratch_ptr[kMaxDevices];
hipError_t g_scratch_err[kMaxDevices];

// The current device's scratch address (set up on the first call on that device).
void *device_scratch(hipError_t &err)
{
    int dev = 0;
    err = hipGetDevice(&dev);
    if (err != hipSuccess) return nullptr;
    if (dev < 0 || dev >= kMaxDevices) {
        err = hipErrorInvalidDevice;
        return nullptr;
    }
    std::call_once(g_scratch_once[dev], [dev] {
        void *p = nullptr;
        g_scratch_err[dev] = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        g_scratch_ptr[dev] = (g_scratch_err[dev] == hipSuccess) ? p : nullptr;
    });
    err = g_scratch_err[dev];
    return g_scratch_ptr[dev];
}

}  // namespace

ProfScope::ProfScope(int c, hipStream_t s) : cls(c), st(s)
{
    if (!g_prof.on || !((g_prof.mask >> c) & 1u)) return;
    std::lock_guard<std::mutex> lk(g_prof.mu);
    a = prof_event();
    if (a) (void)hipEventRecord(a, st);
}

ProfScope::~ProfScope()
{
    if (!a) return;
    std::lock_guard<std::mutex> lk(g_prof.mu);
    hipEvent_t b = prof_event();
    if (!b) return;
    (void)hipEventRecord(b, st);
    g_prof.recs.push_back({cls, a, b});
}

namespace {
}  // namespace
}  // namespace tsqr

using namespace tsqr;

// Row-chunked QR: one more level of the Sec. III-C recursion above per-chunk direct TSQR.  Chunk
// c (rows [c h, c h + h), a short last chunk merged into the one before) is factored by tsqr_qr
// with its level-0 factors kept in its rows of Q, A_c = Q_c R_c; the stacked R_c are factored,
// [R_1; ...; R_C] = [Q2_1; ...; Q2_C] R; then Q_c <- Q_c Q2_c in place (each row block of Q_c is
// read before it is written).  Workspace: the stack and Q2 (C n x n each) and the larger of one
// chunk's and the stack's tsqr_qr workspace, reused by every call in turn.
namespace {

struct ChunkLayout {
    int64_t nchunk = 0, h = 0, last = 0;     // chunks, rows per chunk, rows of the last chunk
    size_t s = 0, q2 = 0, info = 0, inner = 0, inner_bytes = 0, total = 0;
};

tsqr_opts chunk_inner_opts(const tsqr_opts *o)
{
    tsqr_opts r;
    tsqr_default_opts(&r);
    if (o) r = *o;
    r.flags |= TSQR_FLAG_REUSE_OUTPUT;
    return r;
}

tsqr_status chunk_layout(int64_t m, int64_t n, int64_t chunk_rows, const tsqr_opts *o,
                         ChunkLayout &L)
{
    if (m <= 0 || n <= 0 || chunk_rows <= 0) return TSQR_ERR_INVALID_ARG;
    if (m < n || n > TSQR_NMAX) return TSQR_ERR_SHAPE;
    tsqr_status vs = validate_opts(o, n);
    if (vs != TSQR_OK) return vs;
    if (o && (o->precision != TSQR_FP64 || o->flags != 0)) return TSQR_ERR_UNSUPPORTED;
    L.h = chunk_rows < n ? n : chunk_rows;
    L.nchunk = ceil_div(m, L.h);
    L.last = m - (L.nchunk - 1) * L.h;
    if (L.nchunk > 1 && L.last < n) {        // a last chunk shorter than n joins the one before
        --L.nchunk;
        L.last += L.h;
    }
    const tsqr_opts io = chunk_inner_opts(o);
    size_t inner = 0;
    for (const int64_t rows : {L.h < m ? L.h : m, L.last}) {
        Plan pc;
        tsqr_status st = build_plan(OP_QR, rows, n, F64, &io, true, false, pc);
        if (st != TSQR_OK) return st;
        inner = std::max(inner, pc.total);
    }
    Plan top;
    tsqr_status st = build_plan(OP_QR, L.nchunk * n, n, F64, o, true, false, top);
    if (st != TSQR_OK) return st;
    inner = std::max(inner, top.total);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t at = off;
        off = align_up(off + (bytes ? bytes : 1));
        return at;
    };
    L.s = take(sizeof(double) * (size_t)L.nchunk * n * n);
    L.q2 = take(sizeof(double) * (size_t)L.nchunk * n * n);
    L.info = take(sizeof(int32_t));
    L.inner = take(inner);
    L.inner_bytes = inner;
    L.total = off;
    return TSQR_OK;
}

}  // namespace

extern "C" {

void tsqr_default_opts(tsqr_opts *opts)
{
    if (!opts) return;
    memset(opts, 0, sizeof(*opts));
    opts->struct_size = (int32_t)sizeof(tsqr_opts);
    opts->precision = TSQR_FP64;
}

tsqr_status tsqr_workspace_bytes(int32_t op, int64_t m, int64_t n, const tsqr_opts *opts,
                                 size_t *bytes)
{
    if (!bytes) return TSQR_ERR_INVALID_ARG;
    tsqr_opts tmp;
    const tsqr_opts *o = opts_or_default(opts, tmp);
    Plan pl;
    tsqr_status s;
    // input element type: FP64, except that the reuse flag under TSQR_FP32 implies FP32 input
    // (the only input whose level-0 factors have the output's element size)
    const int in_dt = (o->precision == TSQR_FP32 && (o->flags & TSQR_FLAG_REUSE_OUTPUT)) ? F32 : F64;
    switch (op) {
    case TSQR_OP_R: s = build_plan(OP_R, m, n, in_dt, o, false, false, pl); break;
    case TSQR_OP_QR: s = build_plan(OP_QR, m, n, in_dt, o, true, false, pl); break;
    case TSQR_OP_SVD: {
        // the larger of the layouts with and without a Q output (with the reuse flag, of those
        // it supports)
        Plan p2;
        s = build_plan(OP_SVD, m, n, in_dt, o, true, true, pl);
        const tsqr_status s2 = build_plan(OP_SVD, m, n, in_dt, o, false, true, p2);
        if (s != TSQR_OK && s2 == TSQR_OK && (o->flags & TSQR_FLAG_REUSE_OUTPUT)) {
            s = s2;
            pl.total = p2.total;
        } else if (s == TSQR_OK && s2 == TSQR_OK && p2.total > pl.total) {
            pl.total = p2.total;
        }
        break;
    }
    case TSQR_OP_QR_BACKWARD:
    case TSQR_OP_SVD_BACKWARD: {
        BwdLayout bl;
        s = build_bwd_layout(op == TSQR_OP_SVD_BACKWARD, m, n, o, bl);
        if (s != TSQR_OK) return s;
        *bytes = bl.total;
        return TSQR_OK;
    }
    default: return TSQR_ERR_INVALID_ARG;
    }
    if (s != TSQR_OK) return s;
    *bytes = pl.total;
    return TSQR_OK;
}

tsqr_status tsqr_r(int64_t m, int64_t n, const double *A, int64_t lda, double *R, int64_t ldr,
                   void *ws, size_t ws_bytes, int32_t *d_info, const tsqr_opts *opts, void *stream)
{
    return do_r(F64, m, n, A, lda, R, nullptr, ldr, ws, ws_bytes, d_info, opts, stream);
}

tsqr_status tsqr_r_noalloc(int64_t m, int64_t n, const double *A, int64_t lda, double *R,
                           int64_t ldr, int32_t *d_info, const tsqr_opts *opts, void *stream)
{
    if (!A || !R || !d_info) return TSQR_ERR_INVALID_ARG;
    if (lda < n || ldr < n) return TSQR_ERR_INVALID_ARG;
    tsqr_opts tmp;
    Plan pl;
    tsqr_status s = build_plan(OP_R, m, n, F64, opts_or_default(opts, tmp), false, false, pl);
    if (s != TSQR_OK) return s;
    if (pl.total > kNoallocScratchBytes) return TSQR_ERR_WORKSPACE;
    hipError_t e = hipSuccess;
    void *ws = device_scratch(e);
    if (e != hipSuccess) {
        set_last_error(e, "hipGetSymbolAddress(scratch)", __LINE__);
        return TSQR_ERR_HIP;
    }
    return do_r(F64, m, n, A, lda, R, nullptr, ldr, ws, kNoallocScratchBytes, d_info, opts, stream);
}

tsqr_status tsqr_r_f32(int64_t m, int64_t n, const float *A, int64_t lda, float *R, int64_t ldr,
                       void *ws, size_t ws_bytes, int32_t *d_info, const tsqr_opts *opts,
                       void *stream)
{
    return do_r(F32, m, n, A, lda, nullptr, R, ldr, ws, ws_bytes, d_info, opts, stream);
}

tsqr_status tsqr_qr(int64_t m, int64_t n, const double *A, int64_t lda, double *Q, int64_t ldq,
                    double *R, int64_t ldr, void *ws, size_t ws_bytes, int32_t *d_info,
                    const tsqr_opts *opts, void *stream)
{
    return do_qr(F64, m, n, A, lda, Q, ldq, R, nullptr, ldr, ws, ws_bytes, d_info, opts, stream);
}


tsqr_status tsqr_qr_chunked_workspace_bytes(int64_t m, int64_t n, int64_t chunk_rows,
                                            const tsqr_opts *opts, size_t *bytes)
{
    if (!bytes) return TSQR_ERR_INVALID_ARG;
    ChunkLayout L;
    tsqr_status s = chunk_layout(m, n, chunk_rows, opts, L);
    if (s != TSQR_OK) return s;
    *bytes = L.total;
    return TSQR_OK;
}

tsqr_status tsqr_qr_chunked(int64_t m, int64_t n, int64_t chunk_rows, const double *A,
                            int64_t lda, double *Q, int64_t ldq, double *R, int64_t ldr,
                            void *ws, size_t ws_bytes, int32_t *d_info, const tsqr_opts *opts,
                            void *stream)
{
    if (!A || !Q || !R || !d_info) return TSQR_ERR_INVALID_ARG;
    if (lda < n || ldq != n || ldr < n) return TSQR_ERR_INVALID_ARG;
    ChunkLayout L;
    tsqr_status s = chunk_layout(m, n, chunk_rows, opts, L);
    if (s != TSQR_OK) return s;
    if (!ws || ws_bytes < L.total) return TSQR_ERR_WORKSPACE;
    hipStream_t st = (hipStream_t)stream;
    char *base = (char *)ws;
    double *S = (double *)(base + L.s), *Q2 = (double *)(base + L.q2);
    int32_t *cinfo = (int32_t *)(base + L.info);
    void *inner = base + L.inner;
    const tsqr_opts io = chunk_inner_opts(opts);
    // a chunk's own rank deficiency is no condition of A (its QR is still exact), so the chunks
    // report into a scratch flag and only the factorization of the stack writes d_info
    for (int64_t c = 0; c < L.nchunk; ++c) {
        const int64_t r0 = c * L.h, rows = (c + 1 < L.nchunk) ? L.h : L.last;
        s = do_qr(F64, rows, n, A + r0 * lda, lda, Q + r0 * ldq, ldq, S + c * n * n, nullptr, n,
                  inner, L.inner_bytes, cinfo, &io, stream);
        if (s != TSQR_OK) return s;
    }
    s = do_qr(F64, L.nchunk * n, n, S, n, Q2, n, R, nullptr, ldr, inner, L.inner_bytes, d_info,
              opts, stream);
    if (s != TSQR_OK) return s;
    ProfScope ps(PC_APPLY0, st);
    for (int64_t c = 0; c < L.nchunk; ++c) {
        const int64_t r0 = c * L.h, rows = (c + 1 < L.nchunk) ? L.h : L.last;
        double *Qc = Q + r0 * ldq;
        TSQR_HIP_CHECK(launch_gemm_mfma(F64, F64, rows, n, 256, Qc, ldq, Q2 + c * n * n, n, 0,
                                        (int)n, Qc, ldq, (int)n, nullptr, 0, 0, st, 1));
    }
    return TSQR_OK;
}

tsqr_status tsqr_qr_f32(int64_t m, int64_t n, const float *A, int64_t lda, float *Q, int64_t ldq,
                        float *R, int64_t ldr, void *ws, size_t ws_bytes, int32_t *d_info,
                        const tsqr_opts *opts, void *stream)
{
    return do_qr(F32, m, n, A, lda, Q, ldq, nullptr, R, ldr, ws, ws_bytes, d_info, opts, stream);
}

tsqr_status tsqr_svd(int64_t m, int64_t n, const double *A, int64_t lda, double *U, int64_t ldu,
                     double *S, double *V, int64_t ldv, double *Q, int64_t ldq, double *R,
                     int64_t ldr, void *ws, size_t ws_bytes, int32_t *d_info,
                     const tsqr_opts *opts, void *stream)
{
    return do_svd(F64, m, n, A, lda, U, ldu, S, V, ldv, Q, ldq, R, ldr, ws, ws_bytes, d_info, opts,
                  stream);
}

tsqr_status tsqr_svd_f32(int64_t m, int64_t n, const float *A, int64_t lda, float *U, int64_t ldu,
                         float *S, float *V, int64_t ldv, float *Q, int64_t ldq, float *R,
                         int64_t ldr, void *ws, size_t ws_bytes, int32_t *d_info,
                         const tsqr_opts *opts, void *stream)
{
    return do_svd(F32, m, n, A, lda, U, ldu, S, V, ldv, Q, ldq, R, ldr, ws, ws_bytes, d_info, opts,
                  stream);
}

tsqr_status tsqr_indirect_workspace_bytes(int32_t method, int32_t refine, int64_t m, int64_t n,
                                          const tsqr_opts *opts, size_t *bytes)
{
    if (!bytes) return TSQR_ERR_INVALID_ARG;
    tsqr_opts tmp;
    IndirLayout L;
    tsqr_status s = build_indirect_layout(method, refine, m, n, opts_or_default(opts, tmp), L);
    if (s != TSQR_OK) return s;
    *bytes = L.total;
    return TSQR_OK;
}

tsqr_status tsqr_qr_indirect(int32_t method, int32_t refine, int64_t m, int64_t n, const double *A,
                             int64_t lda, double *Q, int64_t ldq, double *R, int64_t ldr, void *ws,
                             size_t ws_bytes, int32_t *d_info, const tsqr_opts *opts, void *stream)
{
    if (!A || !Q || !R || !d_info) return TSQR_ERR_INVALID_ARG;
    if (lda < n || ldq < n || ldr < n) return TSQR_ERR_INVALID_ARG;
    tsqr_opts tmp;
    IndirLayout L;
    tsqr_status s = build_indirect_layout(method, refine, m, n, opts_or_default(opts, tmp), L);
    if (s != TSQR_OK) return s;
    if (!ws || ws_bytes < L.total) return TSQR_ERR_WORKSPACE;
    hipStream_t st = (hipStream_t)stream;
    double *R1 = (double *)wsp(ws, L.r1), *R2 = (double *)wsp(ws, L.r2);
    if (!refine) {
        if ((s = one_indirect_qr(method, L, m, n, A, lda, Q, ldq, R1, ws, d_info, 0, st)) != TSQR_OK)
            return s;
        TSQR_HIP_CHECK(launch_trmul_small(n, nullptr, R1, R, ldr, st));
        return TSQR_OK;
    }
    // iterative refinement (Sec. I): Q1 R1 = A, Q R2 = Q1, R = R2 R1
    double *Q1 = (double *)wsp(ws, L.q1);
    if ((s = one_indirect_qr(method, L, m, n, A, lda, Q1, n, R1, ws, d_info, 0, st)) != TSQR_OK)
        return s;
    if ((s = one_indirect_qr(method, L, m, n, Q1, n, Q, ldq, R2, ws, d_info, 1, st)) != TSQR_OK)
        return s;
    TSQR_HIP_CHECK(launch_trmul_small(n, R2, R1, R, ldr, st));
    return TSQR_OK;
}

tsqr_status tsqr_plan_levels(int32_t op, int64_t m, int64_t n, const tsqr_opts *opts,
                             int32_t max_levels, int32_t *nlevels, int64_t *rows,
                             int32_t *panel_rows)
{
    if (!nlevels || max_levels < 0 || (max_levels > 0 && (!rows || !panel_rows)))
        return TSQR_ERR_INVALID_ARG;
    tsqr_opts tmp;
    const tsqr_opts *o = opts_or_default(opts, tmp);
    Plan pl;
    tsqr_status s;
    switch (op) {
    case TSQR_OP_R: s = build_plan(OP_R, m, n, F64, o, false, false, pl); break;
    case TSQR_OP_QR: s = build_plan(OP_QR, m, n, F64, o, true, false, pl); break;
    case TSQR_OP_SVD: s = build_plan(OP_SVD, m, n, F64, o, true, true, pl); break;
    default: return TSQR_ERR_INVALID_ARG;
    }
    if (s != TSQR_OK) return s;
    *nlevels = pl.nlev;
    for (int L = 0; L < pl.nlev && L < max_levels; ++L) {
        rows[L] = pl.lev[L].rows;
        panel_rows[L] = pl.lev[L].b;
    }
    return TSQR_OK;
}

tsqr_status tsqr_qr_backward(int64_t m, int64_t n, const double *A, int64_t lda,
                             const double *dQ, int64_t lddq, const double *dR, int64_t lddr,
                             double *dA, int64_t ldda, void *ws, size_t ws_bytes,
                             int32_t *d_info, const tsqr_opts *opts, void *stream)
{
    if (!A || !dA || !d_info) return TSQR_ERR_INVALID_ARG;
    if (lda < n || ldda < n || (dQ && lddq < n) || (dR && lddr < n)) return TSQR_ERR_INVALID_ARG;
    tsqr_opts tmp;
    const tsqr_opts *o = opts_or_default(opts, tmp);
    BwdLayout bl;
    tsqr_status s = build_bwd_layout(false, m, n, o, bl);
    if (s != TSQR_OK) return s;
    if (!ws || ws_bytes < bl.total) return TSQR_ERR_WORKSPACE;
    hipStream_t st = (hipStream_t)stream;
    double *Q = (double *)wsp(ws, bl.q), *R = (double *)wsp(ws, bl.r);
    double *W2 = (double *)wsp(ws, bl.w2);
    // recompute Q and R from A (the forward kernels; Q1_i is never kept across calls)
    if ((s = run_factor_levels(bl.fwd, A, lda, ws, st)) != TSQR_OK) return s;
    {
        ProfScope ps(PC_FINALIZE, st);
        TSQR_HIP_CHECK(launch_finalize(n, (const double *)wsp(ws, bl.fwd.lev[bl.fwd.nlev - 1].s), R,
                                       nullptr, n, (double *)wsp(ws, bl.fwd.wtop), bl.fwd.k, 1, 0,
                                       nullptr, nullptr, nullptr, nullptr, 0, nullptr, nullptr,
                                       d_info, st));
    }
    if ((s = run_apply_levels(bl.fwd, ws, F64, Q, n, (int)n, nullptr, 0, st)) != TSQR_OK) return s;
    if (dQ) {
        ProfScope ps(PC_BWD_GRAM, st);
        TSQR_HIP_CHECK(launch_gram(m, n, dQ, lddq, Q, n, (double *)wsp(ws, bl.part),
                                   (double *)wsp(ws, bl.g), st));
    }
    {
        ProfScope ps(PC_BWD_SMALL, st);
        TSQR_HIP_CHECK(launch_qr_bwd_small(n, R, dR, lddr, dQ ? (double *)wsp(ws, bl.g) : nullptr,
                                           W2, (double *)wsp(ws, bl.scratch), d_info, st));
    }
    ProfScope ps(PC_BWD_GEMM, st);
    TSQR_HIP_CHECK(launch_gemm_mfma(F64, F64, m, n, kBwdPanel, Q, n, W2 + n * n, n, 0, (int)n, dA,
                                    ldda, (int)n, nullptr, 0, 0, st));
    if (dQ)
        TSQR_HIP_CHECK(launch_gemm_mfma(F64, F64, m, n, kBwdPanel, dQ, lddq, W2, n, 0, (int)n, dA,
                                        ldda, (int)n, nullptr, 0, 1, st));
    return TSQR_OK;
}

tsqr_status tsqr_svd_backward(int64_t m, int64_t n, const double *A, int64_t lda,
                              const double *dU, int64_t lddu, const double *dS,
                              const double *dV, int64_t lddv, double *dA, int64_t ldda,
                              void *ws, size_t ws_bytes, int32_t *d_info,
                              const tsqr_opts *opts, void *stream)
{
    if (!A || !dA || !d_info) return TSQR_ERR_INVALID_ARG;
    if (lda < n || ldda < n || (dU && lddu < n) || (dV && lddv < n)) return TSQR_ERR_INVALID_ARG;
    tsqr_opts tmp;
    const tsqr_opts *o = opts_or_default(opts, tmp);
    BwdLayout bl;
    tsqr_status s = build_bwd_layout(true, m, n, o, bl);
    if (s != TSQR_OK) return s;
    if (!ws || ws_bytes < bl.total) return TSQR_ERR_WORKSPACE;
    hipStream_t st = (hipStream_t)stream;
    double *U = (double *)wsp(ws, bl.q), *S = (double *)wsp(ws, bl.s), *V = (double *)wsp(ws, bl.v);
    double *W2 = (double *)wsp(ws, bl.w2);
    if ((s = run_factor_levels(bl.fwd, A, lda, ws, st)) != TSQR_OK) return s;
    {
        ProfScope ps(PC_FINALIZE, st);
        TSQR_HIP_CHECK(launch_finalize(n, (const double *)wsp(ws, bl.fwd.lev[bl.fwd.nlev - 1].s),
                                       nullptr, nullptr, 0, (double *)wsp(ws, bl.fwd.wtop),
                                       bl.fwd.k, 0, 1, S, nullptr, V, nullptr, n,
                                       (double *)wsp(ws, bl.fwd.svd_g),
                                       (double *)wsp(ws, bl.fwd.svd_v), d_info, st));
    }
    if ((s = run_apply_levels(bl.fwd, ws, F64, U, n, (int)n, nullptr, 0, st)) != TSQR_OK) return s;
    if (dU) {
        ProfScope ps(PC_BWD_GRAM, st);
        TSQR_HIP_CHECK(launch_gram(m, n, U, n, dU, lddu, (double *)wsp(ws, bl.part),
                                   (double *)wsp(ws, bl.g), st));
    }
    {
        ProfScope ps(PC_BWD_SMALL, st);
        TSQR_HIP_CHECK(launch_svd_bwd_small(n, S, V, dS, dV, lddv,
                                            dU ? (double *)wsp(ws, bl.g) : nullptr, W2,
                                            (double *)wsp(ws, bl.scratch), d_info, st));
    }
    ProfScope ps(PC_BWD_GEMM, st);
    TSQR_HIP_CHECK(launch_gemm_mfma(F64, F64, m, n, kBwdPanel, U, n, W2, n, 0, (int)n, dA, ldda,
                                    (int)n, nullptr, 0, 0, st));
    if (dU)
        TSQR_HIP_CHECK(launch_gemm_mfma(F64, F64, m, n, kBwdPanel, dU, lddu, W2 + n * n, n, 0,
                                        (int)n, dA, ldda, (int)n, nullptr, 0, 1, st));
    return TSQR_OK;
}

const char *tsqr_status_string(tsqr_status status)
{
    switch (status) {
    case TSQR_OK: return "TSQR_OK";
    case TSQR_ERR_INVALID_ARG: return "TSQR_ERR_INVALID_ARG";
    case TSQR_ERR_SHAPE: return "TSQR_ERR_SHAPE";
    case TSQR_ERR_WORKSPACE: return "TSQR_ERR_WORKSPACE";
    case TSQR_ERR_UNSUPPORTED: return "TSQR_ERR_UNSUPPORTED";
    case TSQR_ERR_HIP: return "TSQR_ERR_HIP";
    }
    return "TSQR_ERR_UNKNOWN";
}

int32_t tsqr_abi_version(void) { return TSQR_ABI_VERSION; }

const char *tsqr_last_error(void) { return g_last_error; }

tsqr_status tsqr_profile_enable(int32_t on)
{
    std::lock_guard<std::mutex> lk(g_prof.mu);
    g_prof.on = on != 0;
    return TSQR_OK;
}

tsqr_status tsqr_profile_set_mask(uint32_t mask)
{
    std::lock_guard<std::mutex> lk(g_prof.mu);
    g_prof.mask = mask;
    return TSQR_OK;
}

int32_t tsqr_profile_num_classes(void) { return PC_COUNT; }

const char *tsqr_profile_class_name(int32_t c)
{
    return (c >= 0 && c < PC_COUNT) ? kProfNames[c] : "";
}

tsqr_status tsqr_profile_collect(double *ms, int64_t *launches, int32_t nclasses)
{
    if (!ms || !launches || nclasses < 0) return TSQR_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(g_prof.mu);
    for (int c = 0; c < nclasses; ++c) { ms[c] = 0.0; launches[c] = 0; }
    tsqr_status st = TSQR_OK;
    for (const ProfRec &r : g_prof.recs) {
        if (hipEventSynchronize(r.b) != hipSuccess) { st = TSQR_ERR_HIP; continue; }
        float t = 0.f;
        if (hipEventElapsedTime(&t, r.a, r.b) != hipSuccess) { st = TSQR_ERR_HIP; continue; }
        if (r.cls < nclasses) { ms[r.cls] += t; launches[r.cls] += 1; }
    }
    g_prof.recs.clear();
    g_prof.next = 0;
    return st;
}

}  // extern "C"
