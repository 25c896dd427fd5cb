// Batched form: many independent direct-TSQR factorizations (Sec. III-B/III-C per matrix) in one
// fixed launch sequence that a HIP graph can capture.
//
// A plan (built once on the host) gives every matrix its own recursive tree of register panels
// and lays all trees out in one workspace.  Matrices with the same n share launches: one launch
// per (n, tree level) factors the level-L panels of every matrix of that width, one launch
// finalizes every matrix, and one launch per (n, level) applies the down-sweep.  A work-group
// finds its (matrix, panel) from a task table in device memory (binary search on the first
// block of each task), so the kernels themselves are the single-matrix bodies.  The sequence has
// no host synchronisation, allocation or memset: capturing one call in a graph gives one graph
// launch for the whole batch.
#include <algorithm>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <vector>

#include "apply_mfma_body.h"
#include "panel_blk_body.h"

namespace tsqr {
namespace {

constexpr int kBatchNmax = 64;

// One (matrix, tree level) of the factor sweep: panels [first_block, first_block + panels).
struct FactorTask {
    int64_t first_block;
    int64_t rows;        // rows of the matrix factored at this level
    int64_t ldx;
    int64_t x_off;       // workspace byte offset of the input (stacked R), -1: the caller's A
    int64_t q1_off;      // explicit Q1 panels (rows x n)
    int64_t s_off;       // stacked R output (panels*n x n, FP64)
    int32_t mat, n;
};

// One (matrix, level) of the down-sweep: out_p = Q1_p W_p.
struct ApplyTask {
    int64_t first_block;
    int64_t rows;
    int64_t q1_off;
    int64_t w_off;       // W of the level above (W_top at the top), FP64, n columns
    int64_t wstride;     // rows of W per panel (n), 0 at the top of the tree
    int64_t out_off;     // workspace X of this level, -1: the caller's Q
    int64_t ld_out;
    int32_t mat, n, b;
};

// Finalize of one matrix: R = D R~, W_top = D, info.
struct FinalTask {
    int64_t s_off, wtop_off, ldr;
    int32_t mat, n;
};

template <typename Task>
__device__ __forceinline__ int find_task(const Task *__restrict__ t, int nt, int64_t blk)
{
    int lo = 0, hi = nt - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (t[mid].first_block <= blk) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Panels of the batched form: the blocked kernel, variant V of the width class NCT
// (V = 0 default height, 1 = half the row tiles per wave, 2 = 512 rows for n <= 16)
template <int NCT, int V> struct BlkShapeB {
    static constexpr int NW = 4;
    static constexpr int RT0 = (NCT <= 2) ? 6 : 4;
    static constexpr int RT = (V == 1) ? RT0 / 2 : ((V == 2 && NCT == 1) ? 8 : RT0);
    static constexpr int TC = NCT;
    static constexpr int B = NW * RT * 16;
    template <typename T> static constexpr size_t lds()
    {
        return sizeof(blkpanel::BlkSmem<T, NCT, RT, NW, TC>);
    }
};

template <typename T, int NCT, int V>
__global__ void __launch_bounds__(256, 2)
k_factor_blk_batched(const FactorTask *__restrict__ tasks, int ntasks, const void *const *A,
                     char *__restrict__ ws)
{
    using C = BlkShapeB<NCT, V>;
    const int64_t blk = blockIdx.x;
    const FactorTask t = tasks[find_task(tasks, ntasks, blk)];
    const T *X = t.x_off < 0 ? (const T *)A[t.mat] : (const T *)(ws + t.x_off);
    blkpanel::factor_blk_panel<T, T, NCT, C::RT, C::NW, C::TC>(t.rows, t.n, X, t.ldx,
                                                               (T *)(ws + t.q1_off),
                                                               (double *)(ws + t.s_off),
                                                               blk - t.first_block);
}

template <typename T, typename To, int NT>
__global__ void __launch_bounds__(mfmaapply::kWaves * 64)
k_apply_batched(const ApplyTask *__restrict__ tasks, int ntasks, void *const *Q,
                char *__restrict__ ws)
{
    const int64_t blk = blockIdx.x;
    const ApplyTask t = tasks[find_task(tasks, ntasks, blk)];
    To *out = t.out_off < 0 ? (To *)Q[t.mat] : (To *)(ws + t.out_off);
    mfmaapply::apply_mfma_panel<T, To, NT>(t.rows, t.n, t.b, (const T *)(ws + t.q1_off), t.n,
                                           (const double *)(ws + t.w_off), t.n, t.wstride, t.n,
                                           out, t.ld_out, t.n, (To *)nullptr, 0, 0,
                                           blk - t.first_block, 0);
}

// Sign fix of every matrix's top R (Sec. III-B with diag(R) > 0), W_top = D, and info.
template <typename To>
__global__ void __launch_bounds__(256)
k_finalize_batched(const FinalTask *__restrict__ tasks, void *const *Rout, char *__restrict__ ws,
                   int32_t *__restrict__ info)
{
    __shared__ double d_s[kBatchNmax];
    __shared__ int s_zero, s_nonfinite;
    const FinalTask t = tasks[blockIdx.x];
    const int n = t.n, tid = threadIdx.x;
    const double *Rt = (const double *)(ws + t.s_off);
    double *Wtop = (double *)(ws + t.wtop_off);
    To *R = (To *)Rout[t.mat];
    if (tid == 0) { s_zero = 0x7fffffff; s_nonfinite = 0; }
    __syncthreads();
    for (int i = tid; i < n; i += blockDim.x) {
        const double rii = Rt[(int64_t)i * n + i];
        d_s[i] = (rii >= 0.0) ? 1.0 : -1.0;
        if (rii == 0.0) atomicMin(&s_zero, i);
    }
    __syncthreads();
    for (int e = tid; e < n * n; e += blockDim.x) {
        const int r = e / n, c = e - r * n;
        const double v = Rt[e];
        if (c >= r && !isfinite(v)) s_nonfinite = 1;
        R[(int64_t)r * t.ldr + c] = (To)(c >= r ? d_s[r] * v : 0.0);
        Wtop[e] = (r == c) ? d_s[r] : 0.0;
    }
    __syncthreads();
    if (tid == 0) info[t.mat] = s_nonfinite ? -1 : (s_zero == 0x7fffffff ? 0 : s_zero + 1);
}

// ---- autotuned panel heights -----------------------------------------------------------------
// Variant (0, 1, 2) of the register panel per (dtype, width class); set by tsqr_tune_set.
constexpr int kClasses = 5;   // n <= 4, 8, 16, 32, 64
std::mutex g_tune_mu;
int g_tune[2][kClasses] = {{0, 0, 0, 0, 0}, {0, 0, 0, 0, 0}};

int width_class(int64_t n)
{
    return n <= 4 ? 0 : n <= 8 ? 1 : n <= 16 ? 2 : n <= 32 ? 3 : 4;
}

// Panel height of variant v for width n (the same for FP64 and FP32 panels).
template <int V> int blk_rows_b(int64_t n)
{
    switch ((n + 15) / 16) {
    case 1: return BlkShapeB<1, V>::B;
    case 2: return BlkShapeB<2, V>::B;
    case 3: return BlkShapeB<3, V>::B;
    default: return BlkShapeB<4, V>::B;
    }
}

int batch_panel_rows(int64_t n, int dtype, int v)
{
    (void)dtype;
    return v == 1 ? blk_rows_b<1>(n) : (v == 2 ? blk_rows_b<2>(n) : blk_rows_b<0>(n));
}

// A variant is usable for width n if its panels shrink every tree level (b >= 3n) and it
// differs from the default height (variant 2 only exists for n <= 16 in FP64).
bool variant_ok(int64_t n, int dtype, int v)
{
    if (v < 0 || v > 2) return false;
    if (v > 0 && batch_panel_rows(n, dtype, v) == batch_panel_rows(n, dtype, 0)) return false;
    return batch_panel_rows(n, dtype, v) >= 3 * n;
}


// ---- launch dispatch on the width class and variant ----------------------------------------
template <typename T, int NCT, int V>
hipError_t factor_blk_batched_cv(const FactorTask *tasks, int nt, int64_t blocks,
                                 const void *const *A, char *ws, hipStream_t st)
{
    using C = BlkShapeB<NCT, V>;
    hipLaunchKernelGGL((k_factor_blk_batched<T, NCT, V>), dim3((unsigned)blocks),
                       dim3(C::NW * 64), C::template lds<T>(), st, tasks, nt, A, ws);
    return hipGetLastError();
}

template <typename T, int NCT>
hipError_t factor_blk_batched_c(int v, const FactorTask *tasks, int nt, int64_t blocks,
                                const void *const *A, char *ws, hipStream_t st)
{
    // only the variants that exist (variant_ok) are instantiated
    if constexpr (NCT < 4)
        if (v == 1) return factor_blk_batched_cv<T, NCT, 1>(tasks, nt, blocks, A, ws, st);
    if constexpr (NCT == 1)
        if (v == 2) return factor_blk_batched_cv<T, NCT, 2>(tasks, nt, blocks, A, ws, st);
    return factor_blk_batched_cv<T, NCT, 0>(tasks, nt, blocks, A, ws, st);
}

template <typename T>
hipError_t factor_blk_batched(int64_t n, int v, const FactorTask *tasks, int nt, int64_t blocks,
                              const void *const *A, char *ws, hipStream_t st)
{
    switch ((n + 15) / 16) {
    case 1: return factor_blk_batched_c<T, 1>(v, tasks, nt, blocks, A, ws, st);
    case 2: return factor_blk_batched_c<T, 2>(v, tasks, nt, blocks, A, ws, st);
    case 3: return factor_blk_batched_c<T, 3>(v, tasks, nt, blocks, A, ws, st);
    default: return factor_blk_batched_c<T, 4>(v, tasks, nt, blocks, A, ws, st);
    }
}

template <typename T, typename To, int NT>
hipError_t apply_batched_nt(int64_t n, const ApplyTask *tasks, int nt, int64_t blocks,
                            void *const *Q, char *ws, hipStream_t st)
{
    const size_t lds = mfmaapply::apply_lds_bytes<T, NT>(n);
    auto kern = k_apply_batched<T, To, NT>;
    hipError_t e = ensure_dynamic_lds((const void *)kern, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3((unsigned)blocks),
                       dim3(mfmaapply::kWaves * 64), lds, st, tasks, nt, Q, ws);
    return hipGetLastError();
}

template <typename T, typename To>
hipError_t apply_batched(int64_t n, const ApplyTask *tasks, int nt, int64_t blocks, void *const *Q,
                         char *ws, hipStream_t st)
{
    // one pass covers all n <= 64 columns: NT = ceil(n / 16) tiles of 16
    if (n <= 32) return apply_batched_nt<T, To, 2>(n, tasks, nt, blocks, Q, ws, st);
    return apply_batched_nt<T, To, 4>(n, tasks, nt, blocks, Q, ws, st);
}

enum LaunchKind { LK_FACTOR = 0, LK_FINAL, LK_APPLY };

struct Launch {
    int kind;
    int level;       // tree level (factor / apply)
    int64_t n;       // width of the group
    int variant;
    int64_t blocks;
    int ntasks;
    size_t tab_off;  // byte offset of the task table in the plan's device buffer
};

}  // namespace
}  // namespace tsqr

struct tsqr_batch_plan_t {
    int32_t batch = 0;
    int dtype = tsqr::F64;
    int device = 0;
    size_t ws_bytes = 0;
    char *d_tables = nullptr;
    std::vector<tsqr::Launch> launches;
};

using namespace tsqr;

extern "C" {

tsqr_status tsqr_tune_set(int32_t dtype, int64_t n, int32_t variant)
{
    if ((dtype != TSQR_DTYPE_F64 && dtype != TSQR_DTYPE_F32) || n < 1 || n > kBatchNmax)
        return TSQR_ERR_INVALID_ARG;
    const int dt = dtype == TSQR_DTYPE_F32 ? F32 : F64;
    if (!variant_ok(n, dt, variant)) return TSQR_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[dt][width_class(n)] = variant;
    return TSQR_OK;
}

tsqr_status tsqr_tune_get(int32_t dtype, int64_t n, int32_t *variant, int32_t *panel_rows)
{
    if ((dtype != TSQR_DTYPE_F64 && dtype != TSQR_DTYPE_F32) || n < 1 || n > kBatchNmax ||
        !variant || !panel_rows)
        return TSQR_ERR_INVALID_ARG;
    const int dt = dtype == TSQR_DTYPE_F32 ? F32 : F64;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    int v = g_tune[dt][width_class(n)];
    if (!variant_ok(n, dt, v)) v = 0;
    *variant = v;
    *panel_rows = batch_panel_rows(n, dt, v);
    return TSQR_OK;
}

tsqr_status tsqr_tune_variants(int32_t dtype, int64_t n, int32_t max, int32_t *panel_rows,
                               int32_t *count)
{
    if ((dtype != TSQR_DTYPE_F64 && dtype != TSQR_DTYPE_F32) || n < 1 || n > kBatchNmax ||
        !count || max < 0 || (max > 0 && !panel_rows))
        return TSQR_ERR_INVALID_ARG;
    const int dt = dtype == TSQR_DTYPE_F32 ? F32 : F64;
    int c = 0;
    for (int v = 0; v <= 2; ++v) {
        const int b = variant_ok(n, dt, v) ? batch_panel_rows(n, dt, v) : 0;
        if (c < max) panel_rows[c] = b;
        ++c;
    }
    *count = c;
    return TSQR_OK;
}

tsqr_status tsqr_batch_plan_create(int32_t batch, const int64_t *m, const int64_t *n,
                                   const int64_t *lda, const int64_t *ldq, const int64_t *ldr,
                                   int32_t dtype, const tsqr_opts *opts, tsqr_batch_plan *plan)
{
    if (!plan) return TSQR_ERR_INVALID_ARG;
    *plan = nullptr;
    if (batch < 1 || !m || !n || !lda || !ldq || !ldr) return TSQR_ERR_INVALID_ARG;
    if (dtype != TSQR_DTYPE_F64 && dtype != TSQR_DTYPE_F32) return TSQR_ERR_INVALID_ARG;
    if (opts && (opts->struct_size != (int32_t)sizeof(tsqr_opts) || opts->flags != 0 ||
                 opts->panel_rows < 0))
        return TSQR_ERR_INVALID_ARG;
    if (opts && opts->precision != (dtype == TSQR_DTYPE_F32 ? TSQR_FP32 : TSQR_FP64))
        return TSQR_ERR_UNSUPPORTED;
    for (int32_t i = 0; i < batch; ++i) {
        if (m[i] <= 0 || n[i] <= 0 || lda[i] < n[i] || ldq[i] < n[i] || ldr[i] < n[i])
            return TSQR_ERR_INVALID_ARG;
        if (n[i] > kBatchNmax || m[i] < n[i]) return TSQR_ERR_SHAPE;
    }
    const int dt = dtype == TSQR_DTYPE_F32 ? F32 : F64;
    const size_t es = dt == F32 ? 4 : 8;

    // panel variant per width and level arithmetic (level 0 in dt, the tree in FP64): an
    // explicit height picks the level-0 variant with that height
    auto pick_variant = [&](int64_t w, int ldt, bool explicit_rows, int *v) -> tsqr_status {
        if (explicit_rows && opts && opts->panel_rows > 0) {
            for (int c = 0; c <= 2; ++c)
                if (variant_ok(w, ldt, c) && batch_panel_rows(w, ldt, c) == opts->panel_rows) {
                    *v = c;
                    return TSQR_OK;
                }
            return TSQR_ERR_UNSUPPORTED;
        }
        std::lock_guard<std::mutex> lk(g_tune_mu);
        *v = g_tune[ldt][width_class(w)];
        if (!variant_ok(w, ldt, *v)) *v = 0;
        return TSQR_OK;
    };

    // per-matrix trees and workspace layout
    struct Lev { int64_t rows, panels, b; size_t q1, s, x; };
    std::vector<std::vector<Lev>> trees(batch);
    std::vector<size_t> wtop(batch);
    std::map<int64_t, int> variant_of;     // width -> level-0 variant
    std::map<int64_t, int> variant_tree;   // width -> variant of the FP64 tree levels
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t at = off;
        off = align_up(off + (bytes ? bytes : 1));
        return at;
    };
    for (int32_t i = 0; i < batch; ++i) {
        const int64_t w = n[i];
        if (!variant_of.count(w)) {
            int v = 0, vt = 0;
            tsqr_status s = pick_variant(w, dt, true, &v);
            if (s == TSQR_OK) s = pick_variant(w, F64, false, &vt);
            if (s != TSQR_OK) return s;
            variant_of[w] = v;
            variant_tree[w] = vt;
        }
        const int64_t B0 = batch_panel_rows(w, dt, variant_of[w]);
        const int64_t Bt = batch_panel_rows(w, F64, variant_tree[w]);
        int64_t rows = m[i];
        for (int L = 0;; ++L) {
            if (L >= kMaxLevels) return TSQR_ERR_UNSUPPORTED;
            const int64_t B = L == 0 ? B0 : Bt;
            Lev lv;
            lv.rows = rows;
            lv.b = rows < B ? rows : B;
            lv.panels = ceil_div(rows, lv.b);
            lv.q1 = take((L == 0 ? es : 8) * (size_t)rows * w);
            lv.s = take(8 * (size_t)lv.panels * w * w);
            lv.x = L >= 1 ? take(8 * (size_t)rows * w) : 0;
            trees[i].push_back(lv);
            if (lv.panels == 1) break;
            rows = lv.panels * w;
        }
        wtop[i] = take(8 * (size_t)w * w);
    }

    // launch groups
    std::vector<Launch> launches;
    std::vector<char> tables;
    auto push_table = [&](const void *p, size_t bytes) {
        size_t at = align_up(tables.size());
        tables.resize(at + bytes);
        memcpy(tables.data() + at, p, bytes);
        return at;
    };
    int maxlev = 0;
    for (auto &t : trees) maxlev = std::max(maxlev, (int)t.size());
    for (auto &kv : variant_of) {
        const int64_t w = kv.first;
        for (int L = 0; L < maxlev; ++L) {
            std::vector<FactorTask> ft;
            int64_t blocks = 0;
            for (int32_t i = 0; i < batch; ++i) {
                if (n[i] != w || (int)trees[i].size() <= L) continue;
                const Lev &lv = trees[i][L];
                FactorTask t;
                t.first_block = blocks;
                t.rows = lv.rows;
                t.ldx = L == 0 ? lda[i] : w;
                t.x_off = L == 0 ? -1 : (int64_t)trees[i][L - 1].s;
                t.q1_off = (int64_t)lv.q1;
                t.s_off = (int64_t)lv.s;
                t.mat = i;
                t.n = (int32_t)w;
                ft.push_back(t);
                blocks += lv.panels;
            }
            if (ft.empty()) continue;
            Launch la{LK_FACTOR, L, w, L == 0 ? kv.second : variant_tree[w], blocks, (int)ft.size(),
                      push_table(ft.data(), ft.size() * sizeof(FactorTask))};
            launches.push_back(la);
        }
    }
    {
        std::vector<FinalTask> fin(batch);
        for (int32_t i = 0; i < batch; ++i) {
            fin[i].s_off = (int64_t)trees[i].back().s;
            fin[i].wtop_off = (int64_t)wtop[i];
            fin[i].ldr = ldr[i];
            fin[i].mat = i;
            fin[i].n = (int32_t)n[i];
        }
        Launch la{LK_FINAL, 0, 0, 0, batch, batch,
                  push_table(fin.data(), fin.size() * sizeof(FinalTask))};
        launches.push_back(la);
    }
    for (auto &kv : variant_of) {
        const int64_t w = kv.first;
        for (int L = maxlev - 1; L >= 0; --L) {
            std::vector<ApplyTask> at;
            int64_t blocks = 0;
            for (int32_t i = 0; i < batch; ++i) {
                if (n[i] != w || (int)trees[i].size() <= L) continue;
                const Lev &lv = trees[i][L];
                const bool top = L + 1 == (int)trees[i].size();
                ApplyTask t;
                t.first_block = blocks;
                t.rows = lv.rows;
                t.q1_off = (int64_t)lv.q1;
                t.w_off = top ? (int64_t)wtop[i] : (int64_t)trees[i][L + 1].x;
                t.wstride = top ? 0 : w;
                t.out_off = L == 0 ? -1 : (int64_t)lv.x;
                t.ld_out = L == 0 ? ldq[i] : w;
                t.mat = i;
                t.n = (int32_t)w;
                t.b = (int32_t)lv.b;
                at.push_back(t);
                blocks += lv.panels;
            }
            if (at.empty()) continue;
            Launch la{LK_APPLY, L, w, L == 0 ? kv.second : variant_tree[w], blocks, (int)at.size(),
                      push_table(at.data(), at.size() * sizeof(ApplyTask))};
            launches.push_back(la);
        }
    }

    tsqr_batch_plan_t *p = new (std::nothrow) tsqr_batch_plan_t;
    if (!p) return TSQR_ERR_INVALID_ARG;
    p->batch = batch;
    p->dtype = dt;
    p->ws_bytes = off;
    p->launches = launches;
    if (hipGetDevice(&p->device) != hipSuccess ||
        hipMalloc((void **)&p->d_tables, tables.size()) != hipSuccess ||
        hipMemcpy(p->d_tables, tables.data(), tables.size(), hipMemcpyHostToDevice) != hipSuccess) {
        set_last_error(hipGetLastError(), "tsqr_batch_plan_create: task tables", __LINE__);
        if (p->d_tables) (void)hipFree(p->d_tables);
        delete p;
        return TSQR_ERR_HIP;
    }
    *plan = p;
    return TSQR_OK;
}

tsqr_status tsqr_batch_plan_destroy(tsqr_batch_plan plan)
{
    if (!plan) return TSQR_ERR_INVALID_ARG;
    if (plan->d_tables) (void)hipFree(plan->d_tables);
    delete plan;
    return TSQR_OK;
}

tsqr_status tsqr_batch_workspace_bytes(tsqr_batch_plan plan, size_t *bytes)
{
    if (!plan || !bytes) return TSQR_ERR_INVALID_ARG;
    *bytes = plan->ws_bytes;
    return TSQR_OK;
}

tsqr_status tsqr_batch_plan_launches(tsqr_batch_plan plan, int32_t *nlaunches)
{
    if (!plan || !nlaunches) return TSQR_ERR_INVALID_ARG;
    *nlaunches = (int32_t)plan->launches.size();
    return TSQR_OK;
}

tsqr_status tsqr_qr_batched(tsqr_batch_plan plan, const void *const *d_A, void *const *d_Q,
                            void *const *d_R, void *ws, size_t ws_bytes, int32_t *d_info,
                            void *stream)
{
    if (!plan || !d_A || !d_Q || !d_R || !d_info) return TSQR_ERR_INVALID_ARG;
    if (!ws || ws_bytes < plan->ws_bytes) return TSQR_ERR_WORKSPACE;
    hipStream_t st = (hipStream_t)stream;
    char *w = (char *)ws;
    const bool f32 = plan->dtype == F32;
    for (const Launch &la : plan->launches) {
        const void *tab = plan->d_tables + la.tab_off;
        if (la.kind == LK_FACTOR) {
            ProfScope ps(la.level == 0 ? PC_FACTOR0 : PC_FACTOR_TREE, st);
            const FactorTask *t = (const FactorTask *)tab;
            if (la.level == 0 && f32)
                TSQR_HIP_CHECK((factor_blk_batched<float>(la.n, la.variant, t, la.ntasks,
                                                          la.blocks, d_A, w, st)));
            else
                TSQR_HIP_CHECK((factor_blk_batched<double>(la.n, la.variant, t, la.ntasks,
                                                           la.blocks, d_A, w, st)));
        } else if (la.kind == LK_FINAL) {
            ProfScope ps(PC_FINALIZE, st);
            const FinalTask *t = (const FinalTask *)tab;
            if (f32)
                hipLaunchKernelGGL(k_finalize_batched<float>, dim3((unsigned)la.blocks),
                                   dim3(256), 0, st, t, d_R, w, d_info);
            else
                hipLaunchKernelGGL(k_finalize_batched<double>, dim3((unsigned)la.blocks),
                                   dim3(256), 0, st, t, d_R, w, d_info);
            TSQR_HIP_CHECK(hipGetLastError());
        } else {
            ProfScope ps(la.level == 0 ? PC_APPLY0 : PC_APPLY_TREE, st);
            const ApplyTask *t = (const ApplyTask *)tab;
            if (la.level == 0 && f32)
                TSQR_HIP_CHECK((apply_batched<float, float>(la.n, t, la.ntasks, la.blocks, d_Q,
                                                            w, st)));
            else
                TSQR_HIP_CHECK((apply_batched<double, double>(la.n, t, la.ntasks, la.blocks,
                                                              d_Q, w, st)));
        }
    }
    return TSQR_OK;
}

}  // extern "C"
