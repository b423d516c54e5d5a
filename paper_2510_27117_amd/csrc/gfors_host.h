// Host-side pieces shared by the libgfors host sources: error reporting,
// workspace carving, tile tables, the problem object and its timers.
#pragma once

#include "gfors_internal.h"
#include "../../include/gfors.h"

#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <functional>
#include <map>
#include <memory>
#include <string>
#include <utility>
#include <vector>

namespace gfh {

using namespace gfors;

struct LuForm;   // device side of the factorised TU reformulation (gfors_lu.cpp)

// The calling thread's last error message (defined in gfors_api.cpp).
std::string &err_slot();

inline int fail(int code, const std::string &msg) {
    err_slot() = msg;
    return code;
}

#define HIP_TRY(expr)                                                                    \
    do {                                                                                 \
        hipError_t e_ = (expr);                                                          \
        if (e_ != hipSuccess)                                                            \
            return fail(GFORS_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

constexpr int kSampleTQ = 256;        // quads per sample tile (1024 variables)
constexpr int kEvalNnz = 4096;        // nnz budget of an evaluation tile
constexpr int kCoverRows = 8192;      // rows per bitwise-evaluated tile (max)
constexpr int kBitwiseNnz = 8192;     // nnz budget of a bitwise-evaluated tile
constexpr int kGeneralRows = 4096;    // rows per general tile (max)
constexpr int kQuadNnz = 4096;        // nnz budget of a Q tile
constexpr int kQuadRows = 64;          // variables per Q tile (max): many tiles keep enough wavefronts in flight
constexpr int kVarTile = 4096;        // variables per FP64 reduction tile
constexpr int kRowNnz = 16384;        // nnz budget of a residual row tile
constexpr int kRowRows = 2048;
constexpr int kMfmaRows = 32;          // rows per dense digit block (one 32 x 32 matrix-core tile)
constexpr int kMfmaMaxSpan = 1 << 23;  // column span of a block: keeps int32 plane sums exact

// Bytes of the densified digit blocks: 3 planes at most, each block at least
// half full (rows x span <= 2 nnz) plus 31 padding columns and 16-byte
// alignment per row.
inline int64_t mf_digit_cap(int64_t nnzK, int64_t m) { return 3 * (2 * nnzK + 48 * m); }

enum RowClass { kCover = 0, kGeneral = 1 };

struct HostTiles {
    std::vector<int32_t> inst, b0, b1, first;
};

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Upper bounds on tile counts used both by the workspace size and the carve.
struct Bounds {
    int64_t st, et, qt, vt, rt;
};
inline Bounds tile_bounds(int64_t n, int64_t m, int64_t nnzK, int64_t nnzQ, int64_t T) {
    Bounds b;
    b.st = ceil_div(n / 4 + T, kSampleTQ) + T + 1;
    // a tile closes when its weight (nnz + rows) reaches the budget or its row
    // count reaches the cap, so tiles <= weight/budget + rows/cap + 1 per run
    b.et = m / kCoverRows + (nnzK + m) / kEvalNnz + (nnzK + m) / kBitwiseNnz + 8 * T + 8;
    b.qt = n / kQuadRows + (nnzQ + n) / kQuadNnz + 2 * T + 2;
    b.vt = n / kVarTile + T + 1;
    b.rt = m / kRowRows + (nnzK + m) / kRowNnz + 4 * T + 4;
    return b;
}

// Bump allocator over the caller's workspace (measure mode when base == null).
struct Carver {
    char *base;
    size_t off = 0;
    size_t cap;
    template <class T>
    T *take(int64_t count) {
        off = (off + 255) & ~static_cast<size_t>(255);
        T *p = base ? reinterpret_cast<T *>(base + off) : nullptr;
        off += static_cast<size_t>(std::max<int64_t>(count, 1)) * sizeof(T);
        return p;
    }
};

}  // namespace gfh

using namespace gfors;

struct gfors_problem {
    hipStream_t stream = nullptr;
    gfors_params prm{};
    int64_t n = 0, m1 = 0, m2 = 0, m = 0, nnzK = 0, nnzQ = 0;
    int T = 1;
    bool unitK = true, hasQ = false, obj64 = false, acc64 = false;
    bool coef24 = true;   // every coefficient of the general rows fits in 24 signed bits
    bool q24 = true;      // every evaluated Q entry below 2^21 in magnitude: 24-bit products and
                          // int32 sums over a staged block of 1024 entries are exact
    LaunchCfg cfg;

    // host copies
    std::vector<int64_t> inst_var0, inst_nvar;
    std::vector<double> rowinv, s_o, s_K, qnorm, tau1, tau2, rmin, rmax, rdelta;
    std::vector<uint8_t> rkind_host;

    // device buffers
    int *rp = nullptr, *ci = nullptr, *val = nullptr;
    int *rpT = nullptr, *ciT = nullptr, *valT = nullptr;
    int *rpQ = nullptr, *ciQ = nullptr, *valQ = nullptr;
    int *rowQ = nullptr;   // row of each Q entry (quadratic objective)
    // the objective's evaluation over the upper triangle of a symmetric Q:
    // entries (i, k) with k > i doubled, the diagonal once
    bool qsym = false;
    int *rpU = nullptr, *ciU = nullptr, *valU = nullptr, *rowU = nullptr;
    float *omega = nullptr, *rt = nullptr, *ct = nullptr;
    double *omega64 = nullptr, *rowinv2_d = nullptr, *rowinv_d = nullptr;
    int64_t *rhs = nullptr, *cost = nullptr;
    int *var_inst = nullptr, *row_inst = nullptr;
    int64_t *d_inst_var0 = nullptr, *d_inst_nvar = nullptr;
    float *xbuf[2] = {nullptr, nullptr}, *xbar = nullptr, *xsave = nullptr;
    float *ybuf[2] = {nullptr, nullptr}, *wy = nullptr;
    int cur = 0;
    uint64_t *X = nullptr;
    int lastK = 0;
    int64_t *zpart = nullptr, *zqpart = nullptr;
    int *vpart = nullptr;
    int32_t *viol = nullptr;
    int64_t *z = nullptr;
    uint8_t *xbest = nullptr;
    DevCounters *ctr = nullptr;
    DevInst di{};
    Tiles st, et, qt, vt, rtile;
    int *cover_ids = nullptr, *general_ids = nullptr;
    int n_cover = 0, n_general = 0;
    bool general_long = false;   // general rows average >= 256 entries: split rows over wavefronts
    // general rows evaluated as dense int8 digit blocks on the matrix cores
    bool mfma = false;
    int mf_npl = 0;              // digit planes (1..3)
    int64_t mf_cap = 0;
    int8_t *mf_dig = nullptr;
    int64_t *mf_off = nullptr;   // per tile: byte offset of its block
    int *mf_c0 = nullptr, *mf_span = nullptr;
    int *rows = nullptr;
    uint8_t *rkind = nullptr;    // per row: evaluation kind << 4 | truth table (pair rows)
    uint8_t *xkind = nullptr;    // per variable, last round: 0 sampled, 1 all zero, 2 all one
    int *dual_order = nullptr;   // constraint rows, longest first (block-per-row dual)
    int *rowc0 = nullptr;        // first column of a row whose columns are one contiguous range, else -1
    uint8_t *rowunit = nullptr;  // 1 where every coefficient of the row is 1 (no coefficient stream)
    int *colT0 = nullptr;        // first row of a variable whose rows are one contiguous range, else -1
    int *primal_order = nullptr; // variables, most rows first (block-per-variable primal)
    int heavy_rows = 0, heavy_cols = 0;   // rows / variables with kHeavyLen+ entries
    // light rows / variables with signed entry-major indices (launch variants
    // dual 5 / primal 6): items [lgt_*0, lgt_*0 + lgt_*n) of lgt_*d entries
    int *lgt_d = nullptr, *lgt_p = nullptr;
    int lgt_d0 = 0, lgt_dn = 0, lgt_dd = 0, lgt_p0 = 0, lgt_pn = 0, lgt_pd = 0;
    // heavy variables in groups of <= kHgWidth with unit-shifted rows (launch
    // variant primal 7 = these groups + the light range of primal 6)
    int *hg_var0 = nullptr, *hg_w = nullptr, *hg_e0 = nullptr, *hg_c0 = nullptr;
    int *hg_chg = nullptr, *hg_chb = nullptr, *hg_che = nullptr, *hg_ord = nullptr;
    float *hg_part = nullptr;
    int64_t hg_cap_g = 0, hg_cap_c = 0;
    int hg_ngroup = 0, hg_nchunk = 0, hg_nslot = 0;
    bool pair_rows_mostly = false;   // most bitwise-evaluated rows have one or two entries
    // node classes of the learned proposal's messages (prefixes of dual_order /
    // primal_order): kGnnHeavyLen+ entries, then more than kGnnShortLen
    int gnn_rh = 0, gnn_rm = 0, gnn_ch = 0, gnn_cm = 0;
    double *pv = nullptr, *pu = nullptr, *pw = nullptr, *part = nullptr, *res = nullptr;
    double *dnorm = nullptr;
    // column-sliced copies for the XCD-sliced SpMV (see k_spmv_part)
    bool slicedK = false, slicedT = false;
    int *rpS = nullptr, *ciS = nullptr, *valS = nullptr;      // Kc, 8 column slices of x
    int *rpST = nullptr, *ciST = nullptr, *valST = nullptr;   // Kc^T, 8 slices of the rows
    float *spart = nullptr;
    DevCounters *ctr_scratch = nullptr;
    // SELL-64 copies: dual fused (rows of K), dual sliced (8 column slices), primal fused
    bool sellK_want = false, sellKS_want = false, sellT_want = false;
    SellView sellK, sellKS, sellT;
    int64_t sellK_cap = 0, sellKS_cap = 0, sellT_cap = 0;
    int *sellK_buf[6] = {}, *sellKS_buf[6] = {}, *sellT_buf[6] = {};
    // the coefficients as int16 for the SpMVs when every |a| <= 32767
    // (exact in FP32 either way; half the bytes of the coefficient stream)
    bool use16 = false;
    bool dense_cols = false;   // some variable's rows are one contiguous range (colT0 is read)
    int colT_deg = 0;          // every variable has this many rows (> 0): row ranges are computed
    // entry-major copy of the transposed rows (ell[u n + i]) for the primal step
    // with wy staged in LDS, and its slice length (0: that variant unavailable)
    int *ell = nullptr;
    int lds_slice = 0;
    // evaluation kernel of the general rows: 0 the creation's choice (matrix
    // cores when the blocks qualify, else row by row), 1 matrix cores, 2 rows
    // split over wavefronts, 3 a wavefront per row and word set (timed by the autotuner)
    int eval_variant = 0;
    // dense-block SpMVs (every row dense over its instance's variables)
    bool dense_block = false;
    BlockView blk;
    int16_t *blk_pval = nullptr;   // its padded int16 coefficients (capacity blk_pval_cap)
    int64_t *blk_pbase = nullptr;
    int64_t blk_pval_cap = 0;
    int16_t *val16 = nullptr, *sellT_val16 = nullptr;
    float *rowinv32 = nullptr;          // 1/||a_j|| (0 for a zero row): the GNN's edge weights
    float gnn_ictmax = 1.f, gnn_irtmax = 1.f;
    uint64_t *bx = nullptr, *by = nullptr;   // nonzero bitmaps of xbar and wy
    // host-side record, while a sequence of steps is being enqueued, of
    // whether bx / by already describe the xbar / wy that the next kernel reads
    bool bx_fresh = false, by_fresh = false;
    int64_t bx_words = 0, by_words = 0;
    int red_S = 1;                  // tile slices of the candidate reduction
    int32_t *red_v = nullptr;
    int64_t *red_z = nullptr;

    // device whose static workspace holds this problem (gfors_create_problem_static), else -1
    int static_dev = -1;
    // relaxed set-partitioning rows repaired on the device (gfors_params.repair_row0):
    // per row, its variables in (cost, index) order
    int n_rep = 0;
    int *rep_rp = nullptr, *rep_var = nullptr;
    int *a3_part = nullptr;   // partial assignment of the 3D-assignment sampler (2 x kA3MaxN)
    // factorised TU reformulation (gfors_create_problem_tu): the products with
    // the reformulated matrix go through the LU of the pivot block; null otherwise
    gfh::LuForm *lu = nullptr;

    // graphs: key = (K, parity)
    std::map<std::pair<int, int>, hipGraphExec_t> graphs;
    void graphs_clear() {
        for (auto &kv : graphs) (void)hipGraphExecDestroy(kv.second);
        graphs.clear();
    }
};

namespace gfh {

// Optional per-launch HIP-event timing (kernel ids of gfors_kernel_times).
struct KTimer {
    hipStream_t s;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev[GFORS_NUM_KERNEL_TIMERS];
    void b(int id) {
        hipEvent_t a, z;
        (void)hipEventCreate(&a);
        (void)hipEventCreate(&z);
        ev[id].push_back({a, z});
        (void)hipEventRecord(a, s);
    }
    void e(int id) { (void)hipEventRecord(ev[id].back().second, s); }
    ~KTimer() {
        for (auto &v : ev)
            for (auto &p : v) {
                (void)hipEventDestroy(p.first);
                (void)hipEventDestroy(p.second);
            }
    }
};
#define TB(id) do { if (tm) tm->b(id); } while (0)
#define TE(id) do { if (tm) tm->e(id); } while (0)

inline int validate_csr(const gfors_csr *M, int64_t ncols_expect, const char *name) {
    if (!M) return GFORS_OK;
    if (M->nrows < 0 || M->ncols != ncols_expect)
        return fail(GFORS_E_ARG, std::string(name) + ": ncols must equal n");
    if (!M->row_ptr || (M->nrows > 0 && M->row_ptr[0] != 0))
        return fail(GFORS_E_ARG, std::string(name) + ": row_ptr[0] must be 0");
    const int64_t nnz = M->row_ptr[M->nrows];
    if (nnz < 0 || nnz >= (int64_t{1} << 31))
        return fail(GFORS_E_OOM, std::string(name) + ": nnz must be < 2^31");
    if (nnz > 0 && !M->col_idx) return fail(GFORS_E_ARG, std::string(name) + ": col_idx is NULL");
    for (int64_t r = 0; r < M->nrows; ++r)
        if (M->row_ptr[r + 1] < M->row_ptr[r])
            return fail(GFORS_E_ARG, std::string(name) + ": row_ptr decreases at row " + std::to_string(r));
    for (int64_t e = 0; e < nnz; ++e)
        if (M->col_idx[e] < 0 || M->col_idx[e] >= ncols_expect)
            return fail(GFORS_E_ARG, std::string(name) + ": column index out of range at entry " + std::to_string(e));
    return GFORS_OK;
}

inline void build_tiles_items(HostTiles &ht, int inst, int64_t count,
                       const std::function<int64_t(int64_t)> *weight, int64_t budget,
                       int64_t max_items, int64_t base) {
    int64_t i = 0;
    while (i < count) {
        int64_t j = i, w = 0;
        while (j < count && (j - i) < max_items && (w < budget || j == i)) {
            w += weight ? (*weight)(j) + 1 : 1;
            ++j;
        }
        ht.inst.push_back(inst);
        ht.b0.push_back(static_cast<int32_t>(base + i));
        ht.b1.push_back(static_cast<int32_t>(base + j));
        i = j;
    }
}

template <class T>
int upload(hipStream_t s, T *dst, const T *src, int64_t count) {
    if (count <= 0) return GFORS_OK;
    HIP_TRY(hipMemcpyAsync(dst, src, static_cast<size_t>(count) * sizeof(T), hipMemcpyHostToDevice, s));
    return GFORS_OK;
}

inline void carve_tiles(Carver &cv, Tiles &t, int64_t count, int64_t bound, int T) {
    t.count = static_cast<int32_t>(count);
    t.inst = cv.take<int32_t>(bound);
    t.b0 = cv.take<int32_t>(bound);
    t.b1 = cv.take<int32_t>(bound);
    t.first = cv.take<int32_t>(T + 1);
}

inline int upload_tiles(hipStream_t s, Tiles &t, const HostTiles &h, int T) {
    int rc;
    if ((rc = upload(s, t.inst, h.inst.data(), t.count))) return rc;
    if ((rc = upload(s, t.b0, h.b0.data(), t.count))) return rc;
    if ((rc = upload(s, t.b1, h.b1.data(), t.count))) return rc;
    if ((rc = upload(s, t.first, h.first.data(), T + 1))) return rc;
    return GFORS_OK;
}

inline void finish_first(HostTiles &h, int T) {
    h.first.assign(T + 1, 0);
    // tiles are appended instance by instance
    std::vector<int32_t> cnt(T, 0);
    for (int32_t t : h.inst) cnt[t]++;
    for (int t = 0; t < T; ++t) h.first[t + 1] = h.first[t] + cnt[t];
}

inline int sync(gfors_problem *P) {
    HIP_TRY(hipStreamSynchronize(P->stream));
    return GFORS_OK;
}


// Buffers of a problem carved from a workspace (measure mode when the carver
// has no base) and the candidate-count rule; defined in gfors_api.cpp.
size_t carve_problem(gfors_problem *P, Carver &cv, int64_t n, int64_t m1, int64_t m2,
                     int64_t nnzK, int64_t nnzQ, int T, const gfors_params *prm);
bool k_ok(int64_t K);

// The factorised TU form's pieces of a PDHG step sequence and of EvalBest,
// called by the generic enqueue functions when P->lu is set (gfors_lu.cpp).
void lu_enqueue_steps(gfors_problem *P, int nsteps, bool want_res, KTimer *tm);
void lu_enqueue_eval(gfors_problem *P, int K, int threshold, KTimer *tm, int trigger);
int lu_refresh_tails(gfors_problem *P);
void lu_destroy(LuForm *L);

}  // namespace gfh
