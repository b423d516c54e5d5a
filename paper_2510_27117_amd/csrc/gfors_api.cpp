// Host side of libgfors: ingest and validation of the integer model (eq. bip),
// transposition, row classification and tiling, Preprocess (Sec. 3) with FP64
// power iterations on the device, the Algorithm 1 loop pieces and HIP-graph
// replay of whole rounds, and the C ABI declared in include/gfors.h.
#include "gfors_host.h"
#include "gnn.h"

#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <functional>
#include <memory>
#include <limits>
#include <map>
#include <mutex>
#include <string>
#include <vector>

using namespace gfors;

namespace gfh {
std::string &err_slot() {
    thread_local std::string s;
    return s;
}
}  // namespace gfh

using namespace gfh;

extern "C" {

void gfors_default_params(gfors_params *p) {
    if (!p) return;
    p->sigma = 0.99;
    p->tau1 = -1.0;
    p->tau2 = -1.0;
    p->rho_min = -1.0;
    p->rho_max = -1.0;
    p->rho_T = 10.0;
    p->rho_p = 2.0;
    p->rho_delta = -1.0;
    p->k_int = 100;
    p->K_max = 1024;
    p->power_iters = 200;
    p->hist_cap = 4096;
    p->autotune = 1;
    p->x0 = 0.0;
    p->seed = 0;
    p->eval_mfma = 1;
    p->repair_row0 = -1;
    p->lu_wide_rows = 4096;
    p->lu_lds = 1;
}

const char *gfors_last_error(void) { return err_slot().c_str(); }

static int check_K(int64_t K) {
    if (K < 64 || K > 4096 || K % 64 != 0 || (K > 1024 && K % 1024 != 0)) return 0;
    return 1;
}

// The XCD-sliced SpMV pays when a row's random gathers span a vector larger than
// one XCD's L2 and rows are long enough to keep ~2+ entries per slice.
static bool want_slices(int64_t rows, int64_t vec_len, int64_t nnz) {
    return nnz > 0 && vec_len >= (int64_t{1} << 19) && nnz >= 16 * rows;
}

// Carve every device buffer; with base == null only measures the size.
static size_t carve(gfors_problem *P, Carver &cv, int64_t n, int64_t m1, int64_t m2,
                    int64_t nnzK, int64_t nnzQ, int T, const gfors_params *prm) {
    const int64_t m = m1 + m2;
    const int Wmax = prm->K_max / 64;
    const Bounds b = tile_bounds(n, m, nnzK, nnzQ, T);
    P->rp = cv.take<int>(m + 1);
    P->ci = cv.take<int>(nnzK);
    P->val = cv.take<int>(nnzK);
    P->rpT = cv.take<int>(n + 1);
    P->ciT = cv.take<int>(nnzK);
    P->valT = cv.take<int>(nnzK);
    P->rpQ = cv.take<int>(n + 1);
    P->ciQ = cv.take<int>(nnzQ);
    P->valQ = cv.take<int>(nnzQ);
    P->rowQ = cv.take<int>(nnzQ);
    P->rpU = cv.take<int>(nnzQ ? n + 1 : 1);
    P->ciU = cv.take<int>(nnzQ);
    P->valU = cv.take<int>(nnzQ);
    P->rowU = cv.take<int>(nnzQ);
    P->omega = cv.take<float>(m);
    P->rt = cv.take<float>(m);
    P->omega64 = cv.take<double>(m);
    P->rowinv_d = cv.take<double>(m);
    P->rowinv2_d = cv.take<double>(m);
    P->rhs = cv.take<int64_t>(m);
    P->row_inst = cv.take<int>(m);
    P->ct = cv.take<float>(n);
    P->cost = cv.take<int64_t>(n);
    P->var_inst = cv.take<int>(n);
    P->d_inst_var0 = cv.take<int64_t>(T);
    P->d_inst_nvar = cv.take<int64_t>(T);
    P->xbuf[0] = cv.take<float>(n);
    P->xbuf[1] = cv.take<float>(n);
    P->xbar = cv.take<float>(n + 1);   // [n] stays 0: target of SELL padding
    P->xsave = cv.take<float>(n);
    P->ybuf[0] = cv.take<float>(m);
    P->ybuf[1] = cv.take<float>(m);
    P->wy = cv.take<float>(m + 1);     // [m] stays 0: target of SELL padding
    P->X = cv.take<uint64_t>(n * Wmax);
    P->xbest = cv.take<uint8_t>(n);
    P->zpart = cv.take<int64_t>(b.st * prm->K_max);
    P->vpart = cv.take<int>(b.et * prm->K_max);
    P->zqpart = cv.take<int64_t>((nnzQ ? b.qt : 1) * prm->K_max);
    P->viol = cv.take<int32_t>(static_cast<int64_t>(T) * prm->K_max);
    P->z = cv.take<int64_t>(static_cast<int64_t>(T) * prm->K_max);
    P->rows = cv.take<int>(m);
    P->rkind = cv.take<uint8_t>(m);
    P->xkind = cv.take<uint8_t>(n);
    P->dual_order = cv.take<int>(m);
    P->rowc0 = cv.take<int>(std::max<int64_t>(m, 1));
    P->rowunit = cv.take<uint8_t>(std::max<int64_t>(m, 1));
    P->colT0 = cv.take<int>(std::max<int64_t>(n, 1));
    P->primal_order = cv.take<int>(n);
    P->cover_ids = cv.take<int>(b.et);
    P->general_ids = cv.take<int>(b.et);
    P->a3_part = cv.take<int>(2 * kA3MaxN);
    P->rep_rp = cv.take<int>(prm->repair_row0 >= 0 ? m1 + 1 : 1);
    P->rep_var = cv.take<int>(prm->repair_row0 >= 0 ? nnzK : 1);
    P->mf_cap = prm->eval_mfma && m > 0 ? mf_digit_cap(nnzK, m) : 0;
    P->mf_dig = cv.take<int8_t>(P->mf_cap);
    P->mf_off = cv.take<int64_t>(b.et);
    P->mf_c0 = cv.take<int>(b.et);
    P->mf_span = cv.take<int>(b.et);
    P->pv = cv.take<double>(n);
    P->pu = cv.take<double>(n);
    P->pw = cv.take<double>(std::max(n, m));
    P->part = cv.take<double>(2 * std::max(b.vt, b.rt) + 2);
    P->res = cv.take<double>(4 * static_cast<int64_t>(T));
    P->dnorm = cv.take<double>(2 * static_cast<int64_t>(T));
    P->ctr = cv.take<DevCounters>(1);
    P->ctr_scratch = cv.take<DevCounters>(1);
    // stage-1 reduction buffers: T * S <= max(T, 64) slices of K_max candidates
    P->red_v = cv.take<int32_t>(std::max<int64_t>(T, 64) * prm->K_max);
    P->red_z = cv.take<int64_t>(std::max<int64_t>(T, 64) * prm->K_max);
    P->slicedK = want_slices(m, n, nnzK);
    P->slicedT = want_slices(n, m, nnzK);
    if (P->slicedK) {
        P->rpS = cv.take<int>(static_cast<int64_t>(kXcdSlices) * (m + 1));
        P->ciS = cv.take<int>(nnzK);
        P->valS = cv.take<int>(nnzK);
    }
    if (P->slicedT) {
        P->rpST = cv.take<int>(static_cast<int64_t>(kXcdSlices) * (n + 1));
        P->ciST = cv.take<int>(nnzK);
        P->valST = cv.take<int>(nnzK);
    }
    // SELL-64 copies for short rows (lane = row); the entry budget allows 50%
    // padding (a larger need disables the layout for that matrix)
    auto sell_carve = [&](bool want, int64_t rows, int Pn, int64_t nnz, int64_t &cap, int *(&buf)[6]) {
        if (!want) return;
        const int64_t nch = ceil_div(rows, 64);
        cap = nnz + nnz / 2 + 2 * 64 * Pn * nch;
        buf[0] = cv.take<int>(Pn * (nch + 1));
        buf[1] = cv.take<int>(cap);
        buf[2] = cv.take<int>(cap);
        buf[3] = cv.take<int>(Pn * nch * 64);
        buf[4] = cv.take<int>(Pn * nch * 64);
        buf[5] = cv.take<int>(Pn * nch * 64);
    };
    P->sellK_want = m > 0 && nnzK <= 32 * m;
    P->sellKS_want = P->slicedK;
    P->sellT_want = m > 0 && nnzK <= 32 * n && nnzQ == 0;
    sell_carve(P->sellK_want, m, 1, nnzK, P->sellK_cap, P->sellK_buf);
    sell_carve(P->sellKS_want, m, kXcdSlices, nnzK, P->sellKS_cap, P->sellKS_buf);
    sell_carve(P->sellT_want, n, 1, nnzK, P->sellT_cap, P->sellT_buf);
    P->val16 = cv.take<int16_t>(nnzK);
    P->ell = cv.take<int>((T == 1 && nnzQ == 0 && nnzK <= 8 * n) ? nnzK : 0);
    P->lgt_d = cv.take<int>((T == 1 && nnzQ == 0) ? nnzK : 0);
    P->lgt_p = cv.take<int>((T == 1 && nnzQ == 0) ? nnzK : 0);
    P->hg_cap_g = (T == 1 && nnzQ == 0) ? nnzK / kHeavyLen + 1 : 0;
    P->hg_cap_c = (T == 1 && nnzQ == 0) ? nnzK / kHgChunk + P->hg_cap_g : 0;
    P->hg_var0 = cv.take<int>(P->hg_cap_g);
    P->hg_w = cv.take<int>(P->hg_cap_g);
    P->hg_e0 = cv.take<int>(P->hg_cap_g);
    P->hg_c0 = cv.take<int>(P->hg_cap_g + 1);
    P->hg_chg = cv.take<int>(P->hg_cap_c);
    P->hg_chb = cv.take<int>(P->hg_cap_c);
    P->hg_che = cv.take<int>(P->hg_cap_c);
    P->hg_ord = cv.take<int>(P->hg_cap_c > 0 ? 2 * P->hg_cap_c + 16 : 0);
    P->hg_part = cv.take<float>(P->hg_cap_c * kHgWidth);
    {
        // dense-block SpMV tables (filled only when the problem qualifies)
        const int64_t tb = n / kBlockCols + T + 1;
        BlockView &bv = P->blk;
        int *tile_inst = cv.take<int>(tb), *tile_c0 = cv.take<int>(tb);
        int *row0 = cv.take<int>(T), *nrow = cv.take<int>(T), *rows = cv.take<int>(m), *rank = cv.take<int>(m);
        int *t0 = cv.take<int>(T), *nt = cv.take<int>(T);
        bv.tile_inst = tile_inst; bv.tile_c0 = tile_c0; bv.row0 = row0; bv.nrow = nrow; bv.rows = rows;
        bv.row_rank = rank; bv.inst_tile0 = t0; bv.inst_ntile = nt;
        bv.pp = cv.take<float>(tb * 64);
        // padded int16 coefficients for the dense-block kernels (Q = 0 only)
        P->blk_pval_cap = nnzQ == 0 ? nnzK + 8 * m : 0;
        P->blk_pval = cv.take<int16_t>(P->blk_pval_cap);
        P->blk_pbase = cv.take<int64_t>(nnzQ == 0 ? m : 0);
    }
    P->sellT_val16 = cv.take<int16_t>(P->sellT_want ? P->sellT_cap : 0);
    P->rowinv32 = cv.take<float>(m);
    P->bx_words = ceil_div(n + 64 * kXcdSlices, 64) + 1;
    P->by_words = ceil_div(m + 64, 64) + 1;
    P->bx = cv.take<uint64_t>(P->bx_words);
    P->by = cv.take<uint64_t>(P->by_words);
    if (P->slicedK || P->slicedT)
        P->spart = cv.take<float>(static_cast<int64_t>(kXcdSlices) * std::max(P->slicedK ? m : 0, P->slicedT ? n : 0));
    DevInst &d = P->di;
    d.rho = cv.take<double>(T);
    d.ntrig = cv.take<int64_t>(T);
    d.zbest = cv.take<int64_t>(T);
    d.inc_k = cv.take<int64_t>(T);
    d.inc_round = cv.take<int64_t>(T);
    d.inc_l = cv.take<int64_t>(T);
    d.improved = cv.take<int32_t>(T);
    d.inc_W = cv.take<int32_t>(T);
    d.rho_min = cv.take<double>(T);
    d.rho_max = cv.take<double>(T);
    d.rho_T = cv.take<double>(T);
    d.rho_p = cv.take<double>(T);
    d.rho_delta = cv.take<double>(T);
    d.tau1 = cv.take<float>(T);
    d.tau2 = cv.take<float>(T);
    d.two_so = cv.take<float>(T);
    d.tau1d = cv.take<double>(T);
    d.tau2d = cv.take<double>(T);
    d.two_sod = cv.take<double>(T);
    d.hist_cap = std::max(1, prm->hist_cap);
    d.hist = cv.take<int64_t>(static_cast<int64_t>(T) * d.hist_cap);
    // tile tables are carved by upload_tiles in the same order (see create)
    return cv.off;
}

static size_t carve_tiles_measure(Carver &cv, int64_t n, int64_t m, int64_t nnzK, int64_t nnzQ, int T) {
    const Bounds b = tile_bounds(n, m, nnzK, nnzQ, T);
    for (int64_t bound : {b.st, b.et, b.qt, b.vt, b.rt}) {
        cv.take<int32_t>(bound);
        cv.take<int32_t>(bound);
        cv.take<int32_t>(bound);
        cv.take<int32_t>(T + 1);
    }
    return cv.off;
}

int gfors_workspace_bytes(int64_t n, int64_t m1, int64_t m2, int64_t nnzA, int64_t nnzB,
                          int64_t nnzQ, int32_t num_instances, const gfors_params *p,
                          size_t *bytes) {
    if (!p || !bytes || n <= 0 || m1 < 0 || m2 < 0 || nnzA < 0 || nnzB < 0 || nnzQ < 0 ||
        num_instances < 1)
        return fail(GFORS_E_ARG, "gfors_workspace_bytes: bad argument");
    if (!check_K(p->K_max)) return fail(GFORS_E_ARG, "K_max must be a multiple of 64, <= 4096 (multiple of 1024 above 1024)");
    gfors_problem tmp;
    Carver cv{nullptr, 0, 0};
    carve(&tmp, cv, n, m1, m2, nnzA + nnzB, nnzQ, num_instances, p);
    carve_tiles_measure(cv, n, m1 + m2, nnzA + nnzB, nnzQ, num_instances);
    *bytes = cv.off + 256;
    return GFORS_OK;
}

static void static_ws_release(gfors_problem *P);

void gfors_destroy_problem(gfors_problem *P) {
    if (!P) return;
    for (auto &kv : P->graphs) (void)hipGraphExecDestroy(kv.second);
    static_ws_release(P);
    if (P->lu) lu_destroy(P->lu);
    delete P;
}

static int device_norms(gfors_problem *P);
static int autotune(gfors_problem *P, bool with_eval);
static void launch_eval_general_rows(gfors_problem *P, int K);
static int setup_repair(gfors_problem *P, const gfors_csr *A, const int64_t *b, const gfors_csr *B,
                        const gfors_csr *Q, const int64_t *c);

int gfors_create_problem(const gfors_csr *A, const int64_t *b, const gfors_csr *B,
                         const int64_t *d, const gfors_csr *Q, const int64_t *c, int64_t n,
                         int32_t num_instances, const int64_t *inst_offsets,
                         const gfors_params *prm, void *ws, size_t ws_bytes, void *stream,
                         gfors_problem **out) {
    if (!out || !prm || !c || n <= 0 || num_instances < 1)
        return fail(GFORS_E_ARG, "gfors_create_problem: NULL argument or n <= 0");
    *out = nullptr;
    if (!check_K(prm->K_max)) return fail(GFORS_E_ARG, "K_max must be a multiple of 64, <= 4096 (multiple of 1024 above 1024)");
    if (!(prm->sigma > 0.0) || prm->k_int < 1 || prm->power_iters < 1 || !(prm->x0 >= 0.0 && prm->x0 <= 1.0))
        return fail(GFORS_E_ARG, "bad params (sigma > 0, k_int >= 1, power_iters >= 1, x0 in [0,1])");
    if (n >= (int64_t{1} << 31) / 64) return fail(GFORS_E_OOM, "n too large");
    int rc;
    if ((rc = validate_csr(A, n, "A"))) return rc;
    if ((rc = validate_csr(B, n, "B"))) return rc;
    if ((rc = validate_csr(Q, n, "Q"))) return rc;
    if (Q && Q->nrows != n) return fail(GFORS_E_ARG, "Q must be n x n");
    if (A && A->nrows > 0 && !b) return fail(GFORS_E_ARG, "b is NULL");
    if (B && B->nrows > 0 && !d) return fail(GFORS_E_ARG, "d is NULL");
    if (!ws) return fail(GFORS_E_ARG, "workspace is NULL");

    auto *P = new gfors_problem();
    std::unique_ptr<gfors_problem, void (*)(gfors_problem *)> guard(P, gfors_destroy_problem);
    P->stream = static_cast<hipStream_t>(stream);
    P->prm = *prm;
    P->n = n;
    P->m1 = A ? A->nrows : 0;
    P->m2 = B ? B->nrows : 0;
    P->m = P->m1 + P->m2;
    const int64_t nnzA = A ? A->row_ptr[A->nrows] : 0;
    const int64_t nnzB = B ? B->row_ptr[B->nrows] : 0;
    P->nnzK = nnzA + nnzB;
    P->nnzQ = Q ? Q->row_ptr[Q->nrows] : 0;
    P->hasQ = P->nnzQ > 0;
    P->T = num_instances;
    const int T = P->T;
    if (P->nnzK >= (int64_t{1} << 31)) return fail(GFORS_E_OOM, "nnz(A)+nnz(B) must be < 2^31");
    if (P->m >= (int64_t{1} << 31)) return fail(GFORS_E_OOM, "too many rows");

    // ---- instance ranges
    std::vector<int64_t> off(static_cast<size_t>(3) * (T + 1), 0);
    if (T == 1) {
        off[3] = n;
        off[4] = P->m1;
        off[5] = P->m2;
    } else {
        if (!inst_offsets) return fail(GFORS_E_ARG, "inst_offsets is NULL with num_instances > 1");
        std::memcpy(off.data(), inst_offsets, off.size() * sizeof(int64_t));
        if (off[0] || off[1] || off[2] || off[3 * T] != n || off[3 * T + 1] != P->m1 || off[3 * T + 2] != P->m2)
            return fail(GFORS_E_ARG, "inst_offsets must start at 0 and end at (n, m1, m2)");
        for (int t = 0; t < T; ++t)
            for (int k = 0; k < 3; ++k)
                if (off[3 * (t + 1) + k] < off[3 * t + k]) return fail(GFORS_E_ARG, "inst_offsets must be non-decreasing");
        for (int t = 0; t < T; ++t)
            if (off[3 * (t + 1)] <= off[3 * t]) return fail(GFORS_E_ARG, "every instance needs >= 1 variable");
    }
    P->inst_var0.resize(T);
    P->inst_nvar.resize(T);
    std::vector<int> var_inst(n), row_inst(P->m);
    for (int t = 0; t < T; ++t) {
        P->inst_var0[t] = off[3 * t];
        P->inst_nvar[t] = off[3 * (t + 1)] - off[3 * t];
        for (int64_t i = off[3 * t]; i < off[3 * (t + 1)]; ++i) var_inst[i] = t;
        for (int64_t j = off[3 * t + 1]; j < off[3 * (t + 1) + 1]; ++j) row_inst[j] = t;
        for (int64_t j = off[3 * t + 2]; j < off[3 * (t + 1) + 2]; ++j) row_inst[P->m1 + j] = t;
    }

    // ---- stacked constraint CSR [A; B] with original coefficients
    const int64_t m = P->m;
    std::vector<int> rp(m + 1, 0), ci(P->nnzK), val(P->nnzK);
    std::vector<int64_t> rhs(m);
    P->unitK = (!A || !A->val) && (!B || !B->val);
    {
        int64_t e = 0;
        auto add_rows = [&](const gfors_csr *M, const int64_t *r, int64_t row0) -> int {
            if (!M) return GFORS_OK;
            for (int64_t j = 0; j < M->nrows; ++j) {
                const int t = row_inst[row0 + j];
                const int64_t lo = P->inst_var0[t], hi = lo + P->inst_nvar[t];
                for (int64_t q = M->row_ptr[j]; q < M->row_ptr[j + 1]; ++q) {
                    const int col = M->col_idx[q];
                    if (col < lo || col >= hi)
                        return fail(GFORS_E_ARG, "row " + std::to_string(row0 + j) + " references a variable outside its instance");
                    ci[e] = col;
                    val[e] = M->val ? M->val[q] : 1;
                    ++e;
                }
                rp[row0 + j + 1] = static_cast<int>(e);
                rhs[row0 + j] = r[j];
            }
            return GFORS_OK;
        };
        if ((rc = add_rows(A, b, 0))) return rc;
        if ((rc = add_rows(B, d, P->m1))) return rc;
    }
    // row norms, infeasible zero rows, classes
    P->rowinv.assign(m, 1.0);
    std::vector<uint8_t> cls(m);
    P->rkind_host.assign(m, 0);
    int64_t npair = 0, nbit = 0;   // pair rows, rows evaluated bitwise
    for (int64_t j = 0; j < m; ++j) {
        double sq = 0.0;
        int64_t absum = 0, amax = 0;
        bool allone = true, allneg = true;
        for (int e = rp[j]; e < rp[j + 1]; ++e) {
            sq += static_cast<double>(val[e]) * static_cast<double>(val[e]);
            absum += std::llabs(static_cast<int64_t>(val[e]));
            amax = std::max<int64_t>(amax, std::llabs(static_cast<int64_t>(val[e])));
            allone = allone && val[e] == 1;
            allneg = allneg && val[e] == -1;
        }
        if (rp[j + 1] == rp[j]) {
            const bool bad = (j < P->m1) ? (rhs[j] > 0) : (rhs[j] != 0);
            if (bad) return fail(GFORS_E_INFEAS_ROW, "row " + std::to_string(j) + " has no coefficient but cannot be satisfied");
        }
        const double nrm = std::sqrt(sq);
        P->rowinv[j] = nrm > 0.0 ? 1.0 / nrm : 1.0;
        // rows whose violation is a bitwise function of the candidate words
        const int64_t len = rp[j + 1] - rp[j];
        const bool ineq = j < P->m1;
        int kind = -1, tt = 0;
        if (len > 0 && ineq && allone && rhs[j] == 1) kind = kEvalCover;              // sum >= 1
        else if (len > 0 && ineq && allneg && rhs[j] == -1) kind = kEvalAtMostOne;     // sum <= 1
        else if (len > 0 && !ineq && ((allone && rhs[j] == 1) || (allneg && rhs[j] == -1)))
            kind = kEvalExactlyOne;                                                    // sum == 1
        else if (len == 1 || len == 2) {
            // truth table over (x_p, x_q), bit 2 bp + bq set when violated
            const int64_t ap = val[rp[j]], aq = len == 2 ? val[rp[j] + 1] : 0;
            for (int bp = 0; bp < 2; ++bp)
                for (int bq = 0; bq < 2; ++bq) {
                    const int bqe = len == 2 ? bq : bp;   // one entry: both read x_p
                    const int64_t v = ap * bp + aq * bqe;
                    const bool bad = ineq ? v < rhs[j] : v != rhs[j];
                    if (bad) tt |= 1 << (2 * bp + bq);
                }
            kind = kEvalPair;
        }
        cls[j] = kind >= 0 ? kCover : kGeneral;
        if (kind == kEvalPair) ++npair;
        if (kind >= 0) ++nbit;
        P->rkind_host[j] = static_cast<uint8_t>(kind >= 0 ? (kind << 4) | tt : 0);
        if (cls[j] == kGeneral && absum > 2147483647LL) P->acc64 = true;
        if (cls[j] == kGeneral && amax >= (1LL << 23)) P->coef24 = false;
    }
    P->pair_rows_mostly = nbit > 0 && 2 * npair > nbit;
    std::vector<uint8_t> rowunit_h(m, 0);
    for (int64_t j = 0; j < m; ++j) {
        bool one = rp[j + 1] > rp[j];
        for (int e = rp[j]; e < rp[j + 1] && one; ++e) one = val[e] == 1;
        rowunit_h[j] = one ? 1 : 0;
    }
    // transpose (counting sort by column; rows ascending within a column)
    std::vector<int> rpT(n + 1, 0), ciT(P->nnzK), valT(P->nnzK);
    for (int64_t e = 0; e < P->nnzK; ++e) rpT[ci[e] + 1]++;
    for (int64_t i = 0; i < n; ++i) rpT[i + 1] += rpT[i];
    {
        std::vector<int> pos(rpT.begin(), rpT.end() - 1);
        for (int64_t j = 0; j < m; ++j)
            for (int e = rp[j]; e < rp[j + 1]; ++e) {
                const int p = pos[ci[e]]++;
                ciT[p] = static_cast<int>(j);
                valT[p] = val[e];
            }
    }
    // Q
    std::vector<int> rpQ, ciQ, valQ;
    if (P->hasQ) {
        rpQ.resize(n + 1);
        ciQ.resize(P->nnzQ);
        valQ.resize(P->nnzQ);
        for (int64_t i = 0; i <= n; ++i) rpQ[i] = static_cast<int>(Q->row_ptr[i]);
        for (int64_t e = 0; e < P->nnzQ; ++e) {
            const int t = var_inst[std::upper_bound(rpQ.begin(), rpQ.end(), static_cast<int>(e)) - rpQ.begin() - 1];
            ciQ[e] = Q->col_idx[e];
            valQ[e] = Q->val ? Q->val[e] : 1;
            if (ciQ[e] < P->inst_var0[t] || ciQ[e] >= P->inst_var0[t] + P->inst_nvar[t])
                return fail(GFORS_E_ARG, "Q entry crosses instances");
        }
    }
    // upper triangle of a symmetric Q for the objective's evaluation:
    // <x, Q x> = 2 sum_{i<k} Q_ik x_i x_k + sum_i Q_ii x_i
    std::vector<int> rpU, ciU, valU;
    if (P->hasQ) {
        std::vector<std::array<int64_t, 3>> a(P->nnzQ), b(P->nnzQ);
        bool small = true;
        for (int64_t i = 0; i < n; ++i)
            for (int e = rpQ[i]; e < rpQ[i + 1]; ++e) {
                a[e] = {i, ciQ[e], valQ[e]};
                b[e] = {ciQ[e], i, valQ[e]};
                small = small && std::llabs(static_cast<int64_t>(valQ[e])) < (1LL << 30);
            }
        std::sort(a.begin(), a.end());
        std::sort(b.begin(), b.end());
        P->qsym = small && a == b;
        if (P->qsym) {
            rpU.assign(n + 1, 0);
            for (int64_t i = 0; i < n; ++i) {
                rpU[i + 1] = rpU[i];
                for (int e = rpQ[i]; e < rpQ[i + 1]; ++e)
                    if (ciQ[e] >= i) {
                        ciU.push_back(ciQ[e]);
                        valU.push_back(ciQ[e] > i ? 2 * valQ[e] : valQ[e]);
                        ++rpU[i + 1];
                    }
            }
        }
        const std::vector<int> &ve = P->qsym ? valU : valQ;
        for (int v : ve)
            if (std::llabs(static_cast<int64_t>(v)) >= (1LL << 21)) P->q24 = false;
    }
    // objective accumulation width in the sampler
    int64_t cmax = 0;
    for (int64_t i = 0; i < n; ++i) cmax = std::max<int64_t>(cmax, std::llabs(c[i]));
    P->obj64 = cmax > 0 && (static_cast<double>(cmax) * 4.0 * kSampleTQ >= 2147483647.0);

    // general rows as dense digit blocks: per instance, the general rows are
    // ordered by column range (the order of rows does not change a count) and
    // cut into greedy runs of at most 32 rows whose entries fill at least
    // half of rows x column span; used when every block qualifies
    struct MfTile { int64_t q0, q1; int c0, span; };
    std::vector<std::vector<MfTile>> mf_tiles(T);
    std::vector<std::vector<int>> mf_rows(T);
    {
        int64_t grows = 0, gnnz = 0;
        for (int64_t j = 0; j < m; ++j)
            if (cls[j] != kCover) { ++grows; gnnz += rp[j + 1] - rp[j]; }
        P->general_long = grows > 0 && gnnz >= 256 * grows;
        const int64_t mf_cap = prm->eval_mfma && m > 0 ? mf_digit_cap(P->nnzK, m) : 0;   // as carved below
        P->mfma = mf_cap > 0 && P->general_long;
        int npl = 1;
        for (int64_t j = 0; j < m && P->mfma; ++j) {
            if (cls[j] == kCover) continue;
            for (int e = rp[j]; e < rp[j + 1]; ++e) {
                int64_t rem = val[e];
                int nd = 0;
                do {
                    const int64_t dgt = static_cast<int8_t>(rem & 255);
                    rem = (rem - dgt) >> 8;
                    ++nd;
                } while (rem != 0);
                npl = std::max(npl, nd);
            }
        }
        if (npl > 3) P->mfma = false;
        P->mf_npl = npl;
        int64_t count = 0, bytes = 0;
        for (int t = 0; t < T && P->mfma; ++t) {
            std::vector<int> L;
            for (int64_t j = off[3 * t + 1]; j < off[3 * (t + 1) + 1]; ++j)
                if (cls[j] != kCover) L.push_back(static_cast<int>(j));
            for (int64_t j = off[3 * t + 2]; j < off[3 * (t + 1) + 2]; ++j)
                if (cls[P->m1 + j] != kCover) L.push_back(static_cast<int>(P->m1 + j));
            const int64_t nL = static_cast<int64_t>(L.size());
            std::vector<int64_t> rlo(nL, INT64_MAX), rhi(nL, -1);
            for (int64_t q = 0; q < nL; ++q)
                for (int e = rp[L[q]]; e < rp[L[q] + 1]; ++e) {
                    rlo[q] = std::min<int64_t>(rlo[q], ci[e]);
                    rhi[q] = std::max<int64_t>(rhi[q], ci[e]);
                }
            std::vector<int64_t> ord(nL);
            for (int64_t q = 0; q < nL; ++q) ord[q] = q;
            std::stable_sort(ord.begin(), ord.end(), [&](int64_t a, int64_t b2) {
                return rlo[a] != rlo[b2] ? rlo[a] < rlo[b2] : rhi[a] < rhi[b2];
            });
            std::vector<int> Ls(nL);
            for (int64_t q = 0; q < nL; ++q) Ls[q] = L[ord[q]];
            for (int64_t q = 0; q < nL && P->mfma;) {
                int64_t lo = INT64_MAX, hi = -1, sum = 0, q1 = q;
                while (q1 < nL && q1 - q < kMfmaRows) {
                    const int j = Ls[q1];
                    const int64_t nlo = std::min(lo, rlo[ord[q1]]), nhi = std::max(hi, rhi[ord[q1]]);
                    const int64_t nsum = sum + rp[j + 1] - rp[j];
                    const int64_t nspan = nhi >= nlo ? nhi - nlo + 1 : 0;
                    if (q1 > q && nspan * (q1 - q + 1) > 2 * nsum) break;
                    lo = nlo; hi = nhi; sum = nsum; ++q1;
                }
                const int64_t span = hi >= lo ? hi - lo + 1 : 0;
                if (span * (q1 - q) > 2 * sum || span > kMfmaMaxSpan) { P->mfma = false; break; }
                mf_tiles[t].push_back({q, q1, static_cast<int>(span ? lo : P->inst_var0[t]), static_cast<int>(span)});
                ++count;
                bytes += (static_cast<int64_t>(npl) * (q1 - q) * ((span + 31) / 32 * 32) + 15) / 16 * 16;
                q = q1;
            }
            mf_rows[t] = std::move(Ls);
        }
        if (count > (P->nnzK + m) / kEvalNnz + 4 * static_cast<int64_t>(T) + 8 || bytes > mf_cap) P->mfma = false;
    }

    // ---- tiles
    HostTiles hs, he, hq, hv, hr;
    std::vector<int> rows_list;
    rows_list.reserve(m);
    std::vector<int> cover_ids, general_ids;
    for (int t = 0; t < T; ++t) {
        const int64_t nq = ceil_div(P->inst_nvar[t], 4);
        build_tiles_items(hs, t, nq, nullptr, kSampleTQ, kSampleTQ, 0);
        // evaluation rows of instance t: covering rows, then general rows
        std::vector<int> rc_list[2];
        for (int64_t j = off[3 * t + 1]; j < off[3 * (t + 1) + 1]; ++j) rc_list[cls[j]].push_back(static_cast<int>(j));
        for (int64_t j = off[3 * t + 2]; j < off[3 * (t + 1) + 2]; ++j) rc_list[cls[P->m1 + j]].push_back(static_cast<int>(P->m1 + j));
        for (int k = 0; k < 2; ++k) {
            const int64_t base = static_cast<int64_t>(rows_list.size());
            const std::vector<int> &L = (k == kGeneral && P->mfma) ? mf_rows[t] : rc_list[k];
            rows_list.insert(rows_list.end(), L.begin(), L.end());
            std::function<int64_t(int64_t)> wfun = [&](int64_t q) -> int64_t { return rp[L[q] + 1] - rp[L[q]]; };
            const size_t before = he.inst.size();
            if (k == kGeneral && P->mfma) {
                for (const MfTile &mt : mf_tiles[t]) {
                    he.inst.push_back(t);
                    he.b0.push_back(static_cast<int32_t>(base + mt.q0));
                    he.b1.push_back(static_cast<int32_t>(base + mt.q1));
                }
            } else {
                build_tiles_items(he, t, static_cast<int64_t>(L.size()), &wfun,
                                  k == kCover ? kBitwiseNnz : kEvalNnz,
                                  k == kCover ? kCoverRows : kGeneralRows, base);
            }
            for (size_t q = before; q < he.inst.size(); ++q)
                (k == kCover ? cover_ids : general_ids).push_back(static_cast<int>(q));
        }
        if (P->hasQ) {
            const int64_t v0 = P->inst_var0[t];
            const std::vector<int> &rpE = P->qsym ? rpU : rpQ;   // the evaluated entries
            std::function<int64_t(int64_t)> wq = [&](int64_t q) -> int64_t { return rpE[v0 + q + 1] - rpE[v0 + q]; };
            build_tiles_items(hq, t, P->inst_nvar[t], &wq, kQuadNnz, kQuadRows, v0);
        }
        build_tiles_items(hv, t, P->inst_nvar[t], nullptr, kVarTile, kVarTile, P->inst_var0[t]);
        for (int part = 0; part < 2; ++part) {
            const int64_t r0 = part == 0 ? off[3 * t + 1] : P->m1 + off[3 * t + 2];
            const int64_t r1 = part == 0 ? off[3 * (t + 1) + 1] : P->m1 + off[3 * (t + 1) + 2];
            std::function<int64_t(int64_t)> wr = [&](int64_t q) -> int64_t { return rp[r0 + q + 1] - rp[r0 + q]; };
            build_tiles_items(hr, t, r1 - r0, &wr, kRowNnz, kRowRows, r0);
        }
    }
    for (HostTiles *h : {&hs, &he, &hq, &hv, &hr}) finish_first(*h, T);
    {
        int maxt = 1;
        for (int t = 0; t < T; ++t)
            for (HostTiles *h : {&hs, &he, &hq})
                maxt = std::max(maxt, h->first[t + 1] - h->first[t]);
        const int cap = T >= 64 ? 1 : std::max(1, 64 / T);
        P->red_S = std::max(1, std::min(cap, static_cast<int>(ceil_div(maxt, 32))));
    }
    P->n_cover = static_cast<int>(cover_ids.size());
    P->n_general = static_cast<int>(general_ids.size());

    // ---- carve the workspace
    Carver cv{static_cast<char *>(ws), 0, ws_bytes};
    // align the base
    {
        const uintptr_t a = reinterpret_cast<uintptr_t>(ws);
        cv.off = (256 - (a & 255)) & 255;
    }
    carve(P, cv, n, P->m1, P->m2, P->nnzK, P->nnzQ, T, prm);
    const Bounds bnd = tile_bounds(n, m, P->nnzK, P->nnzQ, T);
    hipStream_t s = P->stream;
    {
        const std::pair<Tiles *, std::pair<const HostTiles *, int64_t>> tl[5] = {
            {&P->st, {&hs, bnd.st}}, {&P->et, {&he, bnd.et}}, {&P->qt, {&hq, bnd.qt}},
            {&P->vt, {&hv, bnd.vt}}, {&P->rtile, {&hr, bnd.rt}}};
        for (const auto &e : tl) {
            if (static_cast<int64_t>(e.second.first->inst.size()) > e.second.second)
                return fail(GFORS_E_OOM, "internal: tile bound exceeded");
            carve_tiles(cv, *e.first, static_cast<int64_t>(e.second.first->inst.size()), e.second.second, T);
        }
    }
    // nothing has touched the device yet: check the size before any copy
    if (cv.off > ws_bytes)
        return fail(GFORS_E_OOM, "workspace too small: need " + std::to_string(cv.off) + " bytes");
    if ((rc = upload_tiles(s, P->st, hs, T))) return rc;
    if ((rc = upload_tiles(s, P->et, he, T))) return rc;
    if ((rc = upload_tiles(s, P->qt, hq, T))) return rc;
    if ((rc = upload_tiles(s, P->vt, hv, T))) return rc;
    if ((rc = upload_tiles(s, P->rtile, hr, T))) return rc;

    // ---- uploads
    if ((rc = upload(s, P->rp, rp.data(), m + 1))) return rc;
    if ((rc = upload(s, P->ci, ci.data(), P->nnzK))) return rc;
    if ((rc = upload(s, P->val, val.data(), P->nnzK))) return rc;
    P->use16 = !P->unitK;
    for (int64_t e = 0; e < P->nnzK && P->use16; ++e) P->use16 = val[e] >= -32767 && val[e] <= 32767;
    if (P->use16) {
        std::vector<int16_t> v16(val.begin(), val.end());
        if ((rc = upload(s, P->val16, v16.data(), P->nnzK))) return rc;
        if ((rc = sync(P))) return rc;
    }
    if ((rc = upload(s, P->rpT, rpT.data(), n + 1))) return rc;
    if ((rc = upload(s, P->ciT, ciT.data(), P->nnzK))) return rc;
    if ((rc = upload(s, P->valT, valT.data(), P->nnzK))) return rc;
    if (P->hasQ) {
        if ((rc = upload(s, P->rpQ, rpQ.data(), n + 1))) return rc;
        if ((rc = upload(s, P->ciQ, ciQ.data(), P->nnzQ))) return rc;
        if ((rc = upload(s, P->valQ, valQ.data(), P->nnzQ))) return rc;
        std::vector<int> rowQ(P->nnzQ);
        for (int64_t i = 0; i < n; ++i)
            for (int e = rpQ[i]; e < rpQ[i + 1]; ++e) rowQ[e] = static_cast<int>(i);
        if ((rc = upload(s, P->rowQ, rowQ.data(), P->nnzQ))) return rc;
        if ((rc = sync(P))) return rc;
        if (P->qsym) {
            const int64_t nu = static_cast<int64_t>(ciU.size());
            std::vector<int> rowU(nu);
            for (int64_t i = 0; i < n; ++i)
                for (int e = rpU[i]; e < rpU[i + 1]; ++e) rowU[e] = static_cast<int>(i);
            if ((rc = upload(s, P->rpU, rpU.data(), n + 1))) return rc;
            if ((rc = upload(s, P->ciU, ciU.data(), nu))) return rc;
            if ((rc = upload(s, P->valU, valU.data(), nu))) return rc;
            if ((rc = upload(s, P->rowU, rowU.data(), nu))) return rc;
            if ((rc = sync(P))) return rc;
        }
    }
    // column-sliced copies: slice q of the variables is [q*ns, (q+1)*ns)
    auto build_sliced = [&](int64_t rows, int64_t cols, const std::vector<int> &rpx,
                            const std::vector<int> &cix, const std::vector<int> &valx,
                            int *d_rp, int *d_ci, int *d_val) -> int {
        const int64_t ns = ceil_div(cols, kXcdSlices);
        std::vector<int> srp(static_cast<size_t>(kXcdSlices) * (rows + 1));
        std::vector<int> sci(cix.size()), sval(cix.size());
        std::vector<int64_t> cnt(kXcdSlices, 0);
        for (size_t e = 0; e < cix.size(); ++e) cnt[cix[e] / ns]++;
        std::vector<int64_t> base(kXcdSlices + 1, 0);
        for (int q = 0; q < kXcdSlices; ++q) base[q + 1] = base[q] + cnt[q];
        std::vector<int64_t> pos(base.begin(), base.end() - 1);
        for (int64_t r = 0; r < rows; ++r) {
            for (int q = 0; q < kXcdSlices; ++q) srp[q * (rows + 1) + r] = static_cast<int>(pos[q]);
            for (int e = rpx[r]; e < rpx[r + 1]; ++e) {
                const int q = static_cast<int>(cix[e] / ns);
                sci[pos[q]] = cix[e];
                sval[pos[q]] = valx[e];
                pos[q]++;
            }
        }
        for (int q = 0; q < kXcdSlices; ++q) srp[q * (rows + 1) + rows] = static_cast<int>(pos[q]);
        int r2;
        if ((r2 = upload(s, d_rp, srp.data(), static_cast<int64_t>(srp.size())))) return r2;
        if ((r2 = upload(s, d_ci, sci.data(), static_cast<int64_t>(sci.size())))) return r2;
        if ((r2 = upload(s, d_val, sval.data(), static_cast<int64_t>(sval.size())))) return r2;
        return sync(P);
    };
    // SELL-64: per column slice, rows sorted by length (descending, stable) inside
    // windows of 8192 rows, chunks of 64 rows padded to the longest row
    auto build_sell = [&](int64_t rows, int64_t cols, int Pn, const std::vector<int> &rpx,
                          const std::vector<int> &cix, const std::vector<int> &valx, int pad_col,
                          int64_t cap, int *(&buf)[6], SellView &sv, int16_t *v16) -> int {
        const int64_t nch = ceil_div(rows, 64);
        const int64_t ns = ceil_div(ceil_div(std::max<int64_t>(cols, 1), Pn), 64) * 64;
        std::vector<int> sptr(static_cast<size_t>(Pn) * (nch + 1)), srow(static_cast<size_t>(Pn) * nch * 64, -1);
        std::vector<int> sc0(static_cast<size_t>(Pn) * nch * 64, -1), slen(static_cast<size_t>(Pn) * nch * 64, 0);
        std::vector<int> sci, sval;
        bool any_dense = false;
        sci.reserve(static_cast<size_t>(cix.size() * 1.2) + 64);
        sval.reserve(sci.capacity());
        std::vector<int> len(rows), order(rows);
        std::vector<std::vector<int>> ent(0);
        for (int q = 0; q < Pn; ++q) {
            for (int64_t r = 0; r < rows; ++r) {
                int cnt = 0;
                for (int e = rpx[r]; e < rpx[r + 1]; ++e) cnt += (cix[e] / ns) == q;
                len[r] = cnt;
                order[r] = static_cast<int>(r);
            }
            const int64_t win = 8192;
            for (int64_t w0 = 0; w0 < rows; w0 += win) {
                const int64_t w1 = std::min(rows, w0 + win);
                std::stable_sort(order.begin() + w0, order.begin() + w1,
                                 [&](int a, int b2) { return len[a] > len[b2]; });
            }
            for (int64_t c = 0; c < nch; ++c) {
                sptr[q * (nch + 1) + c] = static_cast<int>(sci.size());
                int L = 0;
                for (int l = 0; l < 64 && c * 64 + l < rows; ++l) L = std::max(L, len[order[c * 64 + l]]);
                const size_t base = sci.size();
                if (static_cast<int64_t>(base) + 64LL * L > cap) { sv = SellView(); return GFORS_OK; }
                sci.resize(base + 64 * static_cast<size_t>(L), pad_col);
                sval.resize(base + 64 * static_cast<size_t>(L), 0);
                for (int l = 0; l < 64 && c * 64 + l < rows; ++l) {
                    const int r = order[c * 64 + l];
                    const size_t slot = (static_cast<size_t>(q) * nch + c) * 64 + l;
                    srow[slot] = r;
                    int k = 0, first = -1;
                    bool contiguous = true;
                    for (int e = rpx[r]; e < rpx[r + 1]; ++e)
                        if ((cix[e] / ns) == q) {
                            sci[base + 64 * k + l] = cix[e];
                            sval[base + 64 * k + l] = valx[e];
                            if (k == 0) first = cix[e];
                            else contiguous = contiguous && cix[e] == first + k;
                            ++k;
                        }
                    slen[slot] = k;
                    if (k > 0 && contiguous) {
                        sc0[slot] = first;
                        any_dense = true;
                    }
                }
            }
            sptr[q * (nch + 1) + nch] = static_cast<int>(sci.size());
        }
        int r2;
        if ((r2 = upload(s, buf[0], sptr.data(), static_cast<int64_t>(sptr.size())))) return r2;
        if ((r2 = upload(s, buf[1], sci.data(), static_cast<int64_t>(sci.size())))) return r2;
        if ((r2 = upload(s, buf[2], sval.data(), static_cast<int64_t>(sval.size())))) return r2;
        if ((r2 = upload(s, buf[3], srow.data(), static_cast<int64_t>(srow.size())))) return r2;
        if ((r2 = upload(s, buf[4], sc0.data(), static_cast<int64_t>(sc0.size())))) return r2;
        if ((r2 = upload(s, buf[5], slen.data(), static_cast<int64_t>(slen.size())))) return r2;
        std::vector<int16_t> sv16;
        if (v16 && P->use16) {
            sv16.assign(sval.begin(), sval.end());
            if ((r2 = upload(s, v16, sv16.data(), static_cast<int64_t>(sv16.size())))) return r2;
        }
        if ((r2 = sync(P))) return r2;
        sv.val16 = (v16 && P->use16) ? v16 : nullptr;
        sv.nrows = static_cast<int>(rows);
        sv.P = Pn;
        sv.nchunk = static_cast<int>(nch);
        sv.ns = static_cast<int>(ns);
        sv.ptr = buf[0];
        sv.ci = buf[1];
        sv.val = buf[2];
        sv.row_of = buf[3];
        sv.c0 = any_dense ? buf[4] : nullptr;
        sv.len = buf[5];
        return GFORS_OK;
    };
    if (P->sellK_want && (rc = build_sell(m, n, 1, rp, ci, val, static_cast<int>(n), P->sellK_cap, P->sellK_buf, P->sellK, nullptr))) return rc;
    if (P->sellKS_want && (rc = build_sell(m, n, kXcdSlices, rp, ci, val, static_cast<int>(n), P->sellKS_cap, P->sellKS_buf, P->sellKS, nullptr))) return rc;
    if (P->sellT_want && (rc = build_sell(n, m, 1, rpT, ciT, valT, static_cast<int>(m), P->sellT_cap, P->sellT_buf, P->sellT, P->sellT_val16))) return rc;
    if (P->slicedK && (rc = build_sliced(m, n, rp, ci, val, P->rpS, P->ciS, P->valS))) return rc;
    if (P->slicedT && (rc = build_sliced(n, m, rpT, ciT, valT, P->rpST, P->ciST, P->valST))) return rc;
    if ((rc = upload(s, P->rhs, rhs.data(), m))) return rc;
    if ((rc = upload(s, P->cost, c, n))) return rc;
    if ((rc = upload(s, P->var_inst, var_inst.data(), n))) return rc;
    if ((rc = upload(s, P->row_inst, row_inst.data(), m))) return rc;
    if ((rc = upload(s, P->d_inst_var0, P->inst_var0.data(), T))) return rc;
    if ((rc = upload(s, P->d_inst_nvar, P->inst_nvar.data(), T))) return rc;
    if ((rc = upload(s, P->rows, rows_list.data(), m))) return rc;
    if ((rc = upload(s, P->rkind, P->rkind_host.data(), m))) return rc;
    if ((rc = upload(s, P->rowunit, rowunit_h.data(), m))) return rc;
    if ((rc = upload(s, P->cover_ids, cover_ids.data(), P->n_cover))) return rc;
    {
        // launch order of the general tiles: most entries first (a tile's time
        // grows with them; the counts of a tile do not depend on the order)
        std::vector<int> gl(general_ids);
        std::vector<int64_t> work(he.inst.size(), 0);
        for (int id : gl)
            for (int q = he.b0[id]; q < he.b1[id]; ++q) work[id] += rp[rows_list[q] + 1] - rp[rows_list[q]];
        std::stable_sort(gl.begin(), gl.end(), [&](int a, int b2) { return work[a] > work[b2]; });
        if ((rc = upload(s, P->general_ids, gl.data(), P->n_general))) return rc;
    }
    if (P->mfma) {
        // densified digit blocks of the general tiles (signed base-256 digits)
        const int npl = P->mf_npl;
        std::vector<int64_t> offh(he.inst.size(), 0);
        std::vector<int> c0h(he.inst.size(), 0), sph(he.inst.size(), 0);
        int64_t total = 0;
        {
            int ti = 0;
            for (int t = 0; t < T; ++t)
                for (const MfTile &mt : mf_tiles[t]) {
                    const int id = general_ids[ti++];
                    offh[id] = total;
                    c0h[id] = mt.c0;
                    sph[id] = mt.span;
                    total += (static_cast<int64_t>(npl) * (mt.q1 - mt.q0) * ((mt.span + 31) / 32 * 32) + 15) / 16 * 16;
                }
        }
        std::vector<int8_t> digh(static_cast<size_t>(total), 0);
        for (int id : general_ids) {
            const int R = he.b1[id] - he.b0[id];
            const int64_t pitch = (sph[id] + 31) / 32 * 32;
            for (int i = 0; i < R; ++i) {
                const int j = rows_list[he.b0[id] + i];
                for (int e = rp[j]; e < rp[j + 1]; ++e) {
                    int64_t rem = val[e];
                    for (int p = 0; p < npl; ++p) {
                        const int8_t dgt = static_cast<int8_t>(rem & 255);
                        rem = (rem - dgt) >> 8;
                        digh[offh[id] + (static_cast<int64_t>(p) * R + i) * pitch + (ci[e] - c0h[id])] = dgt;
                    }
                }
            }
        }
        if ((rc = upload(s, P->mf_dig, digh.data(), total))) return rc;
        if ((rc = upload(s, P->mf_off, offh.data(), static_cast<int64_t>(offh.size())))) return rc;
        if ((rc = upload(s, P->mf_c0, c0h.data(), static_cast<int64_t>(c0h.size())))) return rc;
        if ((rc = upload(s, P->mf_span, sph.data(), static_cast<int64_t>(sph.size())))) return rc;
        if ((rc = sync(P))) return rc;
    }
    {
        std::vector<int> ord(m);
        for (int64_t j = 0; j < m; ++j) ord[j] = static_cast<int>(j);
        std::stable_sort(ord.begin(), ord.end(),
                         [&](int a, int b2) { return rp[a + 1] - rp[a] > rp[b2 + 1] - rp[b2]; });
        if ((rc = upload(s, P->dual_order, ord.data(), m))) return rc;
        std::vector<int> c0v(m, -1);
        for (int64_t j = 0; j < m; ++j) {
            const int b0 = rp[j], b1 = rp[j + 1];
            bool dense = b1 > b0;
            for (int e = b0 + 1; e < b1 && dense; ++e) dense = ci[e] == ci[b0] + (e - b0);
            if (dense) c0v[j] = ci[b0];
        }
        if ((rc = upload(s, P->rowc0, c0v.data(), m))) return rc;
        // dense blocks: every row of every instance spans all its instance's
        // variables, at most 64 rows per instance, no Q
        {
            bool ok = !P->hasQ && m > 0;
            std::vector<std::vector<int>> irows(T);
            for (int64_t j = 0; j < m && ok; ++j) {
                const int t = row_inst[j];
                ok = c0v[j] == P->inst_var0[t] && rp[j + 1] - rp[j] == P->inst_nvar[t];
                irows[t].push_back(static_cast<int>(j));
            }
            for (int t = 0; t < T && ok; ++t) ok = !irows[t].empty() && irows[t].size() <= 64;
            if (ok) {
                // instances with more rows first (their tiles take longest):
                // the dispatcher hands out tiles in this order, so the last
                // ones to start are short and the tail shrinks; the tiles of
                // one instance stay consecutive and in column order
                std::vector<int> tinst, tc0, row0(T), nrow(T), rows, rank(m), t0(T), nt(T), ord(T);
                for (int t = 0; t < T; ++t) ord[t] = t;
                std::stable_sort(ord.begin(), ord.end(),
                                 [&](int u, int v) { return irows[u].size() > irows[v].size(); });
                for (int t : ord) {
                    row0[t] = static_cast<int>(rows.size());
                    nrow[t] = static_cast<int>(irows[t].size());
                    for (size_t r = 0; r < irows[t].size(); ++r) {
                        rows.push_back(irows[t][r]);
                        rank[irows[t][r]] = static_cast<int>(r);
                    }
                    t0[t] = static_cast<int>(tinst.size());
                    for (int64_t c = P->inst_var0[t]; c < P->inst_var0[t] + P->inst_nvar[t]; c += kBlockCols) {
                        tinst.push_back(t);
                        tc0.push_back(static_cast<int>(c));
                    }
                    nt[t] = static_cast<int>(tinst.size()) - t0[t];
                }
                BlockView &bv = P->blk;
                bv.ntile = static_cast<int>(tinst.size());
                if ((rc = upload(s, const_cast<int *>(bv.tile_inst), tinst.data(), bv.ntile))) return rc;
                if ((rc = upload(s, const_cast<int *>(bv.tile_c0), tc0.data(), bv.ntile))) return rc;
                if ((rc = upload(s, const_cast<int *>(bv.row0), row0.data(), T))) return rc;
                if ((rc = upload(s, const_cast<int *>(bv.nrow), nrow.data(), T))) return rc;
                if ((rc = upload(s, const_cast<int *>(bv.rows), rows.data(), m))) return rc;
                if ((rc = upload(s, const_cast<int *>(bv.row_rank), rank.data(), m))) return rc;
                if ((rc = upload(s, const_cast<int *>(bv.inst_tile0), t0.data(), T))) return rc;
                if ((rc = upload(s, const_cast<int *>(bv.inst_ntile), nt.data(), T))) return rc;
                if ((rc = sync(P))) return rc;
                P->dense_block = true;
                // int16 coefficients: a copy with every row at a multiple of 8
                // entries (aligned 16-byte loads of 8 consecutive columns)
                if (P->use16 && P->blk_pval_cap > 0) {
                    std::vector<int16_t> pv;
                    std::vector<int64_t> pb(m);
                    for (int t = 0; t < T; ++t) {
                        const int64_t nv = P->inst_nvar[t], stride = (nv + 7) / 8 * 8;
                        for (int r = 0; r < nrow[t]; ++r) {
                            const int j = rows[row0[t] + r];
                            pb[row0[t] + r] = static_cast<int64_t>(pv.size());
                            for (int e = rp[j]; e < rp[j + 1]; ++e) pv.push_back(static_cast<int16_t>(val[e]));
                            pv.resize(pb[row0[t] + r] + stride, 0);
                        }
                    }
                    if (static_cast<int64_t>(pv.size()) <= P->blk_pval_cap) {
                        if ((rc = upload(s, P->blk_pval, pv.data(), static_cast<int64_t>(pv.size())))) return rc;
                        if ((rc = upload(s, P->blk_pbase, pb.data(), m))) return rc;
                        if ((rc = sync(P))) return rc;
                        bv.pval = P->blk_pval;
                        bv.pbase = P->blk_pbase;
                    }
                }
            }
        }
        std::vector<int> r0v(n, -1);
        for (int64_t i = 0; i < n; ++i) {
            const int b0 = rpT[i], b1 = rpT[i + 1];
            bool dense = b1 > b0;
            for (int e = b0 + 1; e < b1 && dense; ++e) dense = ciT[e] == ciT[b0] + (e - b0);
            if (dense) r0v[i] = ciT[b0];
            P->dense_cols = P->dense_cols || dense;
        }
        if ((rc = upload(s, P->colT0, r0v.data(), n))) return rc;
        if ((rc = sync(P))) return rc;
        P->heavy_rows = 0;
        while (P->heavy_rows < m && rp[ord[P->heavy_rows] + 1] - rp[ord[P->heavy_rows]] >= kHeavyLen) ++P->heavy_rows;
        std::vector<int> ordT(n);
        for (int64_t i = 0; i < n; ++i) ordT[i] = static_cast<int>(i);
        std::stable_sort(ordT.begin(), ordT.end(),
                         [&](int a, int b2) { return rpT[a + 1] - rpT[a] > rpT[b2 + 1] - rpT[b2]; });
        if ((rc = upload(s, P->primal_order, ordT.data(), n))) return rc;
        P->heavy_cols = 0;
        while (P->heavy_cols < n && rpT[ordT[P->heavy_cols] + 1] - rpT[ordT[P->heavy_cols]] >= kHeavyLen) ++P->heavy_cols;
        // light part with signed indices: one instance, no Q, every |a| = 1,
        // the items below kHeavyLen entries one contiguous range of D <= 8
        // entries each (the heavy ones keep a workgroup each)
        if (T == 1 && !P->hasQ && m > 0 && P->lgt_d && P->lgt_p) {
            bool unit_mag = true;
            for (int64_t e = 0; e < P->nnzK && unit_mag; ++e) unit_mag = val[e] == 1 || val[e] == -1;
            auto light_range = [&](const std::vector<int> &ptr, const std::vector<int> &ix, const std::vector<int> &vv,
                                   int64_t cnt, int *dst, int &i0, int &L, int &D) -> int {
                i0 = L = D = 0;
                if (!unit_mag) return GFORS_OK;
                int64_t lo = -1, hi = -1, nl = 0;
                int d = -1;
                for (int64_t i = 0; i < cnt; ++i) {
                    const int len = ptr[i + 1] - ptr[i];
                    if (len >= kHeavyLen) continue;
                    if (d < 0) d = len;
                    if (len != d) return GFORS_OK;
                    if (lo < 0) lo = i;
                    hi = i;
                    ++nl;
                }
                // heavy items inside the range (at most one in eight) are
                // holes marked kLightHole; the light kernels skip them
                const int64_t span = hi - lo + 1;
                if (nl == 0 || d < 1 || d > 8 || span > nl + nl / 8 || static_cast<int64_t>(d) * span > P->nnzK)
                    return GFORS_OK;
                std::vector<int> h(static_cast<size_t>(d) * span, kLightHole);
                for (int64_t k = 0; k < span; ++k) {
                    if (ptr[lo + k + 1] - ptr[lo + k] >= kHeavyLen) continue;
                    for (int u = 0; u < d; ++u) {
                        const int64_t e = ptr[lo + k] + u;
                        h[static_cast<size_t>(u) * span + k] =
                            static_cast<int>(static_cast<uint32_t>(ix[e]) | (vv[e] < 0 ? 0x80000000u : 0u));
                    }
                }
                nl = span;
                int rc2 = upload(s, dst, h.data(), static_cast<int64_t>(h.size()));
                if (rc2) return rc2;
                if ((rc2 = sync(P))) return rc2;
                i0 = static_cast<int>(lo);
                L = static_cast<int>(nl);
                D = d;
                return GFORS_OK;
            };
            if ((rc = light_range(rp, ci, val, m, P->lgt_d, P->lgt_d0, P->lgt_dn, P->lgt_dd))) return rc;
            if ((rc = light_range(rpT, ciT, valT, n, P->lgt_p, P->lgt_p0, P->lgt_pn, P->lgt_pd))) return rc;
        }
        // heavy variables grouped: consecutive heavy variables (up to kHgWidth) of one
        // length whose rows are those of the group's first variable shifted by
        // their distance to it, with the same coefficients
        P->hg_ngroup = P->hg_nchunk = 0;
        if (P->lgt_pd > 0 && P->hg_cap_g > 0) {
            std::vector<int> hv;
            for (int64_t i = 0; i < n; ++i)
                if (rpT[i + 1] - rpT[i] >= kHeavyLen) hv.push_back(static_cast<int>(i));
            std::vector<int> gv0, gw, ge0, gc0, chg, chb, che;
            size_t k = 0;
            while (k < hv.size()) {
                const int v0 = hv[k], len = rpT[v0 + 1] - rpT[v0];
                int w = 1;
                while (w < kHgWidth && k + w < hv.size() && hv[k + w] == v0 + w) {
                    const int v = v0 + w;
                    bool same = rpT[v + 1] - rpT[v] == len;
                    for (int e = 0; e < len && same; ++e)
                        same = ciT[rpT[v] + e] == ciT[rpT[v0] + e] + w && valT[rpT[v] + e] == valT[rpT[v0] + e];
                    if (!same) break;
                    ++w;
                }
                gc0.push_back(static_cast<int>(chg.size()));
                for (int b = 0; b < len; b += kHgChunk) {
                    chg.push_back(static_cast<int>(gv0.size()));
                    chb.push_back(b);
                    che.push_back(std::min(len, b + kHgChunk));
                }
                gv0.push_back(v0);
                gw.push_back(w);
                ge0.push_back(rpT[v0]);
                k += w;
            }
            gc0.push_back(static_cast<int>(chg.size()));
            // worth it only when the groups are wide on average
            const bool useful = !gv0.empty() && hv.size() >= 4 * gv0.size();
            // launch order: the chunks of groups 2k and 2k + 1 (same chunk
            // count) in units of 16 slots, eight of each group, so that
            // chunk i of both lands on one XCD; other groups in units of 8;
            // empty slots -1
            std::vector<int> ord;
            for (size_t g = 0; g < gv0.size();) {
                const int c0 = gc0[g], nc = gc0[g + 1] - gc0[g];
                const bool pair = g + 1 < gv0.size() && gc0[g + 2] - gc0[g + 1] == nc;
                for (int cb = 0; cb < nc; cb += 8) {
                    for (int i = 0; i < 8; ++i) ord.push_back(cb + i < nc ? c0 + cb + i : -1);
                    if (pair)
                        for (int i = 0; i < 8; ++i) ord.push_back(cb + i < nc ? gc0[g + 1] + cb + i : -1);
                }
                g += pair ? 2 : 1;
            }
            if (useful && static_cast<int64_t>(gv0.size()) <= P->hg_cap_g &&
                static_cast<int64_t>(chg.size()) <= P->hg_cap_c &&
                static_cast<int64_t>(ord.size()) <= 2 * P->hg_cap_c + 16) {
                const int64_t G = static_cast<int64_t>(gv0.size()), C = static_cast<int64_t>(chg.size());
                if ((rc = upload(s, P->hg_ord, ord.data(), static_cast<int64_t>(ord.size())))) return rc;
                P->hg_nslot = static_cast<int>(ord.size());
                if ((rc = upload(s, P->hg_var0, gv0.data(), G))) return rc;
                if ((rc = upload(s, P->hg_w, gw.data(), G))) return rc;
                if ((rc = upload(s, P->hg_e0, ge0.data(), G))) return rc;
                if ((rc = upload(s, P->hg_c0, gc0.data(), G + 1))) return rc;
                if ((rc = upload(s, P->hg_chg, chg.data(), C))) return rc;
                if ((rc = upload(s, P->hg_chb, chb.data(), C))) return rc;
                if ((rc = upload(s, P->hg_che, che.data(), C))) return rc;
                if ((rc = sync(P))) return rc;
                P->hg_ngroup = static_cast<int>(G);
                P->hg_nchunk = static_cast<int>(C);
            }
        }
        P->colT_deg = n > 0 ? rpT[1] - rpT[0] : 0;
        for (int64_t i = 1; i < n && P->colT_deg; ++i)
            if (rpT[i + 1] - rpT[i] != P->colT_deg) P->colT_deg = 0;
        // the primal step with wy staged in LDS: unit coefficients, every
        // variable in the same number (<= 8) of rows, one instance, no Q
        if (P->unitK && !P->hasQ && T == 1 && m > 0 && P->colT_deg >= 1 && P->colT_deg <= 8 &&
            P->nnzK <= 8 * n) {
            const int deg = P->colT_deg;
            std::vector<int> ell(static_cast<size_t>(deg) * n);
            for (int64_t i = 0; i < n; ++i)
                for (int u = 0; u < deg; ++u) ell[static_cast<size_t>(u) * n + i] = ciT[static_cast<size_t>(i) * deg + u];
            if ((rc = upload(s, P->ell, ell.data(), static_cast<int64_t>(ell.size())))) return rc;
            if ((rc = sync(P))) return rc;
            int dev = 0, lds_max = 0;
            HIP_TRY(hipGetDevice(&dev));
            HIP_TRY(hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
            P->lds_slice = primal_lds_slice(static_cast<size_t>(lds_max));
        }
        auto classes = [](const std::vector<int> &o, const std::vector<int> &ptr, int64_t cnt, int &h, int &md) {
            int64_t k = 0;
            while (k < cnt && ptr[o[k] + 1] - ptr[o[k]] >= kGnnHeavyLen) ++k;
            h = static_cast<int>(k);
            while (k < cnt && ptr[o[k] + 1] - ptr[o[k]] > kGnnShortLen) ++k;
            md = static_cast<int>(k) - h;
        };
        classes(ord, rp, m, P->gnn_rh, P->gnn_rm);
        classes(ordT, rpT, n, P->gnn_ch, P->gnn_cm);
    }
    if ((rc = upload(s, P->rowinv_d, P->rowinv.data(), m))) return rc;
    {
        std::vector<double> r2(m);
        for (int64_t j = 0; j < m; ++j) r2[j] = P->rowinv[j] * P->rowinv[j];
        if ((rc = upload(s, P->rowinv2_d, r2.data(), m))) return rc;
        if ((rc = sync(P))) return rc;   // host vectors die at scope end
    }

    // ---- Preprocess on the device: spectral norms by FP64 power iteration
    if ((rc = device_norms(P))) return rc;
    std::vector<double> kn(T), qn(T);
    HIP_TRY(hipMemcpyAsync(kn.data(), P->dnorm, T * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(qn.data(), P->dnorm + T, T * sizeof(double), hipMemcpyDeviceToHost, s));
    if ((rc = sync(P))) return rc;

    P->s_o.resize(T); P->s_K.resize(T); P->qnorm.resize(T); P->tau1.resize(T); P->tau2.resize(T);
    P->rmin.resize(T); P->rmax.resize(T); P->rdelta.resize(T);
    std::vector<float> omega(m), rtv(m), ctv(n);
    std::vector<double> om64(m);
    std::vector<float> t1f(T), t2f(T), tsof(T);
    std::vector<double> tsod(T), rT(T, prm->rho_T), rp_(T, prm->rho_p);
    for (int t = 0; t < T; ++t) {
        const int64_t v0 = P->inst_var0[t], nv = P->inst_nvar[t];
        double csq = 0.0;
        int64_t cm = 0;
        for (int64_t i = v0; i < v0 + nv; ++i) {
            csq += static_cast<double>(c[i]) * static_cast<double>(c[i]);
            cm = std::max<int64_t>(cm, std::llabs(c[i]));
        }
        P->qnorm[t] = qn[t];
        P->s_K[t] = kn[t];
        P->s_o[t] = qn[t] + std::sqrt(csq);
        const double so = P->s_o[t];
        const double Qn = so > 0 ? qn[t] / so : 0.0;
        const double cinf = so > 0 ? static_cast<double>(cm) / so : static_cast<double>(cm);
        const double g = cinf + Qn;
        P->rmin[t] = prm->rho_min >= 0 ? prm->rho_min : 1e-3 * g;
        P->rmax[t] = prm->rho_max >= 0 ? prm->rho_max : g;
        P->rdelta[t] = prm->rho_delta >= 0 ? prm->rho_delta : 1e-4 * g;
        const double sq = std::sqrt(prm->sigma);
        bool q_here = false;
        if (P->hasQ) q_here = rpQ[v0 + nv] > rpQ[v0];
        if (!q_here) {
            P->tau1[t] = P->tau2[t] = sq;
        } else {
            const double L = 2.0 * (Qn + P->rmax[t]);
            P->tau1[t] = std::min(sq, 1.0 / (2.0 * L));
            P->tau2[t] = prm->sigma / P->tau1[t];
        }
        if (prm->tau1 > 0) P->tau1[t] = prm->tau1;
        if (prm->tau2 > 0) P->tau2[t] = prm->tau2;
        for (int64_t i = v0; i < v0 + nv; ++i)
            ctv[i] = static_cast<float>(so > 0 ? static_cast<double>(c[i]) / so : static_cast<double>(c[i]));
        t1f[t] = static_cast<float>(P->tau1[t]);
        t2f[t] = static_cast<float>(P->tau2[t]);
        tsod[t] = so > 0 ? 2.0 / so : 2.0;
        tsof[t] = static_cast<float>(tsod[t]);
    }
    for (int64_t j = 0; j < m; ++j) {
        const double sk = P->s_K[row_inst[j]];
        const double w64 = sk > 0 ? P->rowinv[j] / sk : P->rowinv[j];
        om64[j] = w64;
        omega[j] = static_cast<float>(w64);
        const double rr = static_cast<double>(rhs[j]) * P->rowinv[j];
        rtv[j] = static_cast<float>(sk > 0 ? rr / sk : rr);
    }
    {
        std::vector<float> ri(m);
        double rtm = 0.0, ctm = 0.0;
        for (int64_t j = 0; j < m; ++j) {
            ri[j] = rp[j + 1] > rp[j] ? static_cast<float>(P->rowinv[j]) : 0.f;
            rtm = std::max(rtm, std::fabs(static_cast<double>(rtv[j])));
        }
        for (int64_t i = 0; i < n; ++i) ctm = std::max(ctm, std::fabs(static_cast<double>(ctv[i])));
        P->gnn_ictmax = ctm > 0 ? static_cast<float>(1.0 / ctm) : 1.f;
        P->gnn_irtmax = rtm > 0 ? static_cast<float>(1.0 / rtm) : 1.f;
        if ((rc = upload(s, P->rowinv32, ri.data(), m))) return rc;
        if ((rc = sync(P))) return rc;
    }
    if ((rc = upload(s, P->omega, omega.data(), m))) return rc;
    if ((rc = upload(s, P->rt, rtv.data(), m))) return rc;
    if ((rc = upload(s, P->omega64, om64.data(), m))) return rc;
    if ((rc = upload(s, P->ct, ctv.data(), n))) return rc;
    DevInst &di = P->di;
    if ((rc = upload(s, di.rho_min, P->rmin.data(), T))) return rc;
    if ((rc = upload(s, di.rho_max, P->rmax.data(), T))) return rc;
    if ((rc = upload(s, di.rho_delta, P->rdelta.data(), T))) return rc;
    if ((rc = upload(s, di.rho_T, rT.data(), T))) return rc;
    if ((rc = upload(s, di.rho_p, rp_.data(), T))) return rc;
    if ((rc = upload(s, di.rho, P->rmin.data(), T))) return rc;
    if ((rc = upload(s, di.tau1, t1f.data(), T))) return rc;
    if ((rc = upload(s, di.tau2, t2f.data(), T))) return rc;
    if ((rc = upload(s, di.two_so, tsof.data(), T))) return rc;
    if ((rc = upload(s, di.tau1d, P->tau1.data(), T))) return rc;
    if ((rc = upload(s, di.tau2d, P->tau2.data(), T))) return rc;
    if ((rc = upload(s, di.two_sod, tsod.data(), T))) return rc;
    {
        std::vector<int64_t> zeros(T, 0), big(T, INT64_MAX), neg(T, -2);
        std::vector<int32_t> z32(T, 0);
        if ((rc = upload(s, di.ntrig, zeros.data(), T))) return rc;
        if ((rc = upload(s, di.zbest, big.data(), T))) return rc;
        if ((rc = upload(s, di.inc_k, neg.data(), T))) return rc;
        if ((rc = upload(s, di.inc_round, neg.data(), T))) return rc;
        if ((rc = upload(s, di.inc_l, neg.data(), T))) return rc;
        if ((rc = upload(s, di.improved, z32.data(), T))) return rc;
        if ((rc = upload(s, di.inc_W, z32.data(), T))) return rc;
        std::vector<int64_t> h(static_cast<size_t>(T) * di.hist_cap, INT64_MAX);
        if ((rc = upload(s, di.hist, h.data(), static_cast<int64_t>(h.size())))) return rc;
        DevCounters c0{};
        if ((rc = upload(s, P->ctr, &c0, 1))) return rc;
        std::vector<uint8_t> xb(n, 0);
        if ((rc = upload(s, P->xbest, xb.data(), n))) return rc;
        if ((rc = sync(P))) return rc;
    }
    launch_fill_f32(s, P->xbuf[0], static_cast<float>(prm->x0), n);
    launch_fill_f32(s, P->xbuf[1], static_cast<float>(prm->x0), n);
    launch_fill_f32(s, P->xbar, static_cast<float>(prm->x0), n);
    launch_fill_f32(s, P->ybuf[0], 0.f, m);
    launch_fill_f32(s, P->ybuf[1], 0.f, m);
    launch_fill_f32(s, P->wy, 0.f, m + 1);
    launch_fill_f32(s, P->xbar + n, 0.f, 1);
    launch_fill_f32(s, reinterpret_cast<float *>(P->bx), 0.f, 2 * P->bx_words);
    launch_fill_f32(s, reinterpret_cast<float *>(P->by), 0.f, 2 * P->by_words);
    HIP_TRY(hipGetLastError());
    // launch shapes: lanes per row ~ average row length (rounded to a power of two)
    auto pick = [](double avg) {
        int l = 1;
        while (l < 64 && l * 2 <= avg) l *= 2;
        return l;
    };
    P->cfg.lpr_dual = pick(m ? static_cast<double>(P->nnzK) / m : 1.0);
    P->cfg.lpr_primal = pick(static_cast<double>(P->nnzK + P->nnzQ) / n);
    if (P->slicedK) {
        P->cfg.slices_dual = kXcdSlices;
        P->cfg.lpr_dual = pick(static_cast<double>(P->nnzK) / m / kXcdSlices);
    }
    if (prm->repair_row0 >= 0 && (rc = setup_repair(P, A, b, B, Q, c))) return rc;
    if ((rc = sync(P))) return rc;
    if (prm->autotune && (rc = autotune(P, true))) return rc;
    *out = guard.release();
    return GFORS_OK;
}

// Relaxed set-partitioning rows [repair_row0, m1) (monotone relaxation,
// Sec. 2.4): checks the conditions under which keeping one variable per row
// maps relaxed-feasible points to feasible points of the rows "= 1" without
// raising the objective, then uploads each row's variables in (c, index) order.
static int setup_repair(gfors_problem *P, const gfors_csr *A, const int64_t *b, const gfors_csr *B,
                        const gfors_csr *Q, const int64_t *c) {
    const int64_t r0 = P->prm.repair_row0, m1 = P->m1, n = P->n;
    if (P->T != 1) return fail(GFORS_E_ARG, "repair_row0: single-instance problems only");
    if (r0 > m1) return fail(GFORS_E_ARG, "repair_row0 beyond the inequality rows");
    if (Q && Q->row_ptr[Q->nrows] > 0) return fail(GFORS_E_ARG, "repair_row0 needs Q = 0");
    std::vector<int> owner(n, -1);
    std::vector<int> rrp(1, 0), rvar;
    for (int64_t j = r0; j < m1; ++j) {
        const int64_t e0 = A->row_ptr[j], e1 = A->row_ptr[j + 1];
        if (e1 == e0 || b[j] != 1) return fail(GFORS_E_ARG, "repair row " + std::to_string(j) + ": empty or b != 1");
        const size_t start = rvar.size();
        for (int64_t e = e0; e < e1; ++e) {
            const int i = A->col_idx[e];
            if ((A->val ? A->val[e] : 1) != 1) return fail(GFORS_E_ARG, "repair row " + std::to_string(j) + ": coefficient != 1");
            if (c[i] < 0) return fail(GFORS_E_ARG, "repair row " + std::to_string(j) + ": variable with c < 0");
            if (owner[i] >= 0) return fail(GFORS_E_ARG, "variable " + std::to_string(i) + " in two repair rows (or twice in one)");
            owner[i] = static_cast<int>(j);
            rvar.push_back(i);
        }
        std::sort(rvar.begin() + static_cast<std::ptrdiff_t>(start), rvar.end(),
                  [&](int a2, int b2) { return c[a2] != c[b2] ? c[a2] < c[b2] : a2 < b2; });
        rrp.push_back(static_cast<int>(rvar.size()));
    }
    for (int64_t j = 0; j < r0; ++j)
        for (int64_t e = A->row_ptr[j]; e < A->row_ptr[j + 1]; ++e)
            if (owner[A->col_idx[e]] >= 0 && (A->val ? A->val[e] : 1) > 0)
                return fail(GFORS_E_ARG, "a repair-row variable has a positive coefficient in inequality row " + std::to_string(j));
    if (B)
        for (int64_t e = 0; e < B->row_ptr[B->nrows]; ++e)
            if (owner[B->col_idx[e]] >= 0) return fail(GFORS_E_ARG, "a repair-row variable lies in an equality row");
    int rc;
    if ((rc = upload(P->stream, P->rep_rp, rrp.data(), static_cast<int64_t>(rrp.size())))) return rc;
    if (!rvar.empty() && (rc = upload(P->stream, P->rep_var, rvar.data(), static_cast<int64_t>(rvar.size())))) return rc;
    if ((rc = sync(P))) return rc;
    P->n_rep = static_cast<int>(m1 - r0);
    return GFORS_OK;
}

// FP64 power iterations (Preprocess, Sec. 3): per instance,
//   ||K||_2 of the row-normalised K and ||Q||_2, from v0 = 1/sqrt(n_t) 1.
static int device_norms(gfors_problem *P) {
    hipStream_t s = P->stream;
    const int T = P->T;
    auto init_v = [&](double *v) {
        for (int t = 0; t < T; ++t)
            launch_fill64(s, v + P->inst_var0[t], 1.0 / std::sqrt(static_cast<double>(P->inst_nvar[t])), P->inst_nvar[t]);
    };
    // constraint matrix: M = -diag(rowinv) [A;B]; M^T M v = A^T (rowinv^2 o (A v))
    if (P->nnzK) {
        double *v = P->pv, *u = P->pu;
        init_v(v);
        for (int it = 0; it < P->prm.power_iters; ++it) {
            launch_spmv64(s, static_cast<int>(P->m), P->rp, P->ci, P->unitK ? nullptr : P->val, P->rowinv2_d, v, P->pw);
            launch_spmv64(s, static_cast<int>(P->n), P->rpT, P->ciT, P->unitK ? nullptr : P->valT, nullptr, P->pw, u);
            launch_tile_sumsq(s, P->vt, u, P->part);
            launch_inst_sum(s, T, P->vt, P->part, 1, 0, P->dnorm, 1, true);
            launch_tile_scale_inv(s, P->vt, u, P->dnorm);
            std::swap(u, v);
        }
        launch_spmv64(s, static_cast<int>(P->m), P->rp, P->ci, P->unitK ? nullptr : P->val, P->rowinv_d, v, P->pw);
        launch_tile_sumsq(s, P->rtile, P->pw, P->part);
        launch_inst_sum(s, T, P->rtile, P->part, 1, 0, P->dnorm, 1, true);
    } else {
        launch_fill64(s, P->dnorm, 0.0, T);
    }
    if (P->hasQ) {
        double *v = P->pv, *u = P->pu;
        init_v(v);
        for (int it = 0; it < P->prm.power_iters; ++it) {
            launch_spmv64(s, static_cast<int>(P->n), P->rpQ, P->ciQ, P->valQ, nullptr, v, P->pw);
            launch_spmv64(s, static_cast<int>(P->n), P->rpQ, P->ciQ, P->valQ, nullptr, P->pw, u);
            launch_tile_sumsq(s, P->vt, u, P->part);
            launch_inst_sum(s, T, P->vt, P->part, 1, 0, P->dnorm + T, 1, true);
            launch_tile_scale_inv(s, P->vt, u, P->dnorm + T);
            std::swap(u, v);
        }
        launch_spmv64(s, static_cast<int>(P->n), P->rpQ, P->ciQ, P->valQ, nullptr, v, P->pw);
        launch_tile_sumsq(s, P->vt, P->pw, P->part);
        launch_inst_sum(s, T, P->vt, P->part, 1, 0, P->dnorm + T, 1, true);
    } else {
        launch_fill64(s, P->dnorm + T, 0.0, T);
    }
    HIP_TRY(hipGetLastError());
    return GFORS_OK;
}

// The dual and primal steps in the launch shape of the configuration.  The
// zero-skipping variants read the nonzero bitmap of the vector they gather;
// it is rebuilt (k_nzbits) unless the kernel that last wrote the vector, in
// the same enqueued sequence, already wrote the bitmap with it.
static void launch_dual_cfg(gfors_problem *P, int lpr, int slices, int sell, const float *y_in,
                            float *y_out) {
    hipStream_t s = P->stream;
    const bool batched = P->T > 1;
    const float tau2 = static_cast<float>(P->tau2[0]);
    const int m = static_cast<int>(P->m), m1 = static_cast<int>(P->m1);
    const uint32_t *bx32 = reinterpret_cast<const uint32_t *>(P->bx);
    auto need_bx = [&] {
        if (!P->bx_fresh) launch_nzbits(s, P->xbar, P->n, ceil_div(P->n, 64), P->bx);
        P->bx_fresh = true;
    };
    auto combine = [&] {
        launch_dual_combine(s, batched, m, m1, slices, P->spart, P->omega, P->rt, y_in, y_out,
                            P->wy, tau2, P->di.tau2, P->row_inst, P->by);
    };
    bool wy_bits = false;
    if (P->cfg.bits_dual == 4 && P->dense_block && !sell && slices == 1) {
        launch_dual_block(s, P->blk, m, m1, P->rp, P->val, P->use16 ? P->val16 : nullptr, P->d_inst_var0,
                          P->d_inst_nvar, P->xbar, P->omega, P->rt, P->di.tau2, P->row_inst, y_in, y_out, P->wy);
    } else if (P->cfg.bits_dual == 5 && P->lgt_dd > 0 && !sell && slices == 1) {
        // heavy rows a workgroup each, the light range a lane per row with signed indices
        launch_dual_long(s, P->unitK, false, P->heavy_rows, m1, P->dual_order, P->rp, P->rowc0, P->ci, P->val,
                         P->use16 ? P->val16 : nullptr, P->rowunit, P->omega, P->rt, P->xbar, y_in, y_out, P->wy, tau2,
                         P->di.tau2, P->row_inst);
        launch_dual_light(s, P->lgt_dd, P->lgt_d0, P->lgt_dn, m1, P->lgt_d, P->omega, P->rt, P->xbar, y_in, y_out,
                          P->wy, tau2);
    } else if (sell && P->cfg.bits_dual >= 2) {
        const int nc = P->cfg.bits_dual == 3 ? 4 : 2;
        need_bx();
        if (slices > 1) {
            launch_sell_bits(s, P->sellKS, 0, P->unitK, batched, static_cast<int>(P->n), P->xbar,
                             bx32, P->spart, 0, nullptr, nullptr, nullptr, nullptr, nullptr, 0.f,
                             nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, 0.f, nullptr,
                             nullptr, nullptr, nullptr, nc);
            combine();
            wy_bits = true;
        } else {
            launch_sell_bits(s, P->sellK, 1, P->unitK, batched, static_cast<int>(P->n), P->xbar,
                             bx32, nullptr, m1, P->omega, P->rt, y_in, y_out, P->wy, tau2,
                             P->di.tau2, P->row_inst, nullptr, nullptr, nullptr, nullptr, 0.f,
                             nullptr, nullptr, nullptr, nullptr, nc);
        }
    } else if (sell && slices > 1 && P->cfg.bits_dual) {
        need_bx();
        launch_sell_part_bits(s, P->sellKS, P->sellKS.ns, static_cast<int>(P->n), P->unitK, P->xbar,
                              bx32, P->spart);
        combine();
        wy_bits = true;
    } else if (sell && slices > 1) {
        launch_sell(s, P->sellKS, 0, P->unitK, batched, P->xbar, P->spart, 0, nullptr, nullptr,
                    nullptr, nullptr, nullptr, 0.f, nullptr, nullptr, nullptr, nullptr, nullptr,
                    nullptr, 0.f, nullptr, nullptr, nullptr, nullptr);
        combine();
        wy_bits = true;
    } else if (sell) {
        launch_sell(s, P->sellK, 1, P->unitK, batched, P->xbar, nullptr, m1, P->omega, P->rt,
                    y_in, y_out, P->wy, tau2, P->di.tau2, P->row_inst, nullptr, nullptr, nullptr,
                    nullptr, 0.f, nullptr, nullptr, nullptr, nullptr);
    } else if (slices > 1) {
        launch_spmv_part(s, lpr, P->unitK, m, slices, P->rpS, P->ciS, P->valS, P->xbar, P->spart);
        combine();
        wy_bits = true;
    } else if (lpr >= kLprBlock) {
        // a workgroup per row for all rows (256) or for the heavy rows only,
        // the others with lpr - 256 lanes each
        const bool all = lpr == kLprBlock;
        launch_dual_long(s, P->unitK, batched, all ? m : P->heavy_rows, m1, P->dual_order, P->rp,
                         P->rowc0, P->ci, P->val, P->use16 ? P->val16 : nullptr, P->rowunit, P->omega, P->rt,
                         P->xbar,
                         y_in, y_out, P->wy, tau2,
                         P->di.tau2, P->row_inst);
        if (!all)
            launch_dual(s, lpr - kLprBlock, P->unitK, batched, m, m1, P->rp, P->ci, P->val,
                        P->use16 ? P->val16 : nullptr,
                        P->omega, P->rt, P->xbar, y_in, y_out, P->wy, tau2, P->di.tau2,
                        P->row_inst, kHeavyLen);
    } else {
        launch_dual(s, lpr, P->unitK, batched, m, m1, P->rp, P->ci, P->val,
                    P->use16 ? P->val16 : nullptr, P->omega, P->rt,
                    P->xbar, y_in, y_out, P->wy, tau2, P->di.tau2, P->row_inst, 0);
    }
    P->by_fresh = wy_bits;
}

static void launch_primal_cfg(gfors_problem *P, int lpr, int slices, int sell, const float *x_in,
                              float *x_out, float *xbar, DevCounters *ctr) {
    hipStream_t s = P->stream;
    const bool batched = P->T > 1;
    const int kmode = P->m == 0 ? 0 : (P->unitK ? 1 : 2);
    const float tau1 = static_cast<float>(P->tau1[0]);
    // the bitmap of xbar is written with it only when xbar is the problem's own
    uint64_t *xbits = xbar == P->xbar ? P->bx : nullptr;
    auto need_by = [&] {
        if (!P->by_fresh) launch_nzbits(s, P->wy, P->m, ceil_div(P->m, 64), P->by);
        P->by_fresh = true;
    };
    bool xbar_bits = false;
    if ((P->cfg.bits_primal == 6 || P->cfg.bits_primal == 7) && P->lgt_pd > 0 && !sell && slices == 1) {
        // heavy variables a workgroup each (6) or in shift groups (7), the
        // light range a lane per variable with signed indices
        if (P->cfg.bits_primal == 7)
            launch_primal_hgroup(s, P->unitK, P->hg_nslot, P->hg_ngroup, P->hg_ord, P->hg_chg, P->hg_chb, P->hg_che,
                                 P->hg_var0, P->hg_w, P->hg_e0, P->hg_c0, P->ciT, P->valT, P->wy, P->hg_part,
                                 x_in, x_out, xbar, P->ct, tau1, P->di.rho);
        else
            launch_primal_long(s, P->unitK, false, P->heavy_cols, P->primal_order, P->rpT, P->ciT, P->valT,
                               P->wy, x_in, x_out, xbar, P->ct, tau1, P->di.tau1, P->di.rho, P->var_inst);
        uint64_t *xb_out = (P->lgt_p0 == 0 && P->lgt_pn == P->n && P->heavy_cols == 0) ? xbits : nullptr;
        launch_primal_light(s, P->lgt_pd, P->lgt_p0, P->lgt_pn, P->lgt_p, P->wy, x_in, x_out, xbar, P->ct, tau1,
                            P->di.rho, ctr, xb_out);
        xbar_bits = xb_out != nullptr;
    } else if (P->cfg.bits_primal == 5 && P->dense_block && !sell && slices == 1) {
        launch_primal_block(s, P->blk, P->rp, P->val, P->use16 ? P->val16 : nullptr, P->d_inst_var0, P->d_inst_nvar,
                            P->wy, x_in, x_out, xbar, P->ct, P->di.tau1, P->di.rho, ctr);
    } else if (P->cfg.bits_primal == 4 && P->lds_slice > 0 && !sell && slices == 1) {
        launch_primal_lds(s, static_cast<int>(P->n), static_cast<int>(P->m), P->colT_deg, P->lds_slice, P->ell,
                          P->wy, x_in, x_out, xbar, P->ct, tau1, P->di.rho, ctr, xbits);
        xbar_bits = xbits != nullptr;
    } else if (P->cfg.bits_primal >= 2 && sell && kmode != 0 && !P->hasQ) {
        need_by();
        launch_sell_bits(s, P->sellT, 2, P->unitK, batched, static_cast<int>(P->m), P->wy,
                         reinterpret_cast<const uint32_t *>(P->by), nullptr, 0, nullptr, nullptr,
                         nullptr, nullptr, nullptr, 0.f, nullptr, nullptr, x_in, x_out, xbar,
                         P->ct, tau1, P->di.tau1, P->di.rho, P->var_inst, ctr,
                         P->cfg.bits_primal == 3 ? 4 : 2);
    } else if (P->cfg.bits_primal == 1 && !sell && slices == 1 && kmode != 0 && !P->hasQ) {
        need_by();
        uint64_t *xb_out = lpr <= 8 ? xbits : nullptr;
        launch_primal_bits(s, lpr, P->unitK, batched, static_cast<int>(P->n), static_cast<int>(P->m),
                           P->rpT, P->ciT, P->valT, P->wy, reinterpret_cast<const uint32_t *>(P->by),
                           x_in, x_out, xbar, P->ct, tau1, P->di.tau1, P->di.rho, P->var_inst, ctr,
                           xb_out, P->colT_deg);
        xbar_bits = xb_out != nullptr;
    } else if (sell) {
        launch_sell(s, P->sellT, 2, P->unitK, batched, P->wy, nullptr, 0, nullptr, nullptr, nullptr,
                    nullptr, nullptr, 0.f, nullptr, nullptr, x_in, x_out, xbar, P->ct, tau1,
                    P->di.tau1, P->di.rho, P->var_inst, ctr);
    } else if (slices > 1) {
        launch_spmv_part(s, lpr, P->unitK, static_cast<int>(P->n), slices, P->rpST, P->ciST,
                         P->valST, P->wy, P->spart);
        launch_primal_combine(s, batched, static_cast<int>(P->n), slices, P->spart, x_in, x_out,
                              xbar, P->ct, tau1, P->di.tau1, P->di.rho, P->var_inst, ctr, xbits);
        xbar_bits = xbits != nullptr;
    } else if (lpr > kLprBlock) {
        // heavy variables a workgroup each, the others lpr - 256 lanes (no Q)
        launch_primal_long(s, P->unitK, batched, P->heavy_cols, P->primal_order, P->rpT, P->ciT,
                           P->valT, P->wy, x_in, x_out, xbar, P->ct, tau1, P->di.tau1, P->di.rho,
                           P->var_inst);
        launch_primal(s, lpr - kLprBlock, kmode, false, batched, static_cast<int>(P->n), P->rpT,
                      P->dense_cols ? P->colT0 : nullptr, P->ciT, P->valT, P->wy, P->rpQ, P->ciQ, P->valQ,
                      x_in, x_out, xbar, P->ct, tau1, 0.f, P->di.tau1, P->di.two_so, P->di.rho,
                      P->var_inst, ctr, kHeavyLen);
    } else {
        launch_primal(s, lpr, kmode, P->hasQ, batched, static_cast<int>(P->n), P->rpT,
                      P->dense_cols ? P->colT0 : nullptr, P->ciT,
                      P->valT, P->wy, P->rpQ, P->ciQ, P->valQ, x_in, x_out, xbar, P->ct, tau1,
                      static_cast<float>(P->s_o[0] > 0 ? 2.0 / P->s_o[0] : 2.0), P->di.tau1,
                      P->di.two_so, P->di.rho, P->var_inst, ctr, 0);
    }
    // the problem's xbar changed: its bitmap is current only if written with it
    if (xbar == P->xbar) P->bx_fresh = xbar_bits;
}

// Zero-operand skipping variants.  bits = 1: sliced SELL dual with the slice
// bitmap in LDS, or fused-CSR primal with the dual bitmap in LDS; bits = 2 / 3:
// k_sell_bits on any SELL copy (batched load issue, 2 / 4 chunks per pass).
// Each needs its bitmap to fit in LDS.
static int bits_ok_dual(gfors_problem *P, int slices, int sell, int bits) {
    if (bits == 0) return 1;
    if (bits == 4) return (P->dense_block && slices == 1 && !sell) ? 1 : 0;   // dense-block tiles
    if (bits == 5) return (P->lgt_dd > 0 && slices == 1 && !sell) ? 1 : 0;    // light rows, signed indices
    if (!sell) return 0;
    if (bits == 1) return (slices > 1 && P->sellKS.ptr && P->sellKS.ns / 8 <= kMaxLdsBitmapBytes) ? 1 : 0;
    if (bits != 2 && bits != 3) return 0;
    const SellView &sv = slices > 1 ? P->sellKS : P->sellK;
    return (sv.ptr && sv.ns / 8 <= kMaxLdsBitmapBytes) ? 1 : 0;
}
static int bits_ok_primal(gfors_problem *P, int slices, int sell, int bits) {
    if (bits == 0) return 1;
    if (P->m == 0 || P->hasQ || slices != 1) return 0;
    if (bits == 1) return (!sell && (P->m + 31) / 32 * 4 <= kMaxLdsBitmapBytes) ? 1 : 0;
    if (bits == 4) return (!sell && P->lds_slice > 0) ? 1 : 0;   // wy staged in LDS slices
    if (bits == 5) return (!sell && P->dense_block) ? 1 : 0;     // dense-block tiles
    if (bits == 6) return (!sell && P->lgt_pd > 0) ? 1 : 0;      // light variables, signed indices
    if (bits == 7) return (!sell && P->lgt_pd > 0 && P->hg_ngroup > 0) ? 1 : 0;   // + heavy shift groups
    if (bits != 2 && bits != 3) return 0;
    return (sell && P->sellT.ptr && P->sellT.ns / 8 <= kMaxLdsBitmapBytes) ? 1 : 0;
}

// Autotuner: time every candidate launch shape of the dual and primal SpMV on
// this problem's own data (HIP events, 1 warm-up + 5 timed launches each) and
// keep the fastest.  Outputs go to buffers that carry no state at this point.
static int autotune(gfors_problem *P, bool with_eval) {
    hipStream_t s = P->stream;
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    auto timeit = [&](const std::function<void()> &f) -> float {
        f();
        (void)hipEventRecord(e0, s);
        for (int r = 0; r < 5; ++r) f();
        (void)hipEventRecord(e1, s);
        (void)hipEventSynchronize(e1);
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        return ms / 5.f;
    };
    const int lprs[] = {1, 2, 4, 8, 16, 32, 64};
    P->cfg.bits_dual = P->cfg.bits_primal = 0;
    P->bx_fresh = P->by_fresh = false;
    if (P->m > 0) {
        float best = 1e30f;
        auto consider = [&](int l, int sl, int se) {
            const float t = timeit([&] { launch_dual_cfg(P, l, sl, se, P->ybuf[P->cur], P->ybuf[1 - P->cur]); });
            if (t < best) { best = t; P->cfg.lpr_dual = l; P->cfg.slices_dual = sl; P->cfg.sell_dual = se; }
        };
        for (int sl : {1, kXcdSlices}) {
            if (sl > 1 && !P->slicedK) continue;
            for (int l : lprs) {
                if (sl > 1 && l > 16) continue;
                consider(l, sl, 0);
            }
        }
        if (P->sellK.ptr) consider(1, 1, 1);
        if (P->sellKS.ptr) consider(1, kXcdSlices, 1);
        if (P->nnzK >= 512 * P->m) consider(kLprBlock, 1, 0);   // long rows: a workgroup per row
        if (P->heavy_rows > 0 && P->heavy_rows < P->m)           // heavy rows apart
            for (int l : {1, 2, 4, 8, 16}) consider(kLprBlock + l, 1, 0);
        // zero-operand skipping: each variant is kept only when it is faster
        int best_bits = 0;
        for (int b : {1, 2, 3}) {
            for (int sl : {kXcdSlices, 1}) {
                if (!bits_ok_dual(P, sl, 1, b)) continue;
                P->cfg.bits_dual = b;
                const float t = timeit([&] { launch_dual_cfg(P, 1, sl, 1, P->ybuf[P->cur], P->ybuf[1 - P->cur]); });
                if (t < best) { best = t; best_bits = b; P->cfg.lpr_dual = 1; P->cfg.slices_dual = sl; P->cfg.sell_dual = 1; }
            }
        }
        for (int b : {4, 5}) {
            if (!bits_ok_dual(P, 1, 0, b)) continue;
            P->cfg.bits_dual = b;
            const float t = timeit([&] { launch_dual_cfg(P, 1, 1, 0, P->ybuf[P->cur], P->ybuf[1 - P->cur]); });
            if (t < best) { best = t; best_bits = b; P->cfg.lpr_dual = 1; P->cfg.slices_dual = 1; P->cfg.sell_dual = 0; }
        }
        P->cfg.bits_dual = best_bits;
    }
    {
        float best = 1e30f;
        float *xs = P->xsave, *xb = reinterpret_cast<float *>(P->pv);
        auto consider = [&](int l, int sl, int se) {
            const float t = timeit([&] { launch_primal_cfg(P, l, sl, se, P->xbuf[P->cur], xs, xb, P->ctr_scratch); });
            if (t < best) { best = t; P->cfg.lpr_primal = l; P->cfg.slices_primal = sl; P->cfg.sell_primal = se; }
        };
        for (int sl : {1, kXcdSlices}) {
            if (sl > 1 && (!P->slicedT || P->hasQ)) continue;
            for (int l : lprs) {
                if (sl > 1 && l > 16) continue;
                consider(l, sl, 0);
            }
        }
        if (P->sellT.ptr) consider(1, 1, 1);
        if (!P->hasQ && P->m > 0 && P->heavy_cols > 0 && P->heavy_cols < P->n)   // heavy variables apart
            for (int l : {1, 2, 4, 8, 16}) consider(kLprBlock + l, 1, 0);
        int best_bits = 0;
        if (bits_ok_primal(P, 1, 0, 1)) {
            P->cfg.bits_primal = 1;
            for (int l : {1, 2, 4, 8, 16}) {
                const float t = timeit([&] { launch_primal_cfg(P, l, 1, 0, P->xbuf[P->cur], xs, xb, P->ctr_scratch); });
                if (t < best) { best = t; best_bits = 1; P->cfg.lpr_primal = l; P->cfg.slices_primal = 1; P->cfg.sell_primal = 0; }
            }
        }
        for (int b : {2, 3}) {
            if (!bits_ok_primal(P, 1, 1, b)) continue;
            P->cfg.bits_primal = b;
            const float t = timeit([&] { launch_primal_cfg(P, 1, 1, 1, P->xbuf[P->cur], xs, xb, P->ctr_scratch); });
            if (t < best) { best = t; best_bits = b; P->cfg.lpr_primal = 1; P->cfg.slices_primal = 1; P->cfg.sell_primal = 1; }
        }
        for (int b : {4, 5, 6, 7}) {
            if (!bits_ok_primal(P, 1, 0, b)) continue;
            P->cfg.bits_primal = b;
            const float t = timeit([&] { launch_primal_cfg(P, 1, 1, 0, P->xbuf[P->cur], xs, xb, P->ctr_scratch); });
            if (t < best) { best = t; best_bits = b; P->cfg.lpr_primal = 1; P->cfg.slices_primal = 1; P->cfg.sell_primal = 0; }
        }
        P->cfg.bits_primal = best_bits;
    }
    // EvalBest's general rows: time each kernel that applies on candidates
    // drawn from p = 1/2 (K = min(K_max, 1024)); the candidates, counts and
    // partial sums are scratch at this point
    if (with_eval && P->n_general > 0) {
        const int K = std::min(P->prm.K_max, 1024);
        const int W = K / 64;
        float *p = P->xsave;
        launch_fill_f32(s, p, 0.5f, P->n);
        launch_sample(s, W, P->obj64, p, P->cost, P->X, P->st, P->d_inst_var0, P->d_inst_nvar, P->zpart, K,
                      static_cast<uint32_t>(P->prm.seed & 0xffffffffu), static_cast<uint32_t>(P->prm.seed >> 32),
                      P->ctr, 0, P->xkind);
        float best = 1e30f;
        int bestv = 0;
        for (int v : {1, 2, 3}) {
            if (v == 1 && !P->mfma) continue;
            if ((v == 2 || v == 3) && !(W <= 16 && (W & (W - 1)) == 0)) continue;
            P->eval_variant = v;
            const float t = timeit([&] { launch_eval_general_rows(P, K); });
            if (t < best) { best = t; bestv = v; }
        }
        P->eval_variant = bestv;
    }
    HIP_TRY(hipGetLastError());
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return sync(P);
}

static void enqueue_steps(gfors_problem *P, int nsteps, bool want_res, KTimer *tm = nullptr) {
    if (P->lu) {
        lu_enqueue_steps(P, nsteps, want_res, tm);
        return;
    }
    hipStream_t s = P->stream;
    // a sequence never relies on bitmaps written before it
    P->bx_fresh = P->by_fresh = false;
    for (int it = 0; it < nsteps; ++it) {
        const bool res = want_res && it == nsteps - 1;
        if (res) launch_copy_f32(s, P->xsave, P->xbar, P->n);
        const int a = P->cur, bnext = 1 - P->cur;
        TB(0);
        if (P->m > 0)
            launch_dual_cfg(P, P->cfg.lpr_dual, P->cfg.slices_dual, P->cfg.sell_dual, P->ybuf[a],
                            P->ybuf[bnext]);
        TE(0);
        TB(1);
        launch_primal_cfg(P, P->cfg.lpr_primal, P->cfg.slices_primal, P->cfg.sell_primal,
                          P->xbuf[a], P->xbuf[bnext], P->xbar, P->ctr);
        TE(1);
        if (res) {
            const int T = P->T;
            launch_res_vars(s, P->vt, P->hasQ ? P->rpQ : nullptr, P->ciQ, P->valQ, P->xbuf[bnext],
                            P->xbuf[a], P->di.rho, P->di.tau1d, P->di.two_sod, P->part);
            launch_inst_sum(s, T, P->vt, P->part, 2, 0, P->res + 0, 4, true);
            launch_inst_sum(s, T, P->vt, P->part, 2, 1, P->res + 3, 4, false);
            if (P->m > 0) {
                launch_res_rows(s, P->rtile, static_cast<int>(P->m1), P->rp, P->ci,
                                P->unitK ? nullptr : P->val, P->omega64, P->rhs, P->xsave,
                                P->xbuf[bnext], P->ybuf[a], P->ybuf[bnext], P->di.tau2d, P->part);
                launch_inst_sum(s, T, P->rtile, P->part, 2, 0, P->res + 1, 4, true);
                launch_inst_sum(s, T, P->rtile, P->part, 2, 1, P->res + 2, 4, true);
            } else {
                for (int t = 0; t < T; ++t) {
                    launch_fill64(s, P->res + 4 * t + 1, 0.0, 2);
                }
            }
        }
        P->cur = bnext;
    }
}

static void enqueue_eval(gfors_problem *P, int K, int threshold, KTimer *tm, int trigger);

// The general rows of EvalBest in the chosen kernel: on the matrix cores
// (digit blocks, when the problem holds them), rows split over wavefronts, or
// a wavefront per row; all give the same exact counts.
static void launch_eval_general_rows(gfors_problem *P, int K) {
    hipStream_t s = P->stream;
    const int W = K / 64;
    const int v = P->eval_variant;
    if (P->mfma && (v == 0 || v == 1)) {
        launch_eval_mfma(s, P->n_general, P->general_ids, P->et, P->mf_npl, P->acc64, P->rows, P->mf_off,
                         P->mf_c0, P->mf_span, P->mf_dig, P->rhs, static_cast<int>(P->m1), P->X, W,
                         P->vpart, K);
        return;
    }
    const bool split = v == 2 ? true : (v == 3 ? false : P->general_long);
    launch_eval_general(s, P->n_general, P->general_ids, P->et, P->acc64, P->rows, P->rp, P->ci,
                        P->unitK ? nullptr : P->val, P->rhs, static_cast<int>(P->m1), P->X,
                        P->xkind, W, P->vpart, K, split, P->coef24);
}

static void enqueue_sample_eval(gfors_problem *P, int K, const float *p_override, int threshold,
                                KTimer *tm = nullptr, int trigger = 1) {
    hipStream_t s = P->stream;
    const int W = K / 64;
    const float *p = p_override ? p_override : P->xbuf[P->cur];
    TB(2);
    launch_sample(s, W, P->obj64, p, P->cost, P->X, P->st, P->d_inst_var0, P->d_inst_nvar,
                  P->zpart, K, static_cast<uint32_t>(P->prm.seed & 0xffffffffu),
                  static_cast<uint32_t>(P->prm.seed >> 32), P->ctr, threshold, P->xkind);
    if (P->n_rep > 0)
        launch_mono_repair(s, P->n_rep, W, K, P->rep_rp, P->rep_var, P->cost, P->X, P->xkind, P->zpart);
    TE(2);
    enqueue_eval(P, K, threshold, tm, trigger);
}

// EvalBest (Sec. 3) of the K candidates in P->X (objective's linear part in
// the per-tile partials): constraint rows, quadratic objective, reduction,
// incumbent update, x_best.
static void enqueue_eval(gfors_problem *P, int K, int threshold, KTimer *tm, int trigger) {
    if (P->lu) {
        lu_enqueue_eval(P, K, threshold, tm, trigger);
        return;
    }
    hipStream_t s = P->stream;
    const int W = K / 64;
    TB(3);
    launch_eval_cover(s, P->n_cover, P->cover_ids, P->et, P->rows, P->rkind, P->rp, P->ci, P->X,
                      P->xkind, W, P->vpart, K, P->pair_rows_mostly);
    TE(3);
    TB(4);
    launch_eval_general_rows(P, K);
    TE(4);
    TB(5);
    if (P->hasQ)
        launch_eval_quad(s, P->qt, P->qsym ? P->rpU : P->rpQ, P->qsym ? P->rowU : P->rowQ,
                         P->qsym ? P->ciU : P->ciQ, P->qsym ? P->valU : P->valQ, P->X, W, P->zqpart, K,
                         P->q24);
    TE(5);
    TB(6);
    launch_reduce_cand(s, P->T, K, P->red_S, P->et, P->vpart, P->st, P->zpart, P->qt, P->zqpart,
                       P->hasQ ? 1 : 0, P->red_v, P->red_z, P->viol, P->z);
    TE(6);
    TB(7);
    launch_argmin_update(s, P->T, K, W, P->viol, P->z, P->di, P->ctr, threshold ? 0 : (trigger ? 1 : 2));
    TE(7);
    TB(8);
    launch_extract_best(s, P->n, P->T, P->var_inst, P->X, P->di, P->xbest);
    TE(8);
    P->lastK = K;
}

int gfors_pdhg_steps(gfors_problem *P, int32_t nsteps, int32_t want_residuals) {
    if (!P || nsteps < 0) return fail(GFORS_E_ARG, "gfors_pdhg_steps: bad argument");
    if (nsteps == 0) return GFORS_OK;
    enqueue_steps(P, nsteps, want_residuals != 0);
    HIP_TRY(hipGetLastError());
    return GFORS_OK;
}

int gfors_sample_eval(gfors_problem *P, int32_t K, const float *p_override, int32_t *viol_dev,
                      int64_t *obj_dev) {
    return gfors_sample_eval_ex(P, K, p_override, viol_dev, obj_dev, 0);
}

int gfors_sample_eval_ex(gfors_problem *P, int32_t K, const float *p_override, int32_t *viol_dev,
                         int64_t *obj_dev, int32_t flags) {
    if (!P) return fail(GFORS_E_ARG, "NULL handle");
    if (!check_K(K) || K > P->prm.K_max)
        return fail(GFORS_E_ARG, "K must be a multiple of 64 in [64, K_max] (multiple of 1024 above 1024)");
    if (flags & ~GFORS_SAMPLE_NO_TRIGGER) return fail(GFORS_E_ARG, "unknown flag");
    enqueue_sample_eval(P, K, p_override, 0, nullptr, (flags & GFORS_SAMPLE_NO_TRIGGER) ? 0 : 1);
    const size_t cnt = static_cast<size_t>(P->T) * K;
    if (viol_dev) HIP_TRY(hipMemcpyAsync(viol_dev, P->viol, cnt * sizeof(int32_t), hipMemcpyDeviceToDevice, P->stream));
    if (obj_dev) HIP_TRY(hipMemcpyAsync(obj_dev, P->z, cnt * sizeof(int64_t), hipMemcpyDeviceToDevice, P->stream));
    HIP_TRY(hipGetLastError());
    return GFORS_OK;
}

int gfors_sample_eval_assign3d(gfors_problem *P, int32_t n, int32_t K, int32_t gamma, int32_t L,
                               const float *p_override, int32_t *viol_dev, int64_t *obj_dev,
                               int32_t flags) {
    if (!P) return fail(GFORS_E_ARG, "NULL handle");
    if (P->lu) return fail(GFORS_E_ARG, "not available on a factorised TU problem");
    if (P->T != 1) return fail(GFORS_E_ARG, "3D-assignment sampling: single-instance problems only");
    if (n < 1 || n > kA3MaxN || static_cast<int64_t>(n) * n * n != P->n)
        return fail(GFORS_E_ARG, "3D-assignment sampling: n must satisfy n^3 = number of variables, 1 <= n <= 1024");
    if (!check_K(K) || K > P->prm.K_max)
        return fail(GFORS_E_ARG, "K must be a multiple of 64 in [64, K_max] (multiple of 1024 above 1024)");
    if (gamma < 0 || static_cast<int64_t>(gamma) * n > kA3MaxTop || L < 0)
        return fail(GFORS_E_ARG, "3D-assignment sampling: need gamma >= 0, gamma n <= 4096, L >= 0");
    if (flags & ~GFORS_SAMPLE_NO_TRIGGER) return fail(GFORS_E_ARG, "unknown flag");
    hipStream_t s = P->stream;
    const int W = K / 64;
    const float *p = p_override ? p_override : P->xbuf[P->cur];
    launch_a3(s, p, n, gamma * n, K, L, static_cast<uint32_t>(P->prm.seed & 0xffffffffu),
              static_cast<uint32_t>(P->prm.seed >> 32), P->ctr, P->cost, P->a3_part, P->X, W, P->zpart,
              static_cast<int64_t>(P->st.count) * K, P->xkind);
    enqueue_eval(P, K, 0, nullptr, (flags & GFORS_SAMPLE_NO_TRIGGER) ? 0 : 1);
    P->lastK = K;
    const size_t cnt = static_cast<size_t>(K);
    if (viol_dev) HIP_TRY(hipMemcpyAsync(viol_dev, P->viol, cnt * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
    if (obj_dev) HIP_TRY(hipMemcpyAsync(obj_dev, P->z, cnt * sizeof(int64_t), hipMemcpyDeviceToDevice, s));
    HIP_TRY(hipGetLastError());
    return GFORS_OK;
}

int gfors_final_round(gfors_problem *P) {
    if (!P) return fail(GFORS_E_ARG, "NULL handle");
    enqueue_sample_eval(P, 64, nullptr, 1);
    HIP_TRY(hipGetLastError());
    return GFORS_OK;
}

int gfors_run_rounds(gfors_problem *P, int32_t nrounds, int32_t K, int32_t use_graph) {
    if (!P || nrounds < 0) return fail(GFORS_E_ARG, "gfors_run_rounds: bad argument");
    if (!check_K(K) || K > P->prm.K_max) return fail(GFORS_E_ARG, "bad K");
    for (int r = 0; r < nrounds; ++r) {
        if (!use_graph) {
            enqueue_steps(P, P->prm.k_int, false);
            enqueue_sample_eval(P, K, nullptr, 0);
            continue;
        }
        const auto key = std::make_pair(static_cast<int>(K), P->cur);
        auto it = P->graphs.find(key);
        const int cur0 = P->cur;
        if (it == P->graphs.end()) {
            hipGraph_t g;
            HIP_TRY(hipStreamBeginCapture(P->stream, hipStreamCaptureModeThreadLocal));
            enqueue_steps(P, P->prm.k_int, false);
            enqueue_sample_eval(P, K, nullptr, 0);
            HIP_TRY(hipStreamEndCapture(P->stream, &g));
            hipGraphExec_t ge;
            HIP_TRY(hipGraphInstantiate(&ge, g, nullptr, nullptr, 0));
            HIP_TRY(hipGraphDestroy(g));
            it = P->graphs.emplace(key, ge).first;
            P->cur = cur0;   // capture did not execute; replay below advances the state
        }
        HIP_TRY(hipGraphLaunch(it->second, P->stream));
        P->cur = (cur0 + P->prm.k_int) & 1;
        P->lastK = K;
    }
    HIP_TRY(hipGetLastError());
    return GFORS_OK;
}

int gfors_best(gfors_problem *P, int32_t inst, int64_t *z_best, uint8_t *x_best_host,
               int32_t *found, int64_t *info) {
    if (!P || inst < 0 || inst >= P->T) return fail(GFORS_E_ARG, "gfors_best: bad instance");
    int64_t zb, k, r, l, nt;
    hipStream_t s = P->stream;
    HIP_TRY(hipMemcpyAsync(&zb, P->di.zbest + inst, 8, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(&k, P->di.inc_k + inst, 8, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(&r, P->di.inc_round + inst, 8, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(&l, P->di.inc_l + inst, 8, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(&nt, P->di.ntrig + inst, 8, hipMemcpyDeviceToHost, s));
    if (x_best_host)
        HIP_TRY(hipMemcpyAsync(x_best_host, P->xbest + P->inst_var0[inst], P->inst_nvar[inst],
                               hipMemcpyDeviceToHost, s));
    int rc = sync(P);
    if (rc) return rc;
    if (z_best) *z_best = zb;
    if (found) *found = zb != INT64_MAX ? 1 : 0;
    if (info) { info[0] = k; info[1] = r; info[2] = l; info[3] = nt; }
    return GFORS_OK;
}

int gfors_get_residuals(gfors_problem *P, double *out) {
    if (!P || !out) return fail(GFORS_E_ARG, "bad argument");
    HIP_TRY(hipMemcpyAsync(out, P->res, 4 * P->T * sizeof(double), hipMemcpyDeviceToHost, P->stream));
    return sync(P);
}

int gfors_get_history(gfors_problem *P, int32_t inst, int64_t *z_hist, int32_t cap, int32_t *count) {
    if (!P || inst < 0 || inst >= P->T || !z_hist || cap < 0) return fail(GFORS_E_ARG, "bad argument");
    DevCounters c;
    HIP_TRY(hipMemcpyAsync(&c, P->ctr, sizeof(c), hipMemcpyDeviceToHost, P->stream));
    const int32_t ncopy = std::min<int32_t>(cap, P->di.hist_cap);
    HIP_TRY(hipMemcpyAsync(z_hist, P->di.hist + static_cast<int64_t>(inst) * P->di.hist_cap,
                           ncopy * sizeof(int64_t), hipMemcpyDeviceToHost, P->stream));
    int rc = sync(P);
    if (rc) return rc;
    if (count) *count = static_cast<int32_t>(c.round);
    return GFORS_OK;
}

int gfors_get_state(gfors_problem *P, float *x, float *x_prev, float *y, double *rho,
                    int64_t *k, int64_t *round, int64_t *ntrig) {
    if (!P) return fail(GFORS_E_ARG, "NULL handle");
    hipStream_t s = P->stream;
    if (x) HIP_TRY(hipMemcpyAsync(x, P->xbuf[P->cur], P->n * 4, hipMemcpyDeviceToHost, s));
    if (x_prev) HIP_TRY(hipMemcpyAsync(x_prev, P->xbuf[1 - P->cur], P->n * 4, hipMemcpyDeviceToHost, s));
    if (y && P->m) HIP_TRY(hipMemcpyAsync(y, P->ybuf[P->cur], P->m * 4, hipMemcpyDeviceToHost, s));
    if (rho) HIP_TRY(hipMemcpyAsync(rho, P->di.rho, P->T * 8, hipMemcpyDeviceToHost, s));
    DevCounters c;
    int64_t nt = 0;
    HIP_TRY(hipMemcpyAsync(&c, P->ctr, sizeof(c), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(&nt, P->di.ntrig, 8, hipMemcpyDeviceToHost, s));
    int rc = sync(P);
    if (rc) return rc;
    if (k) *k = c.k;
    if (round) *round = c.round;
    if (ntrig) *ntrig = nt;
    return GFORS_OK;
}

int gfors_set_state(gfors_problem *P, const float *x, const float *x_prev, const float *y,
                    const double *rho, int64_t k, int64_t round, int64_t ntrig) {
    if (!P || !x || !x_prev || (P->m && !y) || !rho) return fail(GFORS_E_ARG, "bad argument");
    hipStream_t s = P->stream;
    HIP_TRY(hipMemcpyAsync(P->xbuf[P->cur], x, P->n * 4, hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(P->xbuf[1 - P->cur], x_prev, P->n * 4, hipMemcpyHostToDevice, s));
    if (P->m) HIP_TRY(hipMemcpyAsync(P->ybuf[P->cur], y, P->m * 4, hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(P->di.rho, rho, P->T * 8, hipMemcpyHostToDevice, s));
    std::vector<int64_t> nt(P->T, ntrig);
    HIP_TRY(hipMemcpyAsync(P->di.ntrig, nt.data(), P->T * 8, hipMemcpyHostToDevice, s));
    DevCounters c{};
    c.k = k;
    c.round = round;
    HIP_TRY(hipMemcpyAsync(P->ctr, &c, sizeof(c), hipMemcpyHostToDevice, s));
    launch_set_xbar(s, P->n, P->xbuf[P->cur], P->xbuf[1 - P->cur], P->xbar);
    HIP_TRY(hipGetLastError());
    if (P->lu) {
        const int rc = lu_refresh_tails(P);
        if (rc) return rc;
    }
    return sync(P);
}

int gfors_reset(gfors_problem *P) {
    if (!P) return fail(GFORS_E_ARG, "NULL handle");
    hipStream_t s = P->stream;
    const int T = P->T;
    int rc;
    const float x0 = static_cast<float>(P->prm.x0);
    launch_fill_f32(s, P->xbuf[0], x0, P->n);
    launch_fill_f32(s, P->xbuf[1], x0, P->n);
    launch_fill_f32(s, P->xbar, x0, P->n);
    launch_fill_f32(s, P->ybuf[0], 0.f, P->m);
    launch_fill_f32(s, P->ybuf[1], 0.f, P->m);
    launch_fill_f32(s, P->wy, 0.f, P->m + 1);
    launch_fill_f32(s, P->xbar + P->n, 0.f, 1);
    std::vector<int64_t> zeros(T, 0), big(T, INT64_MAX), neg(T, -2);
    std::vector<int32_t> z32(T, 0);
    std::vector<int64_t> h(static_cast<size_t>(T) * P->di.hist_cap, INT64_MAX);
    std::vector<uint8_t> xb(P->n, 0);
    DevCounters c0{};
    if ((rc = upload(s, P->di.rho, P->rmin.data(), T))) return rc;
    if ((rc = upload(s, P->di.ntrig, zeros.data(), T))) return rc;
    if ((rc = upload(s, P->di.zbest, big.data(), T))) return rc;
    if ((rc = upload(s, P->di.inc_k, neg.data(), T))) return rc;
    if ((rc = upload(s, P->di.inc_round, neg.data(), T))) return rc;
    if ((rc = upload(s, P->di.inc_l, neg.data(), T))) return rc;
    if ((rc = upload(s, P->di.improved, z32.data(), T))) return rc;
    if ((rc = upload(s, P->di.hist, h.data(), static_cast<int64_t>(h.size())))) return rc;
    if ((rc = upload(s, P->xbest, xb.data(), P->n))) return rc;
    if ((rc = upload(s, P->ctr, &c0, 1))) return rc;
    HIP_TRY(hipGetLastError());
    if (P->lu && (rc = lu_refresh_tails(P))) return rc;
    return sync(P);
}

int gfors_get_candidates(gfors_problem *P, uint64_t *bits_host, int32_t *K_out) {
    if (!P) return fail(GFORS_E_ARG, "NULL handle");
    if (!P->lastK) return fail(GFORS_E_STATE, "no sampling round yet");
    if (K_out) *K_out = P->lastK;
    if (bits_host)
        HIP_TRY(hipMemcpyAsync(bits_host, P->X, P->n * (P->lastK / 64) * 8, hipMemcpyDeviceToHost, P->stream));
    return sync(P);
}

int gfors_get_scales(gfors_problem *P, double *row_scale, double *obj_scale, double *K_norm,
                     double *Q_norm, double *tau1, double *tau2, double *rho_min, double *rho_max,
                     double *rho_delta) {
    if (!P) return fail(GFORS_E_ARG, "NULL handle");
    const size_t T = P->T;
    if (row_scale) std::copy(P->rowinv.begin(), P->rowinv.end(), row_scale);
    if (obj_scale) std::copy(P->s_o.begin(), P->s_o.begin() + T, obj_scale);
    if (K_norm) std::copy(P->s_K.begin(), P->s_K.begin() + T, K_norm);
    if (Q_norm) std::copy(P->qnorm.begin(), P->qnorm.begin() + T, Q_norm);
    if (tau1) std::copy(P->tau1.begin(), P->tau1.begin() + T, tau1);
    if (tau2) std::copy(P->tau2.begin(), P->tau2.begin() + T, tau2);
    if (rho_min) std::copy(P->rmin.begin(), P->rmin.begin() + T, rho_min);
    if (rho_max) std::copy(P->rmax.begin(), P->rmax.begin() + T, rho_max);
    if (rho_delta) std::copy(P->rdelta.begin(), P->rdelta.begin() + T, rho_delta);
    return GFORS_OK;
}

int gfors_kernel_times(gfors_problem *P, int32_t nsteps, int32_t K, double *avg_ms, int32_t *launches) {
    if (!P || nsteps < 1 || !avg_ms) return fail(GFORS_E_ARG, "bad argument");
    if (!check_K(K) || K > P->prm.K_max) return fail(GFORS_E_ARG, "bad K");
    KTimer tm;
    tm.s = P->stream;
    enqueue_steps(P, nsteps, false, &tm);
    enqueue_sample_eval(P, K, nullptr, 0, &tm);
    HIP_TRY(hipGetLastError());
    int rc = sync(P);
    if (rc) return rc;
    for (int id = 0; id < GFORS_NUM_KERNEL_TIMERS; ++id) {
        double tot = 0.0;
        for (auto &p : tm.ev[id]) {
            float ms = 0.f;
            HIP_TRY(hipEventElapsedTime(&ms, p.first, p.second));
            tot += ms;
        }
        const size_t cnt = tm.ev[id].size();
        avg_ms[id] = cnt ? tot / static_cast<double>(cnt) : 0.0;
        if (launches) launches[id] = static_cast<int32_t>(cnt);
    }
    return GFORS_OK;
}

int gfors_philox_throughput(void *hip_stream, int64_t calls, void *dev_sink, double *calls_per_s) {
    if (calls <= 0 || !dev_sink || !calls_per_s) return fail(GFORS_E_ARG, "bad argument");
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    const int blocks = 8 * 256;                         // 8 workgroups of 256 lanes per CU
    const int64_t lanes = static_cast<int64_t>(blocks) * 256;
    const int64_t it64 = (calls + lanes - 1) / lanes;
    if (it64 > (1LL << 30)) return fail(GFORS_E_ARG, "calls too large");
    const int iters = static_cast<int>(it64);
    uint32_t *sink = static_cast<uint32_t *>(dev_sink);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    launch_philox_peak(s, blocks, iters, sink);        // warm-up
    HIP_TRY(hipEventRecord(e0, s));
    launch_philox_peak(s, blocks, iters, sink);
    HIP_TRY(hipEventRecord(e1, s));
    HIP_TRY(hipEventSynchronize(e1));
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
    HIP_TRY(hipEventDestroy(e0));
    HIP_TRY(hipEventDestroy(e1));
    HIP_TRY(hipGetLastError());
    *calls_per_s = ms > 0.f ? static_cast<double>(lanes) * iters / (ms * 1e-3) : 0.0;
    return GFORS_OK;
}

int gfors_read_throughput(void *hip_stream, const void *dev_buf, int64_t bytes, int32_t workgroups,
                          void *dev_sink, double *bytes_per_s) {
    if (!dev_buf || !dev_sink || !bytes_per_s || bytes <= 0 || bytes % 16 != 0 || workgroups < 1 ||
        (reinterpret_cast<uintptr_t>(dev_buf) & 15u) != 0)
        return fail(GFORS_E_ARG, "bad argument (bytes > 0 and a multiple of 16, buffer 16-byte aligned, workgroups >= 1)");
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    uint32_t *sink = static_cast<uint32_t *>(dev_sink);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    launch_read_peak(s, workgroups, dev_buf, bytes / 16, sink);   // warm-up
    HIP_TRY(hipEventRecord(e0, s));
    for (int r = 0; r < 5; ++r) launch_read_peak(s, workgroups, dev_buf, bytes / 16, sink);
    HIP_TRY(hipEventRecord(e1, s));
    HIP_TRY(hipEventSynchronize(e1));
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
    HIP_TRY(hipEventDestroy(e0));
    HIP_TRY(hipEventDestroy(e1));
    HIP_TRY(hipGetLastError());
    *bytes_per_s = ms > 0.f ? 5.0 * static_cast<double>(bytes) / (ms * 1e-3) : 0.0;
    return GFORS_OK;
}

int gfors_autotune(gfors_problem *P) {
    if (!P) return fail(GFORS_E_ARG, "NULL handle");
    if (P->lu) return GFORS_OK;   // one launch shape (the lifted rows are short)
    P->graphs_clear();
    return autotune(P, false);
}

int gfors_eval_planes(gfors_problem *P, int32_t *planes) {
    if (!P || !planes) return fail(GFORS_E_ARG, "bad argument");
    *planes = (P->mfma && (P->eval_variant == 0 || P->eval_variant == 1)) ? P->mf_npl : 0;
    return GFORS_OK;
}

int gfors_get_launch_cfg(gfors_problem *P, int32_t *out) {
    if (!P || !out) return fail(GFORS_E_ARG, "bad argument");
    out[0] = P->cfg.lpr_dual;
    out[1] = P->cfg.lpr_primal;
    out[2] = P->cfg.slices_dual;
    out[3] = P->cfg.slices_primal;
    out[4] = P->cfg.sell_dual;
    out[5] = P->cfg.sell_primal;
    out[6] = P->cfg.bits_dual;
    out[7] = P->cfg.bits_primal;
    return GFORS_OK;
}

int gfors_set_launch_cfg(gfors_problem *P, const int32_t *cfg) {
    if (!P || !cfg) return fail(GFORS_E_ARG, "bad argument");
    if (P->lu) return fail(GFORS_E_ARG, "not available on a factorised TU problem");
    auto pow2 = [](int v) { return v >= 1 && v <= 64 && (v & (v - 1)) == 0; };
    const bool fused_dual = cfg[2] == 1 && cfg[4] == 0 && cfg[6] == 0;
    const bool block_dual = fused_dual && (cfg[0] == kLprBlock || pow2(cfg[0] - kLprBlock));
    const bool block_primal = cfg[3] == 1 && cfg[5] == 0 && cfg[7] == 0 && !P->hasQ && P->m > 0 &&
                              pow2(cfg[1] - kLprBlock);
    if ((!pow2(cfg[0]) && !block_dual) || (!pow2(cfg[1]) && !block_primal))
        return fail(GFORS_E_ARG, "lanes per row must be a power of two in [1, 64], or 256 (dual only) / "
                                 "256 + a power of two (heavy rows a workgroup each) with the fused CSR "
                                 "layout, no skipping, and for the primal Q = 0");
    if (cfg[2] != 1 && !(cfg[2] == kXcdSlices && (P->slicedK || P->sellKS.ptr) && cfg[0] <= 16))
        return fail(GFORS_E_ARG, "dual slices must be 1, or 8 when the sliced copy exists (lanes <= 16)");
    if (cfg[3] != 1 && !(cfg[3] == kXcdSlices && P->slicedT && !P->hasQ && cfg[1] <= 16))
        return fail(GFORS_E_ARG, "primal slices must be 1, or 8 when the sliced copy exists, Q = 0 (lanes <= 16)");
    if (cfg[4] && !((cfg[2] == 1 && P->sellK.ptr) || (cfg[2] == kXcdSlices && P->sellKS.ptr)))
        return fail(GFORS_E_ARG, "no SELL copy of the constraint rows for this slicing");
    if (cfg[5] && !(cfg[3] == 1 && P->sellT.ptr))
        return fail(GFORS_E_ARG, "no SELL copy of the transposed rows");
    if (cfg[6] < 0 || cfg[6] > 5 || !bits_ok_dual(P, cfg[2], cfg[4], cfg[6]))
        return fail(GFORS_E_ARG, "bitmap dual: 1 needs the sliced SELL layout, 2 a SELL layout, and the slice bitmap must fit in LDS; 4 (dense-block tiles) needs rows dense over their instance's variables, <= 64 rows per instance, Q = 0, 1 slice, no SELL; 5 (light rows with signed indices) needs one instance, Q = 0, every |a| = 1 and the rows below 256 entries one range of <= 8 entries each, 1 slice, no SELL");
    if (cfg[7] < 0 || cfg[7] > 7 || !bits_ok_primal(P, cfg[3], cfg[5], cfg[7]))
        return fail(GFORS_E_ARG, "bitmap primal: 1 needs the fused CSR layout, 2 the SELL layout; both need Q = 0 and a dual bitmap that fits in LDS; 4 (wy staged in LDS) needs the fused layout, unit coefficients, every variable in the same number (<= 8) of rows, one instance and Q = 0; 6 (light variables with signed indices) as dual 5 for the variables; 7 = 6 with the heavy variables in groups of up to 16 whose rows are unit shifts of each other");
    P->cfg.lpr_dual = cfg[0];
    P->cfg.lpr_primal = cfg[1];
    P->cfg.slices_dual = cfg[2];
    P->cfg.slices_primal = cfg[3];
    P->cfg.sell_dual = cfg[4] ? 1 : 0;
    P->cfg.sell_primal = cfg[5] ? 1 : 0;
    P->cfg.bits_dual = cfg[6];
    P->cfg.bits_primal = cfg[7];
    P->graphs_clear();
    return GFORS_OK;
}

// ===========================================================================
// Learned sampling proposal (network defined in gnn.h)
// ===========================================================================
}  // extern "C"

struct gfors_gnn {
    float *theta = nullptr, *grad = nullptr, *m = nullptr, *v = nullptr;
    uint16_t *wf = nullptr, *wb = nullptr;     // BF16 operand copies (see k_gnn_pack)
    float *part = nullptr, *loss = nullptr;
    int64_t t = 0;                             // Adam steps taken
    hipStream_t stream = nullptr;
    // the parameters are shared by problems on different streams: every call
    // waits for the previous one (event) and records its own completion
    hipEvent_t ev = nullptr;
    bool ev_valid = false;
    void begin(hipStream_t s) {
        if (ev_valid) (void)hipStreamWaitEvent(s, ev, 0);
    }
    void end(hipStream_t s) {
        (void)hipEventRecord(ev, s);
        ev_valid = true;
    }
    ~gfors_gnn() {
        if (ev) (void)hipEventDestroy(ev);
    }
};

namespace {

struct GnnAct {
    uint16_t *Hv[kGnnL + 1], *Hc[kGnnL + 1], *Sc[kGnnL], *Sv[kGnnL];
    float *dHv, *dHvp, *dHc, *dHcp, *dS;
    uint16_t *dZ;
    float *logit, *p;
};

size_t gnn_ws_carve(gfors_gnn *G, Carver &cv) {
    G->theta = cv.take<float>(kGnnNumParams);
    G->grad = cv.take<float>(kGnnNumParams);
    G->m = cv.take<float>(kGnnNumParams);
    G->v = cv.take<float>(kGnnNumParams);
    G->wf = cv.take<uint16_t>(kGnnL * 2 * 128 * 64);
    G->wb = cv.take<uint16_t>(kGnnL * 2 * 128 * 64);
    G->part = cv.take<float>(static_cast<int64_t>(kGnnMaxParts) * 128 * 64);
    G->loss = cv.take<float>(4);
    return cv.off;
}

// Training keeps every round's activations; inference ping-pongs two buffers.
size_t gnn_act_carve(gfors_problem *P, bool training, GnnAct &a, Carver &cv) {
    const int64_t n = P->n, m = P->m, H = kGnnH;
    const int keep = training ? kGnnL + 1 : 2;
    for (int l = 0; l <= kGnnL; ++l) {
        a.Hv[l] = l < keep ? cv.take<uint16_t>(n * H) : a.Hv[l % 2];
        a.Hc[l] = l < keep ? cv.take<uint16_t>(std::max<int64_t>(m, 1) * H) : a.Hc[l % 2];
    }
    for (int l = 0; l < kGnnL; ++l) {
        a.Sc[l] = (training || l == 0) ? cv.take<uint16_t>(std::max<int64_t>(m, 1) * H) : a.Sc[0];
        a.Sv[l] = (training || l == 0) ? cv.take<uint16_t>(n * H) : a.Sv[0];
    }
    if (training) {
        a.dHv = cv.take<float>(n * H);
        a.dHvp = cv.take<float>(n * H);
        a.dHc = cv.take<float>(std::max<int64_t>(m, 1) * H);
        a.dHcp = cv.take<float>(std::max<int64_t>(m, 1) * H);
        a.dS = cv.take<float>(std::max(n, m) * H);
        a.dZ = cv.take<uint16_t>(std::max(n, m) * H);
    } else {
        a.dHv = a.dHvp = a.dHc = a.dHcp = a.dS = nullptr;
        a.dZ = nullptr;
    }
    a.logit = cv.take<float>(n);
    a.p = cv.take<float>(n);
    return cv.off;
}

// Forward pass; in training mode also the loss and the full backward pass
// (gradient left in G->grad).
int gnn_run(gfors_gnn *G, gfors_problem *P, const float *x, const float *y, const float *target,
            void *act, size_t act_bytes, bool training, float *p_out, float *logit_out) {
    GnnAct a;
    Carver cv{static_cast<char *>(act), 0, act_bytes};
    const uintptr_t al = reinterpret_cast<uintptr_t>(act);
    cv.off = (256 - (al & 255)) & 255;
    gnn_act_carve(P, training, a, cv);
    if (cv.off > act_bytes) return fail(GFORS_E_OOM, "GNN activation workspace too small");
    hipStream_t s = P->stream;
    G->begin(s);
    const int64_t n = P->n, m = P->m;
    const float *xs = x ? x : P->xbuf[P->cur];
    const float *ys = y ? y : P->ybuf[P->cur];
    const int *val = P->unitK ? nullptr : P->val;
    const int *valT = P->unitK ? nullptr : P->valT;
    launch_gnn_embed(s, n, m, static_cast<int>(P->m1), xs, ys, P->ct, P->rt, P->gnn_ictmax,
                     P->gnn_irtmax, G->theta, a.Hv[0], a.Hc[0]);
    for (int l = 0; l < kGnnL; ++l) {
        const float *lay = G->theta + kGnnOffLayer + l * kGnnLayerSize;
        const uint16_t *wfc = G->wf + static_cast<int64_t>(2 * l) * 128 * 64;
        const uint16_t *wfv = G->wf + static_cast<int64_t>(2 * l + 1) * 128 * 64;
        // constraint side: Hc = relu([Hc | E Hv] W + bc)
        launch_gnn_spmm(s, true, true, 0, m, P->dual_order, P->gnn_rh, P->gnn_rm, P->rp, P->ci, val,
                        P->rowinv32, a.Hv[l], a.Sc[l]);
        launch_gnn_dense_fwd(s, m, a.Hc[l], a.Sc[l], wfc, lay + 2 * 4096, a.Hc[l + 1]);
        // variable side: Hv = relu([Hv | E^T Hc] W + bv)
        launch_gnn_spmm(s, false, true, 0, n, P->primal_order, P->gnn_ch, P->gnn_cm, P->rpT, P->ciT, valT,
                        P->rowinv32, a.Hc[l + 1], a.Sv[l]);
        launch_gnn_dense_fwd(s, n, a.Hv[l], a.Sv[l], wfv, lay + 8256 + 2 * 4096, a.Hv[l + 1]);
    }
    launch_gnn_out(s, n, a.Hv[kGnnL], G->theta, logit_out ? logit_out : a.logit, p_out ? p_out : a.p,
                   training ? target : nullptr, a.dHv, G->part, kGnnMaxParts, G->grad, G->loss);
    if (!training) {
        G->end(s);
        HIP_TRY(hipGetLastError());
        return GFORS_OK;
    }
    launch_fill_f32(s, a.dHc, 0.f, std::max<int64_t>(m, 1) * kGnnH);
    for (int l = kGnnL - 1; l >= 0; --l) {
        float *glay = G->grad + kGnnOffLayer + l * kGnnLayerSize;
        const uint16_t *wbc = G->wb + static_cast<int64_t>(2 * l) * 128 * 64;
        const uint16_t *wbv = G->wb + static_cast<int64_t>(2 * l + 1) * 128 * 64;
        // variable side of round l
        launch_gnn_mask(s, n, a.dHv, a.Hv[l + 1], a.dZ, G->part, kGnnMaxParts, glay + 8256 + 2 * 4096);
        launch_gnn_wgrad(s, n, a.Hv[l], a.Sv[l], a.dZ, G->part, kGnnMaxParts, glay + 8256, glay + 8256 + 4096);
        launch_gnn_dense_bwd_in(s, n, a.dZ, wbv, a.dHvp, a.dS, 0);
        launch_gnn_spmm(s, true, false, 2, m, P->dual_order, P->gnn_rh, P->gnn_rm, P->rp, P->ci, val,
                        P->rowinv32, a.dS, a.dHc);
        // constraint side of round l
        launch_gnn_mask(s, m, a.dHc, a.Hc[l + 1], a.dZ, G->part, kGnnMaxParts, glay + 2 * 4096);
        launch_gnn_wgrad(s, m, a.Hc[l], a.Sc[l], a.dZ, G->part, kGnnMaxParts, glay, glay + 4096);
        launch_gnn_dense_bwd_in(s, m, a.dZ, wbc, a.dHcp, a.dS, 0);
        launch_gnn_spmm(s, false, false, 2, n, P->primal_order, P->gnn_ch, P->gnn_cm, P->rpT, P->ciT, valT,
                        P->rowinv32, a.dS, a.dHvp);
        std::swap(a.dHv, a.dHvp);
        std::swap(a.dHc, a.dHcp);
    }
    launch_gnn_embed_bwd(s, n, 1, static_cast<int>(P->m1), xs, P->ct, P->gnn_ictmax, a.Hv[0], a.dHv,
                         G->part, kGnnMaxParts, G->grad + kGnnOffUv, G->grad + kGnnOffuv);
    launch_gnn_embed_bwd(s, m, 0, static_cast<int>(P->m1), ys, P->rt, P->gnn_irtmax, a.Hc[0], a.dHc,
                         G->part, kGnnMaxParts, G->grad + kGnnOffUc, G->grad + kGnnOffuc);
    G->end(s);
    HIP_TRY(hipGetLastError());
    return GFORS_OK;
}

}  // namespace

extern "C" {

int gfors_gnn_workspace_bytes(size_t *bytes) {
    if (!bytes) return fail(GFORS_E_ARG, "NULL argument");
    gfors_gnn tmp;
    Carver cv{nullptr, 0, 0};
    *bytes = gnn_ws_carve(&tmp, cv) + 256;
    return GFORS_OK;
}

int gfors_gnn_create(const float *params_host, void *ws, size_t ws_bytes, void *stream,
                     gfors_gnn **out) {
    if (!params_host || !ws || !out) return fail(GFORS_E_ARG, "NULL argument");
    auto *G = new gfors_gnn();
    G->stream = static_cast<hipStream_t>(stream);
    if (hipEventCreateWithFlags(&G->ev, hipEventDisableTiming) != hipSuccess) {
        delete G;
        return fail(GFORS_E_HIP, "hipEventCreate failed");
    }
    Carver cv{static_cast<char *>(ws), 0, ws_bytes};
    cv.off = (256 - (reinterpret_cast<uintptr_t>(ws) & 255)) & 255;
    if (gnn_ws_carve(G, cv) > ws_bytes) {
        delete G;
        return fail(GFORS_E_OOM, "GNN workspace too small");
    }
    hipStream_t s = G->stream;
    std::vector<float> zero(kGnnNumParams, 0.f);
    int rc;
    if ((rc = upload(s, G->theta, params_host, kGnnNumParams)) ||
        (rc = upload(s, G->m, zero.data(), kGnnNumParams)) ||
        (rc = upload(s, G->v, zero.data(), kGnnNumParams)) ||
        (rc = upload(s, G->grad, zero.data(), kGnnNumParams))) {
        delete G;
        return rc;
    }
    launch_gnn_pack(s, G->theta, G->wf, G->wb);
    if (hipStreamSynchronize(s) != hipSuccess || hipGetLastError() != hipSuccess) {
        delete G;
        return fail(GFORS_E_HIP, "GNN creation failed");
    }
    *out = G;
    return GFORS_OK;
}

void gfors_gnn_destroy(gfors_gnn *G) { delete G; }

int gfors_gnn_act_bytes(gfors_problem *P, int32_t training, size_t *bytes) {
    if (!P || !bytes) return fail(GFORS_E_ARG, "NULL argument");
    if (P->lu) return fail(GFORS_E_ARG, "not available on a factorised TU problem");
    if (P->T != 1) return fail(GFORS_E_ARG, "the learned proposal runs on single-instance problems");
    GnnAct a;
    Carver cv{nullptr, 0, 0};
    *bytes = gnn_act_carve(P, training != 0, a, cv) + 256;
    return GFORS_OK;
}

int gfors_gnn_forward(gfors_gnn *G, gfors_problem *P, const float *x_dev, const float *y_dev,
                      void *act, size_t act_bytes, float *p_dev, float *logit_dev) {
    if (!G || !P || !act || !p_dev) return fail(GFORS_E_ARG, "NULL argument");
    if (P->lu) return fail(GFORS_E_ARG, "not available on a factorised TU problem");
    if (P->T != 1) return fail(GFORS_E_ARG, "the learned proposal runs on single-instance problems");
    return gnn_run(G, P, x_dev, y_dev, nullptr, act, act_bytes, false, p_dev, logit_dev);
}

int gfors_gnn_grad(gfors_gnn *G, gfors_problem *P, const float *x_dev, const float *y_dev,
                   const float *target_dev, void *act, size_t act_bytes, float *loss_host) {
    if (!G || !P || !act || !target_dev) return fail(GFORS_E_ARG, "NULL argument");
    if (P->lu) return fail(GFORS_E_ARG, "not available on a factorised TU problem");
    if (P->T != 1) return fail(GFORS_E_ARG, "the learned proposal runs on single-instance problems");
    int rc = gnn_run(G, P, x_dev, y_dev, target_dev, act, act_bytes, true, nullptr, nullptr);
    if (rc) return rc;
    if (loss_host) {
        HIP_TRY(hipMemcpyAsync(loss_host, G->loss, sizeof(float), hipMemcpyDeviceToHost, P->stream));
        return sync(P);
    }
    return GFORS_OK;
}

static int gnn_adam_on(gfors_gnn *G, hipStream_t s, float lr);

int gfors_gnn_adam(gfors_gnn *G, float lr) {
    if (!G || !(lr > 0.f)) return fail(GFORS_E_ARG, "bad argument");
    return gnn_adam_on(G, G->stream, lr);
}

static int gnn_adam_on(gfors_gnn *G, hipStream_t s, float lr) {
    G->begin(s);
    G->t += 1;
    const double b1 = 0.9, b2 = 0.999;
    const float c1 = static_cast<float>(1.0 - std::pow(b1, static_cast<double>(G->t)));
    const float c2 = static_cast<float>(1.0 - std::pow(b2, static_cast<double>(G->t)));
    launch_gnn_adam(s, kGnnNumParams, G->theta, G->grad, G->m, G->v, lr, 0.9f, 0.999f, 1e-8f, c1, c2);
    launch_gnn_pack(s, G->theta, G->wf, G->wb);
    G->end(s);
    HIP_TRY(hipGetLastError());
    return GFORS_OK;
}

int gfors_gnn_train_step(gfors_gnn *G, gfors_problem *P, const float *x_dev, const float *y_dev,
                         const float *target_dev, void *act, size_t act_bytes, float lr,
                         float *loss_host) {
    if (!(lr > 0.f)) return fail(GFORS_E_ARG, "bad learning rate");
    int rc = gfors_gnn_grad(G, P, x_dev, y_dev, target_dev, act, act_bytes, loss_host);
    if (rc) return rc;
    return gnn_adam_on(G, P->stream, lr);
}

int gfors_gnn_get_params(gfors_gnn *G, float *host) {
    if (!G || !host) return fail(GFORS_E_ARG, "NULL argument");
    G->begin(G->stream);
    HIP_TRY(hipMemcpyAsync(host, G->theta, kGnnNumParams * sizeof(float), hipMemcpyDeviceToHost, G->stream));
    HIP_TRY(hipStreamSynchronize(G->stream));
    return GFORS_OK;
}

int gfors_gnn_set_params(gfors_gnn *G, const float *host) {
    if (!G || !host) return fail(GFORS_E_ARG, "NULL argument");
    G->begin(G->stream);
    HIP_TRY(hipMemcpyAsync(G->theta, host, kGnnNumParams * sizeof(float), hipMemcpyHostToDevice, G->stream));
    launch_gnn_pack(G->stream, G->theta, G->wf, G->wb);
    HIP_TRY(hipStreamSynchronize(G->stream));
    return GFORS_OK;
}

int gfors_gnn_get_grad(gfors_gnn *G, float *host) {
    if (!G || !host) return fail(GFORS_E_ARG, "NULL argument");
    G->begin(G->stream);
    HIP_TRY(hipMemcpyAsync(host, G->grad, kGnnNumParams * sizeof(float), hipMemcpyDeviceToHost, G->stream));
    HIP_TRY(hipStreamSynchronize(G->stream));
    return GFORS_OK;
}

int gfors_gnn_set_grad(gfors_gnn *G, const float *host) {
    if (!G || !host) return fail(GFORS_E_ARG, "NULL argument");
    G->begin(G->stream);
    HIP_TRY(hipMemcpyAsync(G->grad, host, kGnnNumParams * sizeof(float), hipMemcpyHostToDevice, G->stream));
    HIP_TRY(hipStreamSynchronize(G->stream));
    return GFORS_OK;
}

int gfors_get_dims(gfors_problem *P, int64_t *n, int64_t *m1, int64_t *m2, int32_t *T) {
    if (!P) return fail(GFORS_E_ARG, "NULL handle");
    if (n) *n = P->n;
    if (m1) *m1 = P->m1;
    if (m2) *m2 = P->m2;
    if (T) *T = P->T;
    return GFORS_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Problems whose device memory is a file-scope array instead of a caller
// workspace, for callers that cannot allocate device memory.  Each GPU the
// library runs on holds one copy of the array for the life of the process and
// serves at most one live problem at a time.
static __device__ __align__(256) unsigned char scratch[GFORS_STATIC_WS_BYTES];

namespace {
struct StaticWs {
    unsigned char *ptr = nullptr;        // device address of this device's copy of `scratch`
    const gfors_problem *owner = nullptr;
};
std::mutex g_static_mu;
std::map<int, StaticWs> g_static;        // by HIP device ordinal
}  // namespace

static void static_ws_release(gfors_problem *P) {
    if (P->static_dev < 0) return;
    std::lock_guard<std::mutex> lk(g_static_mu);
    auto it = g_static.find(P->static_dev);
    if (it != g_static.end() && it->second.owner == P) it->second.owner = nullptr;
    P->static_dev = -1;
}

extern "C" {

int gfors_create_problem_static(const gfors_csr *A, const int64_t *b, const gfors_csr *B,
                                const int64_t *d, const gfors_csr *Q, const int64_t *c, int64_t n,
                                int32_t num_instances, const int64_t *inst_offsets,
                                const gfors_params *prm, void *stream, gfors_problem **out) {
    if (!out || !prm || !c || n <= 0 || num_instances < 1)
        return fail(GFORS_E_ARG, "gfors_create_problem_static: NULL argument or n <= 0");
    *out = nullptr;
    int rc;
    if ((rc = validate_csr(A, n, "A"))) return rc;
    if ((rc = validate_csr(B, n, "B"))) return rc;
    if ((rc = validate_csr(Q, n, "Q"))) return rc;
    const int64_t m1 = A ? A->nrows : 0, m2 = B ? B->nrows : 0;
    const int64_t nnzA = A ? A->row_ptr[A->nrows] : 0, nnzB = B ? B->row_ptr[B->nrows] : 0;
    const int64_t nnzQ = Q ? Q->row_ptr[Q->nrows] : 0;
    // the launch shapes come from the size heuristic: the autotuner's timing
    // events are runtime objects this entry point does not create
    gfors_params p = *prm;
    p.autotune = 0;
    size_t need = 0;
    if ((rc = gfors_workspace_bytes(n, m1, m2, nnzA, nnzB, nnzQ, num_instances, &p, &need))) return rc;
    if (need > sizeof(scratch))
        return fail(GFORS_E_OOM, "gfors_create_problem_static: the problem needs " + std::to_string(need) +
                                     " bytes of device memory; the static workspace holds " +
                                     std::to_string(sizeof(scratch)) + " (GFORS_STATIC_WS_BYTES)");
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    unsigned char *base = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_static_mu);
        StaticWs &w = g_static[dev];
        if (!w.ptr) {
            // once per device, with that device current: the array's device address
            void *ptr = nullptr;
            HIP_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
            if (!ptr) return fail(GFORS_E_HIP, "hipGetSymbolAddress returned NULL for the static workspace");
            w.ptr = static_cast<unsigned char *>(ptr);
        }
        if (w.owner)
            return fail(GFORS_E_STATE, "gfors_create_problem_static: the static workspace of device " +
                                           std::to_string(dev) + " holds a live problem; destroy it first");
        base = w.ptr;
        w.owner = reinterpret_cast<const gfors_problem *>(&w);   // reserved while creating
    }
    gfors_problem *P = nullptr;
    rc = gfors_create_problem(A, b, B, d, Q, c, n, num_instances, inst_offsets, &p, base, sizeof(scratch),
                              stream, &P);
    std::lock_guard<std::mutex> lk(g_static_mu);
    StaticWs &w = g_static[dev];
    if (rc != GFORS_OK) {
        w.owner = nullptr;
        return rc;
    }
    P->static_dev = dev;
    w.owner = P;
    *out = P;
    return GFORS_OK;
}

}  // extern "C"

namespace gfh {
size_t carve_problem(gfors_problem *P, Carver &cv, int64_t n, int64_t m1, int64_t m2,
                     int64_t nnzK, int64_t nnzQ, int T, const gfors_params *prm) {
    return carve(P, cv, n, m1, m2, nnzK, nnzQ, T, prm);
}
bool k_ok(int64_t K) { return check_K(K) != 0; }
}  // namespace gfh
