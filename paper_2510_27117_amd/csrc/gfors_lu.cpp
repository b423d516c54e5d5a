// Device problems in the factorised TU form (Theorem and Remark of Sec.
// 2.4.1): gfors_create_problem_tu builds a GFORS problem on the kept variables
// of a GFORS_TU_FACTORED handle whose reformulated rows are applied through
// the LU of the pivot block at every step, and the Algorithm 1 pieces that
// differ from the explicit form:
//   * Preprocess: the reformulated rows' 2-norms come exactly from the host;
//     ||K'|| and ||Q'|| by FP64 power iteration with lifted products;
//   * FirstOrderStep: the dual step is the ordinary fused kernel on the lifted
//     rows (the lifted part of xbar is kept current); the primal step adds
//     S^T of the pivot part of the gradient (two transposed solves) and lifts
//     the new x_k (two solves);
//   * residuals (Theorem 2) on FP64 lifts;
//   * EvalBest: each candidate's pivot variables are solved for exactly in
//     int32 and the rows are checked on the lifted integer point.
#include "gfors_host.h"
#include "gfors_lu.h"

#include <limits>

using namespace gfors;
using namespace gfh;

namespace gfh {

struct LuDevSolve {
    int *row = nullptr, *ptr = nullptr, *ent = nullptr, *lvl = nullptr;
    std::vector<LuSeg> seg;
    std::vector<int> hlvl, hptr_at_lvl;   // host: level starts, entry start of each level
    int r = 0, use_lds = 1;
    LuSolve view() const {
        LuSolve v;
        v.r = r;
        v.use_lds = use_lds;
        v.nseg = static_cast<int>(seg.size());
        v.row = row;
        v.ptr = ptr;
        v.ent = ent;
        v.lvl = lvl;
        v.seg = seg.data();
        v.hlvl = hlvl.data();
        v.hptr_at_lvl = hptr_at_lvl.data();
        return v;
    }
};

struct LuForm {
    int64_t nk = 0, r = 0, nfull = 0;
    bool hasQ = false;
    int *BJrp = nullptr, *BJci = nullptr, *BJval = nullptr;
    int *BJTrp = nullptr, *BJTci = nullptr, *BJTval = nullptr;
    int64_t *dJ = nullptr;
    LuDevSolve Lf, Ub, Utf, Ltb;
    float *v32 = nullptr;                          // pivot part of the gradient (r)
    double *w64a = nullptr, *w64b = nullptr, *w64c = nullptr;   // FP64 lifted work vectors (nfull)
    int *XI = nullptr;                             // candidates' pivot values, r x K
    int64_t *rhs_orig = nullptr;
    // evaluation chunks of the lifted rows; rows in several chunks get a slot
    int nch = 0, nslot = 0;
    int *ch_row = nullptr, *ch_e0 = nullptr, *ch_e1 = nullptr, *ch_slot = nullptr, *slot_row = nullptr;
    int64_t *rsum = nullptr;
    // chunks of the lifted Q rows (objective)
    int nqch = 0;
    int *qch_row = nullptr, *qch_e0 = nullptr, *qch_e1 = nullptr;
    int64_t *c_tail = nullptr;
    int64_t c0 = 0;
    int lpr_dual = 1, lpr_bj = 1, lpr_bjt = 1, lpr_tail = 1, lpr_primal = 1;
    int heavy_rows = 0;   // lifted rows of kHeavyLen+ entries (a prefix of dual_order)
    // their chunks of kLuRowChunk entries (a workgroup each) and chunk sums
    int nhch = 0;
    int *hch_row = nullptr, *hch_e0 = nullptr, *hch_e1 = nullptr, *hch_first = nullptr;
    float *hpart = nullptr;
    std::vector<int> h_hch_row, h_hch_e0, h_hch_e1, h_hch_first;
    // host copies
    std::vector<int> h_ch_row, h_ch_e0, h_ch_e1, h_ch_slot, h_slot_row, h_qch_row, h_qch_e0, h_qch_e1;
};

void lu_destroy(LuForm *L) { delete L; }

}  // namespace gfh

namespace {

constexpr int kLuChunk = 256;      // entries per evaluation chunk of a row (a wavefront each)
constexpr int kLuRowChunk = 4096;  // entries per chunk of a long row in the dual step (a workgroup each)

int pick_lpr(double avg) {
    if (avg >= 48) return 64;
    if (avg >= 12) return 16;
    if (avg >= 3) return 4;
    return 1;
}

// Runs of the level order: a level of `wide` rows or more is a launch of its
// own, consecutive narrower levels share one one-workgroup launch.
std::vector<LuSeg> plan_segments(const std::vector<int32_t> &lvl, int wide) {
    std::vector<LuSeg> seg;
    const int nl = static_cast<int>(lvl.size()) - 1;
    int l = 0;
    while (l < nl) {
        if (lvl[l + 1] - lvl[l] >= wide) {
            seg.push_back({1, lvl[l], lvl[l + 1]});
            ++l;
            continue;
        }
        int e = l;
        while (e < nl && lvl[e + 1] - lvl[e] < wide) ++e;
        seg.push_back({0, l, e});
        l = e;
    }
    return seg;
}

void chunk_rows(const std::vector<int32_t> &rp, std::vector<int> &row, std::vector<int> &e0,
                std::vector<int> &e1, std::vector<int> *slot, std::vector<int> *slot_row, bool skip_empty) {
    const int64_t nr = static_cast<int64_t>(rp.size()) - 1;
    for (int64_t j = 0; j < nr; ++j) {
        const int b0 = rp[j], b1 = rp[j + 1];
        if (b1 == b0 && skip_empty) continue;
        const bool multi = b1 - b0 > kLuChunk;
        const int sl = multi ? static_cast<int>(slot_row->size()) : -1;
        if (multi) slot_row->push_back(static_cast<int>(j));
        int a = b0;
        do {
            const int b = std::min(b1, a + kLuChunk);
            row.push_back(static_cast<int>(j));
            e0.push_back(a);
            e1.push_back(b);
            if (slot) slot->push_back(sl);
            a = b;
        } while (a < b1);
    }
}

gfors_params lu_params(const gfors_params *prm) {
    gfors_params p = *prm;
    p.eval_mfma = 0;
    p.repair_row0 = -1;
    return p;
}

// Every device buffer of a factorised problem (measure mode without a base).
size_t lu_carve(gfors_problem *P, Carver &cv, const gftu::TuFactored &F, const gfors_params &prm) {
    LuForm &L = *P->lu;
    const int64_t nk = F.nk, r = F.r, nfull = nk + r;
    const int64_t m1 = F.mA + F.nlow + F.nup, m2 = F.mB, m = m1 + m2;
    const int64_t nnzK = static_cast<int64_t>(F.KLci.size()), nnzQ = static_cast<int64_t>(F.QLci.size());
    carve_problem(P, cv, nfull, m1, m2, nnzK, nnzQ, 1, &prm);
    const Bounds bnd = tile_bounds(nfull, m, nnzK, nnzQ, 1);
    carve_tiles(cv, P->st, P->st.count, bnd.st, 1);
    carve_tiles(cv, P->et, 1, 1, 1);
    carve_tiles(cv, P->qt, 1, 1, 1);
    carve_tiles(cv, P->vt, P->vt.count, bnd.vt, 1);
    carve_tiles(cv, P->rtile, P->rtile.count, bnd.rt, 1);
    const int64_t nbj = static_cast<int64_t>(F.BJci.size());
    L.BJrp = cv.take<int>(r + 1);
    L.BJci = cv.take<int>(nbj);
    L.BJval = cv.take<int>(nbj);
    L.BJTrp = cv.take<int>(nk + 1);
    L.BJTci = cv.take<int>(nbj);
    L.BJTval = cv.take<int>(nbj);
    L.dJ = cv.take<int64_t>(r);
    const gftu::HostTrsv *hs[4] = {&F.Lf, &F.Ub, &F.Utf, &F.Ltb};
    LuDevSolve *ds[4] = {&L.Lf, &L.Ub, &L.Utf, &L.Ltb};
    for (int q = 0; q < 4; ++q) {
        ds[q]->row = cv.take<int>(r);
        ds[q]->ptr = cv.take<int>(r + 1);
        ds[q]->ent = cv.take<int>(static_cast<int64_t>(hs[q]->ent.size()));
        ds[q]->lvl = cv.take<int>(static_cast<int64_t>(hs[q]->lvl.size()));
    }
    L.v32 = cv.take<float>(r);
    L.w64a = cv.take<double>(nfull);
    L.w64b = cv.take<double>(nfull);
    L.w64c = cv.take<double>(nfull);
    L.XI = cv.take<int>(r * prm.K_max);
    L.rhs_orig = cv.take<int64_t>(m);
    L.ch_row = cv.take<int>(L.nch);
    L.ch_e0 = cv.take<int>(L.nch);
    L.ch_e1 = cv.take<int>(L.nch);
    L.ch_slot = cv.take<int>(L.nch);
    L.slot_row = cv.take<int>(L.nslot);
    L.rsum = cv.take<int64_t>(static_cast<int64_t>(L.nslot) * prm.K_max);
    L.qch_row = cv.take<int>(L.nqch);
    L.qch_e0 = cv.take<int>(L.nqch);
    L.qch_e1 = cv.take<int>(L.nqch);
    L.c_tail = cv.take<int64_t>(r);
    L.hch_row = cv.take<int>(L.nhch);
    L.hch_e0 = cv.take<int>(L.nhch);
    L.hch_e1 = cv.take<int>(L.nhch);
    L.hch_first = cv.take<int>(L.heavy_rows + 1);
    L.hpart = cv.take<float>(L.nhch);
    return cv.off;
}

// Host-side plan shared by the size query and the creation.
void lu_plan(gfors_problem *P, const gftu::TuFactored &F, const gfors_params &prm) {
    LuForm &L = *P->lu;
    L.nk = F.nk;
    L.r = F.r;
    L.nfull = F.nk + F.r;
    L.hasQ = !F.QLci.empty();
    chunk_rows(F.KLrp, L.h_ch_row, L.h_ch_e0, L.h_ch_e1, &L.h_ch_slot, &L.h_slot_row, false);
    std::vector<int> dummy;
    chunk_rows(F.QLrp, L.h_qch_row, L.h_qch_e0, L.h_qch_e1, nullptr, &dummy, true);
    L.nch = static_cast<int>(L.h_ch_row.size());
    {
        // long lifted rows (kHeavyLen+ entries), longest first, and their chunks
        const int64_t m = static_cast<int64_t>(F.KLrp.size()) - 1;
        std::vector<int> ord(m);
        for (int64_t j = 0; j < m; ++j) ord[j] = static_cast<int>(j);
        std::stable_sort(ord.begin(), ord.end(), [&](int a2, int b2) {
            return F.KLrp[a2 + 1] - F.KLrp[a2] > F.KLrp[b2 + 1] - F.KLrp[b2];
        });
        L.heavy_rows = 0;
        while (L.heavy_rows < m && F.KLrp[ord[L.heavy_rows] + 1] - F.KLrp[ord[L.heavy_rows]] >= kHeavyLen) ++L.heavy_rows;
        L.h_hch_first.assign(1, 0);
        for (int h = 0; h < L.heavy_rows; ++h) {
            const int j = ord[h];
            for (int e = F.KLrp[j]; e < F.KLrp[j + 1]; e += kLuRowChunk) {
                L.h_hch_row.push_back(j);
                L.h_hch_e0.push_back(e);
                L.h_hch_e1.push_back(std::min(F.KLrp[j + 1], e + kLuRowChunk));
            }
            L.h_hch_first.push_back(static_cast<int>(L.h_hch_row.size()));
        }
        L.nhch = static_cast<int>(L.h_hch_row.size());
    }
    L.nslot = static_cast<int>(L.h_slot_row.size());
    L.nqch = static_cast<int>(L.h_qch_row.size());
    const gftu::HostTrsv *hs[4] = {&F.Lf, &F.Ub, &F.Utf, &F.Ltb};
    LuDevSolve *ds[4] = {&L.Lf, &L.Ub, &L.Utf, &L.Ltb};
    for (int q = 0; q < 4; ++q) {
        // a solve with no entries and a unit diagonal is the identity: nothing to launch
        bool ident = hs[q]->ent.empty();
        for (size_t p = 0; p < hs[q]->row.size() && ident; ++p) ident = (hs[q]->row[p] & 1) == 0;
        ds[q]->seg = ident ? std::vector<LuSeg>() : plan_segments(hs[q]->lvl, std::max(1, prm.lu_wide_rows));
        ds[q]->r = static_cast<int>(F.r);
        ds[q]->use_lds = prm.lu_lds ? 1 : 0;
        ds[q]->hlvl.assign(hs[q]->lvl.begin(), hs[q]->lvl.end());
        ds[q]->hptr_at_lvl.resize(hs[q]->lvl.size());
        for (size_t l = 0; l < hs[q]->lvl.size(); ++l) ds[q]->hptr_at_lvl[l] = hs[q]->ptr[hs[q]->lvl[l]];
    }
    HostTiles hs_, hv;
    build_tiles_items(hs_, 0, ceil_div(F.nk, 4), nullptr, kSampleTQ, kSampleTQ, 0);
    build_tiles_items(hv, 0, F.nk, nullptr, kVarTile, kVarTile, 0);
    P->st.count = static_cast<int32_t>(hs_.inst.size());
    P->vt.count = static_cast<int32_t>(hv.inst.size());
    const int64_t m = F.mA + F.nlow + F.nup + F.mB;
    HostTiles hr;
    std::function<int64_t(int64_t)> wr = [&](int64_t q) -> int64_t { return F.KLrp[q + 1] - F.KLrp[q]; };
    build_tiles_items(hr, 0, m, &wr, kRowNnz, kRowRows, 0);
    P->rtile.count = static_cast<int32_t>(hr.inst.size());
}

// x (nfull, FP64): x[nk..) = M^{-1} (-B_JIbar x[0..nk)) = S x[0..nk)
void lift64(gfors_problem *P, double *x) {
    LuForm &L = *P->lu;
    hipStream_t s = P->stream;
    launch_lu_mv_f64(s, L.lpr_bj, static_cast<int>(L.r), L.BJrp, L.BJci, L.BJval, x, x + L.nk, -1.0, false);
    launch_lu_trsv<double>(s, L.Lf.view(), x + L.nk);
    launch_lu_trsv<double>(s, L.Ub.view(), x + L.nk);
}
// x (nfull, FP64): x[0..nk) += S^T x[nk..) = -B_JIbar^T M^{-T} x[nk..) (the tail is overwritten)
void project64(gfors_problem *P, double *x) {
    LuForm &L = *P->lu;
    hipStream_t s = P->stream;
    launch_lu_trsv<double>(s, L.Utf.view(), x + L.nk);
    launch_lu_trsv<double>(s, L.Ltb.view(), x + L.nk);
    launch_lu_mv_f64(s, L.lpr_bjt, static_cast<int>(L.nk), L.BJTrp, L.BJTci, L.BJTval, x + L.nk, x, -1.0, true);
}
// FP32 lift of an iterate in place (x[nk..) = S x[0..nk)).
void lift32(gfors_problem *P, float *x) {
    LuForm &L = *P->lu;
    hipStream_t s = P->stream;
    launch_lu_mv_f32(s, L.lpr_bj, static_cast<int>(L.r), L.BJrp, L.BJci, L.BJval, x, x + L.nk, -1.f);
    launch_lu_trsv<float>(s, L.Lf.view(), x + L.nk);
    launch_lu_trsv<float>(s, L.Ub.view(), x + L.nk);
}

// Preprocess norms (Sec. 3) of the reformulated data by FP64 power iteration
// (v <- M^T M v / ||.||, then ||M v||) with lifted products:
//   K' row-normalised: M^T M v = project(KL^T (rowinv^2 o KL lift(v))),
//   Q':                M^T M v = Q'(Q' v),  Q' v = project(QL lift(v)).
int lu_device_norms(gfors_problem *P) {
    LuForm &L = *P->lu;
    hipStream_t s = P->stream;
    const int nk = static_cast<int>(L.nk), nfull = static_cast<int>(L.nfull), m = static_cast<int>(P->m);
    double *v = L.w64a, *u = L.w64b, *w = L.w64c;
    auto init_v = [&](double *x) { launch_fill64(s, x, 1.0 / std::sqrt(static_cast<double>(nk)), nk); };
    if (P->nnzK > 0 && m > 0) {
        init_v(v);
        for (int it = 0; it < P->prm.power_iters; ++it) {
            lift64(P, v);
            launch_spmv64(s, m, P->rp, P->ci, P->val, P->rowinv2_d, v, P->pw);
            launch_spmv64(s, nfull, P->rpT, P->ciT, P->valT, nullptr, P->pw, u);
            project64(P, u);
            launch_tile_sumsq(s, P->vt, u, P->part);
            launch_inst_sum(s, 1, P->vt, P->part, 1, 0, P->dnorm, 1, true);
            launch_tile_scale_inv(s, P->vt, u, P->dnorm);
            std::swap(u, v);
        }
        lift64(P, v);
        launch_spmv64(s, m, P->rp, P->ci, P->val, P->rowinv_d, v, P->pw);
        launch_tile_sumsq(s, P->rtile, P->pw, P->part);
        launch_inst_sum(s, 1, P->rtile, P->part, 1, 0, P->dnorm, 1, true);
    } else {
        launch_fill64(s, P->dnorm, 0.0, 1);
    }
    if (L.hasQ) {
        init_v(v);
        for (int it = 0; it < P->prm.power_iters; ++it) {
            lift64(P, v);
            launch_spmv64(s, nfull, P->rpQ, P->ciQ, P->valQ, nullptr, v, w);
            project64(P, w);
            lift64(P, w);
            launch_spmv64(s, nfull, P->rpQ, P->ciQ, P->valQ, nullptr, w, u);
            project64(P, u);
            launch_tile_sumsq(s, P->vt, u, P->part);
            launch_inst_sum(s, 1, P->vt, P->part, 1, 0, P->dnorm + 1, 1, true);
            launch_tile_scale_inv(s, P->vt, u, P->dnorm + 1);
            std::swap(u, v);
        }
        lift64(P, v);
        launch_spmv64(s, nfull, P->rpQ, P->ciQ, P->valQ, nullptr, v, w);
        project64(P, w);
        launch_tile_sumsq(s, P->vt, w, P->part);
        launch_inst_sum(s, 1, P->vt, P->part, 1, 0, P->dnorm + 1, 1, true);
    } else {
        launch_fill64(s, P->dnorm + 1, 0.0, 1);
    }
    HIP_TRY(hipGetLastError());
    return GFORS_OK;
}

// Lanes per row of the SpMV-like kernels of a step, timed on the problem
// (HIP events, 5 launches each after one untimed); the state is reset after.
int lu_autotune(gfors_problem *P) {
    LuForm &L = *P->lu;
    hipStream_t s = P->stream;
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    auto timeit = [&](const std::function<void()> &f) -> float {
        f();
        (void)hipEventRecord(e0, s);
        for (int q = 0; q < 5; ++q) f();
        (void)hipEventRecord(e1, s);
        (void)hipEventSynchronize(e1);
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        return ms;
    };
    const int nk = static_cast<int>(L.nk), r = static_cast<int>(L.r), m = static_cast<int>(P->m);
    const int m1 = static_cast<int>(P->m1);
    const float tau2 = static_cast<float>(P->tau2[0]);
    auto best_of = [&](std::initializer_list<int> opts, int &slot, const std::function<void(int)> &run) {
        float bt = 1e30f;
        int bl = slot;
        for (int l : opts) {
            const float t = timeit([&] { run(l); });
            if (t < bt) { bt = t; bl = l; }
        }
        slot = bl;
    };
    if (m > L.heavy_rows)
        best_of({1, 2, 4, 8, 16, 32, 64}, L.lpr_dual, [&](int l) {
            launch_dual(s, l, false, false, m, m1, P->rp, P->ci, P->val, nullptr, P->omega, P->rt, P->xbar,
                        P->ybuf[0], P->ybuf[1], P->wy, tau2, P->di.tau2, P->row_inst, L.heavy_rows > 0 ? kHeavyLen : 0);
        });
    if (r > 0) {
        best_of({1, 4, 16, 64}, L.lpr_tail, [&](int l) {
            launch_lu_tail_grad(s, l, L.hasQ, r, nk, P->rpT, P->ciT, P->valT, P->wy, P->rpQ, P->ciQ, P->valQ,
                                P->xbuf[0], P->di.two_so, L.v32);
        });
        best_of({1, 4, 16, 64}, L.lpr_bj, [&](int l) {
            launch_lu_mv_f32(s, l, r, L.BJrp, L.BJci, L.BJval, P->xbuf[0], P->xbuf[1] + nk, -1.f);
        });
    }
    best_of({1, 4, 16, 64}, L.lpr_primal, [&](int l) {
        launch_lu_primal(s, l, L.hasQ, nk, P->rpT, P->ciT, P->valT, P->wy, P->rpQ, P->ciQ, P->valQ, L.BJTrp,
                         L.BJTci, L.BJTval, L.v32, P->xbuf[0], P->xbuf[1], P->xbar, P->ct, P->di.tau1,
                         P->di.two_so, P->di.rho, P->ctr_scratch);
    });
    HIP_TRY(hipGetLastError());
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return sync(P);
}

}  // namespace

namespace gfh {

// The lifted parts of x_k, x_{k-1} and xbar after the host replaced the iterate.
int lu_refresh_tails(gfors_problem *P) {
    LuForm &L = *P->lu;
    lift32(P, P->xbuf[0]);
    lift32(P, P->xbuf[1]);
    launch_lu_xbar_tail(P->stream, static_cast<int>(L.r), static_cast<int>(L.nk), P->xbuf[P->cur],
                        P->xbuf[1 - P->cur], P->xbar);
    HIP_TRY(hipGetLastError());
    return GFORS_OK;
}

void lu_enqueue_steps(gfors_problem *P, int nsteps, bool want_res, KTimer *tm) {
    LuForm &L = *P->lu;
    hipStream_t s = P->stream;
    const int nk = static_cast<int>(L.nk), r = static_cast<int>(L.r), m = static_cast<int>(P->m);
    const int m1 = static_cast<int>(P->m1), nfull = static_cast<int>(L.nfull);
    const float tau2 = static_cast<float>(P->tau2[0]);
    for (int it = 0; it < nsteps; ++it) {
        const bool res = want_res && it == nsteps - 1;
        if (res) launch_copy_f32(s, P->xsave, P->xbar, nfull);
        const int a = P->cur, bn = 1 - P->cur;
        TB(0);
        if (m > 0) {
            if (L.heavy_rows > 0)
                launch_lu_dual_heavy(s, L.nhch, L.heavy_rows, m1, L.hch_row, L.hch_e0, L.hch_e1, L.hch_first,
                                     P->dual_order, P->rowc0, P->rp, P->ci, P->val, P->xbar, L.hpart, P->omega,
                                     P->rt, tau2, P->ybuf[a], P->ybuf[bn], P->wy);
            if (L.heavy_rows < m)
                launch_dual(s, L.lpr_dual, false, false, m, m1, P->rp, P->ci, P->val, nullptr, P->omega, P->rt,
                            P->xbar, P->ybuf[a], P->ybuf[bn], P->wy, tau2, P->di.tau2, P->row_inst,
                            L.heavy_rows > 0 ? kHeavyLen : 0);
        }
        TE(0);
        TB(1);
        launch_lu_tail_grad(s, L.lpr_tail, L.hasQ, r, nk, P->rpT, P->ciT, P->valT, P->wy, P->rpQ, P->ciQ,
                            P->valQ, P->xbuf[a], P->di.two_so, L.v32);
        launch_lu_trsv<float>(s, L.Utf.view(), L.v32);
        launch_lu_trsv<float>(s, L.Ltb.view(), L.v32);
        launch_lu_primal(s, L.lpr_primal, L.hasQ, nk, P->rpT, P->ciT, P->valT, P->wy, P->rpQ, P->ciQ, P->valQ,
                         L.BJTrp, L.BJTci, L.BJTval, L.v32, P->xbuf[a], P->xbuf[bn], P->xbar, P->ct,
                         P->di.tau1, P->di.two_so, P->di.rho, P->ctr);
        // lift of x_k; the last run also writes xbar's lifted part 2 t(x_k) - t(x_{k-1})
        launch_lu_mv_f32(s, L.lpr_bj, r, L.BJrp, L.BJci, L.BJval, P->xbuf[bn], P->xbuf[bn] + nk, -1.f);
        launch_lu_trsv<float>(s, L.Lf.view(), P->xbuf[bn] + nk);
        launch_lu_trsv<float>(s, L.Ub.view(), P->xbuf[bn] + nk, P->xbuf[a] + nk, P->xbar + nk);
        TE(1);
        if (res) {
            // s^y and the primal gap on lift(xbar_{k-1} - x_k), lift(x_k)
            launch_lu_diff64(s, nk, P->xsave, P->xbuf[bn], L.w64a);
            lift64(P, L.w64a);
            launch_lu_diff64(s, nk, P->xbuf[bn], nullptr, L.w64b);
            lift64(P, L.w64b);
            if (m > 0) {
                launch_lu_res_rows(s, P->rtile, m1, P->rp, P->ci, P->val, P->omega64, P->rhs, L.w64a, L.w64b,
                                   P->ybuf[a], P->ybuf[bn], P->di.tau2d, P->part);
                launch_inst_sum(s, 1, P->rtile, P->part, 2, 0, P->res + 1, 4, true);
                launch_inst_sum(s, 1, P->rtile, P->part, 2, 1, P->res + 2, 4, true);
            } else {
                launch_fill64(s, P->res + 1, 0.0, 2);
            }
            // s^x with (Q' dx) = project(QL lift(x_k - x_{k-1}))
            const double *qd = nullptr;
            if (L.hasQ) {
                launch_lu_diff64(s, nk, P->xbuf[bn], P->xbuf[a], L.w64c);
                lift64(P, L.w64c);
                launch_spmv64(s, nfull, P->rpQ, P->ciQ, P->valQ, nullptr, L.w64c, L.w64a);
                project64(P, L.w64a);
                qd = L.w64a;
            }
            launch_lu_res_vars(s, P->vt, qd, P->xbuf[bn], P->xbuf[a], P->di.rho, P->di.tau1d, P->di.two_sod,
                               P->part);
            launch_inst_sum(s, 1, P->vt, P->part, 2, 0, P->res + 0, 4, true);
            launch_inst_sum(s, 1, P->vt, P->part, 2, 1, P->res + 3, 4, false);
        }
        P->cur = bn;
    }
}

void lu_enqueue_eval(gfors_problem *P, int K, int threshold, KTimer *tm, int trigger) {
    LuForm &L = *P->lu;
    hipStream_t s = P->stream;
    const int W = K / 64, r = static_cast<int>(L.r), nk = static_cast<int>(L.nk);
    TB(3);
    launch_lu_fill_i32(s, P->vpart, 0, K);
    launch_lu_eval_rhs(s, r, K, L.BJrp, L.BJci, L.BJval, L.dJ, P->X, L.XI);
    launch_lu_trsm(s, L.Lf.view(), L.XI, K);
    launch_lu_trsm(s, L.Ub.view(), L.XI, K);
    if (L.nslot) launch_lu_fill_i64(s, L.rsum, 0, static_cast<int64_t>(L.nslot) * K);
    launch_lu_eval_rows(s, L.nch, K, nk, static_cast<int>(P->m1), L.ch_row, L.ch_e0, L.ch_e1, L.ch_slot, P->ci,
                        P->val, L.rhs_orig, P->X, L.XI, P->vpart, L.rsum);
    launch_lu_eval_multi(s, L.nslot, K, static_cast<int>(P->m1), L.slot_row, L.rhs_orig, L.rsum, P->vpart);
    TE(3);
    TB(5);
    launch_lu_eval_obj(s, r, K, L.c_tail, L.c0, L.XI, L.nqch, nk, L.qch_row, L.qch_e0, L.qch_e1, P->ciQ, P->valQ,
                       P->X, P->zqpart);
    TE(5);
    TB(6);
    launch_reduce_cand(s, 1, K, P->red_S, P->et, P->vpart, P->st, P->zpart, P->qt, P->zqpart, 1, P->red_v,
                       P->red_z, P->viol, P->z);
    TE(6);
    TB(7);
    launch_argmin_update(s, 1, K, W, P->viol, P->z, P->di, P->ctr, threshold ? 0 : (trigger ? 1 : 2));
    TE(7);
    TB(8);
    launch_extract_best(s, P->n, 1, P->var_inst, P->X, P->di, P->xbest);
    TE(8);
    P->lastK = K;
}

}  // namespace gfh

extern "C" {

int gfors_workspace_bytes_tu(gfors_tu *U, const gfors_params *prm, size_t *bytes) {
    if (!U || !prm || !bytes) return fail(GFORS_E_ARG, "NULL argument");
    const gftu::TuFactored *F = gfors_tu_factored_data(U);
    if (!F) return fail(GFORS_E_ARG, "the handle is not a factorised reformulation (GFORS_TU_FACTORED)");
    if (!k_ok(prm->K_max)) return fail(GFORS_E_ARG, "K_max must be a multiple of 64, <= 4096 (multiple of 1024 above 1024)");
    gfors_problem tmp;
    std::unique_ptr<LuForm> hold(new LuForm());
    tmp.lu = hold.get();
    lu_plan(&tmp, *F, *prm);
    Carver cv{nullptr, 0, 0};
    const gfors_params p = lu_params(prm);
    *bytes = lu_carve(&tmp, cv, *F, p) + 256;
    tmp.lu = nullptr;
    return GFORS_OK;
}

int gfors_create_problem_tu(gfors_tu *U, const gfors_params *prm, void *ws, size_t ws_bytes, void *stream,
                            gfors_problem **out) {
    if (!U || !prm || !ws || !out) return fail(GFORS_E_ARG, "NULL argument");
    *out = nullptr;
    const gftu::TuFactored *Fp = gfors_tu_factored_data(U);
    if (!Fp) return fail(GFORS_E_ARG, "the handle is not a factorised reformulation (GFORS_TU_FACTORED)");
    const gftu::TuFactored &F = *Fp;
    if (!k_ok(prm->K_max)) return fail(GFORS_E_ARG, "K_max must be a multiple of 64, <= 4096 (multiple of 1024 above 1024)");
    if (!(prm->sigma > 0.0) || prm->k_int < 1 || prm->power_iters < 1 || !(prm->x0 >= 0.0 && prm->x0 <= 1.0))
        return fail(GFORS_E_ARG, "bad params (sigma > 0, k_int >= 1, power_iters >= 1, x0 in [0,1])");
    if (prm->repair_row0 >= 0) return fail(GFORS_E_ARG, "repair_row0 is not available on a factorised TU problem");
    if (F.infeasible_row >= 0)
        return fail(GFORS_E_INFEAS_ROW, "reformulated row " + std::to_string(F.infeasible_row) +
                                            " has no coefficient but cannot be satisfied");
    const int64_t nk = F.nk, r = F.r, nfull = nk + r;
    if (nfull >= (int64_t{1} << 31) / 64) return fail(GFORS_E_OOM, "n too large");
    if (r * prm->K_max >= (int64_t{1} << 31)) return fail(GFORS_E_OOM, "pivots x K_max must be < 2^31");
    const int64_t m1 = F.mA + F.nlow + F.nup, m2 = F.mB, m = m1 + m2;
    const int64_t nnzK = static_cast<int64_t>(F.KLci.size()), nnzQ = static_cast<int64_t>(F.QLci.size());

    auto *P = new gfors_problem();
    std::unique_ptr<gfors_problem, void (*)(gfors_problem *)> guard(P, gfors_destroy_problem);
    P->lu = new LuForm();
    LuForm &L = *P->lu;
    P->stream = static_cast<hipStream_t>(stream);
    P->prm = lu_params(prm);
    P->n = nk;
    P->m1 = m1;
    P->m2 = m2;
    P->m = m;
    P->nnzK = nnzK;
    P->nnzQ = nnzQ;
    P->hasQ = nnzQ > 0;
    P->T = 1;
    P->unitK = false;
    P->inst_var0 = {0};
    P->inst_nvar = {nk};
    lu_plan(P, F, *prm);
    L.c0 = F.c0;
    int64_t cmax = 0;
    for (int64_t i = 0; i < nk; ++i) cmax = std::max<int64_t>(cmax, std::llabs(F.c_keep[i]));
    P->obj64 = cmax > 0 && (static_cast<double>(cmax) * 4.0 * kSampleTQ >= 2147483647.0);

    // tiles: sampler over the kept variables, one evaluation tile and one
    // objective tile (the candidates' sums), FP64 reductions over variables and rows
    HostTiles hs, he, hq, hv, hr;
    build_tiles_items(hs, 0, ceil_div(nk, 4), nullptr, kSampleTQ, kSampleTQ, 0);
    he.inst = {0}; he.b0 = {0}; he.b1 = {0};
    hq.inst = {0}; hq.b0 = {0}; hq.b1 = {0};
    build_tiles_items(hv, 0, nk, nullptr, kVarTile, kVarTile, 0);
    std::function<int64_t(int64_t)> wr = [&](int64_t q) -> int64_t { return F.KLrp[q + 1] - F.KLrp[q]; };
    build_tiles_items(hr, 0, m, &wr, kRowNnz, kRowRows, 0);
    for (HostTiles *h : {&hs, &he, &hq, &hv, &hr}) finish_first(*h, 1);
    P->red_S = std::max(1, std::min(64, static_cast<int>(ceil_div(static_cast<int64_t>(hs.inst.size()), 32))));

    Carver cv{static_cast<char *>(ws), 0, ws_bytes};
    {
        const uintptr_t a = reinterpret_cast<uintptr_t>(ws);
        cv.off = (256 - (a & 255)) & 255;
    }
    lu_carve(P, cv, F, P->prm);
    if (cv.off > ws_bytes) return fail(GFORS_E_OOM, "workspace too small: need " + std::to_string(cv.off) + " bytes");
    hipStream_t s = P->stream;
    int rc;
    if ((rc = upload_tiles(s, P->st, hs, 1))) return rc;
    if ((rc = upload_tiles(s, P->et, he, 1))) return rc;
    if ((rc = upload_tiles(s, P->qt, hq, 1))) return rc;
    if ((rc = upload_tiles(s, P->vt, hv, 1))) return rc;
    if ((rc = upload_tiles(s, P->rtile, hr, 1))) return rc;

    // lifted rows and their transpose (one row per lifted column), lifted Q
    std::vector<int> rpT(nfull + 1, 0), ciT(nnzK), valT(nnzK);
    for (int64_t e = 0; e < nnzK; ++e) rpT[F.KLci[e] + 1]++;
    for (int64_t i = 0; i < nfull; ++i) rpT[i + 1] += rpT[i];
    {
        std::vector<int> pos(rpT.begin(), rpT.end() - 1);
        for (int64_t j = 0; j < m; ++j)
            for (int e = F.KLrp[j]; e < F.KLrp[j + 1]; ++e) {
                const int p = pos[F.KLci[e]]++;
                ciT[p] = static_cast<int>(j);
                valT[p] = F.KLval[e];
            }
    }
    if ((rc = upload(s, P->rp, F.KLrp.data(), m + 1))) return rc;
    if ((rc = upload(s, P->ci, F.KLci.data(), nnzK))) return rc;
    if ((rc = upload(s, P->val, F.KLval.data(), nnzK))) return rc;
    if ((rc = upload(s, P->rpT, rpT.data(), nfull + 1))) return rc;
    if ((rc = upload(s, P->ciT, ciT.data(), nnzK))) return rc;
    if ((rc = upload(s, P->valT, valT.data(), nnzK))) return rc;
    if (P->hasQ) {
        if ((rc = upload(s, P->rpQ, F.QLrp.data(), nfull + 1))) return rc;
        if ((rc = upload(s, P->ciQ, F.QLci.data(), nnzQ))) return rc;
        if ((rc = upload(s, P->valQ, F.QLval.data(), nnzQ))) return rc;
    }
    if ((rc = upload(s, P->rhs, F.rhs_ref.data(), m))) return rc;
    if ((rc = upload(s, P->cost, F.c_keep.data(), nk))) return rc;
    {
        std::vector<int> zi(std::max<int64_t>(nfull, m), 0);
        if ((rc = upload(s, P->var_inst, zi.data(), nk))) return rc;
        if ((rc = upload(s, P->row_inst, zi.data(), m))) return rc;
        if ((rc = sync(P))) return rc;
    }
    if ((rc = upload(s, P->d_inst_var0, P->inst_var0.data(), 1))) return rc;
    if ((rc = upload(s, P->d_inst_nvar, P->inst_nvar.data(), 1))) return rc;
    // B_JIbar (rows k) and its transpose (rows = kept variables, columns k)
    const int64_t nbj = static_cast<int64_t>(F.BJci.size());
    std::vector<int> bt_rp(nk + 1, 0), bt_ci(nbj), bt_val(nbj);
    for (int64_t e = 0; e < nbj; ++e) bt_rp[F.BJci[e] + 1]++;
    for (int64_t i = 0; i < nk; ++i) bt_rp[i + 1] += bt_rp[i];
    {
        std::vector<int> pos(bt_rp.begin(), bt_rp.end() - 1);
        for (int64_t k = 0; k < r; ++k)
            for (int e = F.BJrp[k]; e < F.BJrp[k + 1]; ++e) {
                const int p = pos[F.BJci[e]]++;
                bt_ci[p] = static_cast<int>(k);
                bt_val[p] = F.BJval[e];
            }
    }
    if ((rc = upload(s, L.BJrp, F.BJrp.data(), r + 1))) return rc;
    if ((rc = upload(s, L.BJci, F.BJci.data(), nbj))) return rc;
    if ((rc = upload(s, L.BJval, F.BJval.data(), nbj))) return rc;
    if ((rc = upload(s, L.BJTrp, bt_rp.data(), nk + 1))) return rc;
    if ((rc = upload(s, L.BJTci, bt_ci.data(), nbj))) return rc;
    if ((rc = upload(s, L.BJTval, bt_val.data(), nbj))) return rc;
    if ((rc = upload(s, L.dJ, F.dJ.data(), r))) return rc;
    {
        const gftu::HostTrsv *hsv[4] = {&F.Lf, &F.Ub, &F.Utf, &F.Ltb};
        LuDevSolve *dsv[4] = {&L.Lf, &L.Ub, &L.Utf, &L.Ltb};
        for (int q = 0; q < 4; ++q) {
            if ((rc = upload(s, dsv[q]->row, hsv[q]->row.data(), r))) return rc;
            if ((rc = upload(s, dsv[q]->ptr, hsv[q]->ptr.data(), r + 1))) return rc;
            if ((rc = upload(s, dsv[q]->ent, hsv[q]->ent.data(), static_cast<int64_t>(hsv[q]->ent.size())))) return rc;
            if ((rc = upload(s, dsv[q]->lvl, hsv[q]->lvl.data(), static_cast<int64_t>(hsv[q]->lvl.size())))) return rc;
        }
    }
    if ((rc = upload(s, L.rhs_orig, F.rhs_orig.data(), m))) return rc;
    if ((rc = upload(s, L.ch_row, L.h_ch_row.data(), L.nch))) return rc;
    if ((rc = upload(s, L.ch_e0, L.h_ch_e0.data(), L.nch))) return rc;
    if ((rc = upload(s, L.ch_e1, L.h_ch_e1.data(), L.nch))) return rc;
    if ((rc = upload(s, L.ch_slot, L.h_ch_slot.data(), L.nch))) return rc;
    if ((rc = upload(s, L.slot_row, L.h_slot_row.data(), L.nslot))) return rc;
    if ((rc = upload(s, L.qch_row, L.h_qch_row.data(), L.nqch))) return rc;
    if ((rc = upload(s, L.qch_e0, L.h_qch_e0.data(), L.nqch))) return rc;
    if ((rc = upload(s, L.qch_e1, L.h_qch_e1.data(), L.nqch))) return rc;
    if ((rc = upload(s, L.c_tail, F.c_tail.data(), r))) return rc;
    // row scales of the reformulated rows (exact norms from the host)
    P->rowinv.assign(m, 1.0);
    for (int64_t j = 0; j < m; ++j) P->rowinv[j] = F.rownorm[j] > 0.0 ? 1.0 / F.rownorm[j] : 1.0;
    {
        std::vector<double> r2(m);
        for (int64_t j = 0; j < m; ++j) r2[j] = P->rowinv[j] * P->rowinv[j];
        if ((rc = upload(s, P->rowinv_d, P->rowinv.data(), m))) return rc;
        if ((rc = upload(s, P->rowinv2_d, r2.data(), m))) return rc;
        if ((rc = sync(P))) return rc;
    }
    // launch shapes; rows of kHeavyLen+ entries a workgroup each, longest first
    auto avg = [](int64_t tot, int64_t cnt) { return cnt > 0 ? static_cast<double>(tot) / cnt : 1.0; };
    {
        std::vector<int> ord(m), c0v(m, -1);
        for (int64_t j = 0; j < m; ++j) ord[j] = static_cast<int>(j);
        std::stable_sort(ord.begin(), ord.end(), [&](int a2, int b2) {
            return F.KLrp[a2 + 1] - F.KLrp[a2] > F.KLrp[b2 + 1] - F.KLrp[b2];
        });
        int64_t light_nnz = 0;
        for (int64_t q = 0; q < m; ++q) {
            const int j = ord[q], len = F.KLrp[j + 1] - F.KLrp[j];
            if (q >= L.heavy_rows) light_nnz += len;
            bool dense = len > 0;
            for (int e = F.KLrp[j] + 1; e < F.KLrp[j + 1] && dense; ++e) dense = F.KLci[e] == F.KLci[F.KLrp[j]] + (e - F.KLrp[j]);
            if (dense) c0v[j] = F.KLci[F.KLrp[j]];
        }
        if ((rc = upload(s, P->dual_order, ord.data(), m))) return rc;
        if ((rc = upload(s, P->rowc0, c0v.data(), m))) return rc;
        if ((rc = upload(s, L.hch_row, L.h_hch_row.data(), L.nhch))) return rc;
        if ((rc = upload(s, L.hch_e0, L.h_hch_e0.data(), L.nhch))) return rc;
        if ((rc = upload(s, L.hch_e1, L.h_hch_e1.data(), L.nhch))) return rc;
        if ((rc = upload(s, L.hch_first, L.h_hch_first.data(), L.heavy_rows + 1))) return rc;
        if ((rc = sync(P))) return rc;
        int lp = 1;
        const double a = avg(light_nnz, m - L.heavy_rows);
        while (lp < 64 && lp * 2 <= a) lp *= 2;
        L.lpr_dual = lp;
    }
    L.lpr_bj = pick_lpr(avg(nbj, r));
    L.lpr_bjt = pick_lpr(avg(nbj, nk));
    L.lpr_tail = pick_lpr(avg(rpT[nfull] - rpT[nk] + (P->hasQ ? F.QLrp[nfull] - F.QLrp[nk] : 0), r));
    L.lpr_primal = pick_lpr(avg(rpT[nk] + (P->hasQ ? F.QLrp[nk] : 0) + nbj, nk));

    // ---- Preprocess on the device
    if ((rc = lu_device_norms(P))) return rc;
    double kn = 0.0, qn = 0.0;
    HIP_TRY(hipMemcpyAsync(&kn, P->dnorm, sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(&qn, P->dnorm + 1, sizeof(double), hipMemcpyDeviceToHost, s));
    if ((rc = sync(P))) return rc;
    P->s_o.assign(1, 0.0); P->s_K.assign(1, kn); P->qnorm.assign(1, qn); P->tau1.assign(1, 0.0);
    P->tau2.assign(1, 0.0); P->rmin.assign(1, 0.0); P->rmax.assign(1, 0.0); P->rdelta.assign(1, 0.0);
    double csq = 0.0;
    int64_t cm = 0;
    for (int64_t i = 0; i < nk; ++i) {
        csq += static_cast<double>(F.c_ref[i]) * static_cast<double>(F.c_ref[i]);
        cm = std::max<int64_t>(cm, std::llabs(F.c_ref[i]));
    }
    P->s_o[0] = qn + std::sqrt(csq);
    const double so = P->s_o[0];
    const double Qn = so > 0 ? qn / so : 0.0;
    const double g = (so > 0 ? static_cast<double>(cm) / so : static_cast<double>(cm)) + Qn;
    P->rmin[0] = prm->rho_min >= 0 ? prm->rho_min : 1e-3 * g;
    P->rmax[0] = prm->rho_max >= 0 ? prm->rho_max : g;
    P->rdelta[0] = prm->rho_delta >= 0 ? prm->rho_delta : 1e-4 * g;
    const double sq = std::sqrt(prm->sigma);
    if (!P->hasQ) {
        P->tau1[0] = P->tau2[0] = sq;
    } else {
        const double Lm = 2.0 * (Qn + P->rmax[0]);
        P->tau1[0] = std::min(sq, 1.0 / (2.0 * Lm));
        P->tau2[0] = prm->sigma / P->tau1[0];
    }
    if (prm->tau1 > 0) P->tau1[0] = prm->tau1;
    if (prm->tau2 > 0) P->tau2[0] = prm->tau2;
    {
        std::vector<float> omega(m), rtv(m), ctv(nk);
        std::vector<double> om64(m);
        for (int64_t j = 0; j < m; ++j) {
            const double w64 = kn > 0 ? P->rowinv[j] / kn : P->rowinv[j];
            om64[j] = w64;
            omega[j] = static_cast<float>(w64);
            const double rr = static_cast<double>(F.rhs_ref[j]) * P->rowinv[j];
            rtv[j] = static_cast<float>(kn > 0 ? rr / kn : rr);
        }
        for (int64_t i = 0; i < nk; ++i)
            ctv[i] = static_cast<float>(so > 0 ? static_cast<double>(F.c_ref[i]) / so : static_cast<double>(F.c_ref[i]));
        if ((rc = upload(s, P->omega, omega.data(), m))) return rc;
        if ((rc = upload(s, P->rt, rtv.data(), m))) return rc;
        if ((rc = upload(s, P->omega64, om64.data(), m))) return rc;
        if ((rc = upload(s, P->ct, ctv.data(), nk))) return rc;
        const float t1f = static_cast<float>(P->tau1[0]), t2f = static_cast<float>(P->tau2[0]);
        const double tsod = so > 0 ? 2.0 / so : 2.0;
        const float tsof = static_cast<float>(tsod);
        DevInst &di = P->di;
        const double rT = prm->rho_T, rpp = prm->rho_p;
        if ((rc = upload(s, di.rho_min, P->rmin.data(), 1))) return rc;
        if ((rc = upload(s, di.rho_max, P->rmax.data(), 1))) return rc;
        if ((rc = upload(s, di.rho_delta, P->rdelta.data(), 1))) return rc;
        if ((rc = upload(s, di.rho_T, &rT, 1))) return rc;
        if ((rc = upload(s, di.rho_p, &rpp, 1))) return rc;
        if ((rc = upload(s, di.tau1, &t1f, 1))) return rc;
        if ((rc = upload(s, di.tau2, &t2f, 1))) return rc;
        if ((rc = upload(s, di.two_so, &tsof, 1))) return rc;
        if ((rc = upload(s, di.tau1d, P->tau1.data(), 1))) return rc;
        if ((rc = upload(s, di.tau2d, P->tau2.data(), 1))) return rc;
        if ((rc = upload(s, di.two_sod, &tsod, 1))) return rc;
        const int32_t z32 = 0;
        if ((rc = upload(s, di.inc_W, &z32, 1))) return rc;
        if ((rc = sync(P))) return rc;
    }
    if ((rc = gfors_reset(P))) return rc;   // iterate, incumbent, counters; lifts the iterate
    if (prm->autotune) {
        if ((rc = lu_autotune(P))) return rc;
        if ((rc = gfors_reset(P))) return rc;
    }
    *out = guard.release();
    return GFORS_OK;
}

}  // extern "C"
