// TU reformulation (Theorem of Sec. 2.4.1), host code.  For pivot equality
// rows J and pivot columns I (one per row) with B_J totally unimodular and
// B_JI invertible, the rows J are solved for x_I:
//   x_I = s + S x_Ibar,   s = B_JI^{-1} d_J,   S = -B_JI^{-1} B_JIbar,
// and x_I is substituted into every other row and into the objective:
//   Q' = S^T Q_II S + S^T Q_IIbar + Q_IIbar^T S + Q_IbarIbar,
//   A' = A_.I S + A_.Ibar,  b' = b - A_.I s,  B' = B_JbarI S + B_JbarIbar,
//   d' = d_Jbar - B_JbarI s,
//   c' = 2 S^T Q_II s + 2 Q_IIbar^T s + S^T c_I + c_Ibar,
//   c'_0 = <s, Q_II s> + <c_I, s>,
// and 0 <= x_p <= 1 becomes the rows  S_p x >= -s_p  and  -S_p x >= s_p - 1.
// A bound row that every point of the box satisfies (sum of its negative
// coefficients >= right-hand side) is left out: it cuts off nothing, neither
// from the relaxation nor from the binary problem.
//
// s and S are computed exactly in integers.  When B_JI is a signed identity
// (each pivot row holds its pivot column with coefficient +-1 and no other
// pivot column) they are read off the rows.  Otherwise Gauss-Jordan
// elimination runs on the rows of B_J: a pivot on a +-1 entry keeps a totally
// unimodular matrix totally unimodular, so every intermediate coefficient stays
// in {-1, 0, 1}; a pivot entry of any other magnitude means B_J is not TU and
// the call fails.  S is stored explicitly (sparse), in place of a factorisation
// of B_JI applied at every step.
#include "../../include/gfors.h"
#include "gfors_lu.h"

#include <algorithm>
#include <cstdlib>
#include <limits>
#include <functional>
#include <map>
#include <memory>
#include <queue>
#include <set>
#include <tuple>
#include <cmath>
#include <string>
#include <utility>
#include <vector>

namespace {
thread_local std::string g_tu_err;
int tu_fail(int code, const std::string &m) {
    g_tu_err = m;
    return code;
}

// A sparse integer row kept sorted by column.
using SRow = std::vector<std::pair<int64_t, int64_t>>;

int64_t row_get(const SRow &r, int64_t col) {
    auto it = std::lower_bound(r.begin(), r.end(), std::make_pair(col, std::numeric_limits<int64_t>::min()));
    return (it != r.end() && it->first == col) ? it->second : 0;
}

// r += f * o (both sorted); drops zeros.
SRow row_axpy(const SRow &r, int64_t f, const SRow &o) {
    SRow out;
    out.reserve(r.size() + o.size());
    size_t i = 0, j = 0;
    while (i < r.size() || j < o.size()) {
        if (j == o.size() || (i < r.size() && r[i].first < o[j].first)) {
            out.push_back(r[i++]);
        } else if (i == r.size() || o[j].first < r[i].first) {
            if (o[j].second * f) out.emplace_back(o[j].first, o[j].second * f);
            ++j;
        } else {
            const int64_t v = r[i].second + f * o[j].second;
            if (v) out.emplace_back(r[i].first, v);
            ++i;
            ++j;
        }
    }
    return out;
}

using gftu::HostTrsv;
using gftu::TuFactored;
using Ent = std::pair<int32_t, int32_t>;   // (column, coefficient)

// Level schedule of an in-place triangular solve whose row k reads the rows
// listed in ents[k] (earlier rows for a forward solve, later for a backward one).
void schedule(int64_t r, const std::vector<std::vector<Ent>> &ents, const std::vector<int32_t> &dg,
              bool forward, HostTrsv &H) {
    std::vector<int32_t> level(r, 0);
    int32_t maxl = -1;
    for (int64_t t = 0; t < r; ++t) {
        const int64_t k = forward ? t : r - 1 - t;
        int32_t lv = 0;
        for (const Ent &e : ents[k]) lv = std::max(lv, level[e.first] + 1);
        level[k] = lv;
        maxl = std::max(maxl, lv);
    }
    const int32_t nl = maxl + 1;
    H.lvl.assign(nl + 1, 0);
    for (int64_t k = 0; k < r; ++k) H.lvl[level[k] + 1]++;
    for (int32_t l = 0; l < nl; ++l) H.lvl[l + 1] += H.lvl[l];
    std::vector<int32_t> pos(H.lvl.begin(), H.lvl.end() - 1), at(r);
    for (int64_t k = 0; k < r; ++k) at[k] = pos[level[k]]++;
    H.row.assign(r, 0);
    H.ptr.assign(r + 1, 0);
    for (int64_t k = 0; k < r; ++k) {
        H.row[at[k]] = static_cast<int32_t>((k << 1) | (dg[k] < 0 ? 1 : 0));
        H.ptr[at[k] + 1] = static_cast<int32_t>(ents[k].size());
    }
    for (int64_t p = 0; p < r; ++p) H.ptr[p + 1] += H.ptr[p];
    H.ent.assign(H.ptr[r], 0);
    for (int64_t k = 0; k < r; ++k) {
        int32_t e = H.ptr[at[k]];
        for (const Ent &x : ents[k]) H.ent[e++] = (x.first << 1) | (x.second < 0 ? 1 : 0);
    }
}

// Sparse M^{-T} alpha (M = L U in position order): U^T z = alpha forward, then
// L^T u = z backward, each touching only the positions the nonzeros reach.
struct SparseSolveT {
    const TuFactored &F;
    std::vector<int64_t> acc;
    std::vector<uint8_t> queued;
    explicit SparseSolveT(const TuFactored &f) : F(f), acc(f.r, 0), queued(f.r, 0) {}
    void run(const std::vector<std::pair<int32_t, int64_t>> &alpha, std::vector<std::pair<int32_t, int64_t>> &u) {
        std::priority_queue<int32_t, std::vector<int32_t>, std::greater<int32_t>> fw;
        for (const auto &a : alpha) {
            acc[a.first] += a.second;
            if (!queued[a.first]) { queued[a.first] = 1; fw.push(a.first); }
        }
        std::vector<std::pair<int32_t, int64_t>> z;
        while (!fw.empty()) {
            const int32_t j = fw.top();
            fw.pop();
            queued[j] = 0;
            const int64_t zj = acc[j] * F.Ud[j];
            acc[j] = 0;
            if (!zj) continue;
            z.emplace_back(j, zj);
            for (int32_t e = F.Urp[j]; e < F.Urp[j + 1]; ++e) {
                const int32_t k = F.Uci[e];
                acc[k] -= F.Uval[e] * zj;
                if (!queued[k]) { queued[k] = 1; fw.push(k); }
            }
        }
        std::priority_queue<int32_t> bw;
        for (const auto &a : z) {
            acc[a.first] += a.second;
            if (!queued[a.first]) { queued[a.first] = 1; bw.push(a.first); }
        }
        u.clear();
        while (!bw.empty()) {
            const int32_t j = bw.top();
            bw.pop();
            queued[j] = 0;
            const int64_t uj = acc[j];
            acc[j] = 0;
            if (!uj) continue;
            u.emplace_back(j, uj);
            for (int32_t e = F.Lrp[j]; e < F.Lrp[j + 1]; ++e) {
                const int32_t k = F.Lci[e];
                acc[k] -= F.Lval[e] * uj;
                if (!queued[k]) { queued[k] = 1; bw.push(k); }
            }
        }
    }
};

// Dense M^{-1} v in exact integers (v and the result in position order).
void solve_M(const TuFactored &F, std::vector<int64_t> &v) {
    const int64_t r = F.r;
    for (int64_t k = 0; k < r; ++k)
        for (int32_t e = F.Lrp[k]; e < F.Lrp[k + 1]; ++e) v[k] -= F.Lval[e] * v[F.Lci[e]];
    for (int64_t k = r - 1; k >= 0; --k) {
        for (int32_t e = F.Urp[k]; e < F.Urp[k + 1]; ++e) v[k] -= F.Uval[e] * v[F.Uci[e]];
        v[k] *= F.Ud[k];
    }
}

// Right-looking sparse LU of the pivot block with Markowitz-style pivots (a
// column of fewest active entries, its shortest active row).  R[q] holds row q
// of B_JI over pivot-column indices.  Every pivot and every updated entry must
// stay in {-1, 0, 1}: B_J is then totally unimodular as far as this block shows.
int factor_block(std::vector<SRow> R, TuFactored &F, std::vector<int32_t> &arow,
                 std::vector<int32_t> &bcol) {
    const int64_t r = F.r;
    std::vector<std::vector<int32_t>> C(r);
    std::vector<int32_t> cnt(r, 0);
    for (int64_t q = 0; q < r; ++q)
        for (const auto &kv : R[q]) {
            C[kv.first].push_back(static_cast<int32_t>(q));
            cnt[kv.first]++;
        }
    std::set<std::pair<int32_t, int32_t>> colq;
    for (int64_t c = 0; c < r; ++c) colq.insert({cnt[c], static_cast<int32_t>(c)});
    std::vector<uint8_t> rdone(r, 0), cdone(r, 0);
    arow.assign(r, -1);
    bcol.assign(r, -1);
    std::vector<std::tuple<int32_t, int32_t, int64_t>> Lrec;
    std::vector<SRow> Urows(r);
    auto setcnt = [&](int64_t col, int delta) {
        if (cdone[col]) return;
        colq.erase({cnt[col], static_cast<int32_t>(col)});
        cnt[col] += delta;
        colq.insert({cnt[col], static_cast<int32_t>(col)});
    };
    const char *not_tu = "an entry other than +-1 met in the LU of B_JI: B_J is not totally unimodular";
    for (int64_t k = 0; k < r; ++k) {
        const auto top = *colq.begin();
        const int32_t c = top.second;
        if (top.first == 0) return tu_fail(GFORS_E_ARG, "pivot block B_JI is singular");
        int32_t p = -1;
        size_t best = SIZE_MAX;
        for (int32_t q : C[c])
            if (!rdone[q] && row_get(R[q], c) != 0 && R[q].size() < best) {
                best = R[q].size();
                p = q;
            }
        if (p < 0) return tu_fail(GFORS_E_ARG, "pivot block B_JI is singular");
        const int64_t piv = row_get(R[p], c);
        if (piv != 1 && piv != -1) return tu_fail(GFORS_E_ARG, not_tu);
        arow[k] = p;
        bcol[k] = c;
        rdone[p] = 1;
        colq.erase({cnt[c], c});
        cdone[c] = 1;
        for (const auto &kv : R[p])
            if (kv.first != c) setcnt(kv.first, -1);
        std::vector<int32_t> rows_c;
        for (int32_t q : C[c])
            if (!rdone[q]) rows_c.push_back(q);
        std::sort(rows_c.begin(), rows_c.end());
        rows_c.erase(std::unique(rows_c.begin(), rows_c.end()), rows_c.end());
        for (int32_t q : rows_c) {
            const int64_t f = row_get(R[q], c);
            if (!f) continue;
            const int64_t mult = f * piv;   // f / piv, piv = +-1
            Lrec.emplace_back(q, static_cast<int32_t>(k), mult);
            SRow nr = row_axpy(R[q], -mult, R[p]);
            // active-column counts: entries that vanished or appeared in row q
            size_t i = 0, j = 0;
            const SRow &o = R[q];
            while (i < o.size() || j < nr.size()) {
                if (j == nr.size() || (i < o.size() && o[i].first < nr[j].first)) {
                    setcnt(o[i].first, -1);
                    ++i;
                } else if (i == o.size() || nr[j].first < o[i].first) {
                    setcnt(nr[j].first, +1);
                    C[nr[j].first].push_back(q);
                    ++j;
                } else {
                    ++i;
                    ++j;
                }
            }
            for (const auto &kv : nr)
                if (kv.second != 1 && kv.second != -1) return tu_fail(GFORS_E_ARG, not_tu);
            R[q].swap(nr);
        }
        Urows[k].swap(R[p]);
    }
    std::vector<int32_t> rowstep(r), colstep(r);
    for (int64_t k = 0; k < r; ++k) {
        rowstep[arow[k]] = static_cast<int32_t>(k);
        colstep[bcol[k]] = static_cast<int32_t>(k);
    }
    std::vector<std::vector<Ent>> Lr(r), Ur(r), Lc(r), Uc(r);
    for (const auto &t : Lrec) {
        const int32_t row = rowstep[std::get<0>(t)], col = std::get<1>(t);
        const int32_t v = static_cast<int32_t>(std::get<2>(t));
        if (v != 1 && v != -1) return tu_fail(GFORS_E_ARG, not_tu);
        Lr[row].emplace_back(col, v);
        Lc[col].emplace_back(row, v);
    }
    F.Ud.assign(r, 0);
    for (int64_t k = 0; k < r; ++k)
        for (const auto &kv : Urows[k]) {
            const int32_t col = colstep[kv.first];
            if (col == k) F.Ud[k] = static_cast<int32_t>(kv.second);
            else {
                Ur[k].emplace_back(col, static_cast<int32_t>(kv.second));
                Uc[col].emplace_back(static_cast<int32_t>(k), static_cast<int32_t>(kv.second));
            }
        }
    auto to_csr = [&](std::vector<std::vector<Ent>> &rows, std::vector<int32_t> &rp, std::vector<int32_t> &ci,
                      std::vector<int32_t> &vv) {
        rp.assign(1, 0);
        for (auto &rw : rows) {
            std::sort(rw.begin(), rw.end());
            for (const Ent &e : rw) {
                ci.push_back(e.first);
                vv.push_back(e.second);
            }
            rp.push_back(static_cast<int32_t>(ci.size()));
        }
    };
    to_csr(Lr, F.Lrp, F.Lci, F.Lval);
    to_csr(Ur, F.Urp, F.Uci, F.Uval);
    std::vector<int32_t> one(r, 1);
    schedule(r, Lr, one, true, F.Lf);
    schedule(r, Ur, F.Ud, false, F.Ub);
    schedule(r, Uc, F.Ud, true, F.Utf);
    schedule(r, Lc, one, false, F.Ltb);
    return GFORS_OK;
}

// Everything the device needs for the factorised form, computed exactly on
// the host without storing S: the LU, s, the lifted rows with the reformulated
// right-hand sides, the 2-norms of the reformulated rows (each row of A', B'
// and S is formed once, in a scratch row, and dropped), which bound rows are
// kept, and the objective pieces c', c'_0.
int build_factored(const gfors_csr *A, const int64_t *b, const gfors_csr *B, const int64_t *d,
                   const gfors_csr *Q, const int64_t *c, int64_t n, const int64_t *pivots,
                   const std::vector<int64_t> &rows_piv, const std::vector<int64_t> &piv_col,
                   const std::vector<int64_t> &piv_index, const std::vector<int64_t> &newidx,
                   const std::vector<int64_t> &keep, const std::vector<SRow> &rowsJ, TuFactored &F) {
    auto coef = [](const gfors_csr *M, int64_t e) -> int64_t { return M->val ? M->val[e] : 1; };
    const int64_t r = static_cast<int64_t>(piv_col.size()), nk = static_cast<int64_t>(keep.size());
    F.n = n;
    F.nk = nk;
    F.r = r;
    F.keep = keep;
    // B_JI over pivot-column indices, B_JIbar over kept indices (rows q)
    std::vector<SRow> RI(r), RK(r);
    for (int64_t q = 0; q < r; ++q)
        for (const auto &kv : rowsJ[q]) {
            const int64_t pq = piv_index[kv.first];
            if (pq >= 0) RI[q].emplace_back(pq, kv.second);
            else RK[q].emplace_back(newidx[kv.first], kv.second);
        }
    for (auto &rw : RI) std::sort(rw.begin(), rw.end());
    for (auto &rw : RK) std::sort(rw.begin(), rw.end());
    for (const auto &rw : RK)
        for (const auto &kv : rw)
            if (kv.second != 1 && kv.second != -1)
                return tu_fail(GFORS_E_ARG, "a pivot row has a coefficient other than +-1: B_J is not totally unimodular");
    std::vector<int32_t> arow, bcol;
    int rc;
    if ((rc = factor_block(RI, F, arow, bcol))) return rc;
    std::vector<int32_t> pos_of(r);   // pivot-column index q' -> position k
    F.tail_var.resize(r);
    for (int64_t k = 0; k < r; ++k) {
        pos_of[bcol[k]] = static_cast<int32_t>(k);
        F.tail_var[k] = piv_col[bcol[k]];
    }
    F.BJrp.assign(1, 0);
    F.dJ.resize(r);
    for (int64_t k = 0; k < r; ++k) {
        for (const auto &kv : RK[arow[k]]) {
            F.BJci.push_back(static_cast<int32_t>(kv.first));
            F.BJval.push_back(static_cast<int32_t>(kv.second));
        }
        F.BJrp.push_back(static_cast<int32_t>(F.BJci.size()));
        F.dJ[k] = d[rows_piv[arow[k]]];
    }
    F.s = F.dJ;
    solve_M(F, F.s);
    // lifted index of an original variable
    auto lifted = [&](int64_t i) -> int64_t {
        const int64_t q = piv_index[i];
        return q < 0 ? newidx[i] : nk + pos_of[q];
    };
    SparseSolveT solver(F);
    std::vector<int64_t> acc(nk, 0);
    std::vector<uint8_t> touched(nk, 0);
    std::vector<int64_t> list;
    std::vector<std::pair<int32_t, int64_t>> alpha, u;
    auto add = [&](int64_t i, int64_t v) {
        if (!touched[i]) { touched[i] = 1; list.push_back(i); }
        acc[i] += v;
    };
    // the reformulated row  base - (M^{-T} alpha)^T B_JIbar  into acc; returns its sum of squares
    struct RowStats { int64_t sq = 0, neg = 0, pos = 0, nnz = 0; };
    auto finish_row = [&]() {
        solver.run(alpha, u);
        for (const auto &kv : u)
            for (int32_t e = F.BJrp[kv.first]; e < F.BJrp[kv.first + 1]; ++e) add(F.BJci[e], -kv.second * F.BJval[e]);
        RowStats st;
        for (int64_t i : list) {
            const int64_t v = acc[i];
            acc[i] = 0;
            touched[i] = 0;
            if (!v) continue;
            st.sq += v * v;
            st.nnz++;
            if (v < 0) st.neg += v;
            else st.pos += v;
        }
        list.clear();
        return st;
    };
    // one original row (A or B_Jbar) lifted: kept entries and position entries
    auto lift_row = [&](const gfors_csr *M, int64_t row, int64_t rh) -> int {
        std::vector<std::pair<int64_t, int64_t>> ents;
        int64_t rref = rh;
        alpha.clear();
        for (int64_t e = M->row_ptr[row]; e < M->row_ptr[row + 1]; ++e) {
            const int64_t i = M->col_idx[e], a = coef(M, e);
            if (!a) continue;
            ents.emplace_back(lifted(i), a);
            const int64_t q = piv_index[i];
            if (q < 0) add(newidx[i], a);
            else {
                rref -= a * F.s[pos_of[q]];
                alpha.emplace_back(pos_of[q], a);
            }
        }
        std::sort(ents.begin(), ents.end());
        std::vector<std::pair<int64_t, int64_t>> merged;
        for (const auto &kv : ents) {
            if (!merged.empty() && merged.back().first == kv.first) merged.back().second += kv.second;
            else merged.push_back(kv);
        }
        for (const auto &kv : merged) {
            if (!kv.second) continue;
            if (kv.second > std::numeric_limits<int32_t>::max() || kv.second < std::numeric_limits<int32_t>::min())
                return tu_fail(GFORS_E_ARG, "coefficient overflows int32");
            F.KLci.push_back(static_cast<int32_t>(kv.first));
            F.KLval.push_back(static_cast<int32_t>(kv.second));
        }
        F.KLrp.push_back(static_cast<int32_t>(F.KLci.size()));
        const RowStats st = finish_row();
        F.rownorm.push_back(std::sqrt(static_cast<double>(st.sq)));
        F.nnz_ref += st.nnz;
        F.rhs_ref.push_back(rref);
        F.rhs_orig.push_back(rh);
        return GFORS_OK;
    };
    F.KLrp.assign(1, 0);
    F.mA = A ? A->nrows : 0;
    for (int64_t i = 0; i < F.mA; ++i)
        if ((rc = lift_row(A, i, b[i]))) return rc;
    // rows of S in pivot order q: S_q = -(M^{-T} e_k)^T B_JIbar, k = position of q
    std::vector<RowStats> Sst(r);
    for (int64_t q = 0; q < r; ++q) {
        alpha.assign(1, {pos_of[q], 1});
        Sst[q] = finish_row();
        F.nnz_S += Sst[q].nnz;
    }
    for (int side = 0; side < 2; ++side)
        for (int64_t q = 0; q < r; ++q) {
            const int64_t k = pos_of[q];
            const int64_t rh = side == 0 ? -F.s[k] : F.s[k] - 1;
            const int64_t negsum = side == 0 ? Sst[q].neg : -Sst[q].pos;
            if (negsum >= rh) continue;   // every point of the box satisfies it
            F.KLci.push_back(static_cast<int32_t>(nk + k));
            F.KLval.push_back(side == 0 ? 1 : -1);
            F.KLrp.push_back(static_cast<int32_t>(F.KLci.size()));
            F.rownorm.push_back(std::sqrt(static_cast<double>(Sst[q].sq)));
            F.nnz_ref += Sst[q].nnz;
            F.rhs_ref.push_back(rh);
            F.rhs_orig.push_back(side == 0 ? 0 : -1);
            (side == 0 ? F.nlow : F.nup)++;
        }
    F.mB = 0;
    for (int64_t rr = 0; rr < B->nrows; ++rr) {
        if (pivots[rr] >= 0) continue;
        if ((rc = lift_row(B, rr, d[rr]))) return rc;
        F.mB++;
    }
    const int64_t m1 = F.mA + F.nlow + F.nup;
    for (int64_t j = 0; j < m1 + F.mB && F.infeasible_row < 0; ++j)
        if (F.rownorm[j] == 0.0 && (j < m1 ? F.rhs_ref[j] > 0 : F.rhs_ref[j] != 0)) F.infeasible_row = j;
    // objective: sigma = (0 on kept, s on pivots); c' = c_Ibar + 2 (Q sigma)_Ibar + S^T (c_I + 2 (Q sigma)_I),
    // c'_0 = <sigma, Q sigma> + <c_I, s>
    F.c_keep.resize(nk);
    for (int64_t i = 0; i < nk; ++i) F.c_keep[i] = c[keep[i]];
    F.c_tail.resize(r);
    for (int64_t k = 0; k < r; ++k) F.c_tail[k] = c[F.tail_var[k]];
    std::vector<int64_t> qs(nk + r, 0);   // Q sigma on the lifted index space
    F.QLrp.assign(1, 0);
    if (Q && Q->row_ptr[Q->nrows] > 0) {
        std::vector<std::vector<Ent>> rows(nk + r);
        std::vector<std::tuple<int64_t, int64_t, int64_t>> ent;
        for (int64_t a = 0; a < n; ++a)
            for (int64_t e = Q->row_ptr[a]; e < Q->row_ptr[a + 1]; ++e) {
                const int64_t v = coef(Q, e);
                if (!v) continue;
                ent.emplace_back(a, Q->col_idx[e], v);
            }
        // the factorised gradient 2 Q' x assumes a symmetric Q
        {
            std::vector<std::tuple<int64_t, int64_t, int64_t>> tr(ent.size());
            for (size_t t = 0; t < ent.size(); ++t) tr[t] = {std::get<1>(ent[t]), std::get<0>(ent[t]), std::get<2>(ent[t])};
            auto a2 = ent;
            std::sort(a2.begin(), a2.end());
            std::sort(tr.begin(), tr.end());
            if (a2 != tr) return tu_fail(GFORS_E_ARG, "the factorised form needs a symmetric Q");
        }
        for (const auto &t : ent) {
            const int64_t a = std::get<0>(t), bb = std::get<1>(t), v = std::get<2>(t);
            if (v > std::numeric_limits<int32_t>::max() || v < std::numeric_limits<int32_t>::min())
                return tu_fail(GFORS_E_ARG, "Q entry overflows int32");
            rows[lifted(a)].emplace_back(static_cast<int32_t>(lifted(bb)), static_cast<int32_t>(v));
            const int64_t qb = piv_index[bb];
            if (qb >= 0) qs[lifted(a)] += v * F.s[pos_of[qb]];
        }
        for (auto &rw : rows) {
            std::sort(rw.begin(), rw.end());
            for (const Ent &e : rw) {
                F.QLci.push_back(e.first);
                F.QLval.push_back(e.second);
            }
            F.QLrp.push_back(static_cast<int32_t>(F.QLci.size()));
        }
    } else {
        F.QLrp.assign(nk + r + 1, 0);
    }
    F.c0 = 0;
    for (int64_t k = 0; k < r; ++k) F.c0 += F.c_tail[k] * F.s[k] + F.s[k] * qs[nk + k];
    // S^T w = -B_JIbar^T M^{-T} w with w = c_I + 2 (Q sigma)_I (dense transposed solve)
    std::vector<int64_t> w(r);
    for (int64_t k = 0; k < r; ++k) w[k] = F.c_tail[k] + 2 * qs[nk + k];
    {
        // z = U^{-T} w: z_k = Ud_k (w_k - sum_{j<k} U_jk z_j), column access through the U^T schedule's rows
        std::vector<int64_t> z(w);
        for (int64_t k = 0; k < r; ++k) {
            z[k] *= F.Ud[k];
            for (int32_t e = F.Urp[k]; e < F.Urp[k + 1]; ++e) z[F.Uci[e]] -= F.Uval[e] * z[k];
        }
        // u = L^{-T} z: u_k = z_k - sum_{j>k} L_jk u_j (rows of L visited from the last)
        for (int64_t k = r - 1; k >= 0; --k)
            for (int32_t e = F.Lrp[k]; e < F.Lrp[k + 1]; ++e) z[F.Lci[e]] -= F.Lval[e] * z[k];
        F.c_ref.resize(nk);
        for (int64_t i = 0; i < nk; ++i) F.c_ref[i] = F.c_keep[i] + 2 * qs[i];
        for (int64_t k = 0; k < r; ++k)
            for (int32_t e = F.BJrp[k]; e < F.BJrp[k + 1]; ++e) F.c_ref[F.BJci[e]] -= z[k] * F.BJval[e];
    }
    return GFORS_OK;
}
}  // namespace

struct gfors_tu {
    int64_t n = 0, n_new = 0;
    std::vector<int64_t> keep;          // new index -> old index
    std::vector<int64_t> newidx;        // old index -> new index (-1 for a pivot)
    std::vector<int64_t> piv_col;       // pivot columns (pivot order)
    std::vector<int64_t> s;             // s_p
    std::vector<int64_t> Srp;           // CSR of S rows (over new indices)
    std::vector<int32_t> Sci;
    std::vector<int64_t> Sval;
    // reformulated model
    std::vector<int64_t> Arp, Brp, Qrp, bvec, dvec, cvec;
    std::vector<int32_t> Aci, Aval, Bci, Bval, Qci, Qval;
    int64_t c0 = 0;
    // GFORS_TU_FACTORED: the LU of the pivot block, no explicit S (Remark of Sec. 2.4.1)
    std::unique_ptr<gftu::TuFactored> fac;
};

const gftu::TuFactored *gfors_tu_factored_data(const gfors_tu *U) { return U ? U->fac.get() : nullptr; }

extern "C" {

const char *gfors_tu_last_error(void) { return g_tu_err.c_str(); }

int gfors_tu_create(const gfors_csr *A, const int64_t *b, const gfors_csr *B, const int64_t *d,
                    const gfors_csr *Q, const int64_t *c, int64_t n, const int64_t *pivots,
                    gfors_tu **out) {
    return gfors_tu_create_ex(A, b, B, d, Q, c, n, pivots, 0, out);
}

int gfors_tu_create_ex(const gfors_csr *A, const int64_t *b, const gfors_csr *B, const int64_t *d,
                       const gfors_csr *Q, const int64_t *c, int64_t n, const int64_t *pivots,
                       int32_t flags, gfors_tu **out) {
    if (flags & ~GFORS_TU_FACTORED) return tu_fail(GFORS_E_ARG, "unknown flag");
    if (!out || !c || n <= 0 || !B || !d || !pivots) return tu_fail(GFORS_E_ARG, "NULL argument");
    *out = nullptr;
    auto check = [&](const gfors_csr *M, const char *nm) -> int {
        if (!M) return GFORS_OK;
        if (M->ncols != n || M->nrows < 0 || !M->row_ptr || M->row_ptr[0] != 0)
            return tu_fail(GFORS_E_ARG, std::string(nm) + ": bad CSR header");
        for (int64_t r = 0; r < M->nrows; ++r)
            if (M->row_ptr[r + 1] < M->row_ptr[r]) return tu_fail(GFORS_E_ARG, std::string(nm) + ": row_ptr decreases");
        for (int64_t e = 0; e < M->row_ptr[M->nrows]; ++e)
            if (M->col_idx[e] < 0 || M->col_idx[e] >= n) return tu_fail(GFORS_E_ARG, std::string(nm) + ": column out of range");
        return GFORS_OK;
    };
    int rc;
    if ((rc = check(A, "A")) || (rc = check(B, "B")) || (rc = check(Q, "Q"))) return rc;
    if (Q && Q->nrows != n) return tu_fail(GFORS_E_ARG, "Q must be n x n");
    if (A && A->nrows > 0 && !b) return tu_fail(GFORS_E_ARG, "b is NULL");
    auto coef = [](const gfors_csr *M, int64_t e) -> int64_t { return M->val ? M->val[e] : 1; };

    auto *U = new gfors_tu();
    std::unique_ptr<gfors_tu> guard(U);
    U->n = n;
    const int64_t m2 = B->nrows;
    std::vector<int64_t> piv_row_of_col(n, -1);
    std::vector<int64_t> rows_piv;      // pivot rows in order
    for (int64_t r = 0; r < m2; ++r) {
        const int64_t p = pivots[r];
        if (p < 0) continue;
        if (p >= n) return tu_fail(GFORS_E_ARG, "pivot column out of range");
        if (piv_row_of_col[p] >= 0) return tu_fail(GFORS_E_ARG, "a column is the pivot of two rows");
        piv_row_of_col[p] = r;
        rows_piv.push_back(r);
        U->piv_col.push_back(p);
    }
    const size_t np = U->piv_col.size();
    U->newidx.assign(n, -1);
    for (int64_t i = 0; i < n; ++i)
        if (piv_row_of_col[i] < 0) {
            U->newidx[i] = static_cast<int64_t>(U->keep.size());
            U->keep.push_back(i);
        }
    U->n_new = static_cast<int64_t>(U->keep.size());
    if (U->n_new == 0) return tu_fail(GFORS_E_ARG, "every variable is a pivot");
    const int64_t nn = U->n_new;
    std::vector<int64_t> piv_index(n, -1);
    for (size_t q = 0; q < np; ++q) piv_index[U->piv_col[q]] = static_cast<int64_t>(q);

    // rows of B_J as sorted sparse rows (duplicates summed)
    std::vector<SRow> rows(np);
    std::vector<int64_t> rhs(np);
    for (size_t q = 0; q < np; ++q) {
        const int64_t r = rows_piv[q];
        SRow &R = rows[q];
        for (int64_t e = B->row_ptr[r]; e < B->row_ptr[r + 1]; ++e) R.emplace_back(B->col_idx[e], coef(B, e));
        std::sort(R.begin(), R.end());
        SRow m;
        for (const auto &kv : R) {
            if (!m.empty() && m.back().first == kv.first) m.back().second += kv.second;
            else m.push_back(kv);
        }
        m.erase(std::remove_if(m.begin(), m.end(), [](const std::pair<int64_t, int64_t> &kv) { return kv.second == 0; }), m.end());
        R.swap(m);
        rhs[q] = d[r];
    }
    if (flags & GFORS_TU_FACTORED) {
        if (np == 0) return tu_fail(GFORS_E_ARG, "no pivot row");
        U->fac.reset(new gftu::TuFactored());
        if ((rc = build_factored(A, b, B, d, Q, c, n, pivots, rows_piv, U->piv_col, piv_index, U->newidx,
                                 U->keep, rows, *U->fac)))
            return rc;
        U->c0 = U->fac->c0;
        *out = guard.release();
        return GFORS_OK;
    }
    // signed identity?
    bool ident = true;
    for (size_t q = 0; q < np && ident; ++q) {
        const int64_t a = row_get(rows[q], U->piv_col[q]);
        if (a != 1 && a != -1) ident = false;
        for (const auto &kv : rows[q])
            if (piv_index[kv.first] >= 0 &&
                (kv.first == U->piv_col[q] ? (kv.second != 1 && kv.second != -1) : true)) {
                ident = false;
                break;
            }
    }
    if (!ident) {
        // Gauss-Jordan on B_J, one pivot column at a time (the column's own row
        // first, else the first unused row holding it)
        std::vector<uint8_t> used(np, 0);
        std::vector<size_t> row_of(np, np);
        for (size_t q = 0; q < np; ++q) {
            const int64_t p = U->piv_col[q];
            size_t r = np;
            if (!used[q] && row_get(rows[q], p) != 0) r = q;
            for (size_t k = 0; k < np && r == np; ++k)
                if (!used[k] && row_get(rows[k], p) != 0) r = k;
            if (r == np) return tu_fail(GFORS_E_ARG, "pivot block B_JI is singular");
            const int64_t a = row_get(rows[r], p);
            if (a != 1 && a != -1)
                return tu_fail(GFORS_E_ARG, "pivot entry " + std::to_string(a) +
                                                " met in the elimination: B_J is not totally unimodular");
            if (a == -1) {
                for (auto &kv : rows[r]) kv.second = -kv.second;
                rhs[r] = -rhs[r];
            }
            used[r] = 1;
            row_of[q] = r;
            for (size_t k = 0; k < np; ++k) {
                if (k == r) continue;
                const int64_t f = row_get(rows[k], p);
                if (!f) continue;
                rows[k] = row_axpy(rows[k], -f, rows[r]);
                rhs[k] -= f * rhs[r];
                for (const auto &kv : rows[k])
                    if (std::llabs(kv.second) > (int64_t{1} << 40))
                        return tu_fail(GFORS_E_ARG, "coefficients grow in the elimination: B_J is not totally unimodular");
            }
        }
        std::vector<SRow> r2(np);
        std::vector<int64_t> h2(np);
        for (size_t q = 0; q < np; ++q) {
            r2[q].swap(rows[row_of[q]]);
            h2[q] = rhs[row_of[q]];
        }
        rows.swap(r2);
        rhs.swap(h2);
    }
    // S and s (pivot order): row q reads  a_q x_pq + sum_{i in Ibar} M_qi x_i = rhs_q
    // with a_q = +-1 and no other pivot column
    U->Srp.assign(np + 1, 0);
    for (size_t q = 0; q < np; ++q) {
        const int64_t bp = row_get(rows[q], U->piv_col[q]);   // +-1 (1 after elimination)
        U->s.push_back(bp * rhs[q]);
        for (const auto &kv : rows[q]) {
            if (kv.first == U->piv_col[q]) continue;
            U->Sci.push_back(static_cast<int32_t>(U->newidx[kv.first]));
            U->Sval.push_back(-bp * kv.second);
        }
        U->Srp[q + 1] = static_cast<int64_t>(U->Sci.size());
    }
    // substitution of one row: dense scratch over new indices + touched list
    std::vector<int64_t> acc(nn, 0);
    std::vector<uint8_t> touched(nn, 0);
    std::vector<int64_t> list;
    auto emit = [&](std::vector<int64_t> &rp, std::vector<int32_t> &ci, std::vector<int32_t> &vv) -> int {
        std::sort(list.begin(), list.end());
        int bad = 0;
        for (int64_t i : list) {
            const int64_t v = acc[i];
            acc[i] = 0;
            touched[i] = 0;
            if (v == 0) continue;
            if (v > std::numeric_limits<int32_t>::max() || v < std::numeric_limits<int32_t>::min()) bad = 1;
            ci.push_back(static_cast<int32_t>(i));
            vv.push_back(static_cast<int32_t>(v));
        }
        list.clear();
        rp.push_back(static_cast<int64_t>(ci.size()));
        return bad ? tu_fail(GFORS_E_ARG, "reformulated coefficient overflows int32") : GFORS_OK;
    };
    auto add = [&](int64_t i, int64_t v) {
        if (!touched[i]) { touched[i] = 1; list.push_back(i); }
        acc[i] += v;
    };
    auto substitute_row = [&](const gfors_csr *M, int64_t r, int64_t rh, std::vector<int64_t> &rp,
                              std::vector<int32_t> &ci, std::vector<int32_t> &vv,
                              std::vector<int64_t> &rv) -> int {
        int64_t nr = rh;
        for (int64_t e = M->row_ptr[r]; e < M->row_ptr[r + 1]; ++e) {
            const int64_t i = M->col_idx[e], a = coef(M, e);
            const int64_t q = piv_index[i];
            if (q < 0) {
                add(U->newidx[i], a);
            } else {
                nr -= a * U->s[q];
                for (int64_t k = U->Srp[q]; k < U->Srp[q + 1]; ++k) add(U->Sci[k], a * U->Sval[k]);
            }
        }
        rv.push_back(nr);
        return emit(rp, ci, vv);
    };
    U->Arp.push_back(0);
    if (A)
        for (int64_t r = 0; r < A->nrows; ++r)
            if ((rc = substitute_row(A, r, b[r], U->Arp, U->Aci, U->Aval, U->bvec))) return rc;
    // bound rows: lower S_p x >= -s_p, then upper -S_p x >= s_p - 1 (trivial ones left out)
    for (int side = 0; side < 2; ++side)
        for (size_t q = 0; q < np; ++q) {
            const int64_t sg = side == 0 ? 1 : -1;
            const int64_t rh = side == 0 ? -U->s[q] : U->s[q] - 1;
            int64_t negsum = 0;
            for (int64_t k = U->Srp[q]; k < U->Srp[q + 1]; ++k)
                if (sg * U->Sval[k] < 0) negsum += sg * U->Sval[k];
            if (negsum >= rh) continue;
            for (int64_t k = U->Srp[q]; k < U->Srp[q + 1]; ++k) add(U->Sci[k], sg * U->Sval[k]);
            U->bvec.push_back(rh);
            if ((rc = emit(U->Arp, U->Aci, U->Aval))) return rc;
        }
    U->Brp.push_back(0);
    for (int64_t r = 0; r < m2; ++r) {
        if (pivots[r] >= 0) continue;
        if ((rc = substitute_row(B, r, d[r], U->Brp, U->Bci, U->Bval, U->dvec))) return rc;
    }
    // objective, linear part: c' = S^T c_I + c_Ibar, c'_0 = <c_I, s>
    U->cvec.assign(nn, 0);
    for (int64_t k = 0; k < nn; ++k) U->cvec[k] = c[U->keep[k]];
    for (size_t q = 0; q < np; ++q) {
        const int64_t cp = c[U->piv_col[q]];
        U->c0 += cp * U->s[q];
        for (int64_t k = U->Srp[q]; k < U->Srp[q + 1]; ++k) U->cvec[U->Sci[k]] += cp * U->Sval[k];
    }
    // quadratic part: every entry Q_ab x_a x_b with x_a, x_b written as affine
    // functions of the kept variables (a kept variable: itself; a pivot: s + S_q x)
    // contributes to c'_0, c' and Q' (this is the theorem's Q', c' and c'_0 terms)
    U->Qrp.push_back(0);
    if (Q && Q->row_ptr[Q->nrows] > 0) {
        std::vector<std::map<int32_t, int64_t>> qrows(nn);
        auto terms = [&](int64_t a, std::vector<std::pair<int32_t, int64_t>> &t, int64_t &cst) {
            t.clear();
            const int64_t q = piv_index[a];
            if (q < 0) {
                cst = 0;
                t.emplace_back(static_cast<int32_t>(U->newidx[a]), 1);
            } else {
                cst = U->s[q];
                for (int64_t k = U->Srp[q]; k < U->Srp[q + 1]; ++k) t.emplace_back(U->Sci[k], U->Sval[k]);
            }
        };
        std::vector<std::pair<int32_t, int64_t>> ta, tb;
        for (int64_t a = 0; a < n; ++a)
            for (int64_t e = Q->row_ptr[a]; e < Q->row_ptr[a + 1]; ++e) {
                const int64_t bcol = Q->col_idx[e], v = coef(Q, e);
                if (!v) continue;
                int64_t ca, cb;
                terms(a, ta, ca);
                terms(bcol, tb, cb);
                U->c0 += v * ca * cb;
                for (const auto &kv : tb) U->cvec[kv.first] += v * ca * kv.second;
                for (const auto &kv : ta) U->cvec[kv.first] += v * cb * kv.second;
                for (const auto &ka : ta)
                    for (const auto &kb : tb) qrows[ka.first][kb.first] += v * ka.second * kb.second;
            }
        for (int64_t k = 0; k < nn; ++k) {
            for (const auto &kv : qrows[k]) {
                if (!kv.second) continue;
                if (kv.second > std::numeric_limits<int32_t>::max() || kv.second < std::numeric_limits<int32_t>::min())
                    return tu_fail(GFORS_E_ARG, "reformulated Q entry overflows int32");
                U->Qci.push_back(kv.first);
                U->Qval.push_back(static_cast<int32_t>(kv.second));
            }
            U->Qrp.push_back(static_cast<int64_t>(U->Qci.size()));
        }
    }
    *out = guard.release();
    return GFORS_OK;
}

int gfors_tu_dims(gfors_tu *U, int64_t *dims) {
    if (!U || !dims) return tu_fail(GFORS_E_ARG, "NULL argument");
    if (U->fac) {
        const gftu::TuFactored &F = *U->fac;
        dims[0] = F.nk;
        dims[1] = F.mA + F.nlow + F.nup;
        dims[2] = F.mB;
        dims[3] = -1;
        dims[4] = -1;
        dims[5] = F.c0;
        dims[6] = -1;
        return GFORS_OK;
    }
    dims[0] = U->n_new;
    dims[1] = static_cast<int64_t>(U->Arp.size()) - 1;
    dims[2] = static_cast<int64_t>(U->Brp.size()) - 1;
    dims[3] = static_cast<int64_t>(U->Aci.size());
    dims[4] = static_cast<int64_t>(U->Bci.size());
    dims[5] = U->c0;
    dims[6] = static_cast<int64_t>(U->Qci.size());
    return GFORS_OK;
}

int gfors_tu_export(gfors_tu *U, int64_t *A_rp, int32_t *A_ci, int32_t *A_val, int64_t *b,
                    int64_t *B_rp, int32_t *B_ci, int32_t *B_val, int64_t *d, int64_t *c,
                    int64_t *kept_vars) {
    if (!U) return tu_fail(GFORS_E_ARG, "NULL handle");
    if (U->fac) {
        if (A_rp || A_ci || A_val || B_rp || B_ci || B_val)
            return tu_fail(GFORS_E_STATE, "a factorised reformulation holds no explicit rows");
        const gftu::TuFactored &F = *U->fac;
        const int64_t m1 = F.mA + F.nlow + F.nup;
        if (b) std::copy(F.rhs_ref.begin(), F.rhs_ref.begin() + m1, b);
        if (d) std::copy(F.rhs_ref.begin() + m1, F.rhs_ref.end(), d);
        if (c) std::copy(F.c_ref.begin(), F.c_ref.end(), c);
        if (kept_vars) std::copy(F.keep.begin(), F.keep.end(), kept_vars);
        return GFORS_OK;
    }
    auto cp = [](auto *dst, const auto &src) {
        if (dst) std::copy(src.begin(), src.end(), dst);
    };
    cp(A_rp, U->Arp); cp(A_ci, U->Aci); cp(A_val, U->Aval); cp(b, U->bvec);
    cp(B_rp, U->Brp); cp(B_ci, U->Bci); cp(B_val, U->Bval); cp(d, U->dvec);
    cp(c, U->cvec); cp(kept_vars, U->keep);
    return GFORS_OK;
}

int gfors_tu_export_q(gfors_tu *U, int64_t *Q_rp, int32_t *Q_ci, int32_t *Q_val) {
    if (!U) return tu_fail(GFORS_E_ARG, "NULL handle");
    if (U->fac) return tu_fail(GFORS_E_STATE, "a factorised reformulation holds no explicit Q'");
    if (U->Qci.empty()) return GFORS_OK;
    if (Q_rp) std::copy(U->Qrp.begin(), U->Qrp.end(), Q_rp);
    if (Q_ci) std::copy(U->Qci.begin(), U->Qci.end(), Q_ci);
    if (Q_val) std::copy(U->Qval.begin(), U->Qval.end(), Q_val);
    return GFORS_OK;
}

int gfors_tu_recover(gfors_tu *U, const uint8_t *x_reduced, uint8_t *x_full) {
    if (!U || !x_reduced || !x_full) return tu_fail(GFORS_E_ARG, "NULL argument");
    if (U->fac) {
        // x_I = M^{-1} (d_J - B_JIbar x_Ibar), exactly
        const gftu::TuFactored &F = *U->fac;
        for (int64_t k = 0; k < F.nk; ++k) x_full[F.keep[k]] = x_reduced[k] ? 1 : 0;
        std::vector<int64_t> v(F.dJ);
        for (int64_t k = 0; k < F.r; ++k)
            for (int32_t e = F.BJrp[k]; e < F.BJrp[k + 1]; ++e) v[k] -= F.BJval[e] * (x_reduced[F.BJci[e]] ? 1 : 0);
        solve_M(F, v);
        int bad = 0;
        for (int64_t k = 0; k < F.r; ++k) {
            if (v[k] != 0 && v[k] != 1) bad = 1;
            x_full[F.tail_var[k]] = v[k] == 1 ? 1 : 0;
        }
        return bad ? tu_fail(GFORS_E_STATE, "reduced point violates a pivot bound") : GFORS_OK;
    }
    for (int64_t k = 0; k < U->n_new; ++k) x_full[U->keep[k]] = x_reduced[k] ? 1 : 0;
    int bad = 0;
    for (size_t q = 0; q < U->piv_col.size(); ++q) {
        int64_t v = U->s[q];
        for (int64_t k = U->Srp[q]; k < U->Srp[q + 1]; ++k) v += U->Sval[k] * (x_reduced[U->Sci[k]] ? 1 : 0);
        if (v != 0 && v != 1) bad = 1;
        x_full[U->piv_col[q]] = v == 1 ? 1 : 0;
    }
    return bad ? tu_fail(GFORS_E_STATE, "reduced point violates a pivot bound") : GFORS_OK;
}

int gfors_tu_factor_info(gfors_tu *U, int64_t *info) {
    if (!U || !info) return tu_fail(GFORS_E_ARG, "NULL argument");
    if (!U->fac) return tu_fail(GFORS_E_STATE, "not a factorised reformulation");
    const gftu::TuFactored &F = *U->fac;
    info[0] = F.r;
    info[1] = static_cast<int64_t>(F.Lci.size());
    info[2] = static_cast<int64_t>(F.Uci.size());
    info[3] = static_cast<int64_t>(F.Lf.lvl.size()) - 1;
    info[4] = static_cast<int64_t>(F.Ub.lvl.size()) - 1;
    info[5] = static_cast<int64_t>(F.Utf.lvl.size()) - 1;
    info[6] = static_cast<int64_t>(F.Ltb.lvl.size()) - 1;
    info[7] = static_cast<int64_t>(F.BJci.size());
    info[8] = F.nnz_S;
    info[9] = F.nnz_ref;
    return GFORS_OK;
}

void gfors_tu_destroy(gfors_tu *U) { delete U; }

}  // extern "C"
