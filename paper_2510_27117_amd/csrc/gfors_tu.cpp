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

#include <algorithm>
#include <cstdlib>
#include <limits>
#include <map>
#include <memory>
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
};

extern "C" {

const char *gfors_tu_last_error(void) { return g_tu_err.c_str(); }

int gfors_tu_create(const gfors_csr *A, const int64_t *b, const gfors_csr *B, const int64_t *d,
                    const gfors_csr *Q, const int64_t *c, int64_t n, const int64_t *pivots,
                    gfors_tu **out) {
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
    if (U->Qci.empty()) return GFORS_OK;
    if (Q_rp) std::copy(U->Qrp.begin(), U->Qrp.end(), Q_rp);
    if (Q_ci) std::copy(U->Qci.begin(), U->Qci.end(), Q_ci);
    if (Q_val) std::copy(U->Qval.begin(), U->Qval.end(), Q_val);
    return GFORS_OK;
}

int gfors_tu_recover(gfors_tu *U, const uint8_t *x_reduced, uint8_t *x_full) {
    if (!U || !x_reduced || !x_full) return tu_fail(GFORS_E_ARG, "NULL argument");
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

void gfors_tu_destroy(gfors_tu *U) { delete U; }

}  // extern "C"
