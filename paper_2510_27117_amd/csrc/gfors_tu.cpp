// TU reformulation (Theorem of Sec. 2.4.1) for pivot blocks B_JI that are a
// signed identity: each pivot equality row r holds its pivot column p with
// coefficient +-1 and no other pivot column.  Then B_JI^{-1} = B_JI and
//   x_p = s_p + S_p x,   s_p = b_rp d_r,   S_p[i] = -b_rp b_ri  (i not a pivot)
// is substituted into every other row and into the objective (Q = 0 here):
//   A' = A_.I S + A_.Ibar,  b' = b - A_.I s,  B' = B_JbarI S + B_JbarIbar,
//   d' = d_Jbar - B_JbarI s,  c' = S^T c_I + c_Ibar,  c'_0 = <c_I, s>,
// and 0 <= x_p <= 1 becomes the rows  S_p x >= -s_p  and  -S_p x >= s_p - 1.
// A bound row that every point of the box satisfies (sum of its negative
// coefficients >= right-hand side) is left out: it cuts off nothing, neither
// from the relaxation nor from the binary problem.  Host code only.
#include "../../include/gfors.h"

#include <algorithm>
#include <cstdlib>
#include <memory>
#include <limits>
#include <string>
#include <vector>

namespace {
thread_local std::string g_tu_err;
int tu_fail(int code, const std::string &m) {
    g_tu_err = m;
    return code;
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
    std::vector<int64_t> Arp, Brp, bvec, dvec, cvec;
    std::vector<int32_t> Aci, Aval, Bci, Bval;
    int64_t c0 = 0;
};

extern "C" {

const char *gfors_tu_last_error(void) { return g_tu_err.c_str(); }

int gfors_tu_create(const gfors_csr *A, const int64_t *b, const gfors_csr *B, const int64_t *d,
                    const gfors_csr *Q, const int64_t *c, int64_t n, const int64_t *pivots,
                    gfors_tu **out) {
    if (!out || !c || n <= 0 || !B || !d || !pivots) return tu_fail(GFORS_E_ARG, "NULL argument");
    *out = nullptr;
    if (Q && Q->row_ptr && Q->row_ptr[Q->nrows] > 0)
        return tu_fail(GFORS_E_ARG, "the TU reformulation here supports Q = 0 only");
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
    if ((rc = check(A, "A")) || (rc = check(B, "B"))) return rc;
    auto coef = [](const gfors_csr *M, int64_t e) -> int64_t { return M->val ? M->val[e] : 1; };

    auto *U = new gfors_tu();
    std::unique_ptr<gfors_tu> guard(U);
    U->n = n;
    const int64_t m2 = B->nrows;
    std::vector<int64_t> piv_row_of_col(n, -1);
    std::vector<int64_t> rows_piv;      // pivot rows in order
    std::vector<int64_t> brp_sign;      // b_rp
    for (int64_t r = 0; r < m2; ++r) {
        const int64_t p = pivots[r];
        if (p < 0) continue;
        if (p >= n) return tu_fail(GFORS_E_ARG, "pivot column out of range");
        if (piv_row_of_col[p] >= 0) return tu_fail(GFORS_E_ARG, "a column is the pivot of two rows");
        int64_t bp = 0;
        for (int64_t e = B->row_ptr[r]; e < B->row_ptr[r + 1]; ++e)
            if (B->col_idx[e] == p) bp += coef(B, e);
        if (bp != 1 && bp != -1) return tu_fail(GFORS_E_ARG, "pivot coefficient must be +1 or -1");
        piv_row_of_col[p] = r;
        rows_piv.push_back(r);
        brp_sign.push_back(bp);
        U->piv_col.push_back(p);
    }
    // B_JI must be diagonal: a pivot row holds no other pivot column
    for (size_t q = 0; q < rows_piv.size(); ++q) {
        const int64_t r = rows_piv[q];
        for (int64_t e = B->row_ptr[r]; e < B->row_ptr[r + 1]; ++e) {
            const int64_t i = B->col_idx[e];
            if (i != U->piv_col[q] && piv_row_of_col[i] >= 0 && coef(B, e) != 0)
                return tu_fail(GFORS_E_ARG, "pivot block B_JI is not a signed identity");
        }
    }
    U->newidx.assign(n, -1);
    for (int64_t i = 0; i < n; ++i)
        if (piv_row_of_col[i] < 0) {
            U->newidx[i] = static_cast<int64_t>(U->keep.size());
            U->keep.push_back(i);
        }
    U->n_new = static_cast<int64_t>(U->keep.size());
    if (U->n_new == 0) return tu_fail(GFORS_E_ARG, "every variable is a pivot");
    const int64_t nn = U->n_new;
    // S and s (pivot order)
    const size_t np = U->piv_col.size();
    std::vector<int64_t> piv_index(n, -1);
    U->Srp.assign(np + 1, 0);
    for (size_t q = 0; q < np; ++q) {
        const int64_t r = rows_piv[q], bp = brp_sign[q];
        piv_index[U->piv_col[q]] = static_cast<int64_t>(q);
        U->s.push_back(bp * d[r]);
        for (int64_t e = B->row_ptr[r]; e < B->row_ptr[r + 1]; ++e) {
            const int64_t i = B->col_idx[e];
            if (i == U->piv_col[q]) continue;
            U->Sci.push_back(static_cast<int32_t>(U->newidx[i]));
            U->Sval.push_back(-bp * coef(B, e));
        }
        U->Srp[q + 1] = static_cast<int64_t>(U->Sci.size());
    }
    // substitution of one row: dense scratch over new indices + touched list
    std::vector<int64_t> acc(nn, 0);
    std::vector<uint8_t> touched(nn, 0);
    std::vector<int64_t> list;
    auto emit = [&](std::vector<int64_t> &rp, std::vector<int32_t> &ci, std::vector<int32_t> &vv) -> int {
        std::sort(list.begin(), list.end());
        for (int64_t i : list) {
            const int64_t v = acc[i];
            acc[i] = 0;
            touched[i] = 0;
            if (v == 0) continue;
            if (v > std::numeric_limits<int32_t>::max() || v < std::numeric_limits<int32_t>::min())
                return tu_fail(GFORS_E_ARG, "reformulated coefficient overflows int32");
            ci.push_back(static_cast<int32_t>(i));
            vv.push_back(static_cast<int32_t>(v));
        }
        list.clear();
        rp.push_back(static_cast<int64_t>(ci.size()));
        return GFORS_OK;
    };
    auto add = [&](int64_t i, int64_t v) {
        if (!touched[i]) { touched[i] = 1; list.push_back(i); }
        acc[i] += v;
    };
    auto substitute_row = [&](const gfors_csr *M, int64_t r, int64_t rhs, std::vector<int64_t> &rp,
                              std::vector<int32_t> &ci, std::vector<int32_t> &vv,
                              std::vector<int64_t> &rv) -> int {
        int64_t nr = rhs;
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
            const int64_t rhs = side == 0 ? -U->s[q] : U->s[q] - 1;
            int64_t negsum = 0;
            for (int64_t k = U->Srp[q]; k < U->Srp[q + 1]; ++k)
                if (sg * U->Sval[k] < 0) negsum += sg * U->Sval[k];
            if (negsum >= rhs) continue;
            for (int64_t k = U->Srp[q]; k < U->Srp[q + 1]; ++k) add(U->Sci[k], sg * U->Sval[k]);
            U->bvec.push_back(rhs);
            if ((rc = emit(U->Arp, U->Aci, U->Aval))) return rc;
        }
    U->Brp.push_back(0);
    for (int64_t r = 0; r < m2; ++r) {
        if (pivots[r] >= 0) continue;
        if ((rc = substitute_row(B, r, d[r], U->Brp, U->Bci, U->Bval, U->dvec))) return rc;
    }
    // objective
    U->cvec.assign(nn, 0);
    for (int64_t k = 0; k < nn; ++k) U->cvec[k] = c[U->keep[k]];
    for (size_t q = 0; q < np; ++q) {
        const int64_t cp = c[U->piv_col[q]];
        U->c0 += cp * U->s[q];
        for (int64_t k = U->Srp[q]; k < U->Srp[q + 1]; ++k) U->cvec[U->Sci[k]] += cp * U->Sval[k];
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
