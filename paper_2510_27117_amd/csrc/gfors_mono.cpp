// Monotone relaxation (Sec. 2.4, "Monotone Relaxation") for set-partitioning
// rows, host only.  With a monotone objective (c >= 0 on the row's variables,
// Q = 0) an equality row  sum_{i in R} x_i = 1  may be relaxed to  >= 1  when
// switching a variable of R off can violate no other row: every other row that
// holds one of its variables is an inequality row with a non-positive
// coefficient on it, and no variable lies in two such rows.  The repair maps a
// point of the relaxed problem back: in every relaxed row with more than one
// variable set, the cheapest one (lowest cost, then lowest index) stays and
// the others are switched off; the result is feasible for the original rows
// whenever the relaxed point was feasible, and costs no more.
#include "../../include/gfors.h"

#include <string>
#include <vector>

namespace {
thread_local std::string g_mono_err;
int mono_fail(int code, const std::string &m) {
    g_mono_err = m;
    return code;
}

int check_csr(const gfors_csr *M, int64_t n, const char *nm) {
    if (!M) return GFORS_OK;
    if (M->ncols != n || M->nrows < 0 || !M->row_ptr || M->row_ptr[0] != 0 ||
        (M->row_ptr[M->nrows] > 0 && !M->col_idx))
        return mono_fail(GFORS_E_ARG, std::string(nm) + ": bad CSR header");
    for (int64_t r = 0; r < M->nrows; ++r) {
        if (M->row_ptr[r + 1] < M->row_ptr[r]) return mono_fail(GFORS_E_ARG, std::string(nm) + ": row_ptr decreases");
        for (int64_t e = M->row_ptr[r]; e < M->row_ptr[r + 1]; ++e)
            if (M->col_idx[e] < 0 || M->col_idx[e] >= n)
                return mono_fail(GFORS_E_ARG, std::string(nm) + ": column index out of range");
    }
    return GFORS_OK;
}

inline int32_t coef(const gfors_csr *M, int64_t e) { return M->val ? M->val[e] : 1; }
}  // namespace

extern "C" {

const char *gfors_mono_last_error(void) { return g_mono_err.c_str(); }

int gfors_mono_rows(const gfors_csr *A, const gfors_csr *B, const int64_t *d, const gfors_csr *Q,
                    const int64_t *c, int64_t n, uint8_t *relax) {
    if (!c || n <= 0) return mono_fail(GFORS_E_ARG, "NULL argument");
    int rc;
    if ((rc = check_csr(A, n, "A")) || (rc = check_csr(B, n, "B")) || (rc = check_csr(Q, n, "Q"))) return rc;
    const int64_t m2 = B ? B->nrows : 0;
    if (m2 > 0 && (!d || !relax)) return mono_fail(GFORS_E_ARG, "NULL argument");
    for (int64_t j = 0; j < m2; ++j) relax[j] = 0;
    if (m2 == 0) return GFORS_OK;
    if (Q && Q->row_ptr[Q->nrows] > 0) return GFORS_OK;            // not monotone in general
    // candidate rows: coefficients all +1, right-hand side 1, not empty
    std::vector<uint8_t> cand(m2, 0);
    std::vector<int32_t> use(n, 0), eq_use(n, 0);
    for (int64_t j = 0; j < m2; ++j) {
        bool ok = d[j] == 1 && B->row_ptr[j + 1] > B->row_ptr[j];
        for (int64_t e = B->row_ptr[j]; e < B->row_ptr[j + 1]; ++e) {
            ok = ok && coef(B, e) == 1;
            ++eq_use[B->col_idx[e]];
        }
        cand[j] = ok ? 1 : 0;
        if (ok)
            for (int64_t e = B->row_ptr[j]; e < B->row_ptr[j + 1]; ++e) ++use[B->col_idx[e]];
    }
    // variables with a positive coefficient in some inequality row
    std::vector<uint8_t> pos_in_A(n, 0);
    if (A)
        for (int64_t r = 0; r < A->nrows; ++r)
            for (int64_t e = A->row_ptr[r]; e < A->row_ptr[r + 1]; ++e)
                if (coef(A, e) > 0) pos_in_A[A->col_idx[e]] = 1;
    for (int64_t j = 0; j < m2; ++j) {
        if (!cand[j]) continue;
        bool ok = true;
        for (int64_t e = B->row_ptr[j]; e < B->row_ptr[j + 1] && ok; ++e) {
            const int32_t v = B->col_idx[e];
            // one qualifying row per variable, in no other equality row, cost >= 0,
            // and no positive coefficient in an inequality row
            ok = use[v] == 1 && eq_use[v] == 1 && c[v] >= 0 && !pos_in_A[v];
        }
        relax[j] = ok ? 1 : 0;
    }
    return GFORS_OK;
}

int gfors_mono_repair(const gfors_csr *B, const uint8_t *relax, const int64_t *c, int64_t n,
                      uint8_t *x) {
    if (!B || !relax || !c || !x || n <= 0) return mono_fail(GFORS_E_ARG, "NULL argument");
    int rc;
    if ((rc = check_csr(B, n, "B"))) return rc;
    for (int64_t j = 0; j < B->nrows; ++j) {
        if (!relax[j]) continue;
        int64_t keep = -1, count = 0;
        for (int64_t e = B->row_ptr[j]; e < B->row_ptr[j + 1]; ++e) {
            const int32_t v = B->col_idx[e];
            if (!x[v]) continue;
            ++count;
            if (keep < 0 || c[v] < c[keep] || (c[v] == c[keep] && v < keep)) keep = v;
        }
        if (count <= 1) continue;
        for (int64_t e = B->row_ptr[j]; e < B->row_ptr[j + 1]; ++e) x[B->col_idx[e]] = 0;
        x[keep] = 1;
    }
    return GFORS_OK;
}

}  // extern "C"
