// Factorised form of the TU reformulation (Theorem and Remark of Sec. 2.4.1).
//
// With pivot rows J (elimination order k), pivot columns I and the kept
// variables Ibar, the pivot block is factorised once, exactly, as
//     M = L U,   M[k][k'] = B[J_{a_k}][I_{b_k'}]   (a, b: row / column order of the elimination)
// with L unit lower and U upper triangular, every entry in {-1, 0, 1} (a pivot
// on a +-1 entry keeps a totally unimodular matrix totally unimodular).  Nothing
// of S = -B_JI^{-1} B_JIbar is stored: the reformulated products are
//     S xbar   = -M^{-1} (B_JIbar xbar)             (rows in order k)
//     S^T v    = -B_JIbar^T M^{-T} v,
// and the reformulated rows are the original rows on the lifted vector
// z = (xbar, t), t = S xbar:  A' xbar = A_.Ibar xbar + A_.I t, the bound rows
// S_p xbar >= -s_p and -S_p xbar >= s_p - 1 read t_p.
#pragma once

#include <cstdint>
#include <vector>

namespace gftu {

// One sparse triangular solve in place, x_k = d_k (x_k - sum_e a_e x_{c_e}),
// with its rows grouped by level (a row reads only rows of earlier levels).
struct HostTrsv {
    std::vector<int32_t> row;   // per position: (k << 1) | (d_k == -1)
    std::vector<int32_t> ptr;   // [r + 1] entries of each position
    std::vector<int32_t> ent;   // (c << 1) | (a == -1)
    std::vector<int32_t> lvl;   // [levels + 1] first position of each level
};

struct TuFactored {
    int64_t n = 0, nk = 0, r = 0;                  // variables, kept variables, pivots
    int64_t mA = 0, nlow = 0, nup = 0, mB = 0;     // reformulated rows: A', S >= -s, -S >= s - 1, B'
    std::vector<int64_t> keep;                     // kept index -> original index
    std::vector<int64_t> tail_var;                 // position k -> original index of I_{b_k}
    // B_JIbar, row k = pivot row J_{a_k}, columns = kept indices; d of that row
    std::vector<int32_t> BJrp, BJci, BJval;
    std::vector<int64_t> dJ;
    std::vector<int64_t> s;                        // s in position order
    std::vector<int32_t> Lrp, Lci, Lval;           // strictly lower part of L, rows k
    std::vector<int32_t> Urp, Uci, Uval, Ud;       // strictly upper part of U, rows k; diagonal
    HostTrsv Lf, Ub, Utf, Ltb;                     // L forward, U backward, U^T forward, L^T backward
    // lifted rows in the reformulated row order (A', kept lower bounds, kept
    // upper bounds, B'): columns < nk kept variables, nk + k position k
    std::vector<int32_t> KLrp, KLci, KLval;
    std::vector<int64_t> rhs_ref;                  // b', -s_p, s_p - 1, d'
    std::vector<int64_t> rhs_orig;                 // b, 0, -1, d (rows on the lifted integer point)
    std::vector<double> rownorm;                   // 2-norm of each reformulated row (exact squares)
    int64_t infeasible_row = -1;                   // a zero reformulated row that no point satisfies
    // objective: Q on the lifted index space (full symmetric), costs
    std::vector<int32_t> QLrp, QLci, QLval;
    std::vector<int64_t> c_keep, c_tail, c_ref;    // c_Ibar, c_I (position order), c'
    int64_t c0 = 0;
    int64_t nnz_ref = 0;                           // entries of the reformulated rows (counted)
    int64_t nnz_S = 0;                             // entries of S (counted)
};

}  // namespace gftu

struct gfors_tu;
// The factorised data of a handle made with GFORS_TU_FACTORED, else null.
const gftu::TuFactored *gfors_tu_factored_data(const gfors_tu *U);
