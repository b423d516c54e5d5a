"""Host-side byte and operation models of bench.py (no GPU): indices charged
only where entries are not one contiguous range, the int16 coefficient size,
and the upper-triangle count of a symmetric Q, each checked against a count
done by brute force on small instances."""
import numpy as np

import bench
from paper_2510_27117_amd import instances as I


def _brute_indexed(bip):
    rows = []
    for M in (bip.A, bip.B):
        if M is None:
            continue
        for j in range(M.nrows):
            rows.append(list(M.col[M.row_ptr[j]:M.row_ptr[j + 1]]))
    row_major = sum(len(r) for r in rows if not (r and r == list(range(r[0], r[0] + len(r)))))
    per_var = {}
    for j, r in enumerate(rows):
        for c in r:
            per_var.setdefault(int(c), []).append(j)
    var_major = sum(len(v) for v in per_var.values() if v != list(range(v[0], v[0] + len(v))))
    return row_major, var_major


def test_indexed_entries_knapsack_batch_is_index_free():
    bip = I.concat_instances(I.knapsack_batch(5, seed=3, n_lo=20, n_hi=60, m_lo=2, m_hi=4))
    assert bench.indexed_entries(bip) == (0, 0) == _brute_indexed(bip)


def test_indexed_entries_mixed():
    for bip in (I.set_cover_bernoulli(60, 30, 0.1, seed=1), I.facility_location(4, 9, seed=2),
                I.knapsack_multi(50, 3, seed=4)):
        assert bench.indexed_entries(bip) == _brute_indexed(bip)


def test_int16_coefficient_bytes():
    small = I.knapsack_multi(50, 3, seed=4)                       # |a| <= 1000
    wide = I.knapsack_multi(50, 3, seed=4, wmax=100_000)          # beyond int16
    nnz = small.A.nnz
    kb_s = bench.kernel_bytes(small, 64, (0, 0))
    kb_w = bench.kernel_bytes(wide, 64, (0, 0))
    assert kb_w["dual"] - kb_s["dual"] == 2 * nnz
    assert kb_w["primal"] - kb_s["primal"] == 2 * nnz


def test_quad_eval_entries_upper_triangle():
    P = I.max_cut_er(300, 6.0, seed=5)                            # symmetric, zero diagonal
    Q = P.Q
    rows = np.repeat(np.arange(Q.nrows), np.diff(Q.row_ptr))
    assert bench.quad_eval_entries(P) == int(np.count_nonzero(Q.col > rows)) == Q.nnz // 2
    # a non-symmetric Q is evaluated in full
    val = Q.values().copy()
    val[0] = 7
    P.Q = I.CSR(Q.nrows, Q.ncols, Q.row_ptr, Q.col, val)
    assert bench.quad_eval_entries(P) == Q.nnz


def test_constant_degree_drops_primal_row_pointers():
    """5 rows per column (the large set cover's structure): no row pointers
    in the primal's bytes; a Bernoulli set cover keeps them."""
    cols = I.set_cover_columns(400, 60, 5, seed=1)
    bern = I.set_cover_bernoulli(400, 60, 0.05, seed=1)
    assert bench.constant_degree(cols) and not bench.constant_degree(bern)
    idx = bench.indexed_entries(cols)
    n, m, nnz = cols.n, cols.m1, cols.A.nnz
    assert bench.kernel_bytes(cols, 64, idx)["primal"] == 16 * n + 4 * idx[1] + 4 * m
