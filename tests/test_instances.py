"""Properties of the seeded synthetic workloads (input recipe)."""
import numpy as np

from paper_2510_27117_amd import instances as I


def test_set_cover_columns_structure():
    P = I.set_cover_columns(5000, 600, 5, seed=0)
    A = P.A
    assert A.val is None and A.nrows == 600 and P.n == 5000
    # each column appears in >= 5 distinct rows (5 drawn + possible repairs)
    rows = np.repeat(np.arange(A.nrows), np.diff(A.row_ptr))
    pairs = rows.astype(np.int64) * P.n + A.col
    assert np.unique(pairs).size == pairs.size          # no duplicates
    per_col = np.bincount(A.col, minlength=P.n)
    assert per_col.min() >= 5
    assert np.all(np.diff(A.row_ptr) >= 1)              # every row coverable
    assert P.c.min() >= 1 and P.c.max() <= 100
    Q = I.set_cover_columns(5000, 600, 5, seed=0)
    assert np.array_equal(Q.A.col, A.col) and np.array_equal(Q.c, P.c)


def test_maxcut_symmetric_and_degree():
    P = I.max_cut_er(2000, 10.0, seed=1)
    D = P.Q
    rows = np.repeat(np.arange(D.nrows), np.diff(D.row_ptr))
    assert np.all(rows != D.col)
    key = rows.astype(np.int64) * P.n + D.col
    keyT = D.col.astype(np.int64) * P.n + rows
    o = np.argsort(key)
    oT = np.argsort(keyT)
    assert np.array_equal(key[o], keyT[oT]) and np.array_equal(D.val[o], D.val[oT])
    deg = np.zeros(P.n, np.int64)
    np.add.at(deg, rows, D.val)
    assert np.array_equal(P.c, -deg)
    assert abs(D.nnz / P.n - 10.0) < 0.5


def test_knapsack_and_ufl_rows():
    P = I.knapsack_multi(50, 4, seed=2)
    W = -I.csr_to_dense(P.A)
    assert W.min() >= 1 and W.max() <= 1000
    assert np.array_equal(-P.b, W.sum(1) // 2)
    F = I.facility_location(3, 4, seed=0)
    assert F.n == 3 + 12 and F.B.nrows == 4 and F.A.nrows == 12
    Bd = I.csr_to_dense(F.B)
    assert np.array_equal(Bd.sum(1), [3, 3, 3, 3])
    Ad = I.csr_to_dense(F.A)
    assert np.all(Ad.sum(1) == 0) and np.all(np.abs(Ad).sum(1) == 2)


def test_concat_offsets():
    parts = I.knapsack_batch(4, seed=3, n_lo=10, n_hi=40, m_lo=2, m_hi=4)
    B = I.concat_instances(parts)
    assert B.num_instances == 4
    assert B.inst_offsets[-1, 0] == sum(p.n for p in parts)
    D = I.csr_to_dense(B.A)
    o = B.inst_offsets
    for t, p in enumerate(parts):
        blk = D[o[t, 1]:o[t + 1, 1], o[t, 0]:o[t + 1, 0]]
        assert np.array_equal(blk, I.csr_to_dense(p.A))
