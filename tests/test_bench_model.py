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


def test_signed_index_variant_bytes_facility_location():
    """Dual 5 / primal 6 / primal 7 on a facility location with heavy
    facilities and assignment rows, against the count written out: light items
    4 bytes per entry; heavy rows two row pointers, no indices (contiguous
    columns) and 2-byte coefficients; heavy variables two row pointers, 4-byte
    indices and 2-byte coefficients (6), or per group of 16 one variable's
    entries and a 16-byte table entry (7); vectors as in kernel_bytes."""
    nf, nc = 300, 257
    P = I.facility_location(nf, nc, 4)
    n, m = nf + nf * nc, nf * nc + nc
    kb = bench.kernel_bytes(P, 1024, bench.indexed_entries(P))
    d5 = bench.signed_index_bytes(P, 5, 0, kb)
    assert d5["dual"] == 4 * 2 * nf * nc + 8 * nc + 2 * nf * nc + 4 * n + 20 * m
    assert d5["primal"] == kb["primal"]
    p6 = bench.signed_index_bytes(P, 0, 6, kb)
    assert p6["primal"] == 4 * 2 * nf * nc + 8 * nf + (4 + 2) * nf * nc + 4 * m + 16 * n
    p7 = bench.signed_index_bytes(P, 0, 7, kb)
    groups = (nf + 15) // 16
    assert p7["primal"] == 4 * 2 * nf * nc + groups * (nc * (4 + 2) + 16) + 4 * m + 16 * n
    assert bench.signed_index_bytes(P, 0, 0, kb) == kb
