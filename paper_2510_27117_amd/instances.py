"""Seeded synthetic instance generators for binary integer programs.

    min <x, Q x> + <c, x>   s.t.  A x >= b,  B x = d,  x in {0,1}^n      (eq. bip, Sec. 1)

This module only builds problem DATA (integer CSR matrices and integer
vectors).  It holds none of the method's arithmetic, so both the CPU oracle
side (tests) and the GPU side (binding, bench) may take inputs from it.

Every generator draws from ``numpy.random.default_rng(seed)`` (PCG64).  The
problem classes are the ones of Sec. 4 (set cover, knapsack, max cut,
facility location); the sizes and distributions are the synthetic workloads
this library is benchmarked on (the paper's own generators are not given).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np


@dataclass
class CSR:
    """Integer CSR matrix: row_ptr int64[nrows+1], col int32[nnz], val int32[nnz] or None (= all ones)."""
    nrows: int
    ncols: int
    row_ptr: np.ndarray
    col: np.ndarray
    val: Optional[np.ndarray] = None

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def values(self) -> np.ndarray:
        """Coefficient array (materialises the implicit ones)."""
        if self.val is None:
            return np.ones(self.nnz, dtype=np.int32)
        return self.val


@dataclass
class BIP:
    """One binary integer program of the form (eq. bip).

    A / B / Q may be None (no inequality rows / no equality rows / Q = 0).
    Q is stored in full symmetric form.  ``inst_offsets`` is set for a batch
    of independent instances concatenated block-diagonally: rows of the
    int64 array [num_instances+1, 3] hold the (variable, inequality row,
    equality row) start offsets of each instance.
    """
    n: int
    c: np.ndarray
    A: Optional[CSR] = None
    b: Optional[np.ndarray] = None
    B: Optional[CSR] = None
    d: Optional[np.ndarray] = None
    Q: Optional[CSR] = None
    name: str = ""
    inst_offsets: Optional[np.ndarray] = None
    meta: dict = field(default_factory=dict)

    @property
    def m1(self) -> int:
        return 0 if self.A is None else self.A.nrows

    @property
    def m2(self) -> int:
        return 0 if self.B is None else self.B.nrows

    @property
    def num_instances(self) -> int:
        return 1 if self.inst_offsets is None else int(self.inst_offsets.shape[0] - 1)


# ----------------------------------------------------------------------------
# CSR assembly helpers (pure data layout)
# ----------------------------------------------------------------------------

def csr_from_coo(nrows: int, ncols: int, rows: np.ndarray, cols: np.ndarray,
                 vals: Optional[np.ndarray]) -> CSR:
    """Sort (row, col) pairs into CSR; duplicate entries must not occur."""
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    order = np.lexsort((cols, rows))
    rows = rows[order]
    cols = cols[order]
    counts = np.bincount(rows, minlength=nrows)
    row_ptr = np.zeros(nrows + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    v = None
    if vals is not None:
        v = np.asarray(vals, dtype=np.int32)[order]
    return CSR(nrows, ncols, row_ptr, cols.astype(np.int32), v)


def csr_from_dense(M: np.ndarray, unit: bool = False) -> CSR:
    M = np.asarray(M, dtype=np.int64)
    r, c = np.nonzero(M)
    vals = None if unit else M[r, c]
    if unit:
        assert np.all(M[r, c] == 1)
    return csr_from_coo(M.shape[0], M.shape[1], r, c, vals)


def csr_to_dense(A: CSR) -> np.ndarray:
    D = np.zeros((A.nrows, A.ncols), dtype=np.int64)
    rows = np.repeat(np.arange(A.nrows), np.diff(A.row_ptr))
    np.add.at(D, (rows, A.col.astype(np.int64)), A.values().astype(np.int64))
    return D


def _vec(x) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(x, dtype=np.int64))


def from_dense(c, A=None, b=None, B=None, d=None, Q=None, name="dense") -> BIP:
    """Build a BIP from small dense integer arrays (tests and examples)."""
    c = _vec(c)
    n = c.shape[0]
    P = BIP(n=n, c=c, name=name)
    if A is not None and np.asarray(A).size:
        P.A = csr_from_dense(np.asarray(A).reshape(-1, n))
        P.b = _vec(b)
    if B is not None and np.asarray(B).size:
        P.B = csr_from_dense(np.asarray(B).reshape(-1, n))
        P.d = _vec(d)
    if Q is not None and np.any(np.asarray(Q)):
        Qd = np.asarray(Q, dtype=np.int64)
        assert np.array_equal(Qd, Qd.T), "Q must be symmetric"
        P.Q = csr_from_dense(Qd)
    return P


# ----------------------------------------------------------------------------
# Problem classes of Sec. 4
# ----------------------------------------------------------------------------

def set_cover_bernoulli(n: int, m: int, density: float, seed: int, cmax: int = 100) -> BIP:
    """Set cover (Sec. 4.2.1): column i covers row j i.i.d. with prob ``density``;
    afterwards every row gets one uniformly chosen column forced to cover it.
    c ~ U{1..cmax}, b = 1, Q = 0."""
    rng = np.random.default_rng(seed)
    M = rng.random((m, n)) < density
    forced = rng.integers(0, n, size=m)
    M[np.arange(m), forced] = True
    c = rng.integers(1, cmax + 1, size=n).astype(np.int64)
    r, cc = np.nonzero(M)
    A = csr_from_coo(m, n, r, cc, None)
    return BIP(n=n, c=c, A=A, b=np.ones(m, dtype=np.int64),
               name=f"setcover_bern_n{n}_m{m}_s{seed}")


def set_cover_columns(n: int, m: int, per_col: int, seed: int, cmax: int = 100) -> BIP:
    """Large set cover: each column covers ``per_col`` distinct uniformly random
    rows (all coefficients 1).  A row left uncovered receives one random
    column.  c ~ U{1..cmax}, b = 1."""
    rng = np.random.default_rng(seed)
    rows = rng.integers(0, m, size=(n, per_col), dtype=np.int64)
    # redraw duplicates inside a column until all are distinct
    for _ in range(64):
        s = np.sort(rows, axis=1)
        dup_mask_sorted = np.zeros_like(s, dtype=bool)
        dup_mask_sorted[:, 1:] = s[:, 1:] == s[:, :-1]
        bad = np.nonzero(dup_mask_sorted.any(axis=1))[0]
        if bad.size == 0:
            break
        rows[bad] = np.sort(rows[bad], axis=1)
        srt = rows[bad]
        dm = np.zeros_like(srt, dtype=bool)
        dm[:, 1:] = srt[:, 1:] == srt[:, :-1]
        srt[dm] = rng.integers(0, m, size=int(dm.sum()))
        rows[bad] = srt
    cols = np.repeat(np.arange(n, dtype=np.int64), per_col)
    rflat = rows.reshape(-1)
    covered = np.bincount(rflat, minlength=m) > 0
    empty = np.nonzero(~covered)[0]
    if empty.size:
        extra_cols = rng.integers(0, n, size=empty.size)
        rflat = np.concatenate([rflat, empty])
        cols = np.concatenate([cols, extra_cols])
        # an extra (row, col) pair cannot duplicate: the row was empty
    c = rng.integers(1, cmax + 1, size=n).astype(np.int64)
    A = csr_from_coo(m, n, rflat, cols, None)
    return BIP(n=n, c=c, A=A, b=np.ones(m, dtype=np.int64),
               name=f"setcover_cols_n{n}_m{m}_k{per_col}_s{seed}")


def knapsack_multi(n: int, m: int, seed: int, wmax: int = 1000, pmax: int = 1000) -> BIP:
    """Multidimensional knapsack (Sec. 4.2.2 with m capacity rows):
    max <profit, x> s.t. W x <= cap, written as  -W x >= -cap,  c = -profit.
    W ~ U{1..wmax} dense, cap = floor(row sum / 2), profit ~ U{1..pmax}."""
    rng = np.random.default_rng(seed)
    W = rng.integers(1, wmax + 1, size=(m, n), dtype=np.int32)
    profit = rng.integers(1, pmax + 1, size=n).astype(np.int64)
    cap = W.sum(axis=1, dtype=np.int64) // 2
    # dense rows: CSR written directly (row j holds columns 0..n-1)
    A = CSR(m, n, np.arange(m + 1, dtype=np.int64) * n,
            np.tile(np.arange(n, dtype=np.int32), m), (-W).reshape(-1))
    return BIP(n=n, c=-profit, A=A, b=-cap, name=f"knapsack_n{n}_m{m}_s{seed}")


def max_cut_er(n: int, avg_degree: float, seed: int) -> BIP:
    """Max cut as an unconstrained BIP (QP form of Sec. 4.2.3).

    Erdos-Renyi G(n, p = avg_degree/(n-1)), weights uniform in {-1, +1}.
    With Q = W (symmetric, zero diagonal) and c_i = -sum_j w_ij,
    <x,Qx> + <c,x> = -sum_{ij in E} w_ij (x_i + x_j - 2 x_i x_j) = -cut(x)."""
    rng = np.random.default_rng(seed)
    p = avg_degree / max(n - 1, 1)
    npairs = n * (n - 1) // 2
    E = int(rng.binomial(npairs, p))
    # sample E distinct unordered pairs uniformly
    keys = np.empty(0, dtype=np.int64)
    while keys.size < E:
        need = E - keys.size
        i = rng.integers(0, n, size=2 * need + 16, dtype=np.int64)
        j = rng.integers(0, n, size=2 * need + 16, dtype=np.int64)
        ok = i != j
        lo = np.minimum(i[ok], j[ok])
        hi = np.maximum(i[ok], j[ok])
        keys = np.unique(np.concatenate([keys, lo * n + hi]))
    if keys.size > E:
        keys = rng.permutation(keys)[:E]
        keys.sort()
    lo = keys // n
    hi = keys % n
    w = rng.choice(np.array([-1, 1], dtype=np.int64), size=E)
    rows = np.concatenate([lo, hi])
    cols = np.concatenate([hi, lo])
    vals = np.concatenate([w, w])
    Q = csr_from_coo(n, n, rows, cols, vals)
    deg = np.zeros(n, dtype=np.int64)
    np.add.at(deg, lo, w)
    np.add.at(deg, hi, w)
    return BIP(n=n, c=-deg, Q=Q, name=f"maxcut_er_n{n}_deg{avg_degree}_s{seed}",
               meta={"edges": (lo, hi, w)})


def facility_location(n_f: int, n_c: int, seed: int, scale: int = 1000,
                      open_lo: int = 500, open_hi: int = 5000) -> BIP:
    """Uncapacitated facility location (Sec. 4.2.5).

    Facilities and customers uniform in the unit square; assignment cost
    rint(scale * distance); opening cost ~ U{open_lo..open_hi}.
    Variables: open_i (n_f of them) first, then assign_ij at index
    n_f + j * n_f + i.  Rows: sum_i assign_ij = 1 (equality, one per customer)
    and open_i - assign_ij >= 0 (inequality, one per pair)."""
    rng = np.random.default_rng(seed)
    F = rng.random((n_f, 2))
    C = rng.random((n_c, 2))
    dist = np.sqrt(((C[:, None, :] - F[None, :, :]) ** 2).sum(-1))  # [n_c, n_f]
    assign_cost = np.rint(scale * dist).astype(np.int64)
    open_cost = rng.integers(open_lo, open_hi + 1, size=n_f).astype(np.int64)
    n = n_f + n_f * n_c
    c = np.concatenate([open_cost, assign_cost.reshape(-1)])
    # equality rows: customer j -> variables n_f + j*n_f + [0, n_f)
    eq_rows = np.repeat(np.arange(n_c, dtype=np.int64), n_f)
    eq_cols = n_f + np.arange(n_f * n_c, dtype=np.int64)
    B = csr_from_coo(n_c, n, eq_rows, eq_cols, None)
    # inequality rows: pair (j, i) -> row j*n_f + i: +1 on open_i, -1 on assign_ij
    npair = n_f * n_c
    pr = np.arange(npair, dtype=np.int64)
    open_col = pr % n_f
    assign_col = n_f + pr
    rows = np.concatenate([pr, pr])
    cols = np.concatenate([open_col, assign_col])
    vals = np.concatenate([np.ones(npair, np.int64), -np.ones(npair, np.int64)])
    A = csr_from_coo(npair, n, rows, cols, vals)
    # one assignment per customer to eliminate by a TU reformulation: the
    # customer's nearest facility (ties to the lowest index)
    nearest = np.argmin(assign_cost, axis=1)
    pivots = n_f + np.arange(n_c, dtype=np.int64) * n_f + nearest
    return BIP(n=n, c=c, A=A, b=np.zeros(npair, dtype=np.int64), B=B,
               d=np.ones(n_c, dtype=np.int64),
               name=f"ufl_f{n_f}_c{n_c}_s{seed}",
               meta={"n_f": n_f, "n_c": n_c, "tu_pivots": pivots})


def assignment_qap_like(n: int, seed: int, q_density: float = 0.02, q_max: int = 5,
                        tree: str = "path", q_per_var: Optional[float] = None) -> BIP:
    """2D assignment with a sparse symmetric quadratic term and one knapsack row.

    Variables x_ij (index i*n + j); equality rows: sum_j x_ij = 1 (row i) then
    sum_i x_ij = 1 (column j), a bipartite incidence matrix (totally
    unimodular).  c_ij ~ U{1..100}; Q symmetric with off-diagonal entries
    ~ U{-q_max..q_max} w.p. q_density, zero diagonal; one row
    -sum w_ij x_ij >= -cap with w ~ U{1..20}, cap = 12 n.
    meta["tu_pivots"]: a spanning tree of the bipartite graph as pivot columns,
    so the pivot block is not a signed identity.  tree="path": row i -> x_ii,
    column j >= 1 -> x_{j-1,j} (a path of 2n - 1 edges: the deepest tree);
    tree="random": a random recursive tree rooted at column 0 (each node, in
    random order, hangs from a uniformly chosen earlier node of the other side:
    depth O(log n)), each node's row pivoting on the edge to its parent.
    Column 0's row is kept either way.  q_per_var: when given, Q has about
    q_per_var entries per variable drawn as random pairs (for sizes where
    scanning all pairs is too slow) instead of each pair w.p. q_density."""
    rng = np.random.default_rng(seed)
    N = n * n
    c = rng.integers(1, 101, size=N).astype(np.int64)
    idx = np.arange(N, dtype=np.int64)
    rows = np.concatenate([idx // n, n + idx % n])
    cols = np.concatenate([idx, idx])
    B = csr_from_coo(2 * n, N, rows, cols, None)
    if q_per_var is None:
        iu, ju = np.triu_indices(N, k=1)
        pick = rng.random(iu.size) < q_density
        iu, ju = iu[pick], ju[pick]
    else:
        cnt = int(q_per_var * N / 2)
        a, b2 = rng.integers(0, N, size=cnt), rng.integers(0, N, size=cnt)
        a, b2 = np.minimum(a, b2), np.maximum(a, b2)
        key = np.unique(a[a != b2] * N + b2[a != b2])
        iu, ju = key // N, key % N
    w = rng.integers(-q_max, q_max + 1, size=iu.size)
    nz = w != 0
    iu, ju, w = iu[nz], ju[nz], w[nz]
    Q = csr_from_coo(N, N, np.concatenate([iu, ju]), np.concatenate([ju, iu]), np.concatenate([w, w]))
    wk = rng.integers(1, 21, size=N)
    A = csr_from_coo(1, N, np.zeros(N, dtype=np.int64), idx, -wk)
    piv = np.empty(2 * n, dtype=np.int64)
    if tree == "path":
        piv[:n] = np.arange(n) * n + np.arange(n)
        piv[n] = -1
        piv[n + 1:] = (np.arange(1, n) - 1) * n + np.arange(1, n)
    elif tree == "random":
        # nodes 0..n-1 = row constraints i, n..2n-1 = column constraints j; root = column 0
        trng = np.random.default_rng(seed + 7919)
        placed = ([], [n])                      # placed row nodes, placed column nodes
        pending = list(trng.permutation(np.r_[np.arange(n), np.arange(n + 1, 2 * n)]))
        piv[n] = -1
        while pending:
            v = int(pending.pop(0))
            other = placed[1] if v < n else placed[0]
            if not other:
                pending.append(v)
                continue
            u = other[int(trng.integers(0, len(other)))]
            i, j = (v, u - n) if v < n else (u, v - n)
            piv[v] = i * n + j
            placed[0 if v < n else 1].append(v)
    else:
        raise ValueError(f"unknown tree {tree!r}")
    return BIP(n=N, c=c, A=A, b=np.array([-12 * n], dtype=np.int64), B=B,
               d=np.ones(2 * n, dtype=np.int64), Q=Q, name=f"assignq_n{n}_s{seed}",
               meta={"tu_pivots": piv})


def assignment_3d(n: int, seed: int, c_hi: int = 100) -> BIP:
    """3D assignment (Sec. 2.4.2, eq. assign3d): x_ijk at index (i n + j) n + k,
    c ~ U{1..c_hi}; equality rows sum_{j,k} x_ijk = 1 (i), then
    sum_{i,k} x_ijk = 1 (j), then sum_{i,j} x_ijk = 1 (k)."""
    rng = np.random.default_rng(seed)
    N = n ** 3
    c = rng.integers(1, c_hi + 1, size=N).astype(np.int64)
    v = np.arange(N, dtype=np.int64)
    i, j, k = v // (n * n), (v // n) % n, v % n
    rows = np.concatenate([i, n + j, 2 * n + k])
    cols = np.concatenate([v, v, v])
    B = csr_from_coo(3 * n, N, rows, cols, None)
    return BIP(n=N, c=c, B=B, d=np.ones(3 * n, dtype=np.int64), name=f"assign3d_n{n}_s{seed}",
               meta={"assign3d_n": n})


def knapsack_batch(num: int, seed: int, n_lo: int = 1000, n_hi: int = 50000,
                   m_lo: int = 5, m_hi: int = 50) -> List[BIP]:
    """Batch of multidimensional knapsacks: n log-uniform in [n_lo, n_hi],
    m ~ U{m_lo..m_hi}; instance t uses seed (seed, t)."""
    rng = np.random.default_rng(seed)
    ns = np.rint(np.exp(rng.uniform(np.log(n_lo), np.log(n_hi), size=num))).astype(np.int64)
    ms = rng.integers(m_lo, m_hi + 1, size=num)
    seeds = rng.integers(0, 2**31 - 1, size=num)
    return [knapsack_multi(int(ns[t]), int(ms[t]), int(seeds[t])) for t in range(num)]


def _stack_csr(mats: Sequence[Optional[CSR]], nrows: Sequence[int], col_off: Sequence[int],
               ncols_total: int) -> Optional[CSR]:
    if all(M is None for M in mats):
        return None
    unit = all(M is None or M.val is None for M in mats)
    rps, cols, vals = [np.zeros(1, dtype=np.int64)], [], []
    base = 0
    for M, nr, co in zip(mats, nrows, col_off):
        if M is None:
            rps.append(np.full(nr, base, dtype=np.int64))
            continue
        rps.append(M.row_ptr[1:] + base)
        cols.append(M.col.astype(np.int64) + co)
        if not unit:
            vals.append(M.values())
        base += M.nnz
    row_ptr = np.concatenate(rps)
    col = np.concatenate(cols).astype(np.int32) if cols else np.zeros(0, np.int32)
    val = None if unit else np.concatenate(vals).astype(np.int32)
    return CSR(int(sum(nrows)), ncols_total, row_ptr, col, val)


def concat_instances(insts: Sequence[BIP]) -> BIP:
    """Block-diagonal concatenation of independent instances (batched form).

    Variables, inequality rows and equality rows of instance t occupy
    contiguous ranges given by ``inst_offsets[t]`` .. ``inst_offsets[t+1]``."""
    T = len(insts)
    off = np.zeros((T + 1, 3), dtype=np.int64)
    for t, P in enumerate(insts):
        off[t + 1] = off[t] + np.array([P.n, P.m1, P.m2])
    n = int(off[-1, 0])
    c = np.concatenate([P.c for P in insts]).astype(np.int64)
    A = _stack_csr([P.A for P in insts], [P.m1 for P in insts], off[:-1, 0], n)
    B = _stack_csr([P.B for P in insts], [P.m2 for P in insts], off[:-1, 0], n)
    Q = _stack_csr([P.Q for P in insts], [P.n if P.Q is not None else P.n for P in insts],
                   off[:-1, 0], n) if any(P.Q is not None for P in insts) else None
    b = np.concatenate([P.b for P in insts if P.A is not None]) if A is not None else None
    d = np.concatenate([P.d for P in insts if P.B is not None]) if B is not None else None
    return BIP(n=n, c=c, A=A, b=b, B=B, d=d, Q=Q, name=f"batch{T}", inst_offsets=off)


# ----------------------------------------------------------------------------
# Named workloads
# ----------------------------------------------------------------------------

def workload(name: str, seed: int = 0) -> BIP:
    """The synthetic workloads, by name.

    setcover_small : n=200, m=100 set cover, density 0.05 + forced cover
    setcover_large : n=2,000,000, m=200,000, 5 distinct rows per column
    maxcut         : n=200,000 Erdos-Renyi, average degree 10, weights +-1
    knapsack_batch : 512 multidimensional knapsacks, n in [1e3, 5e4], m in [5, 50]
    ufl            : 1,000 facilities x 10,000 customers
    qap_tu         : 2D assignment n = 300 (90,000 variables) with a quadratic
                     term of ~10 entries per variable and a knapsack row; its
                     meta["tu_pivots"] a random recursive spanning tree (599 pivots)
    """
    if name == "setcover_small":
        return set_cover_bernoulli(200, 100, 0.05, seed)
    if name == "setcover_large":
        return set_cover_columns(2_000_000, 200_000, 5, seed)
    if name == "maxcut":
        return max_cut_er(200_000, 10.0, seed)
    if name == "knapsack_batch":
        return concat_instances(knapsack_batch(512, seed))
    if name == "ufl":
        return facility_location(1000, 10000, seed)
    if name == "qap_tu":
        return assignment_qap_like(300, seed, tree="random", q_per_var=10.0)
    raise KeyError(name)
