"""Exact evaluation (EvalBest, Sec. 3) of long general rows as dense int8
digit blocks on the matrix cores: violation counts and objectives identical
to the oracle's row-by-row evaluation, with 1, 2 and 3 signed base-256 digit
planes, several 32-row blocks per instance, blocks cut by the half-full rule,
zero padding inside blocks, equality rows, batches, and candidate widths from
one word to 64.  The row-by-row path (eval_mfma = 0) is checked on the same
draws, and its variants for wide coefficients (64-bit sums; coefficients
beyond 24 bits) as well as the quadratic objective's."""
import numpy as np
import pytest

from oracle import gfors_oracle as O
from paper_2510_27117_amd import instances as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def G():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2510_27117_amd import gfors
    gfors.load_library()
    return gfors


def long_rows_bip(n, m1, m2, wmax, seed, layout="full", density=1.0):
    """n variables, m1 inequality and m2 equality rows of coefficients in
    [-wmax, wmax] \\ {0}.  layout: "full" (every row spans all variables),
    "bands" (rows cover one of four disjoint quarters), "mixed" (random
    sub-ranges of at least half the variables).  density: chance that a
    variable of the row's range has an entry (at least 3 entries per row)."""
    rng = np.random.default_rng(seed)
    m = m1 + m2
    rp, cols, vals = [0], [], []
    for j in range(m):
        if layout == "full":
            lo, hi = 0, n
        elif layout == "bands":
            q = j % 4
            lo, hi = q * n // 4, (q + 1) * n // 4
        else:
            w = int(rng.integers(n // 2, n + 1))
            lo = int(rng.integers(0, n - w + 1))
            hi = lo + w
        cj = np.arange(lo, hi)
        if density < 1.0:
            keep = rng.random(cj.size) < density
            keep[:3] = True
            cj = cj[keep]
        a = rng.integers(1, wmax + 1, size=cj.size) * rng.choice([-1, 1], size=cj.size)
        cols.append(cj)
        vals.append(a)
        rp.append(rp[-1] + cj.size)
    rp = np.asarray(rp, dtype=np.int64)
    col = np.concatenate(cols).astype(np.int32)
    val = np.concatenate(vals).astype(np.int64)
    # right-hand sides near the mean of a half-one candidate so that both
    # outcomes occur; equality rows hit by a random candidate
    x0 = rng.random(n) < 0.5
    rhs = np.array([int(val[rp[j]:rp[j + 1]][x0[col[rp[j]:rp[j + 1]]]].sum()) for j in range(m)],
                   dtype=np.int64)
    rhs[:m1] += rng.integers(-wmax, wmax + 1, size=m1)

    def part(j0, j1):
        if j1 == j0:
            return None
        r = rp[j0:j1 + 1] - rp[j0]
        return I.CSR(j1 - j0, n, r, col[rp[j0]:rp[j1]].copy(), val[rp[j0]:rp[j1]].astype(np.int32))

    c = rng.integers(-50, 51, size=n).astype(np.int64)
    return I.BIP(n=n, c=c, A=part(0, m1), b=rhs[:m1] if m1 else None,
                 B=part(m1, m), d=rhs[m1:] if m2 else None, name=f"longrows_{seed}")


def _check_round(G, P, parts, K, planes, seed):
    import torch
    res = []
    for mf in (1, 0):
        # autotune off: the matrix-core kernel is the one under test (the timed
        # choice between it and the row kernels is tested below)
        prob = G.Problem(P, G.default_params(k_int=20, K_max=max(K, 1024), eval_mfma=mf, autotune=0))
        assert prob.eval_planes() == (planes if mf else 0)
        p = np.random.default_rng(seed).random(P.n).astype(np.float32)
        prob.set_state(p, p, np.zeros(P.m1 + P.m2), 0.0, k=0, round=2)
        v, z = prob.sample_eval(K, p_override=torch.from_numpy(p).to("cuda:0"), outputs=True)
        v, z = v.cpu().numpy(), z.cpu().numpy()
        off = P.inst_offsets if P.inst_offsets is not None else np.array([[0, 0, 0], [P.n, P.m1, P.m2]])
        for t, Pt in enumerate(parts):
            pt = p[off[t, 0]:off[t + 1, 0]].astype(np.float64)
            X = O.sample_bits(pt, K, seed=0, rnd=2, instance=t)
            vo, zo = O.evaluate(Pt, X)
            assert np.array_equal(v[t], vo), (mf, t, np.flatnonzero(v[t] != vo)[:8])
            assert np.array_equal(z[t], zo), (mf, t)
        res.append((v, z))
        prob.close()
    return res


@pytest.mark.parametrize("wmax,planes,n", [(100, 1, 700), (1000, 2, 700), (20000, 2, 700),
                                           (3_000_000, 3, 700), (3_000_000, 3, 2500)])
def test_digit_planes(G, wmax, planes, n):
    """n = 2500 with coefficients up to 3e6: row sums of |a| beyond 2^31
    (64-bit row sums)."""
    P = long_rows_bip(n, 5, 2, wmax, seed=wmax + n)
    _check_round(G, P, [P], 512, planes, seed=1)


@pytest.mark.parametrize("K", [64, 192, 1024, 4096])
def test_candidate_widths(G, K):
    P = long_rows_bip(1100, 40, 3, 1000, seed=K)        # two row blocks (32 + 11)
    _check_round(G, P, [P], K, 2, seed=K)


@pytest.mark.parametrize("layout,density", [("bands", 1.0), ("mixed", 1.0), ("full", 0.6), ("mixed", 0.7)])
def test_block_shapes(G, layout, density):
    """Blocks cut by the half-full rule, zero padding inside a block, rows of
    different ranges in one block."""
    P = long_rows_bip(1500, 70, 0, 1000, seed=7, layout=layout, density=density)
    _check_round(G, P, [P], 256, 2, seed=3)


def test_batch_of_knapsacks(G):
    """A block-diagonal batch of knapsacks of 300 to 4000 variables and 1 to 70
    rows (up to three row blocks) and one instance of rows over different
    ranges with equality rows."""
    rng = np.random.default_rng(4)
    parts = []
    for t in range(9):
        n = int(rng.integers(300, 4001))
        m = int(rng.integers(1, 71))
        parts.append(I.knapsack_multi(n, m, seed=100 + t))
    parts.append(long_rows_bip(900, 3, 2, 1000, seed=5, layout="mixed"))
    P = I.concat_instances(parts)
    _check_round(G, P, parts, 512, 2, seed=9)


def test_not_eligible_falls_back(G):
    """Sparse long rows (far below half full over their span) stay row by row."""
    P = long_rows_bip(4000, 6, 0, 1000, seed=2, layout="full", density=0.1)
    prob = G.Problem(P, G.default_params(k_int=20, K_max=1024))
    assert prob.eval_planes() == 0
    prob.close()
    _check_round(G, P, [P], 128, 0, seed=2)


def test_rowwise_wide_coefficients(G):
    """A coefficient of 9e6 (beyond 24 bits and beyond three base-256 digits)
    in each long row: 32-bit row-by-row sums without the 24-bit multiply-add."""
    P = long_rows_bip(600, 4, 1, 100, seed=11)
    for M in (P.A, P.B):
        v = M.val.astype(np.int64)
        v[M.row_ptr[:-1]] = np.where(np.arange(M.nrows) % 2 == 0, 9_000_000, -9_000_000)
        M.val = v.astype(np.int32)
    _check_round(G, P, [P], 512, 0, seed=4)


def test_quadratic_wide_weights(G):
    """Max cut with weights of +-9e6 (beyond 24 bits): the quadratic
    objective summed with 64-bit selects."""
    import torch
    P = I.max_cut_er(3000, 10.0, seed=21)
    P.Q.val = (P.Q.values().astype(np.int64) * 9_000_000).astype(np.int32)
    P.c = P.c.astype(np.int64) * 9_000_000
    prob = G.Problem(P, G.default_params(k_int=20, K_max=1024))
    p = np.random.default_rng(6).random(P.n).astype(np.float32)
    prob.set_state(p, p, np.zeros(P.m1 + P.m2), 0.0, k=0, round=1)
    v, z = prob.sample_eval(1024, p_override=torch.from_numpy(p).to("cuda:0"), outputs=True)
    X = O.sample_bits(p.astype(np.float64), 1024, seed=0, rnd=1)
    vo, zo = O.evaluate(P, X)
    assert np.array_equal(v.cpu().numpy()[0], vo)
    assert np.array_equal(z.cpu().numpy()[0], zo)
    prob.close()


def _quad_bip(n, seed, symmetric):
    """Random Q with a diagonal part and entries in [-5, 5]: symmetric, or
    with (k, i) differing from (i, k)."""
    import scipy.sparse as sp
    rng = np.random.default_rng(seed)
    E = 6 * n
    i = rng.integers(0, n, size=E)
    k = rng.integers(0, n, size=E)
    v = rng.integers(1, 6, size=E) * rng.choice([-1, 1], size=E)
    d = rng.choice(n, size=n // 3, replace=False)
    dv = rng.integers(-5, 6, size=d.size)
    if symmetric:
        rows = np.concatenate([i, k, d])
        cols = np.concatenate([k, i, d])
        vals = np.concatenate([v, v, dv])
    else:
        v2 = rng.integers(1, 6, size=E) * rng.choice([-1, 1], size=E)
        rows = np.concatenate([i, k, d])
        cols = np.concatenate([k, i, d])
        vals = np.concatenate([v, v2, dv])
    M = sp.coo_matrix((vals, (rows, cols)), shape=(n, n)).tocsr()
    M.eliminate_zeros()
    M.sort_indices()
    Q = I.CSR(n, n, M.indptr.astype(np.int64), M.indices.astype(np.int32), M.data.astype(np.int32))
    c = rng.integers(-20, 21, size=n).astype(np.int64)
    return I.BIP(n=n, c=c, Q=Q, name=f"quad_{seed}")


@pytest.mark.parametrize("symmetric", [True, False])
def test_quadratic_triangle(G, symmetric):
    """<x, Q x> from the upper triangle (off-diagonal entries doubled, the
    diagonal once) for a symmetric Q; the full storage otherwise."""
    import torch
    P = _quad_bip(5000, seed=31 if symmetric else 32, symmetric=symmetric)
    prob = G.Problem(P, G.default_params(k_int=20, K_max=1024))
    p = np.random.default_rng(8).random(P.n).astype(np.float32)
    prob.set_state(p, p, np.zeros(0), 0.0, k=0, round=3)
    v, z = prob.sample_eval(512, p_override=torch.from_numpy(p).to("cuda:0"), outputs=True)
    X = O.sample_bits(p.astype(np.float64), 512, seed=0, rnd=3)
    vo, zo = O.evaluate(P, X)
    assert np.array_equal(v.cpu().numpy()[0], vo)
    assert np.array_equal(z.cpu().numpy()[0], zo)
    prob.close()


def test_timed_choice_of_the_evaluation_kernel(G):
    """With autotune the creation times the matrix-core kernel against the
    row-by-row kernels and keeps one; the counts and objectives are the
    oracle's whichever it keeps, and eval_planes reports the choice."""
    import torch
    parts = I.knapsack_batch(4, seed=21, n_lo=800, n_hi=4000, m_lo=3, m_hi=12)
    P = I.concat_instances(parts)
    prob = G.Problem(P, G.default_params(k_int=20, K_max=1024))
    assert prob.eval_planes() in (0, 2)
    p = np.random.default_rng(3).random(P.n).astype(np.float32)
    prob.set_state(p, p, np.zeros(P.m1 + P.m2), 0.0, k=0, round=4)
    v, z = prob.sample_eval(512, p_override=torch.from_numpy(p).to("cuda:0"), outputs=True)
    v, z = v.cpu().numpy(), z.cpu().numpy()
    off = P.inst_offsets
    for t, Pt in enumerate(parts):
        X = O.sample_bits(p[off[t, 0]:off[t + 1, 0]].astype(np.float64), 512, seed=0, rnd=4, instance=t)
        vo, zo = O.evaluate(Pt, X)
        assert np.array_equal(v[t], vo) and np.array_equal(z[t], zo), t
    prob.close()
