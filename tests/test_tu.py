"""TU reformulation (Theorem of Sec. 2.4.1): the oracle's version is pinned by
brute force (same optimum, exact objective shift, recovered points feasible),
and the library's host implementation equals it exactly."""
import itertools

import numpy as np
import pytest

from oracle import gfors_oracle as O
from paper_2510_27117_amd import instances as I


def _all(n):
    return np.array(list(itertools.product([0, 1], repeat=n)), dtype=bool)


@pytest.mark.parametrize("nf,nc,seed", [(2, 3, 0), (3, 3, 1), (2, 5, 2)])
def test_oracle_tu_preserves_the_problem(nf, nc, seed):
    P = I.facility_location(nf, nc, seed)
    piv = P.meta["tu_pivots"]
    Pn, c0, rec = O.tu_reformulate(P, piv)
    assert Pn.n == P.n - nc and Pn.B is None
    Xo, Xn = _all(P.n), _all(Pn.n)
    vo, zo = O.evaluate(P, Xo)
    vn, zn = O.evaluate(Pn, Xn)
    # same optimum (objective shifted by c'_0)
    assert int(zo[vo == 0].min()) == int(zn[vn == 0].min()) + c0
    # every feasible reduced point maps to a feasible original point, same value
    for l in np.nonzero(vn == 0)[0]:
        x = rec(Xn[l])
        assert set(np.unique(x)) <= {0, 1}
        v1, z1 = O.evaluate(P, x[None, :].astype(bool))
        assert v1[0] == 0 and z1[0] == zn[l] + c0
    # and every feasible original point is hit by its reduced image
    feas_o = Xo[vo == 0]
    keep = np.setdiff1d(np.arange(P.n), piv)
    vk, zk = O.evaluate(Pn, feas_o[:, keep])
    assert np.all(vk == 0) and np.array_equal(zk + c0, zo[vo == 0])


def test_oracle_tu_general_block_and_dropped_rows():
    """A 2x2 pivot block that is not diagonal (inverse computed) and a kept row."""
    B = [[1, 1, 0, 1, 0], [0, 1, 0, 0, 1], [1, 0, 1, 1, 1]]
    P = I.from_dense([3, -2, 4, 1, 5], A=[[1, 1, 1, 1, 1]], b=[1], B=B, d=[1, 1, 2])
    Pn, c0, rec = O.tu_reformulate(P, np.array([0, 1, -1]))
    X = _all(P.n)
    vo, zo = O.evaluate(P, X)
    vn, zn = O.evaluate(Pn, _all(Pn.n))
    assert int(zo[vo == 0].min()) == int(zn[vn == 0].min()) + c0


def _quad_tu_case(seed):
    """Equality rows with a TU (interval) matrix whose pivot block is lower
    triangular, not an identity; an inequality row; a symmetric integer Q with
    a diagonal."""
    rng = np.random.default_rng(seed)
    B = [[1, 1, 0, 0, 1, 0, 0], [0, 1, 1, 0, 0, 1, 0], [0, 0, 1, 1, 0, 0, 1]]
    Q = rng.integers(-4, 5, size=(7, 7))
    Q = Q + Q.T
    np.fill_diagonal(Q, rng.integers(-3, 4, size=7))
    c = rng.integers(-6, 7, size=7)
    P = I.from_dense(c, A=[[1, 0, 1, 0, 1, 1, 0]], b=[1], B=B, d=[1, 1, 1], Q=Q)
    return P, np.array([1, 2, 3])          # B_JI = [[1,0,0],[1,1,0],[0,1,1]]


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_oracle_tu_with_quadratic_objective(seed):
    """With Q != 0 (Q' = S^T Q_II S + S^T Q_IIbar + Q_IIbar^T S + Q_IbarIbar,
    c' and c'_0 with the quadratic terms): same optimum up to c'_0, and every
    feasible point on either side maps to a feasible point of equal value."""
    P, piv = _quad_tu_case(seed)
    Pn, c0, rec = O.tu_reformulate(P, piv)
    Xo, Xn = _all(P.n), _all(Pn.n)
    vo, zo = O.evaluate(P, Xo)
    vn, zn = O.evaluate(Pn, Xn)
    assert int(zo[vo == 0].min()) == int(zn[vn == 0].min()) + c0
    for l in np.nonzero(vn == 0)[0]:
        x = rec(Xn[l])
        v1, z1 = O.evaluate(P, x[None, :].astype(bool))
        assert set(np.unique(x)) <= {0, 1} and v1[0] == 0 and z1[0] == zn[l] + c0
    keep = np.setdiff1d(np.arange(P.n), piv)
    vk, zk = O.evaluate(Pn, Xo[vo == 0][:, keep])
    assert np.all(vk == 0) and np.array_equal(zk + c0, zo[vo == 0])
    # every point of {0,1}^n' (feasible or not) has the value of its recovery
    # whenever the recovery is binary: the objective map is exact
    for l in range(Xn.shape[0]):
        x = rec(Xn[l])
        if set(np.unique(x)) <= {0, 1}:
            assert O.evaluate(P, x[None, :].astype(bool))[1][0] == zn[l] + c0


@pytest.mark.parametrize("nf,nc,seed", [(2, 3, 0), (4, 7, 3), (6, 40, 5)])
def test_library_tu_equals_oracle(nf, nc, seed):
    from paper_2510_27117_amd import gfors
    P = I.facility_location(nf, nc, seed)
    piv = P.meta["tu_pivots"]
    Pn, c0, rec = O.tu_reformulate(P, piv)
    T = gfors.TUReformulation(P, piv)
    M = T.model
    assert T.constant == c0 and M.n == Pn.n
    assert np.array_equal(M.c, Pn.c)
    assert np.array_equal(I.csr_to_dense(M.A), I.csr_to_dense(Pn.A)) and np.array_equal(M.b, Pn.b)
    assert M.B is None and Pn.B is None
    rng = np.random.default_rng(seed)
    X = _all(M.n) if M.n <= 12 else (rng.random((64, M.n)) < 0.1)
    v, _ = O.evaluate(Pn, X)
    for l in np.nonzero(v == 0)[0][:20]:
        assert np.array_equal(T.recover(X[l].astype(np.uint8)), rec(X[l]).astype(np.uint8))


def test_library_tu_rejects_bad_pivots():
    from paper_2510_27117_amd import gfors
    P = I.from_dense([1, 2, 3], B=[[2, 1, 0], [0, 1, 1]], d=[2, 1])
    with pytest.raises(gfors.GforsError, match="not totally unimodular"):
        gfors.TUReformulation(P, [0, -1])
    P2 = I.from_dense([1, 2, 3], B=[[1, 1, 0], [1, 1, 1]], d=[1, 1])
    with pytest.raises(gfors.GforsError, match="singular"):
        gfors.TUReformulation(P2, [0, 1])
    P3 = I.from_dense([1, 2, 3, 4], B=[[1, 1, 0, 0], [0, 1, 1, 0]], d=[1, 1])
    with pytest.raises(gfors.GforsError, match="pivot of two rows"):
        gfors.TUReformulation(P3, [1, 1])


def _model_dense(M, n):
    return (I.csr_to_dense(M.A) if M.A is not None else None,
            I.csr_to_dense(M.B) if M.B is not None else None,
            I.csr_to_dense(M.Q) if M.Q is not None else np.zeros((n, n), np.int64))


@pytest.mark.parametrize("case", ["tri0", "tri1", "tri2", "interval", "kept_row"])
def test_library_general_tu_equals_oracle(case):
    """General pivot blocks (Gauss-Jordan in integers) and Q != 0: the library's
    reformulated model, constant and recovery equal the oracle's exactly."""
    from paper_2510_27117_amd import gfors
    if case.startswith("tri"):
        P, piv = _quad_tu_case(int(case[3:]))
    elif case == "interval":
        B = [[1, 1, 0, 1, 0], [0, 1, 0, 0, 1], [1, 0, 1, 1, 1]]
        P = I.from_dense([3, -2, 4, 1, 5], A=[[1, 1, 1, 1, 1]], b=[1], B=B, d=[1, 1, 2])
        piv = np.array([0, 1, -1])
    else:
        P = I.from_dense([1, 2, 3, 4], A=[[1, 0, 0, 1]], b=[1], B=[[1, 1, 0, 0], [0, 1, 1, 0], [1, 1, 1, 1]],
                         d=[1, 1, 2])
        piv = np.array([1, 2, -1])
    Pn, c0, rec = O.tu_reformulate(P, piv)
    T = gfors.TUReformulation(P, piv)
    M = T.model
    assert T.constant == c0 and M.n == Pn.n and np.array_equal(M.c, Pn.c)
    got, ref = _model_dense(M, M.n), _model_dense(Pn, Pn.n)
    for g, r in zip(got, ref):
        assert (g is None) == (r is None) and (g is None or np.array_equal(g, r))
    if Pn.A is not None:
        assert np.array_equal(M.b, Pn.b)
    if Pn.B is not None:
        assert np.array_equal(M.d, Pn.d)
    X = _all(M.n)
    v, _ = O.evaluate(Pn, X)
    for l in np.nonzero(v == 0)[0]:
        assert np.array_equal(T.recover(X[l].astype(np.uint8)), rec(X[l]).astype(np.uint8))
