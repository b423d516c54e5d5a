"""Factorised TU reformulation (Remark of Sec. 2.4.1), host side: the handle
made with GFORS_TU_FACTORED forms no S, yet its reformulated model (b', d',
c', c'_0, row and entry counts, the entries of S it counts) and its recovery
x_I = s + S x_Ibar equal the oracle's explicit reformulation exactly."""
import itertools

import numpy as np
import pytest

from oracle import gfors_oracle as O
from paper_2510_27117_amd import instances as I


def _all(n):
    return np.array(list(itertools.product([0, 1], repeat=n)), dtype=bool)


def _quad_tu_case(seed):
    rng = np.random.default_rng(seed)
    B = [[1, 1, 0, 0, 1, 0, 0], [0, 1, 1, 0, 0, 1, 0], [0, 0, 1, 1, 0, 0, 1]]
    Q = rng.integers(-4, 5, size=(7, 7))
    Q = Q + Q.T
    np.fill_diagonal(Q, rng.integers(-3, 4, size=7))
    c = rng.integers(-6, 7, size=7)
    P = I.from_dense(c, A=[[1, 0, 1, 0, 1, 1, 0]], b=[1], B=B, d=[1, 1, 1], Q=Q)
    return P, np.array([1, 2, 3])


def case(name):
    if name.startswith("fl"):
        nf, nc, seed = {"fl0": (2, 3, 0), "fl1": (4, 7, 3)}[name]
        P = I.facility_location(nf, nc, seed)
        return P, P.meta["tu_pivots"]
    if name.startswith("tri"):
        return _quad_tu_case(int(name[3:]))
    if name == "interval":
        B = [[1, 1, 0, 1, 0], [0, 1, 0, 0, 1], [1, 0, 1, 1, 1]]
        return I.from_dense([3, -2, 4, 1, 5], A=[[1, 1, 1, 1, 1]], b=[1], B=B, d=[1, 1, 2]), np.array([0, 1, -1])
    if name == "kept_row":
        P = I.from_dense([1, 2, 3, 4], A=[[1, 0, 0, 1]], b=[1], B=[[1, 1, 0, 0], [0, 1, 1, 0], [1, 1, 1, 1]],
                         d=[1, 1, 2])
        return P, np.array([1, 2, -1])
    if name == "interval_fill":
        # interval rows [0,1], [1,3], [0,4] (consecutive ones: TU); the pivot
        # block [[1,1,0],[0,1,1],[1,1,1]] leaves a multiplier in L
        P = I.from_dense([4, -1, 3, 2, -2, 1], A=[[1, 0, 1, 0, 1, 1], [-1, -1, 0, 0, 0, -1]], b=[1, -2],
                         B=[[1, 1, 0, 0, 0, 0], [0, 1, 1, 1, 0, 0], [1, 1, 1, 1, 1, 0]], d=[1, 1, 2])
        return P, np.array([0, 1, 2])
    if name.startswith("qap"):
        n, seed, tree = {"qap_path4": (4, 0, "path"), "qap_path6": (6, 1, "path"),
                         "qap_rand5": (5, 2, "random"), "qap_rand8": (8, 3, "random")}[name]
        P = I.assignment_qap_like(n, seed, q_density=0.05, tree=tree)
        return P, P.meta["tu_pivots"]
    raise KeyError(name)


CASES = ["fl0", "fl1", "tri0", "tri1", "tri2", "interval", "interval_fill", "kept_row", "qap_path4",
         "qap_path6", "qap_rand5", "qap_rand8"]


def _S_from_recover(rec, P, piv, nred):
    """S column by column from the oracle's recovery (x_I = s + S x_Ibar)."""
    I_ = np.asarray(piv)[np.asarray(piv) >= 0]
    s = rec(np.zeros(nred, np.int64))[I_]
    S = np.zeros((I_.size, nred), np.int64)
    for j in range(nred):
        e = np.zeros(nred, np.int64)
        e[j] = 1
        S[:, j] = rec(e)[I_] - s
    return S


@pytest.mark.parametrize("name", CASES)
def test_factored_model_equals_oracle(name):
    from paper_2510_27117_amd import gfors
    P, piv = case(name)
    Pn, c0, rec = O.tu_reformulate(P, piv)
    T = gfors.TUReformulation(P, piv, factored=True)
    assert T.model is None
    assert (T.n_reduced, T.m1, T.m2) == (Pn.n, Pn.m1, Pn.m2)
    assert T.constant == c0
    assert np.array_equal(T.c, Pn.c)
    if Pn.m1:
        assert np.array_equal(T.b, Pn.b)
    if Pn.m2:
        assert np.array_equal(T.d, Pn.d)
    nnz_ref = (0 if Pn.A is None else Pn.A.nnz) + (0 if Pn.B is None else Pn.B.nnz)
    assert T.info["nnz_reformulated_rows"] == nnz_ref
    S = _S_from_recover(rec, P, piv, Pn.n)
    assert T.info["nnz_S"] == int(np.count_nonzero(S))
    r = int(np.sum(np.asarray(piv) >= 0))
    assert T.info["pivots"] == r
    if name == "interval_fill":
        assert T.info["nnz_L"] > 0       # the L solves are not the identity here
    # the same handle without the flag agrees
    E = gfors.TUReformulation(P, piv)
    assert np.array_equal(E.model.c, T.c) and E.constant == T.constant


@pytest.mark.parametrize("name", CASES)
def test_factored_recovery_equals_oracle(name):
    """x_I = M^{-1}(d_J - B_JIbar x_Ibar) exactly: equal to the oracle's
    s + S x_Ibar whenever that is binary; E_STATE otherwise."""
    from paper_2510_27117_amd import gfors
    P, piv = case(name)
    Pn, c0, rec = O.tu_reformulate(P, piv)
    T = gfors.TUReformulation(P, piv, factored=True)
    rng = np.random.default_rng(7)
    X = _all(Pn.n) if Pn.n <= 10 else (rng.random((300, Pn.n)) < rng.random((300, 1)))
    hit_bin = hit_bad = 0
    for x in X:
        ref = rec(x.astype(np.int64))
        if set(np.unique(ref)) <= {0, 1}:
            assert np.array_equal(T.recover(x.astype(np.uint8)), ref.astype(np.uint8))
            hit_bin += 1
        else:
            with pytest.raises(gfors.GforsError, match="pivot bound"):
                T.recover(x.astype(np.uint8))
            hit_bad += 1
    assert hit_bin > 0
    if name.startswith("qap"):
        assert hit_bad > 0


def test_factored_levels_follow_the_tree_depth():
    """A path-shaped pivot tree gives solves of depth ~ its length; a random
    recursive tree gives shallow ones (levels of the four solves reported)."""
    from paper_2510_27117_amd import gfors
    Pp = I.assignment_qap_like(12, 0, q_density=0.0, tree="path")
    Pr = I.assignment_qap_like(12, 0, q_density=0.0, tree="random")
    Tp = gfors.TUReformulation(Pp, Pp.meta["tu_pivots"], factored=True)
    Tr = gfors.TUReformulation(Pr, Pr.meta["tu_pivots"], factored=True)
    r = 2 * 12 - 1
    assert Tp.info["pivots"] == Tr.info["pivots"] == r
    # a tree incidence block factorises without fill: L = I, U bidiagonal on the path
    assert Tp.info["nnz_L"] == 0 and Tp.info["nnz_U"] == r - 1
    assert max(Tp.info[k] for k in ("levels_U", "levels_Ut")) == r
    assert max(Tr.info[k] for k in ("levels_U", "levels_Ut")) < r // 2


def test_factored_rejects_non_tu_and_asymmetric_q():
    from paper_2510_27117_amd import gfors
    P = I.from_dense([1, 2, 3], B=[[2, 1, 0], [0, 1, 1]], d=[2, 1])
    with pytest.raises(gfors.GforsError, match="totally unimodular"):
        gfors.TUReformulation(P, [0, -1], factored=True)
    P2 = I.from_dense([1, 2, 3], B=[[1, 1, 0], [1, 1, 1]], d=[1, 1])
    with pytest.raises(gfors.GforsError, match="singular"):
        gfors.TUReformulation(P2, [0, 1], factored=True)
    P3 = I.from_dense([1, 2, 3], B=[[1, 1, 0]], d=[1])
    P3.Q = I.csr_from_dense(np.array([[0, 1, 0], [0, 0, 0], [0, 0, 0]]))   # not symmetric
    with pytest.raises(gfors.GforsError, match="symmetric"):
        gfors.TUReformulation(P3, [0], factored=True)
