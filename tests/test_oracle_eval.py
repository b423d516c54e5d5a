"""Pins of the oracle's exact evaluation and incumbent rule (EvalBest, Sec. 3)."""
import itertools

import numpy as np
import pytest
import scipy.optimize as so

from oracle import gfors_oracle as O
from paper_2510_27117_amd import instances as I


def _all_binary(n):
    return np.array(list(itertools.product([0, 1], repeat=n)), dtype=bool)


def _milp_opt(P):
    n = P.n
    cons = []
    if P.A is not None:
        cons.append(so.LinearConstraint(I.csr_to_dense(P.A), P.b, np.inf))
    if P.B is not None:
        cons.append(so.LinearConstraint(I.csr_to_dense(P.B), P.d, P.d))
    res = so.milp(P.c.astype(float), constraints=cons, integrality=np.ones(n),
                  bounds=so.Bounds(0, 1))
    return res


@pytest.mark.parametrize("maker", [
    lambda s: I.set_cover_bernoulli(12, 8, 0.2, s),
    lambda s: I.knapsack_multi(12, 3, s),
    lambda s: I.facility_location(2, 5, s),
])
@pytest.mark.parametrize("seed", [0, 1])
def test_brute_force_optimum_matches_milp(maker, seed):
    P = maker(seed)
    X = _all_binary(P.n)
    viol, z = O.evaluate(P, X)
    res = _milp_opt(P)
    assert res.status == 0
    assert (viol == 0).any()
    assert int(z[viol == 0].min()) == int(round(res.fun))
    # every candidate's violation count matches a row-by-row count
    Ad = I.csr_to_dense(P.A) if P.A is not None else np.zeros((0, P.n), np.int64)
    Bd = I.csr_to_dense(P.B) if P.B is not None else np.zeros((0, P.n), np.int64)
    sel = np.random.default_rng(seed).choice(X.shape[0], 64, replace=False)
    for l in sel:
        x = X[l].astype(np.int64)
        v = sum(int(Ad[j] @ x < P.b[j]) for j in range(Ad.shape[0]))
        v += sum(int(Bd[j] @ x != P.d[j]) for j in range(Bd.shape[0]))
        assert v == viol[l]
        assert int(P.c @ x) == z[l]


def test_hand_set_cover():
    # rows {1,2,3}; S1={1,2}, S2={2,3}, S3={1,3} cost 3, S4={1,2,3} cost 5
    A = [[1, 0, 1, 1], [1, 1, 0, 1], [0, 1, 1, 1]]
    P = I.from_dense([3, 3, 3, 5], A=A, b=[1, 1, 1])
    X = np.array([[1, 0, 0, 0], [1, 1, 0, 0], [0, 0, 0, 1]], dtype=bool)
    viol, z = O.evaluate(P, X)
    assert viol.tolist() == [1, 0, 0] and z.tolist() == [3, 6, 5]
    Xa = _all_binary(4)
    v, zz = O.evaluate(P, Xa)
    assert int(zz[v == 0].min()) == 5


def test_hand_knapsack():
    # weights (2,3,4,5), profits (3,4,5,6), capacity 5
    P = I.from_dense([-3, -4, -5, -6], A=[[-2, -3, -4, -5]], b=[-5])
    viol, z = O.evaluate(P, np.array([[1, 1, 0, 0], [1, 0, 1, 0]], dtype=bool))
    assert viol.tolist() == [0, 1] and z.tolist() == [-7, -8]
    v, zz = O.evaluate(P, _all_binary(4))
    assert int(zz[v == 0].min()) == -7


def test_max_cut_identity():
    """With Q = W and c = -deg_w: <x,Qx> + <c,x> = -cut(x)  (Sec. 4.2.3 QP)."""
    # triangle w12 = w13 = 1, w23 = -1
    Q = np.array([[0, 1, 1], [1, 0, -1], [1, -1, 0]])
    P = I.from_dense([-2, 0, 0], Q=Q)
    X = np.array([[1, 0, 0], [1, 1, 0], [0, 1, 1]], dtype=bool)
    _, z = O.evaluate(P, X)
    assert z.tolist() == [-2, 0, -2]
    for seed in range(3):
        G = I.max_cut_er(11, 4.0, seed)
        lo, hi, w = G.meta["edges"]
        X = _all_binary(G.n)
        _, z = O.evaluate(G, X)
        for l in range(0, X.shape[0], 37):
            x = X[l]
            cut = sum(int(wi) for a, b_, wi in zip(lo, hi, w) if x[a] != x[b_])
            assert z[l] == -cut


def test_incumbent_rule_lowest_index_and_strict():
    inc = O.Incumbent()
    X = np.eye(4, dtype=bool)
    assert O.incumbent_update(inc, X, np.array([1, 0, 0, 0]), np.array([-9, 5, 3, 3]), 0, 10)
    assert (inc.z, inc.l, inc.rnd) == (3, 2, 0)
    # equal value later does not replace
    assert not O.incumbent_update(inc, X, np.array([0, 0, 0, 0]), np.array([3, 4, 4, 4]), 1, 20)
    assert (inc.l, inc.rnd) == (2, 0)
    # strictly better replaces
    assert O.incumbent_update(inc, X, np.array([0, 0, 0, 0]), np.array([4, 2, 2, 7]), 2, 30)
    assert (inc.z, inc.l, inc.rnd, inc.k) == (2, 1, 2, 30)
    # nothing feasible: unchanged
    assert not O.incumbent_update(inc, X, np.ones(4), np.zeros(4), 3, 40)


def test_gfors_loop_finds_small_optima():
    """End-to-end Algorithm 1 on tiny instances reaches the brute-force optimum."""
    for P in [I.set_cover_bernoulli(14, 8, 0.2, 0), I.knapsack_multi(14, 2, 1)]:
        inc, st, S, _ = O.run_gfors(P, O.Params(k_int=10), iters=400, K=256)
        X = _all_binary(P.n)
        v, z = O.evaluate(P, X)
        assert inc.z is not None and inc.z == int(z[v == 0].min())
        vv, zz = O.evaluate(P, inc.x[None, :])
        assert vv[0] == 0 and zz[0] == inc.z
