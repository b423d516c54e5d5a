"""Pins of the 3D-assignment sampler oracle (Algorithm 4, Sec. 2.4.2):
feasibility of every candidate, the greedy partial assignment's defining
property, uniform random completions (chi-square), the local steps never
raising the cost and ending at pairwise-interchange optima, a 0/1 p at an
assignment reproduced, and the brute-force optimum reached for n = 3."""
import itertools

import numpy as np
import pytest
from scipy import stats

from oracle import assign3d_oracle as A3
from oracle import gfors_oracle as O
from paper_2510_27117_amd import instances as I


@pytest.mark.parametrize("n,gamma,L", [(3, 1, 0), (4, 2, 5), (6, 3, 20), (7, 0, 3), (5, 40, 8)])
def test_every_candidate_is_an_assignment(n, gamma, L):
    P = I.assignment_3d(n, seed=n)
    p = np.random.default_rng(n).random(n ** 3)
    X, z = A3.assign3d_sample(p, P.c, n, 16, gamma, L, seed=3, rnd=1)
    v, zo = O.evaluate(P, X)
    assert np.all(v == 0) and np.array_equal(z, zo)
    assert np.all(X.sum(axis=1) == n)


def test_greedy_partial_assignment_property():
    """Taken entries are conflict-free, and an entry of the top list is left
    out exactly when it conflicts with an entry taken before it."""
    rng = np.random.default_rng(1)
    for n, gamma in [(5, 2), (6, 3), (8, 1), (4, 16)]:
        p = np.round(rng.random(n ** 3), 1)          # many ties
        J0, K0 = A3.partial_assignment(p, n, gamma)
        top = A3.top_entries(p, gamma * n)
        # the top list: positive entries sorted by p descending, ties by index,
        # and no larger p left out
        assert top.size == min(gamma * n, int(np.count_nonzero(p > 0))) and np.all(p[top] > 0)
        assert np.all(np.diff(p[top]) <= 0)
        for a, b in zip(top[:-1], top[1:]):
            assert p[a] > p[b] or a < b
        rest = np.setdiff1d(np.arange(n ** 3), top)
        assert rest.size == 0 or top.size == 0 or p[rest].max() <= p[top].min()
        taken = {(i, J0[i], K0[i]) for i in range(n) if J0[i] >= 0}
        assert len({t[1] for t in taken}) == len(taken) == len({t[2] for t in taken})
        seen = []
        for v in top:
            t = (v // (n * n), (v // n) % n, v % n)
            conflict = any(t[0] == s[0] or t[1] == s[1] or t[2] == s[2] for s in seen)
            assert (t in taken) == (not conflict)
            if t in taken:
                seen.append(t)


def test_random_completion_is_uniform():
    """gamma = 0 (nothing fixed), L = 0: the 3!^2 = 36 assignments of n = 3 are
    equally likely (chi-square at 1 %); with one triple fixed by p, the 2!^2 = 4
    completions are."""
    n = 3
    c = np.ones(n ** 3, dtype=np.int64)
    X, _ = A3.assign3d_sample(np.zeros(n ** 3), c, n, 3600, 0, 0, seed=11, rnd=0)
    keys = [tuple(np.nonzero(x)[0]) for x in X]
    cnt = np.array(list({k: keys.count(k) for k in set(keys)}.values()))
    assert cnt.size == 36
    assert stats.chisquare(cnt).pvalue > 0.01
    p = np.zeros(n ** 3)
    p[(1 * n + 2) * n + 0] = 1.0                       # fixes (1, 2, 0)
    X, _ = A3.assign3d_sample(p, c, n, 800, 1, 0, seed=12, rnd=0)
    assert np.all(X[:, (1 * n + 2) * n + 0])
    keys = [tuple(np.nonzero(x)[0]) for x in X]
    cnt = np.array(list({k: keys.count(k) for k in set(keys)}.values()))
    assert cnt.size == 4 and stats.chisquare(cnt).pvalue > 0.01


def _pairwise_optimal(x, C, n):
    idx = np.nonzero(x)[0]
    J = np.empty(n, dtype=np.int64)
    K = np.empty(n, dtype=np.int64)
    for v in idx:
        J[v // (n * n)], K[v // (n * n)] = (v // n) % n, v % n
    for a in range(n):
        for b in range(n):
            if a == b:
                continue
            cur = C[a, J[a], K[a]] + C[b, J[b], K[b]]
            if C[a, J[b], K[a]] + C[b, J[a], K[b]] < cur or C[a, J[a], K[b]] + C[b, J[b], K[a]] < cur:
                return False
    return True


def test_local_steps_never_raise_cost_and_reach_interchange_optima():
    n = 6
    P = I.assignment_3d(n, seed=2)
    C = P.c.reshape(n, n, n)
    p = np.random.default_rng(2).random(n ** 3)
    X0, z0 = A3.assign3d_sample(p, P.c, n, 32, 2, 0, seed=5, rnd=3)
    X1, z1 = A3.assign3d_sample(p, P.c, n, 32, 2, 4, seed=5, rnd=3)
    X2, z2 = A3.assign3d_sample(p, P.c, n, 32, 2, 300, seed=5, rnd=3)
    assert np.all(z1 <= z0) and np.all(z2 <= z1) and np.any(z2 < z0)
    assert all(_pairwise_optimal(x, C, n) for x in X2)


def test_zero_one_p_at_an_assignment_is_reproduced():
    n = 5
    P = I.assignment_3d(n, seed=4)
    J, K = np.array([3, 0, 4, 1, 2]), np.array([1, 4, 0, 2, 3])
    p = np.zeros(n ** 3)
    p[(np.arange(n) * n + J) * n + K] = 1.0
    X, z = A3.assign3d_sample(p, P.c, n, 8, 1, 0, seed=1, rnd=0)
    assert np.all(X == (p == 1.0)[None, :])
    assert np.all(z == int(P.c[(np.arange(n) * n + J) * n + K].sum()))


def test_best_candidate_reaches_the_brute_force_optimum():
    n = 3
    for seed in range(4):
        P = I.assignment_3d(n, seed=seed)
        C = P.c.reshape(n, n, n)
        best = min(sum(C[i, pj[i], pk[i]] for i in range(n))
                   for pj in itertools.permutations(range(n)) for pk in itertools.permutations(range(n)))
        X, z = A3.assign3d_sample(np.zeros(n ** 3), P.c, n, 64, 0, 20, seed=seed, rnd=0)
        assert int(z.min()) == best


@pytest.mark.parametrize("c_hi", [100, 2])
def test_one_step_is_the_best_interchange_at_the_drawn_triple(c_hi):
    """L = 1 from the L = 0 completion: the triple a is drawn from word 0 of
    Philox(counter = (l, n, round, TAG)) as floor(u n); among all j / k
    interchanges of a with another triple the least cost change (ties: lower
    b, then j) is applied iff negative; with all costs equal nothing moves."""
    n = 5
    P = I.assignment_3d(n, seed=9, c_hi=c_hi)        # c_hi = 2: many tied changes
    C = P.c.reshape(n, n, n)
    p = np.random.default_rng(9).random(n ** 3)
    X0, z0 = A3.assign3d_sample(p, P.c, n, 24, 1, 0, seed=7, rnd=2)
    X1, z1 = A3.assign3d_sample(p, P.c, n, 24, 1, 1, seed=7, rnd=2)
    for l in range(24):
        idx = np.nonzero(X0[l])[0]
        J, K = (idx // n) % n, idx % n                 # idx sorted by i
        U = int(O.philox4x32_10(l, n, 2, 0xA5513D00, 7, 0)[0])
        a = ((U >> 8) * n) >> 24
        cand = []
        for b in range(n):
            if b != a:
                cur = C[a, J[a], K[a]] + C[b, J[b], K[b]]
                cand.append((C[a, J[b], K[a]] + C[b, J[a], K[b]] - cur, b, 0))
                cand.append((C[a, J[a], K[b]] + C[b, J[b], K[a]] - cur, b, 1))
        d, b, t = min(cand)
        J2, K2 = J.copy(), K.copy()
        if d < 0:
            if t == 0:
                J2[a], J2[b] = J[b], J[a]
            else:
                K2[a], K2[b] = K[b], K[a]
        exp = np.zeros(n ** 3, dtype=bool)
        exp[(np.arange(n) * n + J2) * n + K2] = True
        assert np.array_equal(X1[l], exp), l
        assert z1[l] == z0[l] + min(d, 0)
    ones = np.ones(n ** 3, dtype=np.int64)
    Xa, _ = A3.assign3d_sample(p, ones, n, 16, 1, 0, seed=7, rnd=2)
    Xb, _ = A3.assign3d_sample(p, ones, n, 16, 1, 30, seed=7, rnd=2)
    assert np.array_equal(Xa, Xb)
