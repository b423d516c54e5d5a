"""Customized sampling for the 3D assignment problem (Algorithm 4, Sec. 2.4.2);
test infrastructure (only tests/, __graft_entry__.smoke() and bench.py's
cpu_baseline leg may use it).

    min <c, x>  s.t.  sum_{j,k} x_ijk = 1 (all i),  sum_{i,k} x_ijk = 1 (all j),
                      sum_{i,j} x_ijk = 1 (all k),  x in {0,1}^{n^3}
    (variable x_ijk at index (i n + j) n + k)

RandSampleStep(p, K): take the gamma n largest entries of p, build from them
a partial assignment without conflicts (greedy, largest first), then for each
of the K candidates complete it at random and improve it with L steps of
pairwise interchange.  Readings (the paper gives the steps, not these details):

  * order of p: descending value, lower index first among equal values;
    the first min(gamma n, #{p > 0}) entries are taken (an entry with p = 0
    carries no information and is left to the random completion);
  * greedy: an entry (i, j, k) is taken when none of i, j, k is used yet;
  * random completion: the r unassigned i's (ascending) are matched with a
    uniformly random permutation of the unassigned j's and of the unassigned
    k's, each drawn by Fisher-Yates from position r-1 down to 1: swap t with
    floor(u (t + 1)), u = (U >> 8) 2^-24 computed exactly as
    ((U >> 8) (t + 1)) >> 24 with U = word 0 (j) / word 1 (k) of
    Philox4x32-10(key = seed, counter = (l, t, round, TAG));
  * local improvement: step q draws triple a = ((U >> 8) n) >> 24 from word 0
    of Philox(counter = (l, n + q, round, TAG)) and considers, for every other
    triple b, the pairwise interchanges that swap the j's or the k's of a and
    b (swapping the i's is the same as swapping both); the one with the
    least cost change (ties: lower b, then the j swap) is applied when the
    change is negative;
  * TAG = 0xA5513D00 keeps these counters apart from Algorithm 3's, whose
    fourth word is an instance id.

Pinned in tests/test_oracle_assign3d.py: every candidate is a 3D assignment;
the greedy partial assignment against a brute definition; the completion is a
uniform permutation (chi-square over all 3!^2 completions of n = 3); the
local steps never raise the cost and stop at pairwise-interchange optima
for large L; a 0/1 p at an assignment reproduces it.
"""
from __future__ import annotations

import numpy as np

from .gfors_oracle import philox4x32_10

TAG = 0xA5513D00


def _words(seed: int, l: int, step: int, rnd: int):
    w = philox4x32_10(l, step, rnd, TAG, seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF)
    return [int(v) for v in w]


def _below(U: int, bound: int) -> int:
    """floor(u * bound) for the 24-bit uniform u = (U >> 8) 2^-24, exactly."""
    return ((U >> 8) * bound) >> 24


def top_entries(p: np.ndarray, m: int) -> np.ndarray:
    """Indices of the (at most) m largest positive entries of p, descending,
    lower index first on ties."""
    p = np.asarray(p, dtype=np.float64)
    order = np.lexsort((np.arange(p.size), -p))
    m = min(m, int(np.count_nonzero(p > 0)))
    return order[:m]


def partial_assignment(p: np.ndarray, n: int, gamma: int):
    """Greedy conflict-free partial assignment from the gamma n largest p:
    J0[i], K0[i] = the j, k assigned to i, or -1."""
    m = gamma * n
    J0 = np.full(n, -1, dtype=np.int64)
    K0 = np.full(n, -1, dtype=np.int64)
    uj = np.zeros(n, dtype=bool)
    uk = np.zeros(n, dtype=bool)
    for v in top_entries(p, m):
        i, j, k = int(v) // (n * n), (int(v) // n) % n, int(v) % n
        if J0[i] < 0 and not uj[j] and not uk[k]:
            J0[i], K0[i] = j, k
            uj[j] = uk[k] = True
    return J0, K0


def _complete(J0, K0, n, seed, l, rnd):
    J, K = J0.copy(), K0.copy()
    Ui = np.nonzero(J0 < 0)[0]
    usedj = np.zeros(n, dtype=bool)
    usedk = np.zeros(n, dtype=bool)
    usedj[J0[J0 >= 0]] = True
    usedk[K0[K0 >= 0]] = True
    pj = list(np.nonzero(~usedj)[0])
    pk = list(np.nonzero(~usedk)[0])
    r = len(Ui)
    for t in range(r - 1, 0, -1):
        w = _words(seed, l, t, rnd)
        a = _below(w[0], t + 1)
        pj[t], pj[a] = pj[a], pj[t]
        b = _below(w[1], t + 1)
        pk[t], pk[b] = pk[b], pk[t]
    for t in range(r):
        J[Ui[t]], K[Ui[t]] = pj[t], pk[t]
    return J, K


def _improve(J, K, C, n, L, seed, l, rnd):
    """L pairwise-interchange steps on the assignment (J, K); C = c as [n, n, n]."""
    if n < 2:
        return J, K
    for q in range(L):
        a = _below(_words(seed, l, n + q, rnd)[0], n)
        base = C[a, J[a], K[a]]
        best = None
        for b in range(n):
            if b == a:
                continue
            cur = base + C[b, J[b], K[b]]
            dj = C[a, J[b], K[a]] + C[b, J[a], K[b]] - cur
            dk = C[a, J[a], K[b]] + C[b, J[b], K[a]] - cur
            for typ, dlt in ((0, dj), (1, dk)):
                if best is None or dlt < best[0]:
                    best = (int(dlt), b, typ)
        if best[0] < 0:
            _, b, typ = best
            if typ == 0:
                J[a], J[b] = J[b], J[a]
            else:
                K[a], K[b] = K[b], K[a]
    return J, K


def assign3d_sample(p, c, n: int, K: int, gamma: int, L: int, seed: int, rnd: int):
    """Algorithm 4: K candidates (bool [K, n^3]) from the fractional point p
    (length n^3) with costs c (integers, length n^3).  Also returns the
    candidates' objectives <c, x> (int64 [K])."""
    C = np.asarray(c, dtype=np.int64).reshape(n, n, n)
    J0, K0 = partial_assignment(p, n, gamma)
    X = np.zeros((K, n ** 3), dtype=bool)
    z = np.zeros(K, dtype=np.int64)
    for l in range(K):
        J, Kk = _complete(J0, K0, n, seed, l, rnd)
        J, Kk = _improve(J, Kk, C, n, L, seed, l, rnd)
        idx = (np.arange(n) * n + J) * n + Kk
        X[l, idx] = True
        z[l] = int(C[np.arange(n), J, Kk].sum())
    return X, z
