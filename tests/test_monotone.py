"""The library's monotone relaxation (host C++, gfors_mono_rows /
gfors_mono_repair) equals the oracle's: the same rows are relaxed, the
relaxed model has the same rows, and the repair maps every point the same
way.  CPU only (host code); needs the built library."""
import itertools

import numpy as np
import pytest

from oracle import gfors_oracle as O
from paper_2510_27117_amd import instances as I


@pytest.fixture(scope="module")
def G():
    from paper_2510_27117_amd import gfors
    try:
        gfors.load_library()
    except RuntimeError:
        pytest.skip("libgfors.so not built")
    return gfors


def _dense(M, n):
    if M is None:
        return np.zeros((0, n), dtype=np.int64)
    return O.I_dense(M)


def _cases():
    rng = np.random.default_rng(0)
    out = [I.facility_location(4, 6, seed=1), I.facility_location(3, 2, seed=2),
           I.from_dense([5, 2, 2, 9], B=[[1, 1, 1, 1]], d=[1]),
           I.from_dense([3, -1, 2], B=[[1, 1, 0], [0, 0, 1]], d=[1, 1]),
           I.from_dense([1, 1, 1], B=[[1, 1, 0], [0, 1, 1]], d=[1, 1]),
           I.from_dense([1, 1, 1], A=[[1, 0, 0]], b=[1], B=[[1, 1, 0]], d=[1]),
           I.from_dense([1, 1], B=[[1, 1]], d=[1], Q=[[0, 1], [1, 0]])]
    for k in range(6):                     # random partition-like problems
        n = 9
        B = np.zeros((3, n), dtype=np.int64)
        for j in range(3):
            B[j, rng.choice(n, size=3, replace=False)] = 1
        A = -(rng.random((2, n)) < 0.3).astype(np.int64)
        if k % 2:
            A[0, rng.integers(0, n)] = 1
        c = rng.integers(-1 if k == 4 else 0, 9, size=n)
        out.append(I.from_dense(c, A=A, b=[-2, -2], B=B, d=[1, 1, 1]))
    return out


def test_library_rows_and_model_equal_oracle(G):
    for P in _cases():
        M = G.MonotoneRelaxation(P)
        ref, mask = O.monotone_relax(P)
        assert np.array_equal(M.relaxed, mask), P.name
        assert np.array_equal(_dense(M.model.A, P.n), _dense(ref.A, P.n)), P.name
        assert np.array_equal(_dense(M.model.B, P.n), _dense(ref.B, P.n)), P.name
        if ref.A is not None:
            assert np.array_equal(np.asarray(M.model.b), ref.b)
        if ref.B is not None:
            assert np.array_equal(np.asarray(M.model.d), ref.d)


def test_library_repair_equals_oracle(G):
    for P in _cases():
        M = G.MonotoneRelaxation(P)
        pts = np.array(list(itertools.product([0, 1], repeat=P.n)), dtype=np.int64) if P.n <= 10 else \
            (np.random.default_rng(1).random((512, P.n)) < 0.4).astype(np.int64)
        for x in pts:
            got = M.repair(x).astype(np.int64)
            ref = O.monotone_repair(P, M.relaxed, x) if M.relaxed.any() else x
            assert np.array_equal(got, ref), (P.name, x)
