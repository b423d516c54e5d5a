"""Pins of the oracle's monotone relaxation and repair (set-partitioning rows
relaxed to covering rows; Sec. 2.4, "Monotone Relaxation"), by brute force
over every binary point of small facility-location and assignment-like
problems."""
import itertools

import numpy as np

from oracle import gfors_oracle as O
from paper_2510_27117_amd import instances as I


def _feasible(P, x):
    v, _ = O.evaluate(P, np.asarray(x, dtype=bool)[None, :])
    return int(v[0]) == 0


def _all_points(n):
    return np.array(list(itertools.product([0, 1], repeat=n)), dtype=np.int64)


def test_facility_location_rows_are_relaxed_and_optimum_kept():
    F = I.facility_location(2, 3, seed=1)          # n = 2 + 6 = 8
    mask = O.monotone_rows(F)
    assert mask.all()                               # every customer row qualifies
    R, mask2 = O.monotone_relax(F)
    assert np.array_equal(mask, mask2) and R.B is None and R.A.nrows == F.A.nrows + F.B.nrows
    X = _all_points(F.n)
    orig = [x for x in X if _feasible(F, x)]
    relx = [x for x in X if _feasible(R, x)]
    assert len(relx) > len(orig)                    # the relaxation admits supersets
    best_o = min(int(F.c @ x) for x in orig)
    best_r = min(int(R.c @ x) for x in relx)
    assert best_o == best_r                         # same optimum (monotone objective)


def test_repair_maps_relaxed_points_to_feasible_cheaper_points():
    F = I.facility_location(3, 2, seed=2)           # n = 3 + 6 = 9
    R, mask = O.monotone_relax(F)
    for x in _all_points(F.n):
        if _feasible(R, x):
            y = O.monotone_repair(F, mask, x)
            assert _feasible(F, y)
            assert F.c @ y <= F.c @ x
            assert np.all(y <= x)                   # only switches variables off
        if _feasible(F, x):
            assert np.array_equal(O.monotone_repair(F, mask, x), x)


def test_repair_keeps_cheapest_with_lowest_index_on_ties():
    # one partition row over x0..x3 with costs 5, 2, 2, 9 and nothing else
    P = I.from_dense([5, 2, 2, 9], B=[[1, 1, 1, 1]], d=[1])
    R, mask = O.monotone_relax(P)
    assert mask.tolist() == [True]
    assert O.monotone_repair(P, mask, [1, 1, 1, 1]).tolist() == [0, 1, 0, 0]
    assert O.monotone_repair(P, mask, [1, 0, 1, 1]).tolist() == [0, 0, 1, 0]
    assert O.monotone_repair(P, mask, [0, 0, 0, 0]).tolist() == [0, 0, 0, 0]


def test_rows_that_must_stay_equalities():
    # negative cost on a row variable: relaxing could lower the optimum
    P = I.from_dense([3, -1, 2], B=[[1, 1, 0], [0, 0, 1]], d=[1, 1])
    assert O.monotone_rows(P).tolist() == [False, True]
    # a variable in two partition rows
    P = I.from_dense([1, 1, 1], B=[[1, 1, 0], [0, 1, 1]], d=[1, 1])
    assert O.monotone_rows(P).tolist() == [False, False]
    # a positive coefficient in a >= row (switching off could violate it)
    P = I.from_dense([1, 1, 1], A=[[1, 0, 0]], b=[1], B=[[1, 1, 0]], d=[1])
    assert O.monotone_rows(P).tolist() == [False]
    # right-hand side other than 1, or coefficients other than +1
    P = I.from_dense([1, 1, 1], B=[[1, 1, 1], [2, 0, 0]], d=[2, 2])
    assert O.monotone_rows(P).tolist() == [False, False]
    # Q != 0: not monotone in general
    P = I.from_dense([1, 1], B=[[1, 1]], d=[1], Q=[[0, 1], [1, 0]])
    assert O.monotone_rows(P).tolist() == [False]
