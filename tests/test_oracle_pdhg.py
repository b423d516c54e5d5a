"""Pins of the oracle's Preprocess, UpdatePenalty, PDHG step and residuals."""
import json
import math
import os

import numpy as np
import pytest
import scipy.optimize as so

from oracle import gfors_oracle as O
from paper_2510_27117_amd import instances as I

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _load(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


# ---------------------------------------------------------------- Preprocess

def test_power_norm_matches_lapack_2norm():
    rng = np.random.default_rng(0)
    for trial in range(5):
        P = I.set_cover_bernoulli(40 + 10 * trial, 30, 0.1, seed=trial)
        A = I.csr_to_dense(P.A).astype(float)
        ref = np.linalg.norm(A, 2)
        got = O.power_norm(O.csr_to_scipy(P.A), 500)
        assert abs(got - ref) <= 1e-9 * ref


def test_preprocess_normalises_rows_and_spectrum():
    P = I.set_cover_bernoulli(60, 40, 0.1, seed=3)
    S = O.preprocess(P, O.Params(power_iters=500))
    Kd = S.K.toarray()
    # after step 3 the matrix has spectral norm one ...
    assert abs(np.linalg.norm(Kd, 2) - 1.0) < 1e-9
    # ... and its rows all have the same 2-norm 1/s_K (step 1 made them unit)
    rn = np.linalg.norm(Kd, axis=1)
    assert np.allclose(rn, 1.0 / S.s_K, rtol=1e-12)
    # K = -A row-scaled; r = b row-scaled the same way
    A = I.csr_to_dense(P.A).astype(float)
    scale = 1.0 / (np.linalg.norm(A, axis=1) * S.s_K)
    assert np.allclose(Kd, -A * scale[:, None], rtol=1e-12)
    assert np.allclose(S.r, P.b * scale, rtol=1e-12)
    # objective scale: ||Q|| + ||c|| with Q = 0
    assert math.isclose(S.s_o, np.linalg.norm(P.c), rel_tol=1e-12)
    assert math.isclose(S.tau1 * S.tau2, 0.99, rel_tol=1e-12)


def test_preprocess_with_q_uses_spectral_norm_and_step_rule():
    P = I.max_cut_er(30, 4.0, seed=1)
    S = O.preprocess(P, O.Params(power_iters=2000))
    Qd = I.csr_to_dense(P.Q).astype(float)
    qn = np.linalg.norm(Qd, 2)
    assert math.isclose(S.s_o, qn + np.linalg.norm(P.c), rel_tol=1e-9)
    assert math.isclose(S.Q_norm, qn / S.s_o, rel_tol=1e-9)
    L_max = 2 * (S.Q_norm + S.rho_max)
    assert S.tau1 <= 1.0 / (2 * L_max) + 1e-15
    assert S.tau1 <= math.sqrt(0.99) + 1e-15


def test_zero_row_is_left_unscaled():
    c = [1, 2]
    A = [[1, 1], [0, 0]]
    b = [1, 0]
    P = I.from_dense(c, A=A, b=b)
    S = O.preprocess(P, O.Params(power_iters=100))
    assert S.row_norm[1] == 0.0
    assert S.K.toarray()[1].tolist() == [0.0, 0.0]


# ----------------------------------------------------------- UpdatePenalty

def test_rho_schedule_hand_values():
    g = _load("rho_schedules.json")
    for case in g["cases"]:
        seq = O.rho_sequence((case["rho_min"], case["rho_max"], case["T"], case["p"],
                              case["delta"]), len(case["rho"]))
        assert np.allclose(seq, case["rho"], rtol=0, atol=1e-12), case["note"]


# -------------------------------------------------------------------- PDHG

def test_pdhg_hand_trace():
    g = _load("pdhg_trace_n1.json")
    pr = g["problem"]
    P = I.from_dense(pr["c"], A=pr["A"], b=pr["b"])
    prm = O.Params(**g["params"], power_iters=50)
    S = O.preprocess(P, prm)
    assert S.tau1 == g["scaled"]["tau1"] and S.tau2 == g["scaled"]["tau2"]
    assert S.c.tolist() == g["scaled"]["c"] and S.r.tolist() == g["scaled"]["r"]
    assert S.K.toarray().tolist() == g["scaled"]["K"]
    st = O.init_state(S)
    for yk, xk, xbk in g["trace_y_x_xbar"]:
        st = O.pdhg_step(S, st, 0.0)
        assert (st.y[0], st.x[0], st.xbar[0]) == (yk, xk, xbk)


def test_separable_qp_closed_form():
    """No constraints, Q = diag(q) >= 0, rho = 0: the iteration is projected
    gradient descent and converges to clip(-c/(2q), 0, 1)."""
    q = np.array([1, 2, 5, 3, 4, 1])
    c = np.array([-1, -8, 3, -3, -2, -5])
    P = I.from_dense(c, Q=np.diag(q))
    S = O.preprocess(P, O.Params(rho_min=0.0, rho_max=0.0, rho_delta=0.0, power_iters=200))
    st = O.init_state(S)
    for _ in range(4000):
        st = O.pdhg_step(S, st, 0.0)
    ref = np.clip(-c / (2.0 * q), 0.0, 1.0)
    assert np.allclose(st.x, ref, atol=1e-9)


def _scaled_lp(S):
    """The LP of the scaled data: min c~ x  s.t.  K~ x + r~ <= 0 (ineq), = 0 (eq)."""
    Kd = S.K.toarray()
    kw = dict(bounds=[(0, 1)] * S.n, method="highs")
    if S.m1:
        kw["A_ub"], kw["b_ub"] = Kd[: S.m1], -S.r[: S.m1]
    if S.m2:
        kw["A_eq"], kw["b_eq"] = Kd[S.m1:], -S.r[S.m1:]
    return so.linprog(S.c, **kw)


def test_lp_limit_matches_highs():
    """Convex special case (Q = 0, rho = 0): PDHG solves the LP relaxation."""
    P = I.set_cover_bernoulli(24, 12, 0.2, seed=4)
    S = O.preprocess(P, O.Params(rho_min=0.0, rho_max=0.0, rho_delta=0.0))
    res = _scaled_lp(S)
    assert res.status == 0
    st = O.init_state(S)
    for _ in range(30000):
        st = O.pdhg_step(S, st, 0.0)
    assert abs(S.c @ st.x - res.fun) <= 1e-6 * abs(res.fun)
    t = S.K @ st.x + S.r
    assert np.max(t) <= 1e-6


def test_prop1c_energy_bound_along_trajectory():
    """Proposition 1(c) (convex case, tau1 tau2 ||K||^2 <= 1/4):
    (1/4tau1) sum ||x_k - x_{k-1}||^2 + (1/2tau2) sum ||y_k - y^{k-1}||^2
        <= (1/2tau1) ||x* - x0||^2 + (1/2tau2) ||y* - y0||^2,
    with y^k = y_k + tau2 K (xbar_k - x_k) and (x*, y*) a saddle point taken
    from HiGHS (primal solution and constraint marginals)."""
    P = I.set_cover_bernoulli(30, 15, 0.2, seed=6)
    prm = O.Params(sigma=0.25, rho_min=0.0, rho_max=0.0, rho_delta=0.0)
    S = O.preprocess(P, prm)
    res = _scaled_lp(S)
    assert res.status == 0
    xs = res.x
    ys = -res.ineqlin.marginals
    assert np.all(ys >= -1e-12)
    st = O.init_state(S)
    lhs = 0.0
    yhat_prev = st.y.copy()            # y^0 = y_0
    x0, y0 = st.x.copy(), st.y.copy()
    rhs = np.dot(xs - x0, xs - x0) / (2 * S.tau1) + np.dot(ys - y0, ys - y0) / (2 * S.tau2)
    for _ in range(3000):
        nxt = O.pdhg_step(S, st, 0.0)
        dx = nxt.x - st.x
        lhs += np.dot(dx, dx) / (4 * S.tau1) + np.dot(nxt.y - yhat_prev, nxt.y - yhat_prev) / (2 * S.tau2)
        yhat_prev = nxt.y + S.tau2 * (S.K @ (nxt.xbar - nxt.x))
        st = nxt
        assert lhs <= rhs * (1 + 1e-9) + 1e-12


def test_iterates_stay_in_box_and_cone():
    P = I.facility_location(3, 5, seed=2)
    S = O.preprocess(P, O.Params())
    st = O.init_state(S)
    for k in range(300):
        st = O.pdhg_step(S, st, O.rho_value(S, k // 20))
        assert st.x.min() >= 0.0 and st.x.max() <= 1.0
        assert st.y[: S.m1].min() >= 0.0


def test_residual_inclusions_of_theorem2():
    """Theorem 2: s^x in grad_x L(x_k, y_k) + dh1(x_k), s^y in -grad_y L(x_k, y_k) + dh2(y_k).
    On free coordinates these are equalities; at the bounds the difference lies
    in the normal cone of the box / of R_+."""
    P = I.knapsack_multi(25, 3, seed=3)
    P.Q = I.csr_from_dense(np.diag(np.arange(25) % 3 - 1))
    S = O.preprocess(P, O.Params())
    st = O.init_state(S)
    rho = 0.3 * S.rho_max
    for _ in range(40):
        st = O.pdhg_step(S, st, rho)
    nxt = O.pdhg_step(S, st, rho)
    R = O.residuals(S, st, nxt, rho)
    gx = S.c + rho + S.K.T @ nxt.y + 2 * (S.Q @ nxt.x) - 2 * rho * nxt.x
    gy = S.K @ nxt.x + S.r
    dxs = R["sx_vec"] - gx
    free = (nxt.x > 0) & (nxt.x < 1)
    assert free.any()
    assert np.allclose(dxs[free], 0.0, atol=1e-12)
    assert np.all(dxs[nxt.x == 0] <= 1e-12) and np.all(dxs[nxt.x == 1] >= -1e-12)
    dys = R["sy_vec"] + gy
    pos = nxt.y[: S.m1] > 0
    assert np.allclose(dys[: S.m1][pos], 0.0, atol=1e-12)
    assert np.all(dys[: S.m1][~pos] <= 1e-12)
    assert math.isclose(R["binary"], float(np.sum(nxt.x * (1 - nxt.x))), rel_tol=1e-15)


# ------------------------------------------------- equality rows (eq. saddle)

def test_pdhg_hand_trace_with_equality_row():
    """Algorithm 2 with an inequality dual clipped at 0 and an equality dual
    that goes negative (h_2 of eq. (saddle) constrains only inequality rows),
    rho > 0; values traced by hand in exact binary fractions."""
    g = _load("pdhg_trace_eq.json")
    pr = g["problem"]
    P = I.from_dense(pr["c"], A=pr["A"], b=pr["b"], B=pr["B"], d=pr["d"])
    S = O.preprocess(P, O.Params(**g["params"], power_iters=50))
    # the spectral norm of K = -[e1; e3; e2] is 1 up to the power iteration's rounding
    assert abs(S.s_K - 1.0) <= 1e-15
    assert (S.m1, S.m2) == (2, 1)
    assert S.tau1 == g["scaled"]["tau1"] and S.tau2 == g["scaled"]["tau2"]
    assert S.c.tolist() == g["scaled"]["c"]
    assert np.allclose(S.K.toarray(), g["scaled"]["K"], rtol=0, atol=1e-15)
    assert np.allclose(S.r, g["scaled"]["r"], rtol=0, atol=1e-15)
    rho = g["rho"]
    st = O.init_state(S)
    states = [st]
    for step in g["trace"]:
        st = O.pdhg_step(S, st, rho)
        states.append(st)
        for key in ("x", "y", "xbar"):
            assert np.allclose(getattr(st, key), step[key], rtol=0, atol=1e-14), (key, step)
    ref = g["residuals_after_step3"]
    R = O.residuals(S, states[2], states[3], rho)
    assert np.allclose(R["sx_vec"], ref["sx_vec"], rtol=0, atol=1e-14)
    assert np.allclose(R["sy_vec"], ref["sy_vec"], rtol=0, atol=1e-14)
    assert abs(R["sx"] - np.linalg.norm(ref["sx_vec"])) <= 1e-14
    assert abs(R["sy"] - np.linalg.norm(ref["sy_vec"])) <= 1e-14
    assert abs(R["primal"] - math.sqrt(ref["primal_sq"])) <= 1e-14
    assert abs(R["binary"] - ref["binary"]) <= 1e-15


def test_primal_gap_hand_values():
    """CheckHalt's primal gap (Sec. 3) at x_k: the positive part of K x + r on
    inequality rows (a satisfied row contributes 0), the signed residual on
    equality rows.  Two variables; rows x1 + x2 >= 1 (violated at the point),
    x1 >= 0 (satisfied), x1 - x2 = 0 (violated, residual of either sign)."""
    P = I.from_dense([1, 1], A=[[1, 1], [1, 0]], b=[1, 0], B=[[1, -1]], d=[0])
    S = O.preprocess(P, O.Params(power_iters=300))
    rn = np.array([math.sqrt(2.0), 1.0, math.sqrt(2.0)]) * S.s_K   # row scale of K
    for x, xprev in (([0.25, 0.5], [0.5, 0.5]), ([0.5, 0.25], [0.0, 1.0])):
        x = np.array(x)
        xprev = np.array(xprev)
        before = O.State(x=xprev, x_prev=xprev, xbar=xprev.copy(), y=np.zeros(3))
        after = O.State(x=x, x_prev=xprev, xbar=2 * x - xprev, y=np.zeros(3))
        R = O.residuals(S, before, after, 0.0)
        # row 1: 1 - x1 - x2 > 0 (violated); row 2: -x1 < 0 (satisfied -> 0);
        # equality: x2 - x1, kept with its sign
        v1 = (1.0 - x[0] - x[1]) / rn[0]
        v3 = (x[1] - x[0]) / rn[2]
        assert v1 > 0 and abs(v3) > 0
        assert abs(R["primal"] - math.hypot(v1, v3)) <= 1e-12 * math.hypot(v1, v3)
        assert abs(R["binary"] - float(np.sum(x * (1 - x)))) <= 1e-15


def _equality_lp_problem():
    """An LP relaxation whose equality rows bind in both directions: row 1's
    variables have negative costs (a '>=' reading would raise their sum above
    its right-hand side), row 2's positive costs (a '<=' reading would lower
    it); plus one capacity row."""
    rng = np.random.default_rng(12)
    n = 16
    c = np.concatenate([-rng.integers(5, 30, size=8), rng.integers(5, 30, size=8)])
    B = np.zeros((2, n), dtype=np.int64)
    B[0, :8] = 1
    B[1, 8:] = 1
    B[1, 3] = 1                       # couple the rows through one variable
    d = np.array([3, 4])
    w = rng.integers(1, 10, size=n)
    A = (-w)[None, :]
    b = np.array([-int(w.sum() // 2)])
    return I.from_dense(c, A=A, b=b, B=B, d=d)


def test_lp_limit_with_equality_rows_matches_highs():
    """Convex special case (Q = 0, rho = 0) with equality rows: the PDHG limit
    solves the scaled LP (HiGHS) and satisfies the equalities; the equality
    duals take both signs at the saddle point."""
    P = _equality_lp_problem()
    S = O.preprocess(P, O.Params(rho_min=0.0, rho_max=0.0, rho_delta=0.0))
    res = _scaled_lp(S)
    assert res.status == 0
    marg = res.eqlin.marginals
    assert np.min(marg) < -1e-6 and np.max(marg) > 1e-6
    st = O.init_state(S)
    for _ in range(40000):
        st = O.pdhg_step(S, st, 0.0)
    assert abs(S.c @ st.x - res.fun) <= 1e-6 * abs(res.fun)
    t = S.K @ st.x + S.r
    assert np.max(t[: S.m1]) <= 1e-7
    assert np.max(np.abs(t[S.m1:])) <= 1e-7
    assert np.min(st.y[S.m1:]) < 0 < np.max(st.y[S.m1:])
