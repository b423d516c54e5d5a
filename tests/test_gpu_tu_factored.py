"""GPU parity of the factorised TU reformulation (Remark of Sec. 2.4.1): the
problem made by gfors_create_problem_tu applies the LU of the pivot block at
every step and never forms S, and is checked against the oracle run on the
EXPLICIT reformulated model (oracle.tu_reformulate: the theorem's formulas
with the inverse written out), with the bars of the explicit path:
  * Preprocess: row scales of the reformulated rows to 1e-15, spectral norms,
    step sizes and rho constants to 1e-10;
  * one teacher-forced PDHG step: x, y within 1e-5 (FP32);
  * residuals reduced in FP64: 1e-9 against the oracle's formulas on the
    device's own FP32 vectors;
  * sampled candidates, violation counts, objectives, incumbent: bit-exact.
Cases cover a signed-identity block (facility location), a path-shaped and a
random recursive spanning tree of a 2D assignment with a quadratic term, an
interval matrix with a kept equality row, and every launch variant of the
level-scheduled solves (one-workgroup runs with the vector in LDS or in
global memory, one launch per level)."""
import numpy as np
import pytest

from oracle import gfors_oracle as O
from paper_2510_27117_amd import instances as I

from _helpers import f32, f32_state, oracle_trajectory, rel_inf

pytestmark = pytest.mark.gpu

TOL_PDHG = 1e-5


@pytest.fixture(scope="module")
def G():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2510_27117_amd import gfors
    gfors.load_library()
    return gfors


def case(name):
    if name == "fl":
        P = I.facility_location(7, 23, seed=5)
        return P, P.meta["tu_pivots"]
    if name == "qap_path":
        P = I.assignment_qap_like(9, seed=7)
        return P, P.meta["tu_pivots"]
    if name == "qap_rand":
        P = I.assignment_qap_like(12, seed=3, tree="random")
        return P, P.meta["tu_pivots"]
    if name == "qap_heavy":
        # the knapsack row has 17^2 = 289 entries: a workgroup per heavy lifted row
        P = I.assignment_qap_like(17, seed=5, q_density=0.01, tree="random")
        return P, P.meta["tu_pivots"]
    if name == "interval_fill":
        # pivot block [[1,1,0],[0,1,1],[1,1,1]] of interval rows: L has a multiplier
        P = I.from_dense([4, -1, 3, 2, -2, 1], A=[[1, 0, 1, 0, 1, 1], [-1, -1, 0, 0, 0, -1]], b=[1, -2],
                         B=[[1, 1, 0, 0, 0, 0], [0, 1, 1, 1, 0, 0], [1, 1, 1, 1, 1, 0]], d=[1, 1, 2])
        return P, np.array([0, 1, 2])
    if name == "interval":
        B = [[1, 1, 0, 1, 0, 0], [0, 1, 0, 0, 1, 1], [1, 0, 1, 1, 1, 0]]
        P = I.from_dense([3, -2, 4, 1, 5, 2], A=[[1, 1, 1, 1, 1, 1], [-1, 0, -1, 0, 0, -1]], b=[1, -2],
                         B=B, d=[1, 1, 2])
        return P, np.array([0, 1, -1])
    raise KeyError(name)


NAMES = ["fl", "qap_path", "qap_rand", "qap_heavy", "interval", "interval_fill"]
# launch plans of the solves: (lu_wide_rows, lu_lds)
PLANS = {"lds": (4096, 1), "global": (4096, 0), "wide": (1, 1)}


def _params(G, plan="lds", **kw):
    wide, lds = PLANS[plan]
    base = dict(k_int=20, K_max=4096, power_iters=200, lu_wide_rows=wide, lu_lds=lds)
    base.update(kw)
    return G.default_params(**base)


def _make(G, name, plan="lds", **kw):
    P, piv = case(name)
    Pn, c0, rec = O.tu_reformulate(P, piv)
    T = G.TUReformulation(P, piv, factored=True)
    prob = T.problem(_params(G, plan, **kw))
    return P, Pn, c0, rec, T, prob


@pytest.mark.parametrize("name", NAMES)
def test_factored_preprocess_matches_explicit_oracle(G, name):
    P, Pn, c0, rec, T, prob = _make(G, name)
    sc = prob.scales()
    S = O.preprocess(Pn, O.Params(power_iters=200))
    ref_rs = np.where(S.row_norm > 0, 1.0 / np.where(S.row_norm > 0, S.row_norm, 1), 1.0)
    assert np.allclose(sc["row_scale"], ref_rs, rtol=1e-15, atol=0)
    for got, ref in [(sc["K_norm"][0], S.s_K), (sc["obj_scale"][0], S.s_o), (sc["Q_norm"][0], S.Q_norm * S.s_o)]:
        assert abs(got - ref) <= 1e-10 * max(abs(ref), 1e-300), (got, ref)
    for key, ref in [("tau1", S.tau1), ("tau2", S.tau2), ("rho_min", S.rho_min),
                     ("rho_max", S.rho_max), ("rho_delta", S.rho_delta)]:
        assert abs(sc[key][0] - ref) <= 1e-10 * max(abs(ref), 1e-300), key
    prob.close()


@pytest.mark.parametrize("plan", list(PLANS))
@pytest.mark.parametrize("name", NAMES)
def test_factored_teacher_forced_step(G, name, plan):
    P, Pn, c0, rec, T, prob = _make(G, name, plan)
    prm = O.Params(k_int=20, power_iters=200)
    S, traj = oracle_trajectory(Pn, prm, steps=120, keep_every=12)
    for st, rho in traj:
        s32 = f32_state(st)
        prob.set_state(s32.x, s32.x_prev, s32.y, rho, k=st.k)
        prob.pdhg_steps(1)
        got = prob.get_state()
        ref = O.pdhg_step(S, s32, rho)
        ex, ey = rel_inf(got["x"], ref.x), rel_inf(got["y"], ref.y)
        assert ex <= TOL_PDHG and ey <= TOL_PDHG, (st.k, ex, ey)
        assert got["x"].min() >= 0.0 and got["x"].max() <= 1.0
        if Pn.m1:
            assert got["y"][: Pn.m1].min() >= 0.0
        assert np.array_equal(got["x_prev"], f32(s32.x))
        assert got["k"] == st.k + 1
    prob.close()


@pytest.mark.parametrize("name", NAMES)
def test_factored_free_running_drift(G, name):
    """60 free-running FP32 steps (the lifted parts of x_k and xbar carried
    from step to step) stay within 1e-4 of the FP64 oracle on the explicit model."""
    P, Pn, c0, rec, T, prob = _make(G, name)
    S = O.preprocess(Pn, O.Params(k_int=20, power_iters=200))
    st = O.init_state(S)
    for k in range(60):
        st = O.pdhg_step(S, st, S.rho_min)
    prob.pdhg_steps(60)
    got = prob.get_state()
    assert rel_inf(got["x"], st.x) <= 1e-4 and rel_inf(got["y"], st.y) <= 1e-4
    prob.close()


@pytest.mark.parametrize("name", NAMES)
def test_factored_residuals_fp64(G, name):
    """Theorem 2's s^x (with Q' dx through FP64 lifts and transposed solves),
    s^y and CheckHalt's gaps, against the oracle's formulas in FP64 on the
    device's own FP32 vectors: 1e-9 (an FP32 lift or reduction would miss it)."""
    P, Pn, c0, rec, T, prob = _make(G, name)
    prm = O.Params(k_int=20, power_iters=200)
    S, traj = oracle_trajectory(Pn, prm, steps=50, keep_every=49)
    st, rho = traj[-1]
    s32 = f32_state(st)
    prob.set_state(s32.x, s32.x_prev, s32.y, rho, k=st.k)
    prob.pdhg_steps(1, want_residuals=True)
    res = prob.residuals()[0]
    got = prob.get_state()
    x32, xp32 = f32(s32.x), f32(s32.x_prev)
    xbar32 = (np.float32(2) * x32 - xp32).astype(np.float64)
    before = O.State(x=s32.x, x_prev=s32.x_prev, xbar=xbar32, y=s32.y)
    gx = got["x"].astype(np.float64)
    after = O.State(x=gx, x_prev=s32.x, xbar=2 * gx - s32.x, y=got["y"].astype(np.float64))
    R = O.residuals(S, before, after, rho)
    for i, key in enumerate(["sx", "sy", "primal", "binary"]):
        assert abs(res[i] - R[key]) <= 1e-9 * abs(R[key]) + 1e-13, (key, res[i], R[key])
    prob.close()


@pytest.mark.parametrize("plan", list(PLANS))
@pytest.mark.parametrize("name", NAMES)
def test_factored_sample_eval_bit_exact(G, name, plan):
    """Candidates drawn from the same p are the oracle's bits; each candidate's
    pivot variables are solved for exactly (any integer, also outside {0,1})
    and its violation count and objective equal the oracle's evaluation on the
    explicit reformulated model."""
    import torch
    P, Pn, c0, rec, T, prob = _make(G, name, plan)
    rng = np.random.default_rng(11)
    K = 1024
    for trial, rnd in enumerate((0, 5)):
        p = f32(rng.random(Pn.n) * (0.4 + 0.5 * trial))
        p[:3] = [0.0, 1.0, 0.5]
        prob.set_state(p, p, np.zeros(Pn.m1 + Pn.m2), 0.0, k=0, round=rnd)
        pt = torch.from_numpy(p).to("cuda:0")
        v, z = prob.sample_eval(K, p_override=pt, outputs=True)
        X = O.sample_bits(p.astype(np.float64), K, seed=0, rnd=rnd)
        assert np.array_equal(prob.candidates(), O.pack_bits(X))
        vr, zr = O.evaluate(Pn, X)
        assert np.array_equal(v.cpu().numpy()[0], vr)
        assert np.array_equal(z.cpu().numpy()[0], zr)
    prob.close()


@pytest.mark.parametrize("name", NAMES)
def test_factored_rounds_incumbent_and_final_round(G, name):
    """Graph-replayed rounds equal eager rounds bit for bit; the incumbent is
    the oracle's EvalBest over the candidates of every round; it maps back to
    a feasible point of the original problem with objective z + c'_0; the final
    rounding evaluates round(x_k) like the oracle."""
    import torch
    # the same launch shapes on both (timed choices could differ and change
    # the FP32 summation order)
    P, Pn, c0, rec, T, a = _make(G, name, k_int=10, seed=3, autotune=0)
    _, _, _, _, T2, b = _make(G, name, k_int=10, seed=3, autotune=0)
    inc = O.Incumbent()
    for r in range(6):
        a.run_rounds(1, 256, use_graph=False)
        b.run_rounds(1, 256, use_graph=True)
        X = O.unpack_bits(a.candidates(), 256)
        vr, zr = O.evaluate(Pn, X)
        O.incumbent_update(inc, X, vr, zr, r, a.get_state()["k"])
    sa, sb = a.get_state(), b.get_state()
    assert np.array_equal(sa["x"], sb["x"]) and np.array_equal(sa["y"], sb["y"])
    ba, bb = a.best(), b.best()
    assert ba["found"] == bb["found"] and ba["z"] == bb["z"]
    assert ba["found"] == (inc.z is not None)
    if inc.z is not None:
        assert ba["z"] == inc.z and np.array_equal(ba["x"].astype(bool), inc.x)
        x_full = T.recover(ba["x"])
        vo, zo = O.evaluate(P, x_full[None, :].astype(bool))
        assert vo[0] == 0 and zo[0] == ba["z"] + c0
    # final rounding of x_k: one more candidate (round -1 in the record when it improves)
    x = a.get_state()["x"]
    Xf = O.round_candidate(x)
    vf, zf = O.evaluate(Pn, Xf)
    before = a.best()
    a.final_round()
    after = a.best()
    improves = vf[0] == 0 and (not before["found"] or zf[0] < before["z"])
    if improves:
        assert after["found"] and after["z"] == zf[0] and after["round"] == -1
        assert np.array_equal(after["x"].astype(bool), Xf[0])
    else:
        assert (after["found"], after["z"], after["round"]) == (before["found"], before["z"], before["round"])
    a.close()
    b.close()
