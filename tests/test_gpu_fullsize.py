"""Parity at the benchmark's full size (set cover n = 2,000,000, m = 200,000,
K = 1024, autotuned launch shapes): scales and a teacher-forced PDHG step on
whole vectors, sampled candidate words and a sample of fully evaluated
candidates from the oracle, and any-size properties of the incumbent."""
import numpy as np
import pytest

from oracle import gfors_oracle as O
from paper_2510_27117_amd import instances as I

from _helpers import f32, f32_state, rel_inf, sample_subset

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def setup():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2510_27117_amd import gfors
    P = I.workload("setcover_large", seed=0)
    prm = O.Params(k_int=100, power_iters=200)
    S = O.preprocess(P, prm)
    st = O.init_state(S)
    rho = O.rho_value(S, 0)
    for _ in range(12):
        st = O.pdhg_step(S, st, rho)
    G = gfors.Problem(P, gfors.default_params(k_int=100, K_max=1024))
    yield gfors, P, S, st, rho, G
    G.close()


def test_full_scales(setup):
    gfors, P, S, st, rho, G = setup
    sc = G.scales()
    assert abs(sc["K_norm"][0] - S.s_K) <= 1e-10 * S.s_K
    assert abs(sc["obj_scale"][0] - S.s_o) <= 1e-10 * S.s_o
    assert abs(sc["tau1"][0] - S.tau1) <= 1e-15 and abs(sc["rho_max"][0] - S.rho_max) <= 1e-10 * S.rho_max


def test_full_teacher_forced_step(setup):
    gfors, P, S, st, rho, G = setup
    s32 = f32_state(st)
    G.set_state(s32.x, s32.x_prev, s32.y, rho, k=st.k)
    G.pdhg_steps(1)
    got = G.get_state()
    ref = O.pdhg_step(S, s32, rho)
    assert rel_inf(got["x"], ref.x) <= 1e-5 and rel_inf(got["y"], ref.y) <= 1e-5


def test_full_sampler_and_eval_sampled(setup):
    import torch
    gfors, P, S, st, rho, G = setup
    p = f32(st.x)
    # make a fraction of the probabilities fractional so that Philox is exercised
    rng = np.random.default_rng(0)
    idx = rng.choice(P.n, size=P.n // 5, replace=False)
    p[idx] = f32(rng.random(idx.size))
    rnd = 7
    G.set_state(p, p, np.zeros(P.m1, np.float32), rho, k=st.k, round=rnd)
    v, z = G.sample_eval(1024, p_override=torch.from_numpy(p).cuda(), outputs=True)
    bits = G.candidates()
    # candidate words of sampled variables
    vs = np.sort(rng.choice(P.n, size=3000, replace=False))
    ii = vs[None, :].astype(np.int64)
    ll = np.arange(1024, dtype=np.int64)[:, None]
    Xs = O.uniforms24(0, rnd, 0, ii, ll) < p[vs].astype(np.float64)[None, :]
    assert np.array_equal(bits[vs], O.pack_bits(Xs))
    # full evaluation of sampled candidates
    cand = np.array([0, 1, 63, 64, 511, 777, 1023])
    Xc = sample_subset(p.astype(np.float64), cand, 0, rnd)
    vo, zo = O.evaluate(P, Xc)
    assert np.array_equal(v.cpu().numpy()[0][cand], vo)
    assert np.array_equal(z.cpu().numpy()[0][cand], zo)


def test_full_rounds_incumbent_properties(setup):
    """After graph-replayed rounds, the reported incumbent is a feasible point
    whose exact objective is the reported value (holds at any size)."""
    gfors, P, S, st, rho, G = setup
    G.reset()
    G.run_rounds(120, 1024, use_graph=True)
    G.final_round()
    b = G.best(0)
    hist = G.history(0, 120)
    assert hist.size == 120 and np.all(np.diff(hist) <= 0)          # incumbent never worsens
    if b["found"]:
        vo, zo = O.evaluate(P, b["x"].astype(bool)[None, :])
        assert vo[0] == 0 and zo[0] == b["z"]
