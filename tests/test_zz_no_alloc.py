"""gfors_create_problem_static (no device allocation) against gfors_create_problem.

The static entry point carves the problem from the library's file-scope device
array instead of a caller workspace; everything else is the same code.  With
the same data and the same launch shapes (autotune off on both) the two
problems must compute identical bits: iterates, residuals, candidates,
violation counts, objectives, incumbent and history.  Two problems are created
in a row on the static array, the second smaller than the first, so the second
starts from whatever the first left in it.
"""
import numpy as np
import pytest

from paper_2510_27117_amd import instances as I

from _helpers import mixed_problem

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def G():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2510_27117_amd import gfors
    gfors.load_library()
    return gfors


def _params(G):
    return G.default_params(k_int=10, K_max=256, autotune=0, hist_cap=64)


def _run(P):
    """Two triggers of Algorithm 1 and the final rounding; returns every output."""
    out = {}
    P.pdhg_steps(25, want_residuals=True)
    out["res"] = P.residuals()
    out["v1"], out["z1"] = (t.cpu().numpy() for t in P.sample_eval(256, outputs=True))
    out["X1"] = P.candidates()
    P.pdhg_steps(10)
    out["v2"], out["z2"] = (t.cpu().numpy() for t in P.sample_eval(128, outputs=True))
    out["X2"] = P.candidates()
    P.final_round()
    out["state"] = P.get_state()
    out["best"] = P.best(0)
    out["hist"] = P.history(0)
    out["scales"] = P.scales()
    return out


def _same(a, b):
    for k in ("res", "v1", "z1", "X1", "v2", "z2", "X2", "hist"):
        assert np.array_equal(a[k], b[k]), k
    for k, v in a["state"].items():
        assert np.array_equal(np.asarray(v), np.asarray(b["state"][k])), "state " + k
    for k in ("z", "found", "round", "l", "k", "ntrig"):
        assert a["best"][k] == b["best"][k], "best " + k
    assert np.array_equal(a["best"]["x"], b["best"]["x"])
    for k, v in a["scales"].items():
        assert np.array_equal(np.asarray(v), np.asarray(b["scales"][k])), "scales " + k


@pytest.mark.parametrize("first,second", [
    (lambda: mixed_problem(400, seed=3), lambda: mixed_problem(150, seed=6)),
    (lambda: I.set_cover_columns(5003, 997, 5, seed=2), lambda: I.facility_location(6, 30, seed=5)),
])
def test_static_equals_workspace_two_calls(G, first, second):
    for make in (first, second):
        bip = make()
        print("static workspace vs caller workspace:", bip.n, bip.m1, bip.m2, flush=True)
        ref = G.Problem(bip, _params(G))
        st = G.Problem(bip, _params(G), static_ws=True)
        try:
            assert st.ws is None
            a, b = _run(ref), _run(st)
        finally:
            st.close()
            ref.close()
        _same(a, b)
        assert a["best"]["found"] or bip.m1 + bip.m2 > 0


def test_static_rejects_a_second_live_problem_and_oversize(G):
    bip = mixed_problem(150, seed=1)
    st = G.Problem(bip, _params(G), static_ws=True)
    try:
        with pytest.raises(G.GforsError, match="GFORS_E_STATE"):
            G.Problem(bip, _params(G), static_ws=True)
    finally:
        st.close()
    # released: a new one can be created
    st = G.Problem(bip, _params(G), static_ws=True)
    st.close()
    # beyond GFORS_STATIC_WS_BYTES: rejected before any device work, with the sizes
    n = 300_000
    big = I.BIP(n=n, c=np.ones(n, dtype=np.int64),
                A=I.CSR(1, n, np.array([0, 1], dtype=np.int64), np.array([0], dtype=np.int32)),
                b=np.ones(1, dtype=np.int64))
    with pytest.raises(G.GforsError, match="GFORS_E_OOM.*static workspace holds"):
        G.Problem(big, G.default_params(K_max=1024, autotune=0), static_ws=True)
