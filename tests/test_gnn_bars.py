"""The learned proposal's GPU bars (tests/gnn_bars.py) against the BF16
storage-point model (tests/gnn_bf16_model.py): the bars cover the model's
spread around the FP64 oracle with a margin of 1.5, and a gradient tensor
scaled by 2 fails them."""
import numpy as np
import pytest

from oracle import gnn_oracle as N

import gnn_bars as B
import gnn_bf16_model as M
from _helpers import gnn_case, gnn_params


def _runs():
    for name in ["ufl", "mixed", "setcover"]:
        P, S, x, y, t = gnn_case(name)
        E = N.edge_matrix(P)
        Fv, Fc = N.features(S.c.astype(np.float32), S.r.astype(np.float32), S.m1, x, y)
        tt = t.astype(np.float64)
        for ps in (1, 2, 3):
            p32 = gnn_params(ps)
            pd = {k: (M.bf16(v) if v.shape == (N.H, N.H) else v.astype(np.float64))
                  for k, v in p32.items()}
            ref = N.loss_and_grad(pd, E, Fv, Fc, tt)
            for js in (0, 1, 2):
                got = M.loss_and_grad({k: v.astype(np.float64) for k, v in p32.items()},
                                      E, Fv, Fc, tt, jitter=3e-7, seed=js)
                yield ref, got


@pytest.fixture(scope="module")
def runs():
    return list(_runs())


def test_model_without_rounding_is_the_oracle():
    """With every rounding taken out the model is the oracle's network (same
    loss, logits and gradient to FP64 rounding), so its spread comes from the
    BF16 storage points alone."""
    for name in ["ufl", "mixed"]:
        P, S, x, y, t = gnn_case(name)
        E = N.edge_matrix(P)
        Fv, Fc = N.features(S.c.astype(np.float32), S.r.astype(np.float32), S.m1, x, y)
        p = {k: v.astype(np.float64) for k, v in gnn_params(4).items()}
        l1, g1, z1 = N.loss_and_grad(p, E, Fv, Fc, t.astype(np.float64))
        l2, g2, z2 = M.loss_and_grad(p, E, Fv, Fc, t.astype(np.float64), exact=True)
        assert abs(l1 - l2) <= 1e-12 and np.allclose(z1, z2, rtol=0, atol=1e-12)
        a, b = N.flatten(g1), N.flatten(g2)
        assert np.max(np.abs(a - b)) <= 1e-12 * np.max(np.abs(a))


def test_bars_cover_the_bf16_model_with_margin(runs):
    worst = {"logit": 0.0, "loss": 0.0, "cos": 1.0, "rel": 0.0, "trel": 0.0, "rlo": 1.0, "rhi": 1.0}
    for (lr, gr, zr), (l, g, z) in runs:
        c = M.compare(g, gr, z, zr, l, lr)
        worst["logit"] = max(worst["logit"], c["logit"])
        worst["loss"] = max(worst["loss"], c["loss"])
        worst["cos"] = min(worst["cos"], c["cos"])
        worst["rel"] = max(worst["rel"], c["rel"])
        for k, v in c["tensor_rel"].items():
            if v is not None:
                worst["trel"] = max(worst["trel"], v)
                worst["rlo"] = min(worst["rlo"], c["tensor_ratio"][k])
                worst["rhi"] = max(worst["rhi"], c["tensor_ratio"][k])
    assert B.LOGIT_REL >= 1.5 * worst["logit"], worst
    assert B.LOSS_REL >= 1.5 * worst["loss"], worst
    assert 1 - B.GRAD_COS_MIN >= 1.5 * (1 - worst["cos"]), worst
    assert B.GRAD_REL_MAX >= 1.5 * worst["rel"], worst
    assert B.TENSOR_REL_MAX >= 1.5 * worst["trel"], worst
    assert 1 - B.TENSOR_RATIO[0] >= 1.5 * (1 - worst["rlo"]), worst
    assert B.TENSOR_RATIO[1] - 1 >= 1.5 * (worst["rhi"] - 1), worst


def test_a_tensor_scaled_by_two_fails_the_bars(runs):
    (lr, gr, zr), (l, g, z) = runs[0]
    assert B.check(M.compare(g, gr, z, zr, l, lr)) == []
    for k in N.PARAM_ORDER:
        if np.linalg.norm(gr[k]) < B.TENSOR_MIN_NORM:
            continue
        g2 = dict(g)
        g2[k] = 2.0 * np.asarray(g[k])
        bad = B.check(M.compare(g2, gr, z, zr, l, lr))
        assert any(name.startswith(k + ":") for name, _ in bad), k
