"""Pins of the learned-proposal oracle: the hand-written backward pass against
central finite differences of the loss, closed forms of single pieces, and
Adam's first step."""
import numpy as np
import pytest

from oracle import gfors_oracle as O
from oracle import gnn_oracle as N
from paper_2510_27117_amd import instances as I


def _setup(seed=0):
    P = I.facility_location(3, 6, seed=seed)
    S = O.preprocess(P, O.Params())
    rng = np.random.default_rng(seed)
    x = rng.random(P.n)
    x[rng.random(P.n) < 0.3] = 0.0
    y = rng.random(S.m) * 2 - 0.5
    Fv, Fc = N.features(S.c, S.r, S.m1, x, y)
    E = N.edge_matrix(P)
    p = {k: rng.normal(0, 0.3, size=s) for k, s in N.param_shapes().items()}
    t = (rng.random(P.n) < 0.4).astype(float)
    return P, E, Fv, Fc, p, t


def test_gradient_matches_central_differences():
    P, E, Fv, Fc, p, t = _setup(0)
    loss, g, _ = N.loss_and_grad(p, E, Fv, Fc, t)
    rng = np.random.default_rng(1)
    h = 1e-6
    for k in N.PARAM_ORDER:
        flat_idx = rng.choice(p[k].size, size=min(6, p[k].size), replace=False)
        for fi in flat_idx:
            idx = np.unravel_index(fi, p[k].shape)
            pp = {kk: v.copy() for kk, v in p.items()}
            pm = {kk: v.copy() for kk, v in p.items()}
            pp[k][idx] += h
            pm[k][idx] -= h
            lp = N.bce_loss(N.forward(pp, E, Fv, Fc)[0], t)
            lm = N.bce_loss(N.forward(pm, E, Fv, Fc)[0], t)
            fd = (lp - lm) / (2 * h)
            an = g[k][idx]
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(fd)) + 1e-9, (k, idx, fd, an)


def test_edge_matrix_and_features():
    P = I.from_dense([1, 2, 3], A=[[3, 4, 0], [0, 0, 0]], b=[1, 0], B=[[1, 1, 1]], d=[1])
    E = N.edge_matrix(P).toarray()
    assert np.allclose(E, [[0.6, 0.8, 0], [0, 0, 0], [1 / np.sqrt(3)] * 3])
    Fv, Fc = N.features(np.array([0.5, -1.0, 0.25]), np.array([2.0, 0.0, -4.0]), 2,
                        np.array([0.0, 0.5, 1.0]), np.array([1.0, 0.0, -3.0]))
    assert np.allclose(Fv[:, 0], [0, 0.5, 1]) and np.allclose(Fv[:, 1], [0, 1, 0])
    assert np.allclose(Fv[:, 2], [0.5, -1.0, 0.25]) and np.all(Fv[:, 3] == 1)
    assert np.allclose(Fc[:, 0], [0.5, 0.0, -0.75]) and np.allclose(Fc[:, 1], [0.5, 0.0, -1.0])
    assert np.allclose(Fc[:, 2], [0, 0, 1])


def test_zero_network_gives_half_and_log2_loss():
    """With all weights zero the logits are bo; with bo = 0 every p = 1/2 and the
    loss is log 2 whatever the targets."""
    P, E, Fv, Fc, p, t = _setup(2)
    z = {k: np.zeros(s) for k, s in N.param_shapes().items()}
    logit, _ = N.forward(z, E, Fv, Fc)
    assert np.all(logit == 0.0)
    assert abs(N.bce_loss(logit, t) - np.log(2.0)) < 1e-15
    # gradient w.r.t. bo is mean(p - t) = 0.5 - mean(t)
    _, g, _ = N.loss_and_grad(z, E, Fv, Fc, t)
    assert abs(g["bo"][0] - (0.5 - t.mean())) < 1e-15


def test_adam_first_step_is_signed_lr():
    """At t = 1 the bias-corrected Adam step is -lr * g / (|g| + eps)."""
    p = {k: np.ones(s) for k, s in N.param_shapes().items()}
    rng = np.random.default_rng(3)
    g = {k: rng.normal(size=s) for k, s in N.param_shapes().items()}
    st = {}
    q = N.adam_step(p, g, st, lr=0.01)
    for k in N.PARAM_ORDER:
        assert np.allclose(q[k], 1.0 - 0.01 * g[k] / (np.abs(g[k]) + 1e-8), rtol=1e-12, atol=1e-15)


def test_flatten_roundtrip_and_size():
    p = {k: np.random.default_rng(0).normal(size=s) for k, s in N.param_shapes().items()}
    v = N.flatten(p)
    assert v.size == 4 * 64 * 2 + 64 * 2 + 3 * (4 * 64 * 64 + 2 * 64) + 64 + 1
    q = N.unflatten(v)
    assert all(np.array_equal(p[k], q[k]) for k in N.PARAM_ORDER)
