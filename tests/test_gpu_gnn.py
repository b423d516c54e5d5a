"""GPU parity of the learned sampling proposal against the FP64 oracle
(oracle/gnn_oracle.py), on the same parameters and inputs.

The device keeps the 64x64 layer weights, activations, messages and dZ in BF16
(MFMA operands) and accumulates in FP32, so the oracle is given the layer
weights rounded to BF16 (round to nearest even), as the device uses them, and
the bars (tests/gnn_bars.py) bound what BF16 storage leaves over: logits,
loss, the whole gradient (cosine and relative L2 error) and, per parameter
tensor, the relative L2 error and the norm ratio |g_k| / |g_ref_k|.  They are
derived from an FP64 model that rounds to BF16 at the kernels' storage points
(tests/gnn_bf16_model.py; checked against the bars in tests/test_gnn_bars.py)
and reject a tensor whose gradient is off by a factor of 2.  Adam is compared
to 1e-6, and training lowers the loss.
"""
import numpy as np
import pytest

from oracle import gnn_oracle as N

import gnn_bars as B
import gnn_bf16_model as M
from _helpers import gnn_case as _case, gnn_params as _params

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def G():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2510_27117_amd import gfors
    gfors.load_library()
    return gfors


def _oracle(P, S, x, y, t, p32):
    E = N.edge_matrix(P)
    Fv, Fc = N.features(S.c.astype(np.float32), S.r.astype(np.float32), S.m1, x, y)
    # the layer weights as the device holds them (BF16); embeddings, biases and
    # the output layer stay FP32 on the device
    pd = {k: (M.bf16(v) if v.shape == (N.H, N.H) else v.astype(np.float64)) for k, v in p32.items()}
    loss, g, logit = N.loss_and_grad(pd, E, Fv, Fc, t.astype(np.float64))
    return loss, g, logit


@pytest.mark.parametrize("pseed", [1, 2])
@pytest.mark.parametrize("name", ["ufl", "mixed", "setcover"])
def test_forward_and_gradient_match_oracle(G, name, pseed):
    import torch
    P, S, x, y, t = _case(name)
    p32 = _params(pseed)
    loss_ref, g_ref, logit_ref = _oracle(P, S, x, y, t, p32)
    prob = G.Problem(P, G.default_params(k_int=20, K_max=1024))
    net = G.GNN(params=N.flatten(p32).astype(np.float32))
    xd = torch.from_numpy(x).cuda()
    yd = torch.from_numpy(y).cuda() if y.size else torch.zeros(1, device="cuda")
    td = torch.from_numpy(t).cuda()
    p, lg = net.forward(prob, xd, yd, with_logits=True)
    prob.synchronize(); net.stream.synchronize()
    lg = lg.cpu().numpy().astype(np.float64)
    assert np.allclose(p.cpu().numpy(), 1 / (1 + np.exp(-lg)), atol=1e-6)
    loss = net.grad(prob, td, xd, yd)
    gg = N.unflatten(net.get_grad().astype(np.float64))
    c = M.compare(gg, g_ref, lg, logit_ref, loss, loss_ref)
    bad = B.check(c)
    assert not bad, (bad, {k: c[k] for k in ("logit", "loss", "cos", "rel")})
    for k in N.PARAM_ORDER:
        if np.linalg.norm(g_ref[k]) < B.TENSOR_MIN_NORM:
            assert np.linalg.norm(gg[k]) <= 1e-5, k
    net.close()
    prob.close()


def test_adam_matches_oracle(G):
    P, S, x, y, t = _case("ufl")
    p32 = _params(2)
    net = G.GNN(params=N.flatten(p32).astype(np.float32))
    rng = np.random.default_rng(5)
    st = {}
    cur = {k: v.astype(np.float64) for k, v in p32.items()}
    for step in range(3):
        g = {k: rng.normal(0, 1e-2, size=s) for k, s in N.param_shapes().items()}
        gv = N.flatten(g).astype(np.float32)
        net.set_grad(gv)
        net.adam(1e-3)
        cur = N.adam_step(cur, N.unflatten(gv.astype(np.float64)), st, lr=1e-3)
        got = net.params().astype(np.float64)
        assert np.max(np.abs(got - N.flatten(cur))) <= 1e-6, step
    net.close()


def test_training_lowers_loss(G):
    import torch
    P, S, x, y, t = _case("ufl")
    prob = G.Problem(P, G.default_params(k_int=20, K_max=1024))
    net = G.GNN(seed=3)
    xd, yd, td = (torch.from_numpy(a).cuda() for a in (x, y, t))
    losses = [net.train_step(prob, td, 1e-2, xd, yd) for _ in range(40)]
    assert losses[-1] < 0.8 * losses[0], losses[::8]
    net.close()
    prob.close()


def test_learned_p_feeds_the_sampler(G):
    """p from the network (in [0, 1]) drives the same Philox sampler through
    p_override: the per-variable frequency over K candidates matches p within
    6 sigma (Proposition x_p = p), and the round is evaluated."""
    P, S, x, y, t = _case("setcover")
    prob = G.Problem(P, G.default_params(k_int=20, K_max=4096))
    net = G.GNN(seed=4)
    p = net.forward(prob)                  # on the problem's current state
    K = 4096
    v, z = prob.sample_eval(K, p_override=p, outputs=True)
    pv = p.cpu().numpy().astype(np.float64)
    assert pv.min() >= 0.0 and pv.max() <= 1.0
    words = prob.candidates()
    freq = np.array([sum(bin(int(w)).count("1") for w in row) for row in words]) / K
    sd = np.sqrt(pv * (1 - pv) / K)
    assert np.all(np.abs(freq - pv) <= 6 * sd + 1e-9)
    assert v.shape == (1, K) and int(v.min()) >= 0
    net.close()
    prob.close()


def test_what_the_trained_network_gains(G):
    """What the trained network gains over the method without it, on held-out
    facility-location instances (100 x 1000, customer rows relaxed to >= 1,
    every candidate repaired on the device): the network is trained on the
    GPU on iterate / incumbent pairs of the plain method on 20 small
    instances, then the plain loop (K from x_k) and the learned loop (K/2 from
    x_k + K/2 from the network) run the same number of triggers.  Shown and
    checked: training lowers the held-out loss below the untrained network's;
    both loops find an incumbent and the learned one is within 0.1 % of the
    plain one (the spec quality bar).  The rounds and wall time each
    needs to reach the plain incumbent are printed: at this size the learned
    loop needs about as many rounds and more time per round (the network's
    forward pass), so its time-to-incumbent ratio is below 1 (the configured
    1,000 x 10,000 record is in profiles/ufl_learned_vs_plain.json)."""
    import torch
    from paper_2510_27117_amd import instances as I
    from paper_2510_27117_amd import learned

    def relaxed(P):
        m = G.MonotoneRelaxation(P)
        prm = G.default_params(k_int=50, K_max=256)
        prm.repair_row0 = P.m1
        return m.model, prm

    train = [relaxed(I.facility_location(40, 400, seed=2000 + s)) for s in range(20)]
    samples = learned.collect([b for b, _ in train], train[0][1], rounds=60, K=256, snapshots=4)
    assert len(samples) >= 40
    held = [relaxed(I.facility_location(40, 400, seed=2100 + s)) for s in range(3)]
    held_samples = learned.collect([b for b, _ in held], held[0][1], rounds=60, K=256, snapshots=4)
    net = G.GNN(seed=5)
    loss0 = learned.mean_loss(net, held_samples)
    learned.train(net, samples, steps=400, lr=3e-3, seed=5)
    loss1 = learned.mean_loss(net, held_samples)
    assert loss1 < 0.5 * loss0, (loss0, loss1)
    out = []
    for sd in (0, 1):
        P = I.facility_location(100, 1000, seed=3000 + sd)
        model, prm = relaxed(P)
        prm.k_int, prm.K_max = 100, 1024
        prob = G.Problem(model, prm)
        R = 150
        plain = learned.run_plain(prob, R, 1024)
        prob.reset()
        lrn = learned.run_learned(prob, net, R, 1024)
        zp, zl = plain.z[-1], lrn.z[-1]
        assert zp != learned.INT64_MAX and zl != learned.INT64_MAX, sd
        assert zl <= zp + 0.001 * abs(zp), (sd, zp, zl)
        target = int(np.floor(zp + 0.001 * abs(zp)))
        rp = next(r for r, z in enumerate(plain.z) if z <= target)
        rl = next(r for r, z in enumerate(lrn.z) if z <= target)
        out.append((sd, zp, zl, rp, rl, plain.time_to(target), lrn.time_to(target)))
        prob.close()
    net.close()
    for sd, zp, zl, rp, rl, tp, tl in out:
        print(f"held-out seed {sd}: plain z={zp} at round {rp} ({tp:.1f} ms), "
              f"learned z={zl} at round {rl} ({tl:.1f} ms), time ratio {tp / tl:.2f}")
