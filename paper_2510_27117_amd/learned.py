"""Learned sampling proposal: data collection from the method's own runs,
GPU training of the network, and the plain / learned loops of Algorithm 1
with per-round HIP-event timing for time-to-incumbent.

Every numerical step runs in libgfors (PDHG, sampling, evaluation, network
forward/backward, Adam); this module only sequences the calls.

Learned loop (k_r = 2 rounds per trigger of Algorithm 1): after the k_int PDHG
steps, K/2 candidates are drawn from the iterate x_k exactly as in the plain
method (the fallback, it also advances rho) and K/2 from the network's p; every
candidate goes through the same exact evaluation and incumbent update.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

from . import gfors


@dataclass
class Sample:
    prob: "gfors.Problem"
    x: object          # device float32 [n]
    y: object          # device float32 [m]
    target: object     # device float32 [n] (0/1 incumbent)


@dataclass
class RunTrace:
    ms: List[float] = field(default_factory=list)      # elapsed ms after each trigger
    z: List[int] = field(default_factory=list)          # incumbent after each trigger (INT64_MAX = none)
    rounds: int = 0

    def time_to(self, target: int) -> Optional[float]:
        for t, z in zip(self.ms, self.z):
            if z <= target:
                return t
        return None


INT64_MAX = np.iinfo(np.int64).max


def _torch():
    import torch
    return torch


def run_plain(prob: "gfors.Problem", rounds: int, K: int) -> RunTrace:
    """Plain Algorithm 1 (eager launches, one round of K per trigger)."""
    torch = _torch()
    s = prob.stream
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(rounds + 1)]
    ev[0].record(s)
    for r in range(rounds):
        prob.run_rounds(1, K, use_graph=False)
        ev[r + 1].record(s)
    prob.synchronize()
    tr = RunTrace(rounds=rounds)
    hist = prob.history(0, rounds)
    tr.ms = [ev[0].elapsed_time(ev[r + 1]) for r in range(rounds)]
    tr.z = [int(v) for v in hist[:rounds]]
    return tr


def run_learned(prob: "gfors.Problem", net: "gfors.GNN", rounds: int, K: int,
                net_every: int = 1) -> RunTrace:
    """Learned Algorithm 1: per trigger K/2 candidates from x_k (rho advances)
    and K/2 from the network's probabilities (extra round, rho unchanged).
    The network runs at every net_every-th trigger; in between, its last p is
    sampled again (fresh Philox rounds, so fresh candidates)."""
    torch = _torch()
    s = prob.stream
    k_int = prob.params.k_int
    Kh = K // 2
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(rounds + 1)]
    ev[0].record(s)
    p = None
    for r in range(rounds):
        prob.pdhg_steps(k_int)
        if r % max(1, net_every) == 0 or p is None:
            p = net.forward(prob)
        prob.sample_eval(Kh, None, trigger=True)
        prob.sample_eval(Kh, p, trigger=False)
        ev[r + 1].record(s)
    prob.synchronize()
    tr = RunTrace(rounds=rounds)
    hist = prob.history(0, 2 * rounds)
    tr.ms = [ev[0].elapsed_time(ev[r + 1]) for r in range(rounds)]
    tr.z = [int(hist[2 * r + 1]) for r in range(rounds)]
    return tr


def collect(bips, params, rounds: int, K: int, snapshots: int = 6, device: str = "cuda:0",
            log=None, window=(None, None)) -> List[Sample]:
    """Run the plain method on each instance and pair the iterate (x_k, y_k) at
    `snapshots` evenly spaced triggers with the run's final incumbent.
    `window` = (first, last) fractions of the run to take snapshots from
    (default: from rounds/snapshots to the end)."""
    torch = _torch()
    out: List[Sample] = []
    lo = rounds // snapshots if window[0] is None else int(window[0] * rounds)
    hi = rounds - 1 if window[1] is None else max(lo, int(window[1] * rounds))
    snap_at = set(np.linspace(lo, hi, snapshots).astype(int).tolist())
    for idx, bip in enumerate(bips):
        prob = gfors.Problem(bip, params, device=device)
        xs = []
        for r in range(rounds):
            prob.run_rounds(1, K, use_graph=False)
            if r in snap_at:
                st = prob.get_state()
                xs.append((st["x"].copy(), st["y"].copy()))
        prob.final_round()
        b = prob.best(0)
        if not b["found"]:
            if log:
                log(f"instance {idx}: no incumbent, skipped")
            prob.close()
            continue
        if log and (idx + 1) % 25 == 0:
            log(f"collected {idx + 1} of {len(bips)} instances")
        t = torch.from_numpy(b["x"].astype(np.float32)).to(device)
        for x, y in xs:
            out.append(Sample(prob, torch.from_numpy(x).to(device),
                              torch.from_numpy(y if y.size else np.zeros(1, np.float32)).to(device), t))
    return out


def train(net: "gfors.GNN", samples: List[Sample], steps: int, lr: float = 3e-3, seed: int = 0,
          log_every: int = 0, log=None) -> List[float]:
    """Adam on single samples drawn in a seeded random order; returns the loss
    of every logged step."""
    rng = np.random.default_rng(seed)
    losses = []
    for it in range(steps):
        smp = samples[int(rng.integers(0, len(samples)))]
        want = bool(log_every) and (it % log_every == 0 or it == steps - 1)
        loss = net.train_step(smp.prob, smp.target, lr, smp.x, smp.y, want_loss=want)
        if want:
            losses.append(loss)
            if log:
                log(f"step {it}: loss {loss:.4f}")
    return losses


def mean_loss(net: "gfors.GNN", samples: List[Sample]) -> float:
    return float(np.mean([net.grad(s.prob, s.target, s.x, s.y) for s in samples]))
