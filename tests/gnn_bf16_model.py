"""Bar-derivation model of the learned proposal's device arithmetic (test helper,
not the oracle).

The oracle (oracle/gnn_oracle.py) states the network in FP64.  The device keeps
some tensors in BF16 (the MFMA operands) and accumulates in FP32, so its
results differ from the oracle by more than FP32 rounding.  This module is the
oracle's network again, in FP64, with a BF16 rounding (round to nearest even)
at every point where the kernels store a BF16 tensor:

  forward   H0 = bf(relu(F U + u));  S = bf(E H) (messages);
            H' = bf(relu([H | S] W_bf + b)) (dense layers; W rounded too);
            logit = H_L wo + bo (H_L in BF16, wo and bo FP32)
  backward  dlogit = (p - t)/n, dH_L = dlogit wo^T;  per dense layer
            Z = dH o [H' > 0]: bias gradient = sum Z (unrounded),
            dZ = bf(Z) is the MFMA operand of the weight gradient
            [H | S]^T dZ and of the input gradient dZ W_bf^T (kept FP32);
            message gradients E dS, E^T dS in FP32; embeddings in FP32.

A relative perturbation of `jitter` times a standard normal is applied before
each rounding, standing for the FP32 accumulation order of the kernels (which
decides some roundings one way or the other).  The GPU tests' bars are taken
from the spread of this model around the oracle (tests/gnn_bars.py); a CPU test
checks that the bars cover it and still reject a gradient tensor scaled by 2.
"""
from __future__ import annotations

import numpy as np

from oracle import gnn_oracle as N


def bf16(a) -> np.ndarray:
    """Round to the nearest BF16 value (ties to even), returned as FP64."""
    u = np.asarray(a, dtype=np.float64).astype(np.float32).view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


class _Round:
    def __init__(self, jitter: float, seed: int, exact: bool):
        self.jitter = jitter
        self.exact = exact
        self.rng = np.random.default_rng(seed)

    def __call__(self, a):
        a = np.asarray(a, dtype=np.float64)
        if self.exact:
            return a
        if self.jitter > 0:
            a = a * (1.0 + self.jitter * self.rng.standard_normal(a.shape))
        return bf16(a)


def loss_and_grad(p, E, Fv, Fc, t, jitter: float = 0.0, seed: int = 0, exact: bool = False):
    """(loss, gradient dict, logits) of the network with the device's BF16
    storage points.  p: FP64 parameters (the FP32 master values).  exact=True
    takes every rounding out (the oracle's arithmetic, as a structural check)."""
    bf = _Round(jitter, seed, exact)
    L = N.L
    W = {k: (bf(v) if np.shape(v) == (N.H, N.H) else np.asarray(v, dtype=np.float64))
         for k, v in p.items()}
    relu = N.relu
    Hv = [bf(relu(Fv @ W["Uv"] + W["uv"]))]
    Hc = [bf(relu(Fc @ W["Uc"] + W["uc"]))]
    Sc, Sv = [], []
    for l in range(L):
        Sc.append(bf(E @ Hv[l]))
        Hc.append(bf(relu(Hc[l] @ W[f"Wcc{l}"] + Sc[l] @ W[f"Wcv{l}"] + W[f"bc{l}"])))
        Sv.append(bf(E.T @ Hc[l + 1]))
        Hv.append(bf(relu(Hv[l] @ W[f"Wvv{l}"] + Sv[l] @ W[f"Wvc{l}"] + W[f"bv{l}"])))
    logit = Hv[L] @ W["wo"] + W["bo"][0]
    loss = N.bce_loss(logit, t)
    n = logit.shape[0]
    g = {}
    dz = (N.sigmoid(logit) - np.asarray(t, dtype=np.float64)) / n
    g["wo"] = Hv[L].T @ dz
    g["bo"] = np.array([dz.sum()])
    dHv = np.outer(dz, W["wo"])
    dHc = np.zeros_like(Hc[L])
    for l in range(L - 1, -1, -1):
        Zv = dHv * (Hv[l + 1] > 0)
        g[f"bv{l}"] = Zv.sum(axis=0)
        dZv = bf(Zv)
        g[f"Wvv{l}"] = Hv[l].T @ dZv
        g[f"Wvc{l}"] = Sv[l].T @ dZv
        dHv_prev = dZv @ W[f"Wvv{l}"].T
        dS = dZv @ W[f"Wvc{l}"].T
        dHc = dHc + E @ dS
        Zc = dHc * (Hc[l + 1] > 0)
        g[f"bc{l}"] = Zc.sum(axis=0)
        dZc = bf(Zc)
        g[f"Wcc{l}"] = Hc[l].T @ dZc
        g[f"Wcv{l}"] = Sc[l].T @ dZc
        dHc_prev = dZc @ W[f"Wcc{l}"].T
        dS = dZc @ W[f"Wcv{l}"].T
        dHv = dHv_prev + E.T @ dS
        dHc = dHc_prev
    dZv0 = dHv * (Hv[0] > 0)
    dZc0 = dHc * (Hc[0] > 0)
    g["Uv"] = Fv.T @ dZv0
    g["uv"] = dZv0.sum(axis=0)
    g["Uc"] = Fc.T @ dZc0
    g["uc"] = dZc0.sum(axis=0)
    return loss, g, logit


def compare(g, g_ref, logit, logit_ref, loss, loss_ref):
    """The quantities the GPU test bounds: logit and loss errors, whole-gradient
    cosine and relative L2 error, and per tensor the relative L2 error and the
    norm ratio |g_k| / |g_ref_k| (tensors whose reference norm is below 1e-7
    are reported as None)."""
    gv, gr = N.flatten(g), N.flatten(g_ref)
    out = {
        "logit": float(np.max(np.abs(logit - logit_ref)) / max(1.0, float(np.max(np.abs(logit_ref))))),
        "loss": float(abs(loss - loss_ref) / max(1.0, abs(loss_ref))),
        "cos": float(gv @ gr / (np.linalg.norm(gv) * np.linalg.norm(gr))),
        "rel": float(np.linalg.norm(gv - gr) / np.linalg.norm(gr)),
        "tensor_rel": {},
        "tensor_ratio": {},
    }
    for k in N.PARAM_ORDER:
        a = np.asarray(g[k], dtype=np.float64).reshape(-1)
        b = np.asarray(g_ref[k], dtype=np.float64).reshape(-1)
        nb = float(np.linalg.norm(b))
        if nb < 1e-7:
            out["tensor_rel"][k] = None
            out["tensor_ratio"][k] = None
            continue
        out["tensor_rel"][k] = float(np.linalg.norm(a - b) / nb)
        out["tensor_ratio"][k] = float(np.linalg.norm(a) / nb)
    return out
