"""CPU oracle of the learned sampling proposal (test infrastructure only).

The paper lets any GPU-compatible routine stand in for RandSampleStep
(customized sampling, Sec. 2.4.2); this library adds one whose per-variable
probabilities come from a small bipartite message-passing network over the
constraint graph.  This file is its plain FP64 statement: features, forward
pass, binary cross-entropy against an incumbent, hand-written backward pass and
Adam.  The HIP kernels are checked against it (parity unpinned beyond the
finite-difference and closed-form checks in tests: the paper has no learned
component to compare with).

Network (hidden width H = 64, L = 3 rounds):
  E      = diag(1/||a_j||) [A; B]          row-normalised constraint matrix (m x n)
  Fv_i   = [x_i, 4 x_i (1 - x_i), c~_i / max|c~|, 1]
  Fc_j   = [y_j / (1 + |y_j|), r~_j / max|r~|, [row j is an equality], 1]
  Hv0 = relu(Fv Uv + uv),  Hc0 = relu(Fc Uc + uc)
  for l = 1..L:
      Sc = E Hv,    Hc = relu(Hc Wcc_l + Sc Wcv_l + bc_l)
      Sv = E^T Hc,  Hv = relu(Hv Wvv_l + Sv Wvc_l + bv_l)
  logit = Hv wo + bo,   p = sigmoid(logit)
  loss  = mean_i [ softplus(logit_i) - t_i logit_i ]   (t = incumbent bits)
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

H = 64
L = 3
DV = 4
DC = 4

PARAM_ORDER = (["Uv", "uv", "Uc", "uc"] +
               [f"{k}{l}" for l in range(L) for k in ("Wcc", "Wcv", "bc", "Wvv", "Wvc", "bv")] +
               ["wo", "bo"])


def param_shapes():
    s = {"Uv": (DV, H), "uv": (H,), "Uc": (DC, H), "uc": (H,), "wo": (H,), "bo": (1,)}
    for l in range(L):
        s.update({f"Wcc{l}": (H, H), f"Wcv{l}": (H, H), f"bc{l}": (H,),
                  f"Wvv{l}": (H, H), f"Wvc{l}": (H, H), f"bv{l}": (H,)})
    return s


def edge_matrix(P) -> sp.csr_matrix:
    """E = diag(1/||a_j||) [A; B] (a zero row stays zero)."""
    blocks = []
    for M in (P.A, P.B):
        if M is not None:
            vals = np.ones(M.nnz) if M.val is None else M.val.astype(np.float64)
            blocks.append(sp.csr_matrix((vals, M.col.astype(np.int64), M.row_ptr.astype(np.int64)),
                                        shape=(M.nrows, M.ncols)))
    if not blocks:
        return sp.csr_matrix((0, P.n))
    E = sp.vstack(blocks).tocsr()
    nrm = np.sqrt(np.asarray(E.multiply(E).sum(axis=1)).reshape(-1))
    inv = np.where(nrm > 0, 1.0 / np.where(nrm > 0, nrm, 1.0), 0.0)
    return (sp.diags(inv) @ E).tocsr()


def features(ct, rt, m1, x, y):
    """Fv, Fc as defined in the module docstring (ct = c~, rt = r~ of Preprocess)."""
    ct = np.asarray(ct, dtype=np.float64)
    rt = np.asarray(rt, dtype=np.float64)
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    cm = float(np.max(np.abs(ct))) if ct.size else 0.0
    cm = cm if cm > 0 else 1.0
    rm = float(np.max(np.abs(rt))) if rt.size else 0.0
    rm = rm if rm > 0 else 1.0
    Fv = np.stack([x, 4.0 * x * (1.0 - x), ct / cm, np.ones_like(x)], axis=1)
    m = rt.shape[0]
    eq = (np.arange(m) >= m1).astype(np.float64)
    Fc = np.stack([y / (1.0 + np.abs(y)), rt / rm, eq, np.ones(m)], axis=1)
    return Fv, Fc


def relu(z):
    return np.maximum(z, 0.0)


def forward(p, E, Fv, Fc):
    cache = {"Hv": [], "Hc": [], "Sc": [], "Sv": []}
    Hv = relu(Fv @ p["Uv"] + p["uv"])
    Hc = relu(Fc @ p["Uc"] + p["uc"])
    cache["Hv"].append(Hv)
    cache["Hc"].append(Hc)
    for l in range(L):
        Sc = E @ Hv
        Hc = relu(Hc @ p[f"Wcc{l}"] + Sc @ p[f"Wcv{l}"] + p[f"bc{l}"])
        Sv = E.T @ Hc
        Hv = relu(Hv @ p[f"Wvv{l}"] + Sv @ p[f"Wvc{l}"] + p[f"bv{l}"])
        cache["Sc"].append(Sc)
        cache["Hc"].append(Hc)
        cache["Sv"].append(Sv)
        cache["Hv"].append(Hv)
    logit = Hv @ p["wo"] + p["bo"][0]
    return logit, cache


def bce_loss(logit, t):
    """mean softplus(z) - t z, computed stably."""
    z = np.asarray(logit, dtype=np.float64)
    sp_ = np.maximum(z, 0.0) + np.log1p(np.exp(-np.abs(z)))
    return float(np.mean(sp_ - np.asarray(t, dtype=np.float64) * z))


def sigmoid(z):
    return 0.5 * (1.0 + np.tanh(0.5 * np.asarray(z, dtype=np.float64)))


def backward(p, E, Fv, Fc, cache, logit, t):
    """Gradients of bce_loss with respect to every parameter (chain rule written out)."""
    n = logit.shape[0]
    g = {}
    dz = (sigmoid(logit) - np.asarray(t, dtype=np.float64)) / n
    Hv_L = cache["Hv"][L]
    g["wo"] = Hv_L.T @ dz
    g["bo"] = np.array([dz.sum()])
    dHv = np.outer(dz, p["wo"])
    dHc = np.zeros_like(cache["Hc"][L])
    for l in range(L - 1, -1, -1):
        Hv_out, Hv_in = cache["Hv"][l + 1], cache["Hv"][l]
        Hc_out, Hc_in = cache["Hc"][l + 1], cache["Hc"][l]
        Sc, Sv = cache["Sc"][l], cache["Sv"][l]
        dZv = dHv * (Hv_out > 0)
        g[f"Wvv{l}"] = Hv_in.T @ dZv
        g[f"Wvc{l}"] = Sv.T @ dZv
        g[f"bv{l}"] = dZv.sum(axis=0)
        dHv_prev = dZv @ p[f"Wvv{l}"].T
        dSv = dZv @ p[f"Wvc{l}"].T
        dHc = dHc + E @ dSv
        dZc = dHc * (Hc_out > 0)
        g[f"Wcc{l}"] = Hc_in.T @ dZc
        g[f"Wcv{l}"] = Sc.T @ dZc
        g[f"bc{l}"] = dZc.sum(axis=0)
        dHc_prev = dZc @ p[f"Wcc{l}"].T
        dSc = dZc @ p[f"Wcv{l}"].T
        dHv_prev = dHv_prev + E.T @ dSc
        dHv, dHc = dHv_prev, dHc_prev
    dZv0 = dHv * (cache["Hv"][0] > 0)
    dZc0 = dHc * (cache["Hc"][0] > 0)
    g["Uv"] = Fv.T @ dZv0
    g["uv"] = dZv0.sum(axis=0)
    g["Uc"] = Fc.T @ dZc0
    g["uc"] = dZc0.sum(axis=0)
    return g


def loss_and_grad(p, E, Fv, Fc, t):
    logit, cache = forward(p, E, Fv, Fc)
    return bce_loss(logit, t), backward(p, E, Fv, Fc, cache, logit, t), logit


def adam_step(p, g, state, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba): m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
    theta -= lr * (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps)."""
    state["t"] = state.get("t", 0) + 1
    tt = state["t"]
    out = {}
    for k in PARAM_ORDER:
        m = state.setdefault("m_" + k, np.zeros_like(p[k]))
        v = state.setdefault("v_" + k, np.zeros_like(p[k]))
        m = b1 * m + (1 - b1) * g[k]
        v = b2 * v + (1 - b2) * g[k] * g[k]
        state["m_" + k], state["v_" + k] = m, v
        mh = m / (1 - b1 ** tt)
        vh = v / (1 - b2 ** tt)
        out[k] = p[k] - lr * mh / (np.sqrt(vh) + eps)
    return out


def flatten(p) -> np.ndarray:
    return np.concatenate([np.asarray(p[k], dtype=np.float64).reshape(-1) for k in PARAM_ORDER])


def unflatten(v) -> dict:
    out, o = {}, 0
    for k in PARAM_ORDER:
        shp = param_shapes()[k]
        sz = int(np.prod(shp))
        out[k] = np.asarray(v[o:o + sz], dtype=np.float64).reshape(shp)
        o += sz
    return out
