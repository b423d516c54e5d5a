"""Shared helpers of the GPU parity tests.  Inputs always originate from the
generators or the oracle; the HIP path only ever produces the values that are
compared."""
import numpy as np

from oracle import gfors_oracle as O
from paper_2510_27117_amd import instances as I


def f32(a):
    return np.asarray(a, dtype=np.float32)


def f32_state(st: O.State) -> O.State:
    """Oracle state rounded to FP32 (what both sides start a teacher-forced step from)."""
    x = f32(st.x).astype(np.float64)
    xp = f32(st.x_prev).astype(np.float64)
    y = f32(st.y).astype(np.float64)
    return O.State(x=x, x_prev=xp, xbar=2.0 * x - xp, y=y, k=st.k, n_trig=st.n_trig, rnd=st.rnd)


def rel_inf(got, ref):
    ref = np.asarray(ref, dtype=np.float64)
    if ref.size == 0:
        return 0.0
    return float(np.max(np.abs(np.asarray(got, dtype=np.float64) - ref)) / max(1.0, float(np.max(np.abs(ref)))))


def oracle_trajectory(P, prm: O.Params, steps: int, keep_every: int = 1):
    """FP64 oracle iterates with the rho schedule of Algorithm 1 (one trigger per
    k_int iterations); returns the scaled data and [(state, rho)] before each kept step."""
    S = O.preprocess(P, prm)
    st = O.init_state(S)
    out = []
    for k in range(steps):
        rho = O.rho_value(S, k // prm.k_int)
        if k % keep_every == 0:
            out.append((st, rho))
        st = O.pdhg_step(S, st, rho)
    return S, out


def sample_subset(p, cand, seed, rnd, inst=0):
    """Oracle Bernoulli bits for candidate indices `cand` only: bool [len(cand), n]."""
    n = p.shape[0]
    ii = np.arange(n, dtype=np.int64)[None, :]
    ll = np.asarray(cand, dtype=np.int64)[:, None]
    u = O.uniforms24(seed, rnd, inst, ii, ll)
    return u < np.asarray(p, dtype=np.float64)[None, :]


def mixed_problem(n=150, seed=0):
    """A small BIP mixing every row kind: covering rows, general integer rows with
    signs, equality rows, an all-zero satisfiable row, and a symmetric Q."""
    rng = np.random.default_rng(seed)
    m1, m2 = 40, 9
    A = np.zeros((m1, n), dtype=np.int64)
    for j in range(m1):
        cols = rng.choice(n, size=rng.integers(1, 12), replace=False)
        if j % 3 == 0:
            A[j, cols] = 1
        else:
            A[j, cols] = rng.integers(-7, 8, size=cols.size)
    A[5, :] = 0                       # zero row with b <= 0: always satisfied
    b = np.where(np.arange(m1) % 3 == 0, 1, rng.integers(-6, 3, size=m1))
    b[5] = 0
    Bm = np.zeros((m2, n), dtype=np.int64)
    for j in range(m2):
        cols = rng.choice(n, size=rng.integers(2, 9), replace=False)
        Bm[j, cols] = rng.integers(1, 3, size=cols.size)
    d = rng.integers(0, 4, size=m2)
    Qd = np.zeros((n, n), dtype=np.int64)
    for _ in range(3 * n):
        i, j = rng.integers(0, n, size=2)
        v = int(rng.integers(-5, 6))
        Qd[i, j] += v
        if i != j:
            Qd[j, i] += v
    c = rng.integers(-50, 60, size=n)
    return I.from_dense(c, A=A, b=b, B=Bm, d=d, Q=Qd, name=f"mixed{seed}")


# --------------------------------------------------------- learned proposal

def gnn_case(name):
    """A problem, its scaled data, an oracle iterate (x, y as FP32) and 0/1
    targets: the inputs of the learned-proposal gradient checks."""
    if name == "ufl":
        P = I.facility_location(6, 40, seed=3)
    elif name == "mixed":
        P = mixed_problem(150, seed=11)
    else:
        P = I.set_cover_bernoulli(700, 260, 0.02, seed=4)
    S, traj = oracle_trajectory(P, O.Params(k_int=20), steps=61, keep_every=60)
    st, _ = traj[-1]
    rng = np.random.default_rng(7)
    x = st.x.astype(np.float32)
    y = st.y.astype(np.float32)
    t = (rng.random(P.n) < 0.3).astype(np.float32)
    return P, S, x, y, t


def gnn_params(seed):
    """Network parameters at the initialiser's scale (std sqrt(2/(fan_in+fan_out))),
    small random biases, as FP32."""
    from oracle import gnn_oracle as N
    rng = np.random.default_rng(seed)
    out = {}
    for k, s in N.param_shapes().items():
        if len(s) == 2:
            out[k] = rng.normal(0, np.sqrt(2.0 / (s[0] + s[1])), size=s)
        elif k == "wo":
            out[k] = rng.normal(0, np.sqrt(2.0 / 65), size=s)
        else:
            out[k] = rng.normal(0, 0.05, size=s)
    return {k: v.astype(np.float32) for k, v in out.items()}
