"""Benchmark of the GFORS hot path on one MI355X.

A step = one trigger period of Algorithm 1: k_int PDHG iterations (Algorithm 2)
followed by one sampling round of K candidates (Algorithm 3) with exact
evaluation and incumbent update (EvalBest), replayed from a captured HIP graph.
Inputs are resident in HBM before the timed region starts.

Prints ONE JSON line (see the keys below).  Also measured:
  * per-kernel HIP-event durations -> roofline of the dominant kernel;
  * time-to-incumbent: wall time (HIP events) until the incumbent is within
    0.1% of the best value reached in a fixed budget of rounds;
  * the CPU oracle on a bounded sample of the same workload (cpu_baseline).
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "PDHG iter/s + candidates/s; time-to-incumbent at fixed gap, learned vs plain"
HBM_PEAK_GBS = 8000.0
# single-instance workloads generated as they are (no reformulation), whose
# time-to-incumbent is also taken over other instance seeds
PLAIN_WORKLOADS = ("setcover_small", "setcover_large", "maxcut", "ufl")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="setcover_large",
                    help="setcover_large (the headline line), setcover_small, maxcut, knapsack_batch, ufl, "
                         "ufl_tu, ufl_mono, ufl_learned, or tu_factored (the factorised TU record alone)")
    ap.add_argument("--K", type=int, default=1024)
    ap.add_argument("--k-int", type=int, default=100)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--tti-rounds", type=int, default=300)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--tti-seeds", default="0,1,2,3,4",
                    help="instance seeds whose time-to-incumbent is reported (median over them); "
                         "single-instance plain workloads only, '' for the main seed alone")
    ap.add_argument("--traffic-file", default=os.path.join(ROOT, "profiles", "hbm_traffic.json"))
    ap.add_argument("--launch-cfg", default=None,
                    help="pin the SpMV launch shapes (8 comma-separated ints: lpr_dual, lpr_primal, "
                         "slices_dual, slices_primal, sell_dual, sell_primal, bits_dual, "
                         "bits_primal) instead of autotuning them")
    ap.add_argument("--calib-copy", action="store_true",
                    help="run a plain 512 MiB device copy first (scale for HBM byte counters)")
    ap.add_argument("--ufl-eval", default="1000,10000",
                    help="ufl_learned: facilities,customers of the evaluation instance")
    ap.add_argument("--relax", choices=["tu", "mono"], default="tu",
                    help="ufl_learned: TU reformulation or monotone relaxation of the customer rows")
    ap.add_argument("--snap-window", default=None,
                    help="ufl_learned: first,last fraction of each training run to take iterates from")
    ap.add_argument("--train-instances", type=int, default=200)
    ap.add_argument("--net-every", type=int, default=1,
                    help="ufl_learned: run the network at every n-th trigger (its p is reused in between)")
    ap.add_argument("--eval-seeds", default="",
                    help="ufl_learned: instance seeds of the evaluation instance (default: --seed)")
    ap.add_argument("--train-steps", type=int, default=3000)
    ap.add_argument("--seq-sample", type=int, default=8,
                    help="batched workloads: instances run one by one for the comparison")
    ap.add_argument("--sub", default="setcover_small_e2e,knapsack_batch,ufl_mono,tu_factored,ufl_learned",
                    help="with the default workload: further workloads measured after it and reported as "
                         "compact sub-records ('' for none)")
    return ap.parse_args()


def _csr_dot(M, x):
    """Row sums M x of an integer CSR (reporting only)."""
    import scipy.sparse as sp
    val = np.ones(M.nnz, dtype=np.int64) if M.val is None else np.asarray(M.val, dtype=np.int64)
    S = sp.csr_matrix((val, np.asarray(M.col), np.asarray(M.row_ptr)), shape=(M.nrows, M.ncols))
    return S @ np.asarray(x, dtype=np.int64)


def indexed_entries(bip):
    """Entries of [A; B] whose index must be read: a row whose columns form one
    contiguous range needs only its first column, and likewise a variable
    whose rows form one (the transposed products).  Returns (row-major,
    variable-major) counts."""
    mats = [M for M in (bip.A, bip.B) if M is not None and M.nrows]
    if not mats:
        return 0, 0
    rp = np.concatenate([np.asarray(mats[0].row_ptr, dtype=np.int64)] +
                        [np.asarray(M.row_ptr[1:], dtype=np.int64) + sum(P.nnz for P in mats[:i])
                         for i, M in enumerate(mats) if i])
    col = np.concatenate([np.asarray(M.col, dtype=np.int64) for M in mats])
    m, ln = len(rp) - 1, np.diff(rp)
    rows = np.repeat(np.arange(m, dtype=np.int64), ln)
    # row-major: a row is contiguous when its last column is first + len - 1
    first = np.where(ln > 0, col[np.minimum(rp[:-1], len(col) - 1)], 0)
    last = np.where(ln > 0, col[np.maximum(rp[1:] - 1, 0)], 0)
    rsorted = np.all(np.diff(col)[np.diff(rows) == 0] > 0) if len(col) > 1 else True
    rcont = (ln > 0) & (last - first + 1 == ln) & bool(rsorted)
    row_major = int(ln[~rcont].sum())
    # variable-major: rows of each variable, by count, min and max
    n = bip.n
    cnt = np.bincount(col, minlength=n)
    lo = np.full(n, np.iinfo(np.int64).max)
    hi = np.full(n, -1)
    np.minimum.at(lo, col, rows)
    np.maximum.at(hi, col, rows)
    ccont = (cnt > 0) & (hi - lo + 1 == cnt)
    var_major = int(cnt[~ccont].sum())
    return row_major, var_major


def constant_degree(bip):
    """Every variable has the same number of rows of [A; B] (> 0)."""
    mats = [M for M in (bip.A, bip.B) if M is not None and M.nrows]
    if not mats:
        return False
    cnt = sum(np.bincount(np.asarray(M.col, dtype=np.int64), minlength=bip.n) for M in mats)
    return bool(cnt[0] > 0 and np.all(cnt == cnt[0]))


def kernel_bytes(bip, K, idx=None):
    """Algorithmic HBM bytes per launch: every array the kernel must touch,
    counted once (gathered vectors by their unique size); indices only where
    the entries are not one contiguous range (idx = indexed_entries)."""
    n, m = bip.n, bip.m1 + bip.m2
    nnzK = (0 if bip.A is None else bip.A.nnz) + (0 if bip.B is None else bip.B.nnz)
    unit = (bip.A is None or bip.A.val is None) and (bip.B is None or bip.B.val is None)
    nnzQ = 0 if bip.Q is None else bip.Q.nnz
    vb = 0 if unit else 4
    if not unit and all(np.abs(M.values().astype(np.int64)).max(initial=0) <= 32767
                        for M in (bip.A, bip.B) if M is not None):
        vb = 2   # the SpMVs read an int16 copy of the coefficients
    ir, ic = (nnzK, nnzK) if idx is None else idx
    W = K // 64
    out = {}
    if m:
        # row_ptr + col (+val) + xbar (unique) + omega, rt, y_in, y_out, wy
        out["dual"] = 4 * (m + 1) + 4 * ir + vb * nnzK + 4 * n + 20 * m
    prim = 16 * n  # x_in, ct read; x_out, xbar written
    if m:
        # row pointers of the transposed CSR, unless every variable has the
        # same number of rows (then the kernels compute the ranges)
        prim += (0 if constant_degree(bip) else 4 * (n + 1)) + 4 * ic + vb * nnzK + 4 * m
    if nnzQ:
        prim += 4 * (n + 1) + 8 * nnzQ
    out["primal"] = prim
    out["sample"] = 8 * n * W + 4 * n + 8 * n          # candidate words + p + cost
    if m:
        out["eval_cover"] = 4 * (m + 1) + 4 * ir + 8 * n * W
        out["eval_general"] = 4 * (m + 1) + 4 * ir + (4 if vb else 0) * nnzK + 8 * n * W + 8 * m
    if nnzQ:
        out["eval_quad"] = 4 * (n + 1) + 8 * nnzQ + 8 * n * W
    return out


def signed_index_bytes(bip, bits_dual, bits_primal, kb):
    """The SpMVs' bytes in the signed-index launch variants (dual 5, primal 6
    and 7): a light item (< 256 entries) reads its D 4-byte signed indices and
    neither a row pointer nor a coefficient; a heavy item its two row pointers,
    its indices (unless its entries are one contiguous range) and
    coefficients; in primal 7 a group of up to 16 heavy variables with
    unit-shifted rows reads the indices and coefficients of its first variable
    only.  Vectors as in kernel_bytes.  Returns kb updated."""
    import scipy.sparse as sp
    if bits_dual != 5 and bits_primal not in (6, 7):
        return kb
    mats = [M for M in (bip.A, bip.B) if M is not None and M.nrows]
    K = sp.vstack([sp.csr_matrix((M.values().astype(np.int64), np.asarray(M.col), np.asarray(M.row_ptr)),
                                 shape=(M.nrows, bip.n)) for M in mats]).tocsr()
    m, n = K.shape
    vb = 2 if np.abs(K.data).max(initial=0) <= 32767 else 4
    heavy = 256
    out = dict(kb)

    def side(M, nvec_other, extra, group):
        ln = np.diff(M.indptr)
        hv = ln >= heavy
        b = int(4 * ln[~hv].sum())                         # light: signed indices
        first = M.indices[np.minimum(M.indptr[:-1], max(M.nnz - 1, 0))]
        last = M.indices[np.maximum(M.indptr[1:] - 1, 0)]
        cont = hv & (last - first + 1 == ln)
        if group:
            idxs = np.flatnonzero(hv)
            k = 0
            while k < len(idxs):
                v0 = idxs[k]
                r0 = M.indices[M.indptr[v0]:M.indptr[v0 + 1]]
                a0 = M.data[M.indptr[v0]:M.indptr[v0 + 1]]
                w = 1
                while w < 16 and k + w < len(idxs) and idxs[k + w] == v0 + w:
                    v = v0 + w
                    r = M.indices[M.indptr[v]:M.indptr[v + 1]]
                    a = M.data[M.indptr[v]:M.indptr[v + 1]]
                    if len(r) != len(r0) or np.any(r != r0 + w) or np.any(a != a0):
                        break
                    w += 1
                b += int(ln[v0]) * (4 + vb) + 16   # first variable's entries; group table
                k += w
        else:
            b += int(8 * hv.sum() + 4 * ln[hv & ~cont].sum() + vb * ln[hv].sum())
        return b + 4 * nvec_other + extra

    if bits_dual == 5 and "dual" in out:
        out["dual"] = side(K, n, 20 * m, False)
    if bits_primal in (6, 7) and "primal" in out:
        out["primal"] = side(K.T.tocsr(), m, 16 * n, bits_primal == 7)
    return out


VALU_LANE_OPS = 256 * 64 * 2.4e9   # lanes x clock of the 256 CUs: one integer op per lane per clock
MFMA_INT8_TOPS = 5000.0             # dense int8 matrix-core peak of the MI355X (TOP/s)


def quad_eval_entries(bip):
    """Q entries the objective's evaluation visits: the upper triangle
    (diagonal included) of a symmetric Q, else all of them."""
    if bip.Q is None:
        return 0
    import scipy.sparse as sp
    Q = bip.Q
    M = sp.csr_matrix((Q.values().astype(np.int64), np.asarray(Q.col), np.asarray(Q.row_ptr)),
                      shape=(Q.nrows, Q.ncols))
    if (M != M.T).nnz:
        return Q.nnz
    rows = np.repeat(np.arange(Q.nrows), np.diff(np.asarray(Q.row_ptr)))
    return int(np.count_nonzero(np.asarray(Q.col) >= rows))


def general_row_nnz(bip):
    """Entries of the rows evaluated lane = candidate (not as bitwise functions
    of the candidate words: covering, at-most-one, exactly-one and rows of one
    or two entries are)."""
    tot = 0
    for M, rhs in ((bip.A, bip.b), (bip.B, bip.d)):
        if M is None or M.nrows == 0:
            continue
        rp = np.asarray(M.row_ptr, dtype=np.int64)
        ln = np.diff(rp)
        v = np.ones(int(rp[-1]), dtype=np.int64) if M.val is None else np.asarray(M.val, dtype=np.int64)
        rows = np.repeat(np.arange(M.nrows), ln)
        allone = np.bincount(rows, weights=(v == 1), minlength=M.nrows) == ln
        allneg = np.bincount(rows, weights=(v == -1), minlength=M.nrows) == ln
        r = np.asarray(rhs, dtype=np.int64)
        # covering / at-most-one (inequalities), exactly-one (equalities), pairs
        bitwise = (ln > 0) & (((allone & (r == 1)) | (allneg & (r == -1))) | (ln <= 2))
        tot += int(ln[~bitwise].sum())
    return tot


def run_tti_rounds(G, R, K, use_graph):
    """R sampling rounds from a reset; elapsed ms after each (HIP events)."""
    import torch
    G.reset()
    stream = G.stream
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(R + 1)]
    evs[0].record(stream)
    for r in range(R):
        G.run_rounds(1, K, use_graph)
        evs[r + 1].record(stream)
    G.synchronize()
    return [evs[0].elapsed_time(evs[r + 1]) for r in range(R)]


def single_tti(G, R, times, k_int):
    """Time to an incumbent within 0.1 % of the value after R rounds."""
    hist = G.history(0, R)
    feas = np.nonzero(hist != np.iinfo(np.int64).max)[0]
    if not feas.size:
        return {"rounds": R, "z_final": None, "note": "no feasible candidate",
                "avg_ms_per_round": round(times[-1] / R, 4)}
    zf = int(hist[-1])
    target = zf + 0.001 * abs(zf)
    r_hit = int(np.nonzero(hist <= target)[0][0])
    return {"rounds": R, "z_final": zf, "target_gap": 0.001, "round_hit": r_hit,
            "ms_to_target": round(times[r_hit], 3), "first_feasible_round": int(feas[0]),
            "ms_to_first_feasible": round(times[int(feas[0])], 3),
            "ms_total": round(times[-1], 3),
            "avg_ms_per_round": round(times[-1] / R, 4),
            "iter_per_s_over_run": round(R * k_int / (times[-1] / 1e3), 1)}


def host_cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(bip, k_int, K, budget_s=8.0):
    """The oracle as it stands (FP64 PDHG, exact int64 evaluation, one host
    core) on a bounded sample of the same workload: one warm-up iteration, then
    up to 10 iterations timed one by one (median); from the resulting iterate
    one sampling round of Kc candidates (64, or 8 above 4M variables) drawn
    at once, evaluated in 4 blocks after a warm-up evaluation of 2 candidates
    (median block time).  Iterations and blocks stop early once budget_s is
    spent (at least 3 iterations and one block).  Scaled to the step of the
    GPU record (k_int iterations + K candidates per instance)."""
    from oracle import gfors_oracle as O
    prm = O.Params(k_int=k_int, power_iters=3)
    S = O.preprocess(bip, prm)
    st = O.init_state(S)
    rho = O.rho_value(S, 0)
    st = O.pdhg_step(S, st, rho)                       # warm-up
    ti = []
    t_start = time.perf_counter()
    while len(ti) < 10 and (len(ti) < 3 or time.perf_counter() - t_start < budget_s):
        t0 = time.perf_counter()
        st = O.pdhg_step(S, st, rho)
        ti.append(time.perf_counter() - t0)
    t_iter = float(np.median(ti))
    kc = 64 if bip.n <= 4_000_000 else 8
    blk = kc // 4
    t0 = time.perf_counter()
    X = O.sample_bits(st.x, kc, 0, 0)
    t_sample = time.perf_counter() - t0
    O.evaluate(bip, X[:2])                              # warm-up
    tb = []
    inc = O.Incumbent()
    t_start = time.perf_counter()
    for q in range(4):
        if q and time.perf_counter() - t_start > budget_s:
            break
        t0 = time.perf_counter()
        viol, z = O.evaluate(bip, X[q * blk:(q + 1) * blk])
        O.incumbent_update(inc, X[q * blk:(q + 1) * blk], viol, z, 0, st.k)
        tb.append(time.perf_counter() - t0)
    t_cand = t_sample / kc + float(np.median(tb)) / blk
    T = bip.num_instances
    step = k_int * t_iter + K * T * t_cand
    return {"value": k_int / step, "unit": "PDHG iter/s", "cores": 1, "kind": "oracle",
            "sample": (f"1 warm-up + {len(ti)} FP64 PDHG iterations timed one by one (median), "
                       f"1 sampling round of {kc} candidates drawn at once and evaluated exactly in "
                       f"{len(tb)} block(s) of {blk} after a warm-up (median), on the full workload; "
                       f"scaled to a step of {k_int} iterations + {K * T} candidates"),
            "candidates_per_s": 1.0 / t_cand, "iter_per_s_pdhg_only": 1.0 / t_iter,
            "host_cpus": os.cpu_count(), "host_cpu_model": host_cpu_model()}


def _pool_instance(args):
    """One knapsack of the batch with the oracle (pool worker): seconds for
    10 FP64 PDHG iterations and for one sampling round of 64 candidates."""
    bip, k_int = args
    from oracle import gfors_oracle as O
    S = O.preprocess(bip, O.Params(k_int=k_int, power_iters=3))
    st = O.init_state(S)
    rho = O.rho_value(S, 0)
    st = O.pdhg_step(S, st, rho)
    t0 = time.perf_counter()
    for _ in range(10):
        st = O.pdhg_step(S, st, rho)
    t1 = time.perf_counter()
    X = O.sample_bits(st.x, 64, 0, 0)
    viol, z = O.evaluate(bip, X)
    O.incumbent_update(O.Incumbent(), X, viol, z, 0, st.k)
    return t1 - t0, time.perf_counter() - t1


def cpu_baseline_pool(parts, k_int, K=512):
    """The oracle on the knapsack batch over all host cores: a process pool
    (one instance per task) runs 10 FP64 iterations and a 64-candidate round
    on a sample of 4 x cores instances (after one warm-up task per worker);
    each instance's time for k_int iterations + K candidates is estimated from
    its own timings, the sample mean is scaled to the whole batch and divided
    by the core count (the pool keeps every core busy).  Must run before the
    process touches the GPU (the pool forks)."""
    import multiprocessing as mp
    cores = os.cpu_count() or 1
    pick = parts[:4 * cores]
    ctx = mp.get_context("fork")
    with ctx.Pool(cores) as pool:
        pool.map(_pool_instance, [(parts[0], k_int)] * cores, chunksize=1)
        t0 = time.perf_counter()
        res = pool.map(_pool_instance, [(P, k_int) for P in pick], chunksize=1)
        wall = time.perf_counter() - t0
    step = [k_int * ti / 10.0 + K * tc / 64.0 for ti, tc in res]
    batch_step = float(np.mean(step)) * len(parts) / cores
    return {"value": k_int / batch_step, "unit": "PDHG iter/s (batched)", "cores": cores,
            "kind": "oracle",
            "sample": (f"{len(pick)} of the {len(parts)} instances, 10 FP64 PDHG iterations + 1 round of "
                       f"64 candidates each, process pool on {cores} cores ({wall:.1f} s); per-instance "
                       f"step ({k_int} iterations + {K} candidates) scaled from its timings, batch = "
                       f"mean x {len(parts)} / {cores}"),
            "instance_iter_per_s": k_int * len(parts) / batch_step,
            "candidates_per_s": len(pick) * 64 / sum(tc for _, tc in res) * cores,
            "host_cpus": cores, "host_cpu_model": host_cpu_model()}


def c1_end_to_end(a):
    """Set cover n=200, m=100 end to end as configured: 2,000 PDHG iterations
    with a round of K=256 candidates every 100 (20 rounds) and the final
    rounding.  GPU: one captured graph per round, median of 5 runs from a
    reset after a warm-up run.  Oracle: the same loop in FP64 on one core.
    Both incumbents against the exact optimum (HiGHS milp)."""
    import torch
    from scipy.optimize import Bounds, LinearConstraint, milp
    from paper_2510_27117_amd import gfors, instances
    from oracle import gfors_oracle as O
    bip = instances.workload("setcover_small", seed=a.seed)
    G = gfors.Problem(bip, gfors.default_params(k_int=100, K_max=256))
    G.run_rounds(20, 256, True)
    G.final_round()
    G.synchronize()
    ms = []
    for _ in range(5):
        G.reset()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(G.stream)
        G.run_rounds(20, 256, True)
        G.final_round()
        e1.record(G.stream)
        G.synchronize()
        ms.append(e0.elapsed_time(e1))
    bg = G.best(0)
    G.close()
    t0 = time.perf_counter()
    inc, _, _, _ = O.run_gfors(bip, O.Params(k_int=100), 2000, 256)
    t_or = time.perf_counter() - t0
    A = np.zeros((bip.m1, bip.n))
    rows = np.repeat(np.arange(bip.m1), np.diff(np.asarray(bip.A.row_ptr)))
    A[rows, np.asarray(bip.A.col)] = bip.A.values()
    res = milp(np.asarray(bip.c, dtype=np.float64), constraints=LinearConstraint(A, lb=np.asarray(bip.b, float)),
               integrality=np.ones(bip.n), bounds=Bounds(0, 1))
    zopt = int(round(res.fun)) if res.success else None
    gap = (lambda z: round((z - zopt) / abs(zopt), 5) if (z is not None and zopt) else None)
    return {"workload": "set cover n=200, m=100 (density 0.05 + forced cover), 2,000 iterations, "
                        "20 rounds x K=256 + final rounding",
            "gpu_ms_end_to_end": round(float(np.median(ms)), 3),
            "gpu_pdhg_iter_per_s": round(2000 / (float(np.median(ms)) / 1e3), 1),
            "gpu_candidates_per_s": round(20 * 256 / (float(np.median(ms)) / 1e3), 1),
            "gpu_z": bg["z"] if bg["found"] else None, "gpu_gap_to_optimum": gap(bg["z"] if bg["found"] else None),
            "cpu_oracle": {"s_end_to_end": round(t_or, 3), "cores": 1, "kind": "oracle",
                           "z": inc.z, "gap_to_optimum": gap(inc.z)},
            "milp_optimum": zopt}


SUB_STEPS = {"knapsack_batch": (512, 50), "ufl_mono": (1024, 200)}


def sub_records(a, subs, pre):
    """Compact records of further workloads (same measurement as the main
    line, fewer steps): the configured small set cover end to end, the
    knapsack batch, facility location under the monotone relaxation, the
    factorised TU reformulation of a 90,000-variable quadratic assignment, and
    the learned proposal against the plain sampler on facility location."""
    import argparse as _ap
    out = {}
    keep = ("value", "unit", "ms_per_step", "candidates_per_s", "instance_iter_per_s", "config",
            "roofline", "eval_alu", "kernels", "time_to_incumbent", "batched_vs_sequential",
            "cpu_baseline", "preprocess_s", "generate_s")
    for w in subs:
        if w == "setcover_small_e2e":
            out[w] = c1_end_to_end(a)
            continue
        if w == "ufl_learned":
            # the learned proposal at the configured facility-location size
            # with a shortened training (50 instances, 1,000 Adam steps) and
            # one evaluation seed, the network run every 4th trigger; the
            # full record (200 instances, 3,000 steps, seeds 0-4, every 1st
            # and 4th trigger) is profiles/ufl_learned_vs_plain.json
            b = _ap.Namespace(**vars(a))
            b.relax, b.train_instances, b.train_steps, b.eval_seeds = "mono", 50, 1000, str(a.seed)
            b.tti_rounds, b.net_every, b.K, b.ufl_eval, b.snap_window = 300, 4, 1024, "1000,10000", None
            r = learned_experiment(b)
            out[w] = {k: r[k] for k in ("config", "train_loss_before", "train_loss_after", "per_seed",
                                        "median_speedup_time_to_incumbent",
                                        "median_learned_round_overhead")}
            continue
        if w == "tu_factored":
            out[w] = tu_factored_record(a)
            continue
        if w not in SUB_STEPS:
            raise SystemExit(f"--sub: unknown workload {w}")
        b = _ap.Namespace(**vars(a))
        b.workload, b.steps, b.warmup, b.tti_seeds, b.seq_sample, b.launch_cfg = w, 5, 2, "", 4, None
        b.K, b.tti_rounds = SUB_STEPS[w]
        b.pre_baseline = pre.get(w)
        r = run_workload(b)
        rec = {k: r[k] for k in keep if k in r}
        if r.get("sampler_alu"):
            rec["sampler_alu_frac"] = r["sampler_alu"]["frac"]
        out[w] = rec
    return out


def tu_factored_record(a, rounds: int = 150, K: int = 1024):
    """The factorised TU reformulation (Remark of Sec. 2.4.1) at a size where
    the explicit one cannot be formed: 2D assignment n = 300 with a quadratic
    term (90,000 variables), pivots on a random recursive spanning tree (599).
    S would hold millions of entries and Q' = S^T Q_II S + ... on the order of
    10^9; the device problem keeps the LU of the 599 x 599 pivot block
    instead.  Records the PDHG rate (graph replay), the per-step kernels, the
    rounds to an incumbent, and checks the recovered incumbent on the ORIGINAL
    model (B x = d, A x >= b, objective = z + c'_0) with plain integer sums."""
    import torch
    from paper_2510_27117_amd import gfors, instances
    t0 = time.perf_counter()
    full = instances.workload("qap_tu", seed=a.seed)
    t_gen = time.perf_counter() - t0
    t0 = time.perf_counter()
    T = gfors.TUReformulation(full, full.meta["tu_pivots"], factored=True)
    t_factor = time.perf_counter() - t0
    prm = gfors.default_params(k_int=a.k_int, K_max=K)
    t0 = time.perf_counter()
    G = T.problem(prm)
    t_pre = time.perf_counter() - t0
    for _ in range(2):
        G.run_rounds(1, K, True)
    G.synchronize()
    steps = 5
    stream = G.stream
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    G.run_rounds(steps, K, True)
    ev1.record(stream)
    G.synchronize()
    ms = ev0.elapsed_time(ev1) / steps
    kt = G.kernel_times(a.k_int, K)
    kernels = {k: {"avg_ms": round(v, 5), "launches": c} for k, (v, c) in kt.items() if c}
    times = run_tti_rounds(G, rounds, K, True)
    tti = single_tti(G, rounds, times, a.k_int)
    check = None
    b = G.best()
    if b["found"]:
        x = T.recover(b["x"]).astype(np.int64)
        def mv(M, v):
            rows = np.repeat(np.arange(M.nrows), np.diff(M.row_ptr))
            vals = np.ones(M.nnz, np.int64) if M.val is None else M.val.astype(np.int64)
            return np.bincount(rows, weights=vals * v[M.col], minlength=M.nrows).astype(np.int64)
        zq = int(x @ mv(full.Q, x)) if full.Q is not None else 0
        check = {"equalities_hold": bool(np.array_equal(mv(full.B, x), full.d)),
                 "inequalities_hold": bool(np.all(mv(full.A, x) >= full.b)),
                 "z_reduced": b["z"], "constant": T.constant,
                 "z_original": int(full.c @ x) + zq,
                 "objective_shift_exact": int(full.c @ x) + zq == b["z"] + T.constant}
    G.close()
    return {"config": {"workload": "2D assignment n=300 + quadratic term + knapsack row, TU-reformulated "
                                   "with the pivot block factorised (random recursive spanning tree)",
                       "n": int(full.n), "n_reduced": T.n_reduced, "m1_reduced": T.m1,
                       "m2_reduced": T.m2, "nnz_Q": int(full.Q.nnz), "K": K, "k_int": a.k_int,
                       "step": f"{a.k_int} PDHG iterations + 1 round of {K} candidates"},
            "value": round(a.k_int / (ms / 1e3) if ms > 0 else 0.0, 1),
            "unit": "PDHG iter/s", "ms_per_step": round(ms, 4),
            "factor": T.info, "workspace_bytes": G.ws_bytes,
            "kernels": kernels, "time_to_incumbent": tti, "incumbent_check": check,
            "generate_s": round(t_gen, 3), "factor_s": round(t_factor, 3), "preprocess_s": round(t_pre, 3)}


def batched_tti(G, bip, R, times):
    """Per-instance rounds (and wall ms of the batched launch) until the
    incumbent is within 0.1% of the instance's best after R rounds."""
    hits, feas = [], 0
    for t in range(bip.num_instances):
        hist = G.history(t, R)
        ok = np.nonzero(hist != np.iinfo(np.int64).max)[0]
        if not ok.size:
            continue
        feas += 1
        zf = int(hist[-1])
        hits.append(int(np.nonzero(hist <= zf + 0.001 * abs(zf))[0][0]))
    if not hits:
        return {"rounds": R, "instances_with_incumbent": 0}
    med = int(np.median(hits))
    return {"rounds": R, "instances_with_incumbent": feas, "target_gap": 0.001,
            "median_round_hit": med, "max_round_hit": int(max(hits)),
            "ms_to_all_targets": round(times[int(max(hits))], 3),
            "ms_total": round(times[-1], 3), "avg_ms_per_round": round(times[-1] / R, 4)}


def sequential_compare(bip, prm, a, R, batched_ms):
    """The same R rounds run instance by instance (each its own problem, graph
    replay) on a sample of instances; the per-instance mean is scaled to the
    whole batch and set against the batched launch."""
    import torch
    from paper_2510_27117_amd import gfors, instances
    off = bip.inst_offsets
    rng = np.random.default_rng(0)
    pick = rng.choice(bip.num_instances, size=min(a.seq_sample, bip.num_instances), replace=False)
    ms = []
    for t in pick:
        sub = instances.BIP(n=int(off[t + 1, 0] - off[t, 0]), c=bip.c[off[t, 0]:off[t + 1, 0]])
        r0, r1 = int(off[t, 1]), int(off[t + 1, 1])
        rp = bip.A.row_ptr[r0:r1 + 1] - bip.A.row_ptr[r0]
        e0, e1 = int(bip.A.row_ptr[r0]), int(bip.A.row_ptr[r1])
        sub.A = instances.CSR(r1 - r0, sub.n, rp, bip.A.col[e0:e1] - int(off[t, 0]),
                              None if bip.A.val is None else bip.A.val[e0:e1])
        sub.b = bip.b[r0:r1]
        P = gfors.Problem(sub, prm)
        P.run_rounds(1, a.K, True)
        P.synchronize()
        e0_, e1_ = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0_.record(P.stream)
        P.run_rounds(R - 1, a.K, True)
        e1_.record(P.stream)
        P.synchronize()
        ms.append(e0_.elapsed_time(e1_) * R / (R - 1))
        P.close()
    per = float(np.mean(ms))
    return {"sampled_instances": int(len(pick)), "mean_ms_per_instance": round(per, 3),
            "sequential_ms_estimate": round(per * bip.num_instances, 1),
            "batched_ms": round(batched_ms, 1),
            "speedup": round(per * bip.num_instances / batched_ms, 2)}


def learned_experiment(a):
    """Learned vs plain proposal on uncapacitated facility location, after the
    TU reformulation (one assignment per customer eliminated, B_JI = I) or the
    monotone relaxation (customer rows relaxed to >= 1, every candidate
    repaired on the device).

    Training: the plain method runs on `--train-instances` small instances
    (40 facilities x 400 customers, seeds 1000..); iterates at 6 triggers are
    paired with the run's final incumbent; the network is trained on the GPU.
    Evaluation, per instance seed of `--eval-seeds` (the configured 1,000 x
    10,000 by default): `--tti-rounds` triggers plain (K per round from x_k)
    and, after a reset, learned (K/2 from x_k + K/2 from the network per
    trigger).  Time-to-incumbent = HIP-event time until the incumbent is
    within 0.1% of the plain run's final value; the median over the seeds is
    reported."""
    import torch
    from paper_2510_27117_amd import gfors, instances, learned
    t0 = time.perf_counter()

    def reform(P):
        if a.relax == "mono":
            m = gfors.MonotoneRelaxation(P)
            return m.model, m, 0
        t = gfors.TUReformulation(P, P.meta["tu_pivots"])
        return t.model, t, t.constant

    def params(P, k_int, K):
        prm = gfors.default_params(k_int=k_int, K_max=K)
        if a.relax == "mono":
            prm.repair_row0 = P.m1      # relaxed rows follow the original inequality rows
        return prm

    bips = []
    for sd in range(1000, 1000 + a.train_instances):
        P = instances.facility_location(40, 400, seed=sd)
        bips.append(reform(P)[0])
    win = tuple(float(v) for v in a.snap_window.split(",")) if a.snap_window else (None, None)
    train_prm = params(instances.facility_location(40, 400, seed=1000), 50, 256)
    samples = learned.collect(bips, train_prm, rounds=60, K=256, snapshots=6, window=win,
                              log=lambda msg: print(f"[ufl_learned] {msg}", file=sys.stderr, flush=True))
    t_collect = time.perf_counter() - t0
    print(f"[ufl_learned] collected {len(samples)} pairs in {t_collect:.1f} s", file=sys.stderr, flush=True)
    net = gfors.GNN(seed=a.seed)
    loss0 = learned.mean_loss(net, samples[:64])
    t0 = time.perf_counter()
    learned.train(net, samples, steps=a.train_steps, lr=3e-3, seed=a.seed)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    loss1 = learned.mean_loss(net, samples[:64])
    print(f"[ufl_learned] trained {a.train_steps} steps in {t_train:.1f} s, loss {loss0:.4f} -> {loss1:.4f}",
          file=sys.stderr, flush=True)

    nf, nc = (int(v) for v in a.ufl_eval.split(","))
    seeds = [int(v) for v in a.eval_seeds.split(",")] if a.eval_seeds else [a.seed]
    R = a.tti_rounds
    per = {}
    for sd in seeds:
        full = instances.facility_location(nf, nc, seed=sd)
        model, rf, c0 = reform(full)
        G = gfors.Problem(model, params(full, a.k_int, a.K))
        plain = learned.run_plain(G, R, a.K)
        G.reset()
        lrn = learned.run_learned(G, net, R, a.K, net_every=a.net_every)
        G.final_round()
        best = G.best(0)
        zp = [z + c0 if z != learned.INT64_MAX else None for z in plain.z]
        zl = [z + c0 if z != learned.INT64_MAX else None for z in lrn.z]
        rec = {"plain": {"first_feasible_round": next((i for i, z in enumerate(zp) if z is not None), None),
                         "z_final": zp[-1], "ms_total": round(plain.ms[-1], 2),
                         "ms_per_round": round(plain.ms[-1] / R, 3)},
               "learned": {"first_feasible_round": next((i for i, z in enumerate(zl) if z is not None), None),
                           "z_final": zl[-1], "ms_total": round(lrn.ms[-1], 2),
                           "ms_per_round": round(lrn.ms[-1] / R, 3)}}
        if zp[-1] is not None:
            target = zp[-1] + 0.001 * abs(zp[-1])
            tp = plain.time_to(int(np.floor(target - c0)))
            tl = lrn.time_to(int(np.floor(target - c0)))
            rec["time_to_incumbent"] = {"target": target, "plain_ms": tp, "learned_ms": tl,
                                        "learned_reached": tl is not None,
                                        "speedup": (round(tp / tl, 3) if tp and tl else None)}
        if best["found"]:
            xfull = rf.repair(best["x"]) if a.relax == "mono" else rf.recover(best["x"])
            rec["recovered_point_objective"] = int(full.c @ xfull.astype(np.int64))
        per[str(sd)] = rec
        print(f"[ufl_learned] seed {sd}: {json.dumps(rec)}", file=sys.stderr, flush=True)
        G.close()
    net.close()
    sp = [r["time_to_incumbent"]["speedup"] for r in per.values()
          if r.get("time_to_incumbent") and r["time_to_incumbent"]["speedup"] is not None]
    over = [r["learned"]["ms_per_round"] / r["plain"]["ms_per_round"] - 1.0 for r in per.values()]
    return {"metric": METRIC, "workload": "ufl_learned",
            "config": {"workload": (f"facility location {nf} x {nc} (TU: {nc} assignments eliminated)"
                                    if a.relax == "tu" else
                                    f"facility location {nf} x {nc} (customer rows relaxed to >= 1, "
                                    f"candidates repaired on the device)"),
                       "K": a.K, "k_int": a.k_int, "rounds": R, "eval_seeds": seeds,
                       "network_every_n_triggers": a.net_every,
                       "train": f"{a.train_instances} instances 40 x 400, {len(samples)} pairs, {a.train_steps} Adam steps",
                       "snapshot_window": list(win)},
            "collect_s": round(t_collect, 2), "train_s": round(t_train, 2),
            "train_loss_before": round(loss0, 5), "train_loss_after": round(loss1, 5),
            "per_seed": per,
            "median_speedup_time_to_incumbent": (round(float(np.median(sp)), 3) if sp else None),
            "seeds_where_learned_reached_target": len(sp),
            "median_learned_round_overhead": round(float(np.median(over)), 3)}


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {a.gpus}); this build has no "
              f"multi-GPU path.", file=sys.stderr)
        sys.exit(2)
    subs = [w for w in a.sub.split(",") if w.strip()] if (a.sub and a.workload == "setcover_large") else []
    # CPU baselines that fork a process pool run before anything touches the GPU
    pre = {}
    if "knapsack_batch" in subs and not a.no_cpu_baseline:
        from paper_2510_27117_amd import instances
        pre["knapsack_batch"] = cpu_baseline_pool(instances.knapsack_batch(512, a.seed), a.k_int)
    import torch

    if a.calib_copy:
        src = torch.ones(128 * 1024 * 1024, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if a.workload == "ufl_learned":
        print(json.dumps(learned_experiment(a)))
        return
    if a.workload == "tu_factored":
        print(json.dumps(tu_factored_record(a)))
        return
    out = run_workload(a)
    if subs:
        out["sub_records"] = sub_records(a, subs, pre)
    print(json.dumps(out))


def run_workload(a):
    """One workload: warm-up, the timed steps, per-kernel rooflines,
    time-to-incumbent and the CPU oracle baseline.  Returns the record."""
    import torch
    from paper_2510_27117_amd import gfors, instances
    t0 = time.perf_counter()
    tu = None
    mono = None
    if a.workload == "ufl_mono":
        # facility location with the customer rows relaxed to ">= 1" (monotone
        # relaxation); incumbents are repaired to the original problem below
        full = instances.workload("ufl", seed=a.seed)
        mono = gfors.MonotoneRelaxation(full)
        bip = mono.model
    elif a.workload == "ufl_tu":
        # facility location after the TU reformulation (one assignment per
        # customer eliminated); objective values below are of the reduced model
        # and differ from the original ones by the constant c0
        full = instances.workload("ufl", seed=a.seed)
        tu = gfors.TUReformulation(full, full.meta["tu_pivots"])
        bip = tu.model
    else:
        bip = instances.workload(a.workload, seed=a.seed)
    t_gen = time.perf_counter() - t0
    pinned = [int(v) for v in a.launch_cfg.split(",")] if a.launch_cfg else None
    if pinned is not None and len(pinned) != 8:
        raise SystemExit("--launch-cfg takes 8 integers")
    prm = gfors.default_params(k_int=a.k_int, K_max=max(a.K, 1024),
                               autotune=0 if pinned else 1)
    if mono is not None:
        # every candidate is repaired on the device before evaluation: the
        # relaxed rows follow the original inequality rows
        prm.repair_row0 = mono.source.m1
    t0 = time.perf_counter()
    G = gfors.Problem(bip, prm)
    t_pre = time.perf_counter() - t0
    if pinned:
        G.set_launch_cfg(*pinned)
    use_graph = not a.no_graph
    stream = G.stream

    # warmup + timed region (graph replay of whole rounds); the launch shapes
    # are re-tuned on the warmed-up iterate (zero-operand skipping needs it)
    for _ in range(a.warmup):
        G.run_rounds(1, a.K, use_graph)
    G.synchronize()
    if a.warmup and not pinned:
        G.autotune()
        G.run_rounds(1, a.K, use_graph)
        G.synchronize()
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(stream)
    G.run_rounds(a.steps, a.K, use_graph)
    ev1.record(stream)
    G.synchronize()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = ev0.elapsed_time(ev1)
    ms_per_step = gpu_ms / a.steps
    iters_per_s = a.steps * a.k_int / (gpu_ms / 1e3)
    cands_per_s = a.steps * a.K * bip.num_instances / (gpu_ms / 1e3)

    # iterate statistics at the measured state (what the sampler sees)
    stt = G.get_state()
    xs = stt["x"]
    xbar = 2.0 * xs - stt["x_prev"]
    xstats = {"frac_zero": float(np.mean(xs == 0.0)), "frac_one": float(np.mean(xs == 1.0)),
              "frac_fractional": float(np.mean((xs > 0) & (xs < 1))),
              "xbar_zero": float(np.mean(xbar == 0.0)),
              "y_zero": float(np.mean(stt["y"] == 0.0)) if stt["y"].size else None}

    # per-kernel HIP-event durations (eager launches, same stream, state advances)
    kt = G.kernel_times(a.k_int, a.K)
    per_step = {k: ms * (a.k_int if k in ("dual", "primal") else 1) for k, (ms, cnt) in kt.items() if cnt}
    kb = kernel_bytes(bip, a.K, indexed_entries(bip))
    lc = G.launch_cfg()
    kb = signed_index_bytes(bip, lc.get("bits_dual", 0), lc.get("bits_primal", 0), kb)
    dom = max((k for k in per_step if k in kb), key=lambda k: per_step[k])
    avg_ms = kt[dom][0]
    achieved = kb[dom] / (avg_ms * 1e-3) / 1e9
    traffic = None
    try:
        with open(a.traffic_file) as f:
            tr = json.load(f)
        # counters taken on the same workload, K and launch shape only
        cfg_now = list(G.launch_cfg().values())
        for wl in tr.get(a.workload, {}).get("runs", []):
            ent = wl.get(dom)
            if ent and ent.get("K") == a.K and wl.get("launch_cfg") == cfg_now:
                traffic = ent.get("bytes_per_launch")
    except (OSError, ValueError):
        pass
    # the device's bare streaming-read rate (1,024 workgroups, 512 MiB), next to the published peak
    stream_ref = gfors.read_throughput(512 << 20, 1024) / 1e9
    roofline = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "measured_stream_read_gbs": round(stream_ref, 1),
                "frac_of_measured_stream_read": round(achieved / stream_ref, 4) if stream_ref > 0 else None,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "traffic_source": ("rocprofv3 FETCH_SIZE + WRITE_SIZE of this kernel on the same workload, K "
                                   "and launch shape, taken from profiles/hbm_traffic.json (not measured in this run)"
                                   if traffic is not None else None),
                "algorithmic_bytes_per_launch": kb[dom], "avg_launch_ms": avg_ms}
    # the sampler is integer-ALU bound (Philox): its generator calls per second
    # at the measured state (fractional variables x K/4 calls per launch)
    # against the generator's own throughput on this device
    sampler_alu = None
    if kt.get("sample", (0.0, 0))[1]:
        calls = int(round(xstats["frac_fractional"] * bip.n)) * (a.K // 4)
        peak = gfors.philox_throughput()
        ach = calls / (kt["sample"][0] * 1e-3)
        sampler_alu = {"bound": "alu", "kernel": "sample", "achieved": round(ach, 1),
                       "peak": round(peak, 1), "unit": "Philox4x32-10 calls/s",
                       "frac": round(ach / peak, 4) if peak > 0 else None,
                       "calls_per_launch": calls, "avg_launch_ms": kt["sample"][0],
                       "peak_source": "gfors_philox_throughput (generator alone, same counter shape)"}
    # integer evaluation (general rows, quadratic objective): entry x candidate
    # products per second against the VALU lane rate (each product costs at
    # least one lane operation, so frac is an upper bound of VALU use)
    eval_alu = None
    cand = [(k, prods) for k, prods in (("eval_general", general_row_nnz(bip) * a.K),
                                        ("eval_quad", quad_eval_entries(bip) * a.K))
            if prods and kt.get(k, (0.0, 0))[1] and kt[k][0] > 0]
    planes = G.eval_planes()
    if cand:
        k, prods = max(cand, key=lambda kp: kt[kp[0]][0])
        ach = prods / (kt[k][0] * 1e-3)
        if k == "eval_general" and planes:
            # dense digit blocks on the int8 matrix cores: one multiply-add
            # (2 ops) per entry, candidate and digit plane, against the dense
            # int8 MFMA peak
            ops = 2 * prods * planes
            acho = ops / (kt[k][0] * 1e-3)
            eval_alu = {"bound": "mfma", "kernel": k, "achieved": round(acho / 1e12, 2),
                        "peak": MFMA_INT8_TOPS, "unit": "TOP/s (int8)",
                        "frac": round(acho / 1e12 / MFMA_INT8_TOPS, 4), "digit_planes": planes,
                        "ops_per_launch": ops, "entry_candidate_products_per_s": round(ach, 1),
                        "avg_launch_ms": kt[k][0]}
        else:
            eval_alu = {"bound": "alu", "kernel": k, "achieved": round(ach, 1), "peak": VALU_LANE_OPS,
                        "unit": "entry-candidate products/s", "frac": round(ach / VALU_LANE_OPS, 4),
                        "products_per_launch": prods, "avg_launch_ms": kt[k][0]}
    kernels = {k: {"avg_ms": round(ms, 5), "launches": cnt,
                   "gbs": (round(kb[k] / (ms * 1e-3) / 1e9, 1) if k in kb and ms > 0 else None)}
               for k, (ms, cnt) in kt.items() if cnt}

    # time-to-incumbent from a fresh start (same problem, reset)
    R = a.tti_rounds
    times = run_tti_rounds(G, R, a.K, use_graph)
    tti = {}
    if bip.num_instances > 1:
        tti = batched_tti(G, bip, R, times)
    else:
        tti = single_tti(G, R, times, a.k_int)
    # the same for other instance seeds (same launch shapes), median reported
    seeds = [int(v) for v in a.tti_seeds.split(",") if v.strip()] if a.tti_seeds else []
    if (seeds and bip.num_instances == 1 and a.workload in PLAIN_WORKLOADS
            and tti.get("z_final") is not None):
        per = {str(a.seed): {k: tti[k] for k in ("z_final", "round_hit", "ms_to_target", "first_feasible_round")}}
        cfg = list(G.launch_cfg().values())
        for sd in seeds:
            if sd == a.seed:
                continue
            Bs = instances.workload(a.workload, seed=sd)
            Gs = gfors.Problem(Bs, gfors.default_params(k_int=a.k_int, K_max=max(a.K, 1024), autotune=0))
            Gs.set_launch_cfg(*cfg)
            ts = single_tti(Gs, R, run_tti_rounds(Gs, R, a.K, use_graph), a.k_int)
            Gs.close()
            del Gs
            per[str(sd)] = {k: ts.get(k) for k in ("z_final", "round_hit", "ms_to_target", "first_feasible_round")}
        hits = [v["ms_to_target"] for v in per.values() if v.get("ms_to_target") is not None]
        tti["seeds"] = per
        tti["median_ms_to_target"] = round(float(np.median(hits)), 3) if hits else None
        tti["median_round_hit"] = float(np.median([v["round_hit"] for v in per.values() if v.get("round_hit") is not None])) if hits else None

    seq = None
    if bip.num_instances > 1 and a.seq_sample:
        seq = sequential_compare(bip, prm, a, R, times[-1])

    base = None
    if not a.no_cpu_baseline:
        base = a.pre_baseline if getattr(a, "pre_baseline", None) else cpu_baseline(bip, a.k_int, a.K)

    nnzK = (0 if bip.A is None else bip.A.nnz) + (0 if bip.B is None else bip.B.nnz)
    out = {
        "metric": METRIC, "value": round(iters_per_s, 2), "unit": "PDHG iter/s",
        "n_gpus": 1, "steps": a.steps, "warmup": a.warmup, "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "fp32",
        "data": "synthetic",
        "config": {"workload": a.workload, "n": bip.n, "m1": bip.m1, "m2": bip.m2,
                   "nnz_constraints": nnzK, "nnz_Q": 0 if bip.Q is None else bip.Q.nnz,
                   "instances": bip.num_instances, "K": a.K, "k_int": a.k_int,
                   "step": f"{a.k_int} PDHG iterations + 1 round of {a.K} candidates",
                   "graph": use_graph, "seed": a.seed},
        "candidates_per_s": round(cands_per_s, 1),
        "wall_s_timed": round(wall, 4),
        "preprocess_s": round(t_pre, 3), "generate_s": round(t_gen, 3),
        "roofline": roofline, "sampler_alu": sampler_alu, "eval_alu": eval_alu, "kernels": kernels, "launch_cfg": G.launch_cfg(),
        "iterate_stats": xstats,
        "time_to_incumbent": tti,
        "cpu_baseline": base,
    }
    if mono is not None:
        out["config"]["relaxed_rows"] = int(mono.relaxed.sum())
        G.final_round()
        b = G.best(0)
        if b["found"]:
            # candidates were repaired on the device, so the incumbent is a
            # point of the original problem; checked here on its rows
            xr = b["x"].astype(np.int64)
            orig = mono.source
            viol = int(np.sum(_csr_dot(orig.A, xr) < orig.b)) if orig.A is not None else 0
            viol += int(np.sum(_csr_dot(orig.B, xr) != orig.d)) if orig.B is not None else 0
            tti["incumbent_original"] = {"z": int(b["z"]), "z_recomputed": int(orig.c @ xr),
                                         "violated_original_rows": viol,
                                         "repair": "every candidate, on the device, before evaluation"}
    if tu is not None:
        out["config"]["objective_constant"] = int(tu.constant)
        if tti.get("z_final") is not None:
            tti["z_final_original"] = int(tti["z_final"]) + int(tu.constant)
    if bip.num_instances > 1:
        out["instance_iter_per_s"] = round(iters_per_s * bip.num_instances, 1)
        out["batched_vs_sequential"] = seq
    G.close()
    return out


if __name__ == "__main__":
    main()
