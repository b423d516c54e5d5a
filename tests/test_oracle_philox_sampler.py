"""Pins of the oracle's Philox4x32-10 and Bernoulli sampler (Algorithm 3).

The Philox stream is pinned to rocRAND's Philox4x32-10 engine, compiled from
rocRAND's public header API on the host (tests/philox_ref/rocrand_ref.cpp).
rocRAND documents a subsequence as 4 * 2^64 numbers, so (subsequence, offset)
address the counter as high 64 bits = subsequence, low 64 bits = offset / 4.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle import gfors_oracle as O

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def rocrand_ref(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    out = tmp_path_factory.mktemp("rr") / "rocrand_ref"
    src = os.path.join(HERE, "philox_ref", "rocrand_ref.cpp")
    subprocess.run([hipcc, "-O1", "-o", str(out), src], check=True,
                   stdout=subprocess.PIPE, stderr=subprocess.PIPE)
    return str(out)


def _rocrand4(exe, seed, c0, c1, c2, c3, count=1):
    sub = (c3 << 32) | c2
    off = 4 * ((c1 << 32) | c0)
    r = subprocess.run([exe, str(seed), str(sub), str(off), str(count)], check=True,
                       stdout=subprocess.PIPE, text=True)
    return [tuple(int(v) for v in line.split()) for line in r.stdout.strip().splitlines()]


def test_philox_matches_rocrand_engine(rocrand_ref):
    rng = np.random.default_rng(123)
    cases = [(0, 0, 0, 0, 0)]
    for _ in range(12):
        seed = int(rng.integers(0, 2**63))
        c = [int(v) for v in rng.integers(0, 2**32, size=4)]
        c[0] = min(c[0], 2**32 - 8)  # consecutive counters stay inside word 0
        c[1] >>= 2                   # rocRAND's offset counts numbers: 4 * counter < 2^64
        cases.append((seed, *c))
    for seed, c0, c1, c2, c3 in cases:
        ref = _rocrand4(rocrand_ref, seed, c0, c1, c2, c3, count=4)
        for j, words in enumerate(ref):
            got = O.philox4x32_10([c0 + j], [c1], [c2], [c3], seed & 0xFFFFFFFF, seed >> 32)
            assert tuple(int(g[0]) for g in got) == words, (seed, c0 + j, c1, c2, c3)


def test_uniform_counter_map_matches_rocrand(rocrand_ref):
    """u(inst, round, i, l) uses counter (l>>2, i, round, inst), word l&3."""
    seed, rnd, inst = 77, 5, 3
    i = np.array([0, 1, 2, 3, 4, 9, 1001])
    l = np.array([0, 0, 7, 63, 64, 1000, 5])
    u = O.uniforms24(seed, rnd, inst, i, l)
    for k in range(i.size):
        words = _rocrand4(rocrand_ref, seed, int(l[k]) >> 2, int(i[k]), rnd, inst)[0]
        U = words[int(l[k]) & 3]
        assert u[k] == (U >> 8) * 2.0 ** -24


def test_philox_bit_balance_and_chi2():
    n = 1 << 16
    w = O.philox4x32_10(np.arange(n), 0, 0, 0, 12345, 0)
    allw = np.concatenate(w).astype(np.uint64)
    # every bit position is one with probability 1/2 (binomial, 6 sigma)
    N = allw.size
    for b in range(32):
        ones = int(np.sum((allw >> np.uint64(b)) & np.uint64(1)))
        assert abs(ones - N / 2) < 6 * np.sqrt(N / 4)
    # chi-square over 256 bins of the top byte
    hist = np.bincount((allw >> np.uint64(24)).astype(np.int64), minlength=256)
    e = N / 256
    chi2 = float(np.sum((hist - e) ** 2 / e))
    assert chi2 < 255 + 6 * np.sqrt(2 * 255)


def test_sampler_mean_equals_p():
    """Proposition (x_p = p), Sec. 2.2: the mean of the product distribution is p."""
    rng = np.random.default_rng(0)
    n, K = 64, 4096
    p = rng.random(n)
    p[:4] = [0.0, 1.0, 0.5, 2.0 ** -24]
    X = O.sample_bits(p, K, seed=9, rnd=2)
    mean = X.mean(axis=0)
    sd = np.sqrt(p * (1 - p) / K)
    assert np.all(np.abs(mean - p) <= 6 * sd + 1e-12)
    assert not X[:, 0].any() and X[:, 1].all()


def test_sampler_is_threshold_of_uniforms():
    rng = np.random.default_rng(1)
    n, K = 37, 128
    p = rng.random(n).astype(np.float32)
    X = O.sample_bits(p.astype(np.float64), K, seed=5, rnd=11, instance=2)
    ii = np.arange(n)[None, :]
    ll = np.arange(K)[:, None]
    u = O.uniforms24(5, 11, 2, ii, ll)
    assert np.array_equal(X, u < p[None, :].astype(np.float64))
    # 24-bit uniforms are exactly representable in FP32
    assert np.array_equal(u.astype(np.float32).astype(np.float64), u)


def test_pack_unpack_roundtrip():
    rng = np.random.default_rng(2)
    X = rng.random((192, 13)) < 0.3
    W = O.pack_bits(X)
    assert W.shape == (13, 3) and W.dtype == np.uint64
    assert np.array_equal(O.unpack_bits(W, 192), X)
    # candidate 64w+b lives in bit b of word w
    assert bool((W[4, 2] >> np.uint64(5)) & np.uint64(1)) == bool(X[128 + 5, 4])


def test_round_candidate_threshold():
    x = np.array([0.0, 0.5, np.nextafter(0.5, 1.0), np.nextafter(0.5, 0.0), 1.0])
    assert O.round_candidate(x).tolist() == [[False, False, True, False, True]]


def test_strict_threshold_at_equal_uniform(rocrand_ref):
    """Algorithm 3 with the strict comparison of the sampler's reading: a
    candidate whose uniform equals p_i exactly samples 0, one ulp of the 24-bit
    grid above it samples 1.  The uniforms come from rocRAND's engine."""
    seed, rnd, inst = 3, 4, 1
    n, K = 6, 8
    l0 = 5
    words = [_rocrand4(rocrand_ref, seed, l0 >> 2, i, rnd, inst)[0][l0 & 3] for i in range(n)]
    u = np.array([(w >> 8) * 2.0 ** -24 for w in words])
    X_eq = O.sample_bits(u, K, seed, rnd, inst)
    X_up = O.sample_bits(u + 2.0 ** -24, K, seed, rnd, inst)
    assert not X_eq[l0].any()
    assert X_up[l0].all()


def test_header_counter_map_replays_the_sampler():
    """The uniform map stated in include/gfors.h (gfors_sample_eval) is read
    from the header text, evaluated with the oracle's Philox4x32-10, and must
    reproduce the oracle's candidates: a caller can replay the uniforms from
    the documented contract alone."""
    import re
    with open(os.path.join(HERE, "..", "include", "gfors.h")) as f:
        txt = " ".join(ln.strip().lstrip("/*").strip() for ln in f)
    txt = " ".join(txt.split())
    m = re.search(r"U = word \(([^)]*)\) of Philox4x32-10\(key = \(([^,]*), ([^)]*)\), "
                  r"counter = \(([^,]*), ([^,]*), ([^,]*), ([^)]*)\)\), taken as u = "
                  r"\(U >> (\d+)\) 2\^-(\d+); candidate bit = \[u < p_i\]", txt)
    assert m, "uniform map sentence not found in gfors.h"
    word, key0, key1, *ctr = m.groups()[:7]
    shift, bits = int(m.group(8)), int(m.group(9))
    seed, rnd, inst = (1 << 33) + 12345, 7, 2
    rng = np.random.default_rng(4)
    p = rng.random(9)
    K = 64
    X = O.sample_bits(p, K, seed, rnd, inst)
    for l in (0, 1, 6, 33, 63):
        for i in range(p.size):
            env = {"l": l, "i": i, "r": rnd, "t": inst, "seed": seed}
            c = [eval(e, {}, env) for e in ctr]
            k0, k1 = eval(key0, {}, env), eval(key1, {}, env)
            w = O.philox4x32_10(*c, k0, k1)[eval(word, {}, env)]
            u = (int(w) >> shift) * 2.0 ** -bits
            assert bool(u < p[i]) == bool(X[l, i]), (l, i)
