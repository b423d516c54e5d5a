// Bernoulli sampling (Algorithm 3) with Philox4x32-10 uniforms and exact
// candidate evaluation (EvalBest, Sec. 3) for gfx950.
//
// Candidate layout: uint64 X[i * W + w] holds candidates 64w .. 64w+63 of
// variable i (bit b = candidate 64w + b); W = K / 64.
//
// Sampler: one Philox call gives the uniforms of four consecutive candidates
// 4g .. 4g+3 of one variable i (counter = (g, i, round, instance), word =
// candidate & 3).  A variable whose p is 0 or 1 needs no uniform at all (its
// candidates are all 0 / all 1), so only the fractional variables cost Philox
// calls.  A workgroup handles 64 variables at a time; its four wavefronts
// split the candidates, lane = group of four candidates; the four bits of a
// lane and of its neighbour form one byte of the variable's candidate row in
// LDS, and the block is written back contiguously.  The linear objective
// sum_i c_i x_i of each candidate is accumulated on the fly, so X is never
// re-read for it.
//
// Evaluation: rows whose coefficients are all one with right-hand side 1
// (covering rows) are checked with bitwise OR over 64 candidates at a time;
// any other row is summed exactly in integers, one candidate per lane.
#include "gfors_internal.h"
#include <type_traits>

namespace gfors {

// Pointers into the constant address space: loads at wave-uniform addresses
// through them become scalar loads.  Only for data no kernel writes while it
// is being read.
template <typename T>
using cptr = const __attribute__((address_space(4))) T *;
template <typename T>
__device__ __forceinline__ cptr<T> to_const(const T *p) {
    return reinterpret_cast<cptr<T>>(reinterpret_cast<uintptr_t>(p));
}

__device__ __forceinline__ void philox10(uint32_t &c0, uint32_t &c1, uint32_t &c2,
                                         uint32_t &c3, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = static_cast<uint64_t>(kPhiloxM0) * c0;
        const uint64_t p1 = static_cast<uint64_t>(kPhiloxM1) * c2;
        const uint32_t hi0 = static_cast<uint32_t>(p0 >> 32), lo0 = static_cast<uint32_t>(p0);
        const uint32_t hi1 = static_cast<uint32_t>(p1 >> 32), lo1 = static_cast<uint32_t>(p1);
        c0 = hi1 ^ c1 ^ k0;
        c1 = lo1;
        c2 = hi0 ^ c3 ^ k1;
        c3 = lo0;
        k0 += kPhiloxW0;
        k1 += kPhiloxW1;
    }
}

// u = (U >> 8) 2^-24 < p  <=>  (U >> 8) < ceil(p 2^24) for p in [0, 1]
// (p 2^24 is exact in FP32); p <= 0 or NaN never samples, p >= 1 always does.
__device__ __forceinline__ uint32_t bern_threshold(float p) {
    if (!(p > 0.f)) return 0u;
    if (p >= 1.f) return 1u << 24;
    return static_cast<uint32_t>(ceilf(p * 16777216.0f));
}

// Lane v's 64-bit value as a wave-uniform one.
__device__ __forceinline__ int64_t readlane64(int64_t x, int v) {
    const uint32_t lo = __builtin_amdgcn_readlane(static_cast<int>(static_cast<uint64_t>(x)), v);
    const uint32_t hi = __builtin_amdgcn_readlane(static_cast<int>(static_cast<uint64_t>(x) >> 32), v);
    return static_cast<int64_t>((static_cast<uint64_t>(hi) << 32) | lo);
}

// A workgroup samples one tile of variables, 64 variables (a sub-tile) at a
// time.  Every wavefront loads the sub-tile's p and costs itself (lane =
// variable, one sub-tile ahead), so the variables' kinds are wave-uniform
// ballots: the candidate loop visits only the fractional variables, whose
// threshold and cost come from their lane.  The four wavefronts split the
// candidate groups (4 candidates per Philox call); a lane's 4 bits and its
// neighbour's form one byte of the variable's row in LDS.  Rows of
// deterministic variables are written as constants during the copy-out.  The
// LDS rows are double-buffered (one barrier per sub-tile) when two buffers fit.
template <typename ACC>
__global__ void __launch_bounds__(256)
k_sample(const float *__restrict__ p, const int64_t *__restrict__ cost,
         uint64_t *__restrict__ X, int W, const int *__restrict__ tile_inst,
         const int *__restrict__ tile_q0, const int *__restrict__ tile_q1,
         const int64_t *__restrict__ inst_var0, const int64_t *__restrict__ inst_nvar,
         int64_t *__restrict__ zpart, int K, uint32_t key0, uint32_t key1,
         const DevCounters *__restrict__ ctr, int threshold_mode, uint8_t *__restrict__ xkind,
         uint64_t wdiv, int nbuf) {
    extern __shared__ uint64_t lds[];   // nbuf buffers of [64 variables][W words]
    const int tile = blockIdx.x;
    const int inst = tile_inst[tile];
    const int q0 = tile_q0[tile], q1 = tile_q1[tile];
    const int64_t v0 = inst_var0[inst];
    const int64_t nv = inst_nvar[inst];
    const uint32_t round = static_cast<uint32_t>(ctr->round);
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    // candidate groups (4 candidates each) of this wavefront: [gb, ge)
    const int G4 = K >> 2;
    const int per = G4 >> 2;            // K is a multiple of 64, so per is a multiple of 4
    const int gb = wave * per, ge = gb + per;
    constexpr int SMAX = 4;             // groups per lane: per <= 256 (K <= 4096)
    ACC zacc[SMAX][4];
#pragma unroll
    for (int t = 0; t < SMAX; ++t)
#pragma unroll
        for (int j = 0; j < 4; ++j) zacc[t][j] = 0;
    ACC zconst = 0;                     // variables sampled as all ones
    const size_t bufw = static_cast<size_t>(64) * W;

    float pn = 0.f;
    int64_t cn = 0;
    {
        const int64_t il = 4LL * q0 + lane;
        if (q0 < q1 && il < nv) { pn = p[v0 + il]; cn = cost[v0 + il]; }
    }
    int buf = 0;
    for (int sq = q0; sq < q1; sq += 16) {
        const int nq = min(16, q1 - sq);
        const int64_t il0 = 4LL * sq;
        const int nvars = static_cast<int>(min<int64_t>(4LL * nq, nv - il0));
        const float pv = pn;
        const int64_t cv = cn;
        {
            const int64_t il = il0 + 64 + lane;
            const bool nx = sq + 16 < q1 && il < nv;
            pn = nx ? p[v0 + il] : 0.f;
            cn = nx ? cost[v0 + il] : 0;
        }
        const bool in = lane < nvars;
        const uint32_t th = in ? bern_threshold(pv) : 0u;
        int d;                          // 0: fractional, 1: all zero, 2: all one
        if (threshold_mode) d = (0x800000u < th) ? 2 : 1;     // u = 1/2: [p > 1/2]
        else d = th == 0u ? 1 : (th == (1u << 24) ? 2 : 0);
        if (!in) d = 1;
        const uint64_t fmask = __ballot(d == 0);
        const uint64_t omask = __ballot(d == 2);
        if (wave == 0 && in) xkind[v0 + il0 + lane] = static_cast<uint8_t>(d);
        if (omask) {                                              // uniform
            // all-one variables add their cost to every candidate
            ACC t = d == 2 ? static_cast<ACC>(cv) : static_cast<ACC>(0);
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o, 64);
            zconst += t;
        }
        uint64_t *rows = lds + (nbuf == 2 ? buf : 0) * bufw;
        uint8_t *lrow = reinterpret_cast<uint8_t *>(rows);
        uint64_t fm = fmask;
        while (fm) {                                              // uniform
            const int v = __builtin_ctzll(fm);
            fm &= fm - 1;
            const uint32_t thv = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(th), v));
            const ACC c = static_cast<ACC>(readlane64(cv, v));
            const uint32_t il = static_cast<uint32_t>(il0 + v);
#pragma unroll
            for (int t = 0; t < SMAX; ++t) {
                const int g = gb + lane + 64 * t;
                if (64 * t >= per) break;                          // uniform
                uint32_t r0 = static_cast<uint32_t>(g), r1 = il, r2 = round, r3 = static_cast<uint32_t>(inst);
                philox10(r0, r1, r2, r3, key0, key1);
                const uint32_t b0 = (r0 >> 8) < thv, b1 = (r1 >> 8) < thv;
                const uint32_t b2 = (r2 >> 8) < thv, b3 = (r3 >> 8) < thv;
                if (b0) zacc[t][0] += c;
                if (b1) zacc[t][1] += c;
                if (b2) zacc[t][2] += c;
                if (b3) zacc[t][3] += c;
                const uint32_t nib = b0 | (b1 << 1) | (b2 << 2) | (b3 << 3);
                const uint32_t other = __shfl_xor(nib, 1, 64);
                if (g < ge && (g & 1) == 0)
                    lrow[static_cast<size_t>(v) * W * 8 + (g >> 1)] = static_cast<uint8_t>(nib | (other << 4));
            }
        }
        __syncthreads();
        const int total = nvars * W;
        uint64_t *dst = X + (v0 + il0) * W;
        for (int idx = threadIdx.x; idx < total; idx += blockDim.x) {
            const int v = static_cast<int>((static_cast<uint64_t>(idx) * wdiv) >> 32);   // idx / W
            const bool fr = (fmask >> v) & 1ull, one = (omask >> v) & 1ull;
            dst[idx] = fr ? rows[idx] : (one ? ~0ull : 0ull);
        }
        if (nbuf == 2) buf ^= 1;
        else __syncthreads();
    }
#pragma unroll
    for (int t = 0; t < SMAX; ++t) {
        const int g = gb + lane + 64 * t;
        if (64 * t >= per) break;
        if (g < ge) {
            int64_t *zp = zpart + static_cast<int64_t>(tile) * K + 4 * static_cast<int64_t>(g);
#pragma unroll
            for (int j = 0; j < 4; ++j) zp[j] = static_cast<int64_t>(zacc[t][j] + zconst);
        }
    }
}

// ---------------------------------------------------------------------------
// Customized sampling for the 3D assignment problem (Algorithm 4, Sec. 2.4.2).
// x_ijk at index (i n + j) n + k.  Uniforms: Philox4x32-10(key = seed,
// counter = (candidate l, step, round, kA3Tag)); Fisher-Yates step t (r-1 down
// to 1) swaps position t of the free j's with floor(u (t + 1)) (word 0) and of
// the free k's with word 1's; local step q draws triple a = floor(u n) from
// word 0 of step n + q; floor(u m) = ((U >> 8) m) >> 24 exactly.
constexpr uint32_t kA3Tag = 0xA5513D00u;

__device__ __forceinline__ uint32_t a3_key(float p) { return p > 0.f ? __float_as_uint(p) : 0u; }

__device__ __forceinline__ uint32_t a3_below(uint32_t U, uint32_t m) {
    return static_cast<uint32_t>((static_cast<uint64_t>(U >> 8) * m) >> 24);
}

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// One workgroup: the min(m, #{p > 0}) largest entries of p (descending, lower
// index first on ties) by a 4-digit radix select of the FP32 bit patterns
// (monotone for p > 0), an index-ordered compaction and a bitonic sort in
// LDS; then the greedy conflict-free partial assignment (largest first).
// part[i] / part[n + i] = j / k of i, or -1.
__global__ void __launch_bounds__(1024)
k_a3_partial(const float *__restrict__ p, int64_t N, int n, int m, int *__restrict__ part) {
    __shared__ uint32_t hist[256];
    __shared__ uint64_t sel[kA3MaxTop];
    __shared__ int J0[kA3MaxN], K0[kA3MaxN];
    __shared__ uint8_t uj[kA3MaxN], uk[kA3MaxN];
    __shared__ uint32_t s_prefix, s_rank, s_npos, s_ngt, s_eqbase;
    __shared__ uint32_t s_wcnt[16];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int nw = blockDim.x >> 6;
    if (tid == 0) { s_npos = 0; s_ngt = 0; s_eqbase = 0; s_prefix = 0; }
    for (int i = tid; i < n; i += blockDim.x) { J0[i] = -1; K0[i] = -1; uj[i] = 0; uk[i] = 0; }
    __syncthreads();
    uint32_t cnt = 0;
    for (int64_t v = tid; v < N; v += blockDim.x) cnt += p[v] > 0.f ? 1u : 0u;
    atomicAdd(&s_npos, cnt);
    __syncthreads();
    const uint32_t meff = min(static_cast<uint32_t>(m), s_npos);
    if (meff > 0) {
        if (tid == 0) s_rank = meff;
        for (int d = 3; d >= 0; --d) {
            for (int b = tid; b < 256; b += blockDim.x) hist[b] = 0;
            __syncthreads();
            const uint32_t pre = s_prefix;
            const int sh = 8 * d;
            const uint32_t himask = d == 3 ? 0u : (0xFFFFFFFFu << (sh + 8));
            for (int64_t v = tid; v < N; v += blockDim.x) {
                const uint32_t key = a3_key(p[v]);
                if (key != 0u && (key & himask) == (pre & himask)) atomicAdd(&hist[(key >> sh) & 255u], 1u);
            }
            __syncthreads();
            if (tid == 0) {
                uint32_t cum = 0;
                const uint32_t r = s_rank;
                int b = 255;
                for (; b > 0; --b) {
                    if (cum + hist[b] >= r) break;
                    cum += hist[b];
                }
                s_prefix = pre | (static_cast<uint32_t>(b) << sh);
                s_rank = r - cum;
            }
            __syncthreads();
        }
        const uint32_t T = s_prefix, need_eq = s_rank, ngt_total = meff - need_eq;
        for (int64_t base = 0; base < N; base += blockDim.x) {
            const int64_t v = base + tid;
            const uint32_t key = v < N ? a3_key(p[v]) : 0u;
            const bool gt = key > T;
            const bool eq = key != 0u && key == T;
            if (gt) {
                const uint32_t slot = atomicAdd(&s_ngt, 1u);
                if (slot < ngt_total) sel[slot] = (static_cast<uint64_t>(~key) << 32) | static_cast<uint64_t>(v);
            }
            const uint64_t bal = __ballot(eq);
            if (lane == 0) s_wcnt[wv] = static_cast<uint32_t>(__popcll(bal));
            __syncthreads();
            uint32_t off = s_eqbase;
            for (int w = 0; w < wv; ++w) off += s_wcnt[w];
            const uint32_t pos = off + static_cast<uint32_t>(__popcll(bal & ((1ull << lane) - 1ull)));
            if (eq && pos < need_eq) sel[ngt_total + pos] = (static_cast<uint64_t>(~key) << 32) | static_cast<uint64_t>(v);
            __syncthreads();
            if (tid == 0) {
                uint32_t tot = 0;
                for (int w = 0; w < nw; ++w) tot += s_wcnt[w];
                s_eqbase += tot;
            }
            __syncthreads();
        }
        int M2 = 1;
        while (M2 < static_cast<int>(meff)) M2 <<= 1;
        for (int i = static_cast<int>(meff) + tid; i < M2; i += blockDim.x) sel[i] = ~0ull;
        __syncthreads();
        for (int k = 2; k <= M2; k <<= 1)
            for (int j = k >> 1; j > 0; j >>= 1) {
                for (int i = tid; i < M2; i += blockDim.x) {
                    const int ixj = i ^ j;
                    if (ixj > i) {
                        const uint64_t a = sel[i], b = sel[ixj];
                        const bool asc = (i & k) == 0;
                        if ((a > b) == asc) {
                            sel[i] = b;
                            sel[ixj] = a;
                        }
                    }
                }
                __syncthreads();
            }
        if (tid == 0) {
            const int64_t nn = static_cast<int64_t>(n) * n;
            for (uint32_t t = 0; t < meff; ++t) {
                const int64_t v = static_cast<int64_t>(sel[t] & 0xFFFFFFFFull);
                const int i = static_cast<int>(v / nn), j = static_cast<int>((v / n) % n), k = static_cast<int>(v % n);
                if (J0[i] < 0 && !uj[j] && !uk[k]) {
                    J0[i] = j;
                    K0[i] = k;
                    uj[j] = 1;
                    uk[k] = 1;
                }
            }
        }
        __syncthreads();
    }
    for (int i = tid; i < n; i += blockDim.x) {
        part[i] = J0[i];
        part[n + i] = K0[i];
    }
}

// Zero the candidate block, the per-tile objective partials and the variable
// kinds (every variable's words are then read by the evaluation).
__global__ void k_a3_clear(uint64_t *__restrict__ X, int64_t nX, int64_t *__restrict__ zpart,
                           int64_t nz, uint8_t *__restrict__ xkind, int64_t nk) {
    const int64_t st = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t t = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; t < nX; t += st) X[t] = 0ull;
    for (int64_t t = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; t < nz; t += st) zpart[t] = 0;
    for (int64_t t = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; t < nk; t += st) xkind[t] = 0;
}

// One wavefront per candidate l: random completion of the partial assignment
// (Fisher-Yates on the free j's and k's, swap indices drawn in parallel, the
// swaps done in order by lane 0), L steps of pairwise interchange (lanes over
// the partner triple, lexicographic (change, 2 b + kind) minimum), then the
// objective into the sampler's partial of tile 0 and the candidate's bits.
__global__ void __launch_bounds__(256)
k_a3_cand(int n, int K, int L, uint32_t key0, uint32_t key1, const DevCounters *__restrict__ ctr,
          const int64_t *__restrict__ cost, const int *__restrict__ part, uint64_t *__restrict__ X,
          int W, int64_t *__restrict__ zpart) {
    extern __shared__ int16_t a3s[];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int l = blockIdx.x * (blockDim.x >> 6) + wv;
    if (l >= K) return;                       // no workgroup barrier below
    int16_t *J = a3s + static_cast<size_t>(wv) * 7 * kA3MaxN;
    int16_t *Kk = J + kA3MaxN, *Ui = Kk + kA3MaxN, *Fj = Ui + kA3MaxN, *Fk = Fj + kA3MaxN;
    int16_t *Aj = Fk + kA3MaxN, *Ak = Aj + kA3MaxN;
    __shared__ uint32_t bits_j[4][kA3MaxN / 32], bits_k[4][kA3MaxN / 32];
    const uint32_t round = static_cast<uint32_t>(ctr->round);
    for (int w = lane; w < kA3MaxN / 32; w += 64) {
        bits_j[wv][w] = 0u;
        bits_k[wv][w] = 0u;
    }
    wave_sync();
    for (int i = lane; i < n; i += 64) {
        const int j = part[i], k = part[n + i];
        J[i] = static_cast<int16_t>(j);
        Kk[i] = static_cast<int16_t>(k);
        if (j >= 0) {
            atomicOr(&bits_j[wv][j >> 5], 1u << (j & 31));
            atomicOr(&bits_k[wv][k >> 5], 1u << (k & 31));
        }
    }
    wave_sync();
    int r = 0, rj = 0, rk = 0;
    for (int base = 0; base < n; base += 64) {
        const int t = base + lane;
        const bool fi = t < n && J[t] < 0;
        const bool fj = t < n && !((bits_j[wv][t >> 5] >> (t & 31)) & 1u);
        const bool fk = t < n && !((bits_k[wv][t >> 5] >> (t & 31)) & 1u);
        const uint64_t below = (1ull << lane) - 1ull;
        const uint64_t bi = __ballot(fi), bj = __ballot(fj), bk = __ballot(fk);
        if (fi) Ui[r + __popcll(bi & below)] = static_cast<int16_t>(t);
        if (fj) Fj[rj + __popcll(bj & below)] = static_cast<int16_t>(t);
        if (fk) Fk[rk + __popcll(bk & below)] = static_cast<int16_t>(t);
        r += __popcll(bi);
        rj += __popcll(bj);
        rk += __popcll(bk);
    }
    for (int t = lane; t < r; t += 64) {
        if (t == 0) continue;
        uint32_t c0 = static_cast<uint32_t>(l), c1 = static_cast<uint32_t>(t), c2 = round, c3 = kA3Tag;
        philox10(c0, c1, c2, c3, key0, key1);
        Aj[t] = static_cast<int16_t>(a3_below(c0, static_cast<uint32_t>(t + 1)));
        Ak[t] = static_cast<int16_t>(a3_below(c1, static_cast<uint32_t>(t + 1)));
    }
    wave_sync();
    if (lane == 0) {
        for (int t = r - 1; t >= 1; --t) {
            const int a = Aj[t], b = Ak[t];
            const int16_t x = Fj[t];
            Fj[t] = Fj[a];
            Fj[a] = x;
            const int16_t y = Fk[t];
            Fk[t] = Fk[b];
            Fk[b] = y;
        }
    }
    wave_sync();
    for (int t = lane; t < r; t += 64) {
        J[Ui[t]] = Fj[t];
        Kk[Ui[t]] = Fk[t];
    }
    wave_sync();
    const int64_t nn = static_cast<int64_t>(n) * n;
    auto cst = [&](int i, int j, int k) -> int64_t { return cost[i * nn + static_cast<int64_t>(j) * n + k]; };
    if (n >= 2) {
        for (int q = 0; q < L; ++q) {
            uint32_t c0 = static_cast<uint32_t>(l), c1 = static_cast<uint32_t>(n + q), c2 = round, c3 = kA3Tag;
            philox10(c0, c1, c2, c3, key0, key1);
            const int a = static_cast<int>(a3_below(c0, static_cast<uint32_t>(n)));
            const int ja = J[a], ka = Kk[a];
            const int64_t ca = cst(a, ja, ka);
            int64_t bd = INT64_MAX;
            int bk = 0x7FFFFFFF;
            for (int b = lane; b < n; b += 64) {
                if (b == a) continue;
                const int jb = J[b], kb = Kk[b];
                const int64_t cur = ca + cst(b, jb, kb);
                const int64_t dj = cst(a, jb, ka) + cst(b, ja, kb) - cur;
                const int64_t dk = cst(a, ja, kb) + cst(b, jb, ka) - cur;
                if (dj < bd || (dj == bd && 2 * b < bk)) { bd = dj; bk = 2 * b; }
                if (dk < bd || (dk == bd && 2 * b + 1 < bk)) { bd = dk; bk = 2 * b + 1; }
            }
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) {
                const int64_t od = static_cast<int64_t>(
                    (static_cast<uint64_t>(static_cast<uint32_t>(__shfl_xor(static_cast<int>(static_cast<uint64_t>(bd) >> 32), o, 64))) << 32) |
                    static_cast<uint32_t>(__shfl_xor(static_cast<int>(static_cast<uint64_t>(bd)), o, 64)));
                const int ok = __shfl_xor(bk, o, 64);
                if (od < bd || (od == bd && ok < bk)) { bd = od; bk = ok; }
            }
            if (bd < 0 && lane == 0) {
                const int b = bk >> 1;
                if ((bk & 1) == 0) {
                    const int16_t x = J[a];
                    J[a] = J[b];
                    J[b] = x;
                } else {
                    const int16_t x = Kk[a];
                    Kk[a] = Kk[b];
                    Kk[b] = x;
                }
            }
            wave_sync();
        }
    }
    int64_t z = 0;
    for (int i = lane; i < n; i += 64) {
        const int64_t v = i * nn + static_cast<int64_t>(J[i]) * n + Kk[i];
        z += cost[v];
        atomicOr(reinterpret_cast<unsigned long long *>(X) + v * W + (l >> 6), 1ull << (l & 63));
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const int64_t oz = static_cast<int64_t>(
            (static_cast<uint64_t>(static_cast<uint32_t>(__shfl_xor(static_cast<int>(static_cast<uint64_t>(z) >> 32), o, 64))) << 32) |
            static_cast<uint32_t>(__shfl_xor(static_cast<int>(static_cast<uint64_t>(z)), o, 64)));
        z += oz;
    }
    if (lane == 0) zpart[l] = z;
}

void launch_a3(hipStream_t s, const float *p, int n, int m, int K, int L, uint32_t key0,
               uint32_t key1, const DevCounters *ctr, const int64_t *cost, int *part, uint64_t *X,
               int W, int64_t *zpart, int64_t nzpart, uint8_t *xkind) {
    const int64_t N = static_cast<int64_t>(n) * n * n;
    k_a3_partial<<<1, 1024, 0, s>>>(p, N, n, m, part);
    int64_t blocks = (N * W + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    k_a3_clear<<<static_cast<int>(blocks), 256, 0, s>>>(X, N * W, zpart, nzpart, xkind, N);
    const size_t lds = static_cast<size_t>(4) * 7 * kA3MaxN * sizeof(int16_t);
    k_a3_cand<<<(K + 3) / 4, 256, lds, s>>>(n, K, L, key0, key1, ctr, cost, part, X, W, zpart);
}

void launch_sample(hipStream_t s, int W, bool obj64, const float *p, const int64_t *cost,
                   uint64_t *X, const Tiles &st, const int64_t *inst_var0,
                   const int64_t *inst_nvar, int64_t *zpart, int K, uint32_t key0,
                   uint32_t key1, const DevCounters *ctr, int threshold_mode, uint8_t *xkind) {
    if (!st.count || W < 1 || W > 64) return;
    // idx / W = (idx * ceil(2^32 / W)) >> 32, exact for idx < 64 W <= 4096
    const uint64_t wdiv = ((1ull << 32) + static_cast<uint64_t>(W) - 1) / static_cast<uint64_t>(W);
    const size_t one = static_cast<size_t>(64) * W * sizeof(uint64_t);
    const int nbuf = 2 * one <= 32 * 1024 ? 2 : 1;
    const size_t lds = nbuf * one;
    if (obj64)
        k_sample<int64_t><<<st.count, 256, lds, s>>>(p, cost, X, W, st.inst, st.b0, st.b1, inst_var0, inst_nvar, zpart, K, key0, key1, ctr, threshold_mode, xkind, wdiv, nbuf);
    else
        k_sample<int32_t><<<st.count, 256, lds, s>>>(p, cost, X, W, st.inst, st.b0, st.b1, inst_var0, inst_nvar, zpart, K, key0, key1, ctr, threshold_mode, xkind, wdiv, nbuf);
}

// Monotone relaxation repair (Sec. 2.4).  Thread (row r, word w) walks the
// row's variables in (cost, index) order with a mask of the candidates that
// already hold a set variable in this row; a later set bit of such a candidate
// is cleared and its cost added to the candidate's LDS sum.  Each variable lies
// in one row, so every (variable, word) is read and written by one thread.
// The LDS sums are then taken off the sampler's partial objectives (one
// 64-bit atomic per candidate and workgroup; integer sums, order-free).
__global__ void __launch_bounds__(256)
k_mono_repair(int nrows, int W, int K, const int *__restrict__ rp, const int *__restrict__ var,
              const int64_t *__restrict__ cost, uint64_t *__restrict__ X,
              uint8_t *__restrict__ xkind, int64_t *__restrict__ zpart) {
    extern __shared__ unsigned long long dz[];   // [K]
    for (int l = threadIdx.x; l < K; l += blockDim.x) dz[l] = 0ull;
    __syncthreads();
    const int rpb = static_cast<int>(blockDim.x) / W;
    const int lr = static_cast<int>(threadIdx.x) / W, w = static_cast<int>(threadIdx.x) - lr * W;
    const int r = blockIdx.x * rpb + lr;
    if (lr < rpb && r < nrows) {
        uint64_t keep = 0;
        const int e0 = rp[r], e1 = rp[r + 1];
        for (int e = e0; e < e1; e += 4) {
            int iv[4];
            uint64_t bits[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) iv[u] = var[min(e + u, e1 - 1)];
#pragma unroll
            for (int u = 0; u < 4; ++u) bits[u] = X[static_cast<int64_t>(iv[u]) * W + w];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                if (e + u >= e1) break;
                const uint64_t clr = bits[u] & keep;
                keep |= bits[u];
                if (clr) {
                    X[static_cast<int64_t>(iv[u]) * W + w] = bits[u] & ~clr;
                    xkind[iv[u]] = 0;
                    const unsigned long long cu = static_cast<unsigned long long>(cost[iv[u]]);
                    uint64_t mk = clr;
                    while (mk) {
                        const int bt = __builtin_ctzll(mk);
                        mk &= mk - 1;
                        atomicAdd(&dz[64 * w + bt], cu);
                    }
                }
            }
        }
    }
    __syncthreads();
    for (int l = threadIdx.x; l < K; l += blockDim.x) {
        const unsigned long long d = dz[l];
        if (d) atomicAdd(reinterpret_cast<unsigned long long *>(zpart) + l, 0ull - d);
    }
}

void launch_mono_repair(hipStream_t s, int nrows, int W, int K, const int *rp, const int *var,
                        const int64_t *cost, uint64_t *X, uint8_t *xkind, int64_t *zpart) {
    if (nrows <= 0 || W < 1 || W > 64) return;
    const int rpb = 256 / W;
    const int blocks = (nrows + rpb - 1) / rpb;
    k_mono_repair<<<blocks, 256, static_cast<size_t>(K) * sizeof(unsigned long long), s>>>(
        nrows, W, K, rp, var, cost, X, xkind, zpart);
}

// Throughput of the uniform generator alone (the sampler's ALU roofline): each
// lane evaluates Philox4x32-10 `iters` times with the sampler's counter shape
// (one word per lane, three wave-uniform words) and folds the outputs into a
// word that is stored only if it hits a fixed value, so nothing is skipped.
__global__ void __launch_bounds__(256)
k_philox_peak(int iters, uint32_t key0, uint32_t key1, uint32_t *__restrict__ sink) {
    const uint32_t g = blockIdx.x * 256u + threadIdx.x;
    uint32_t acc = 0u;
    for (int it = 0; it < iters; ++it) {
        uint32_t r0 = g, r1 = static_cast<uint32_t>(it), r2 = key1 ^ 0x5bd1e995u, r3 = 0u;
        philox10(r0, r1, r2, r3, key0, key1);
        acc ^= (r0 ^ r1) ^ (r2 ^ r3);
    }
    if (acc == 0x9e3779b9u) sink[0] = g;
}

void launch_philox_peak(hipStream_t s, int blocks, int iters, uint32_t *sink) {
    if (blocks > 0 && iters > 0) k_philox_peak<<<blocks, 256, 0, s>>>(iters, 0x243f6a88u, 0x85a308d3u, sink);
}

// Streaming read of n 16-byte words (grid-stride, one load per lane and
// step, results folded so the loads are not dropped): the device's
// achievable read bandwidth for a given number of workgroups, a reference
// next to the published HBM peak.
__global__ void __launch_bounds__(256)
k_read_peak(const int4 *__restrict__ p, int64_t n, uint32_t *__restrict__ sink) {
    const int64_t st = static_cast<int64_t>(gridDim.x) * 256;
    uint32_t acc = 0u;
    for (int64_t i = blockIdx.x * 256LL + threadIdx.x; i < n; i += st) {
        const int4 q = p[i];
        acc ^= static_cast<uint32_t>(q.x ^ q.y ^ q.z ^ q.w);
    }
    if (acc == 0x9e3779b9u) sink[0] = acc;
}

void launch_read_peak(hipStream_t s, int blocks, const void *p, int64_t n16, uint32_t *sink) {
    if (blocks > 0 && n16 > 0) k_read_peak<<<blocks, 256, 0, s>>>(static_cast<const int4 *>(p), n16, sink);
}

// ---------------------------------------------------------------------------
// Rows whose violation is a bitwise function of the candidate words (64
// candidates per word):
//   covering     (sum x >= 1, coefficients 1):   violated = ~OR
//   at-most-one  (-sum x >= -1):                  violated = "two or more"
//   exactly-one  (sum x == 1, coefficients +-1):  violated = ~one | two
//   pair         (one or two entries, any integer coefficients, >= or =):
//                violated = the row's truth table over (x_p, x_q)
// where one / two are the running "at least one / at least two set" masks.
// A group of Wp (power of two >= W) lanes owns a row, lane w of the group word
// w.  Each lane keeps per-candidate violation counts bit-sliced in 8 planes
// (ripple-carry adds of 64-bit masks) and flushes them to LDS counters every
// 255 rows.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void flush_planes(uint64_t (&c)[8], int *cnt, int w) {
    for (int b = 0; b < 64; ++b) {
        int v = 0;
#pragma unroll
        for (int pl = 0; pl < 8; ++pl) v |= static_cast<int>((c[pl] >> b) & 1ull) << pl;
        if (v) atomicAdd(&cnt[64 * w + b], v);
    }
#pragma unroll
    for (int pl = 0; pl < 8; ++pl) c[pl] = 0;
}

// Word `sub` of variable c's candidates: variables the sampler found
// deterministic (p = 0 / p = 1: all candidates 0 / 1) are answered from the
// per-variable kind byte (an L2-resident n-byte array) instead of the 8n W-byte
// candidate block.
constexpr int kCoverBatch = 8;    // entries per load stage in the bitwise row evaluation (16 is slower)

__device__ __forceinline__ uint64_t cand_word(const uint64_t *__restrict__ X,
                                              const uint8_t *__restrict__ xkind, int c, int W,
                                              int sub) {
    const uint8_t k = xkind[c];
    if (k == 1) return 0ull;
    if (k == 2) return ~0ull;
    return X[static_cast<int64_t>(c) * W + sub];
}

template <int RU>
__global__ void __launch_bounds__(256)
k_eval_cover(const int *__restrict__ tile_ids, const int *__restrict__ tb0,
             const int *__restrict__ tb1, const int *__restrict__ rows,
             const uint8_t *__restrict__ rkind, const int *__restrict__ rp,
             const int *__restrict__ ci, const uint64_t *__restrict__ X,
             const uint8_t *__restrict__ xkind, int W, int lgWp, int *__restrict__ vpart, int K) {
    __shared__ int cnt[4096];
    const int tile = tile_ids[blockIdx.x];
    const int r0 = tb0[tile], r1 = tb1[tile];
    for (int l = threadIdx.x; l < K; l += blockDim.x) cnt[l] = 0;
    __syncthreads();
    const int sub = threadIdx.x & ((1 << lgWp) - 1);
    const int grp = threadIdx.x >> lgWp;
    const int ngrp = blockDim.x >> lgWp;
    uint64_t c[8];
#pragma unroll
    for (int pl = 0; pl < 8; ++pl) c[pl] = 0;
    int since = 0;
    // RU rows per group and pass: their row data, and the two words of pair
    // rows, are loaded together (a row's count does not depend on the order
    // in which rows are added).  Four pay on pair rows (two entries, a chain
    // of dependent loads each); on long covering rows they cost occupancy.
    for (int rb = r0 + grp; rb < r1; rb += RU * ngrp) {
        if (sub < W) {
            int j[RU], kd[RU], e0[RU], e1[RU];
#pragma unroll
            for (int u = 0; u < RU; ++u) j[u] = rb + u * ngrp < r1 ? rows[rb + u * ngrp] : -1;
#pragma unroll
            for (int u = 0; u < RU; ++u) {
                kd[u] = j[u] >= 0 ? rkind[j[u]] : 0;
                e0[u] = j[u] >= 0 ? rp[j[u]] : 0;
                e1[u] = j[u] >= 0 ? rp[j[u] + 1] : 0;
            }
            uint64_t P[RU], Q[RU];
            {
                int c0[RU], c1[RU];
                uint8_t k0[RU], k1[RU];
#pragma unroll
                for (int u = 0; u < RU; ++u) {
                    const bool pr = j[u] >= 0 && (kd[u] >> 4) == kEvalPair;
                    c0[u] = pr ? ci[e0[u]] : -1;
                    c1[u] = pr ? ci[e1[u] - 1] : -1;
                }
#pragma unroll
                for (int u = 0; u < RU; ++u) {
                    k0[u] = c0[u] >= 0 ? xkind[c0[u]] : 1;
                    k1[u] = c1[u] >= 0 ? xkind[c1[u]] : 1;
                }
#pragma unroll
                for (int u = 0; u < RU; ++u) {
                    P[u] = k0[u] == 0 ? X[static_cast<int64_t>(c0[u]) * W + sub] : (k0[u] == 2 ? ~0ull : 0ull);
                    Q[u] = k1[u] == 0 ? X[static_cast<int64_t>(c1[u]) * W + sub] : (k1[u] == 2 ? ~0ull : 0ull);
                }
            }
#pragma unroll
            for (int u = 0; u < RU; ++u) {
                if (j[u] < 0) break;
                const int kind = kd[u] >> 4;
                uint64_t viol;
                if (kind == kEvalPair) {
                    const int k = kd[u];
                    viol = ((k & 1) ? (~P[u] & ~Q[u]) : 0ull) | ((k & 2) ? (~P[u] & Q[u]) : 0ull) |
                           ((k & 4) ? (P[u] & ~Q[u]) : 0ull) | ((k & 8) ? (P[u] & Q[u]) : 0ull);
                } else {
                    // "at least one / at least two set" do not depend on the
                    // order of the entries: kCoverBatch at a time, their column
                    // indices, kind bytes and words each loaded together
                    uint64_t one = 0, two = 0;
                    int e = e0[u];
                    const int ee1 = e1[u];
                    for (; e + kCoverBatch <= ee1; e += kCoverBatch) {
                        int cc[kCoverBatch];
                        uint8_t kk[kCoverBatch];
                        uint64_t xx[kCoverBatch];
#pragma unroll
                        for (int v = 0; v < kCoverBatch; ++v) cc[v] = ci[e + v];
#pragma unroll
                        for (int v = 0; v < kCoverBatch; ++v) kk[v] = xkind[cc[v]];
#pragma unroll
                        for (int v = 0; v < kCoverBatch; ++v)
                            xx[v] = kk[v] == 0 ? X[static_cast<int64_t>(cc[v]) * W + sub] : (kk[v] == 2 ? ~0ull : 0ull);
#pragma unroll
                        for (int v = 0; v < kCoverBatch; ++v) {
                            two |= one & xx[v];
                            one |= xx[v];
                        }
                    }
                    for (; e < ee1; ++e) {
                        const uint64_t x = cand_word(X, xkind, ci[e], W, sub);
                        two |= one & x;
                        one |= x;
                    }
                    viol = kind == kEvalCover ? ~one : (kind == kEvalAtMostOne ? two : (~one | two));
                }
                uint64_t carry = viol;
#pragma unroll
                for (int pl = 0; pl < 8; ++pl) {
                    const uint64_t t = c[pl] & carry;
                    c[pl] ^= carry;
                    carry = t;
                }
                if (++since == 255) { flush_planes(c, cnt, sub); since = 0; }
            }
        }
    }
    if (sub < W && since) flush_planes(c, cnt, sub);
    __syncthreads();
    for (int l = threadIdx.x; l < K; l += blockDim.x)
        vpart[static_cast<int64_t>(tile) * K + l] = cnt[l];
}

void launch_eval_cover(hipStream_t s, int ntiles, const int *tile_ids, const Tiles &et,
                       const int *rows, const uint8_t *rkind, const int *rp, const int *ci,
                       const uint64_t *X, const uint8_t *xkind, int W, int *vpart, int K, bool pair_rows) {
    if (!ntiles) return;
    int lg = 0;
    while ((1 << lg) < W) ++lg;
    if (pair_rows)
        k_eval_cover<4><<<ntiles, 256, 0, s>>>(tile_ids, et.b0, et.b1, rows, rkind, rp, ci, X, xkind, W, lg, vpart, K);
    else
        k_eval_cover<1><<<ntiles, 256, 0, s>>>(tile_ids, et.b0, et.b1, rows, rkind, rp, ci, X, xkind, W, lg, vpart, K);
}

// ---------------------------------------------------------------------------
// General rows: lane = candidate.  For row j and word w the wavefront walks
// the row (column index, coefficient and candidate word are uniform across
// the wave, so they are scalar loads) and each lane adds a_ji when its bit is
// set.  Violation: sum < rhs on inequality rows, sum != rhs on equality rows.
// ---------------------------------------------------------------------------
template <typename ACC>
__global__ void __launch_bounds__(1024)
k_eval_general(const int *__restrict__ tile_ids, const int *__restrict__ tb0,
               const int *__restrict__ tb1, const int *__restrict__ rows,
               const int *__restrict__ rp, const int *__restrict__ ci,
               const int *__restrict__ val, const int64_t *__restrict__ rhs, int m1,
               const uint64_t *__restrict__ X, int W, int *__restrict__ vpart, int K) {
    const int tile = tile_ids[blockIdx.x];
    const int r0 = tb0[tile], r1 = tb1[tile];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int NW = blockDim.x >> 6;
    const int sh = lane & 31;
    const bool hi = lane >= 32;
    for (int w = wave; w < W; w += NW) {
        int cntv = 0;
        for (int rr = r0; rr < r1; ++rr) {
            const int j = rows[rr];
            ACC acc = 0;
            const int e1 = rp[j + 1];
            for (int e = rp[j]; e < e1; ++e) {
                const uint64_t word = X[static_cast<int64_t>(ci[e]) * W + w];
                const uint32_t half = hi ? static_cast<uint32_t>(word >> 32) : static_cast<uint32_t>(word);
                const int bit = static_cast<int>((half >> sh) & 1u);
                const int a = val ? val[e] : 1;
                acc += static_cast<ACC>(bit * a);
            }
            const int64_t b = rhs[j];
            const bool bad = (j < m1) ? (static_cast<int64_t>(acc) < b) : (static_cast<int64_t>(acc) != b);
            cntv += bad ? 1 : 0;
        }
        vpart[static_cast<int64_t>(tile) * K + 64 * w + lane] = cntv;
    }
}

// General rows, all words at once: a wavefront owns one row and all W words
// (lane = candidate 64w + lane, W accumulators per lane), so the row's column
// indices and coefficients are read once and a variable's W candidate words
// come in one wide uniform load.  Four wavefronts per workgroup share LDS
// counters for the tile.
template <int WW, typename ACC>
__global__ void __launch_bounds__(256)
k_eval_rows_allw(const int *__restrict__ tile_ids, const int *__restrict__ tb0,
                 const int *__restrict__ tb1, const int *__restrict__ rows,
                 const int *__restrict__ rp, const int *__restrict__ ci,
                 const int *__restrict__ val, const int64_t *__restrict__ rhs, int m1,
                 const uint64_t *__restrict__ X, int *__restrict__ vpart, int K) {
    __shared__ int cnt[64 * WW];
    const int tile = tile_ids[blockIdx.x];
    const int r0 = tb0[tile], r1 = tb1[tile];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int sh = lane & 31;
    const bool hi = lane >= 32;
    for (int l = threadIdx.x; l < 64 * WW; l += blockDim.x) cnt[l] = 0;
    __syncthreads();
    int vc[WW];
#pragma unroll
    for (int w = 0; w < WW; ++w) vc[w] = 0;
    for (int rr = r0 + wave; rr < r1; rr += 4) {
        const int j = rows[rr];
        ACC acc[WW];
#pragma unroll
        for (int w = 0; w < WW; ++w) acc[w] = 0;
        const int e1 = rp[j + 1];
        for (int e = rp[j]; e < e1; ++e) {
            const uint64_t *xr = X + static_cast<int64_t>(ci[e]) * WW;
            const int a = val ? val[e] : 1;
#pragma unroll
            for (int w = 0; w < WW; ++w) {
                const uint64_t word = xr[w];
                const uint32_t half = hi ? static_cast<uint32_t>(word >> 32) : static_cast<uint32_t>(word);
                acc[w] += static_cast<ACC>(static_cast<int>((half >> sh) & 1u) * a);
            }
        }
        const int64_t b = rhs[j];
#pragma unroll
        for (int w = 0; w < WW; ++w) {
            const bool bad = (j < m1) ? (static_cast<int64_t>(acc[w]) < b) : (static_cast<int64_t>(acc[w]) != b);
            vc[w] += bad ? 1 : 0;
        }
    }
#pragma unroll
    for (int w = 0; w < WW; ++w)
        if (vc[w]) atomicAdd(&cnt[64 * w + lane], vc[w]);
    __syncthreads();
    for (int l = threadIdx.x; l < K; l += blockDim.x)
        vpart[static_cast<int64_t>(tile) * K + l] = cnt[l];
}

// Long general rows (hundreds of entries and more): the workgroup's four
// wavefronts split each row's entries into four contiguous quarters, each
// wavefront adds its quarter for all W words (lane = candidate), and
// wavefront 0 adds the four partial sums (exact integers) and tests the row.
// A wavefront walks its quarter in blocks of B = 512 / W entries: the block's
// candidate words (a variable's W words contiguous, lane = (entry, word)) are
// fetched with vector loads into registers while the previous block is summed
// from the wavefront's LDS buffer, then stored to the other buffer as two
// planes, low and high 32-bit halves; lanes 0-31 read the low plane, lanes
// 32-63 the high one, four words per 16-byte read (two addresses per
// wavefront).  Bit (lane & 31) of the half times the coefficient (a scalar
// load) is added: one 24-bit multiply-add when every coefficient fits in 24
// signed bits and the sums in 32 (MAD24), else a select and an add.  The
// sampler writes every variable's words, constant rows included, so no kind
// lookup is needed.
template <int WW, typename ACC, bool MAD24>
__global__ void __launch_bounds__(256)
k_eval_rows_split(const int *__restrict__ tile_ids, const int *__restrict__ tb0,
                  const int *__restrict__ tb1, const int *__restrict__ rows,
                  const int *__restrict__ rp, const int *__restrict__ ci,
                  const int *__restrict__ val, const int64_t *__restrict__ rhs, int m1,
                  const uint64_t *__restrict__ X, int *__restrict__ vpart, int K) {
    constexpr int B = 512 / WW;                  // entries per block
    __shared__ ACC part[4][WW][64];
    __shared__ uint32_t stage[4][2][2][512];     // per wavefront: two blocks, low / high planes
    const int tile = tile_ids[blockIdx.x];
    const int r0 = tb0[tile], r1 = tb1[tile];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x >> 6));   // wave-uniform
    const unsigned sh = lane & 31;
    const int half = lane >> 5;                  // plane this lane reads
    const cptr<int> val_c = to_const(val), rows_c = to_const(rows), rp_c = to_const(rp);
    int vc[WW];
#pragma unroll
    for (int w = 0; w < WW; ++w) vc[w] = 0;
    for (int rr = r0; rr < r1; ++rr) {
        const int j = rows_c[rr];
        const int e0 = rp_c[j], len = rp_c[j + 1] - e0;
        const int q0 = e0 + static_cast<int>((static_cast<int64_t>(len) * wave) / 4);
        const int q1 = e0 + static_cast<int>((static_cast<int64_t>(len) * (wave + 1)) / 4);
        ACC acc[WW];
#pragma unroll
        for (int w = 0; w < WW; ++w) acc[w] = 0;
        uint64_t reg[8];
        // words of the block starting at entry blk: pair 64 t + lane is
        // (entry (64 t + lane) / WW, word (64 t + lane) % WW); entries past
        // q1 load a clamped (valid) index and are never read
        auto load_block = [&](int blk) {
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                const int idx = 64 * t + lane;
                const int e = min(blk + idx / WW, q1 - 1);
                reg[t] = X[static_cast<int64_t>(ci[e]) * WW + (idx % WW)];
            }
        };
        auto store_block = [&](int b) {
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                stage[wave][b][0][64 * t + lane] = static_cast<uint32_t>(reg[t]);
                stage[wave][b][1][64 * t + lane] = static_cast<uint32_t>(reg[t] >> 32);
            }
        };
        if (q0 < q1) {
            load_block(q0);
            store_block(0);
        }
        __builtin_amdgcn_wave_barrier();
        int cur = 0;
        for (int blk = q0; blk < q1; blk += B) {
            const int nxt = blk + B;
            if (nxt < q1) load_block(nxt);                       // in flight during the sum
            const uint32_t *pl = stage[wave][cur][half];
            const int ne = min(B, q1 - blk);
#pragma unroll 4
            for (int e = 0; e < ne; ++e) {
                const int a = val ? val_c[blk + e] : 1;
                uint32_t hw[WW];
                if constexpr (WW >= 4) {
#pragma unroll
                    for (int w = 0; w < WW; w += 4) {
                        const uint4 q4 = *reinterpret_cast<const uint4 *>(pl + e * WW + w);
                        hw[w] = q4.x; hw[w + 1] = q4.y; hw[w + 2] = q4.z; hw[w + 3] = q4.w;
                    }
                } else {
#pragma unroll
                    for (int w = 0; w < WW; ++w) hw[w] = pl[e * WW + w];
                }
#pragma unroll
                for (int w = 0; w < WW; ++w) {
                    if constexpr (MAD24) {
                        acc[w] += __mul24(a, static_cast<int>(__builtin_amdgcn_ubfe(hw[w], sh, 1u)));
                    } else {
                        // a select, not a mask: widening (a & sign-extended bit)
                        // to 64 bits was compiled as a zero extension
                        acc[w] += __builtin_amdgcn_ubfe(hw[w], sh, 1u) ? static_cast<ACC>(a) : ACC(0);
                    }
                }
            }
            __builtin_amdgcn_wave_barrier();
            if (nxt < q1) store_block(cur ^ 1);
            __builtin_amdgcn_wave_barrier();
            cur ^= 1;
        }
#pragma unroll
        for (int w = 0; w < WW; ++w) part[wave][w][lane] = acc[w];
        __syncthreads();
        if (wave == 0) {
            const int64_t b = rhs[j];
#pragma unroll
            for (int w = 0; w < WW; ++w) {
                const int64_t sum = static_cast<int64_t>(part[0][w][lane]) + part[1][w][lane] +
                                    part[2][w][lane] + part[3][w][lane];
                vc[w] += ((j < m1) ? (sum < b) : (sum != b)) ? 1 : 0;
            }
        }
        __syncthreads();
    }
    if (wave == 0) {
#pragma unroll
        for (int w = 0; w < WW; ++w)
            if (64 * w + lane < K) vpart[static_cast<int64_t>(tile) * K + 64 * w + lane] = vc[w];
    }
}

// Dense blocks of general rows on the int8 matrix cores.  A tile holds up to
// 32 rows of one instance whose entries fill at least half of the block
// rows x [c0, c0 + span); its coefficients are stored once, densified, as
// NPL planes of signed base-256 digits (a = sum_p d_p 256^p, d_p in
// [-128, 127]) in int8, plane-major then row-major with the span padded to
// a multiple of 32.  Then row sums over the candidates of one word are the
// product  C_p = D_p (R x span) . Xbits (span x 64)  with exact int32
// accumulation (|C_p| <= 128 span < 2^31), combined as sum_p C_p 256^p in
// int64: the same integers as the entry-by-entry sums.
// A workgroup takes one tile and one candidate word; its four wavefronts
// split the span into quarters of 32-variable k-steps.  Per k-step a lane
// (row i = lane & 31, k-half g = lane >> 5) loads 16 digits of each plane
// (one 16-byte load) as the A operand of v_mfma_i32_32x32x32_i8, and builds
// the B operands of the word's two 32-candidate halves from the candidate
// bits of the same 16 variables (the k-step's 32 words staged per wavefront
// in LDS, fetched one k-step ahead with the digits): byte b of the lane is
// bit (32 t + (lane & 31)) of variable 16 g + b.  A and B use the same (g, byte) -> variable map, so the
// contraction does not depend on how the instruction orders k.  The four
// partial products are added in LDS and wavefront 0 tests each row for each
// candidate.  Workgroups of one tile share an XCD (blockIdx % 8) so that the
// tile's digits are read from HBM once per word group, then from L2.
typedef int gf_v4i __attribute__((ext_vector_type(4)));
typedef int gf_v16i __attribute__((ext_vector_type(16)));

__device__ __forceinline__ int gf_bytes_of_bits(uint32_t h0, uint32_t h1, uint32_t h2, uint32_t h3,
                                                unsigned sh) {
    return static_cast<int>(__builtin_amdgcn_ubfe(h0, sh, 1u) | (__builtin_amdgcn_ubfe(h1, sh, 1u) << 8) |
                            (__builtin_amdgcn_ubfe(h2, sh, 1u) << 16) | (__builtin_amdgcn_ubfe(h3, sh, 1u) << 24));
}

template <int NPL, bool W64>
__global__ void __launch_bounds__(256)
k_eval_mfma(int ntiles, int W, const int *__restrict__ tile_ids, const int *__restrict__ tb0,
            const int *__restrict__ tb1, const int *__restrict__ rows,
            const int64_t *__restrict__ mf_off, const int *__restrict__ mf_c0,
            const int *__restrict__ mf_span, const int8_t *__restrict__ dig,
            const int64_t *__restrict__ rhs, int m1, const uint64_t *__restrict__ X,
            int *__restrict__ vpart, int K) {
    __shared__ uint64_t xs[4][128];
    // row sums of the four wavefronts: 64-bit, or 32-bit when every row's sum
    // of |a| is below 2^31 (then every partial sum and the plane combination
    // taken modulo 2^32 are the exact values)
    using RT = typename std::conditional<W64, unsigned long long, unsigned>::type;
    __shared__ RT red[2][16][64];
    const int b = blockIdx.x;
    const int r = b >> 3;
    const int w = r % W;
    const int ti = (r / W) * 8 + (b & 7);
    if (ti >= ntiles) return;                      // whole workgroup, before any barrier
    for (int q = threadIdx.x; q < 2 * 16 * 64; q += 256) (&red[0][0][0])[q] = 0;
    const int tile = tile_ids[ti];
    const int r0 = tb0[tile], R = tb1[tile] - r0;
    const int c0 = mf_c0[tile], span = mf_span[tile];
    const int nk = (span + 31) >> 5;               // k-steps; digits padded to 32 nk per row
    const int8_t *dt = dig + mf_off[tile];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x >> 6));
    const int i = lane & 31, g = lane >> 5;
    const unsigned sh = static_cast<unsigned>(i);
    const int k0 = (nk * wave) >> 2, k1 = (nk * (wave + 1)) >> 2;
    const int64_t pitch = static_cast<int64_t>(nk) * 32;
    gf_v16i acc[2][NPL];
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int p = 0; p < NPL; ++p) acc[t][p] = gf_v16i{};
    const int8_t *arow = dt + static_cast<int64_t>(i) * pitch + 16 * g;
    const bool live = i < R;
    // operands of the next KS k-steps are fetched while the current KS are
    // multiplied: the candidate words of their 32 KS variables (clamped to
    // the span's last variable, whose digits there are zero) and the digit
    // fragments
    constexpr int KS = 4;
    uint64_t xn[KS / 2];
    gf_v4i an[KS][NPL];
    auto fetch = [&](int kk) {
#pragma unroll
        for (int h = 0; h < KS / 2; ++h) {
            const int v = min(c0 + 32 * kk + 64 * h + lane, c0 + span - 1);
            xn[h] = X[static_cast<int64_t>(v) * W + w];
        }
#pragma unroll
        for (int s2 = 0; s2 < KS; ++s2)
#pragma unroll
            for (int p = 0; p < NPL; ++p)
                an[s2][p] = (live && kk + s2 < k1)
                                ? *reinterpret_cast<const gf_v4i *>(arow + p * R * pitch + 32 * (kk + s2))
                                : gf_v4i{};
    };
    if (k0 < k1) fetch(k0);
    for (int ks = k0; ks < k1; ks += KS) {
#pragma unroll
        for (int h = 0; h < KS / 2; ++h) xs[wave][64 * h + lane] = xn[h];
        gf_v4i a[KS][NPL];
#pragma unroll
        for (int s2 = 0; s2 < KS; ++s2)
#pragma unroll
            for (int p = 0; p < NPL; ++p) a[s2][p] = an[s2][p];
        if (ks + KS < k1) fetch(ks + KS);
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int s2 = 0; s2 < KS; ++s2) {
            if (ks + s2 < k1) {
                const uint64_t *xv = &xs[wave][32 * s2 + 16 * g];
                gf_v4i bl, bh;
#pragma unroll
                for (int d = 0; d < 4; ++d) {
                    const uint64_t x0 = xv[4 * d], x1 = xv[4 * d + 1], x2 = xv[4 * d + 2], x3 = xv[4 * d + 3];
                    bl[d] = gf_bytes_of_bits(static_cast<uint32_t>(x0), static_cast<uint32_t>(x1),
                                             static_cast<uint32_t>(x2), static_cast<uint32_t>(x3), sh);
                    bh[d] = gf_bytes_of_bits(static_cast<uint32_t>(x0 >> 32), static_cast<uint32_t>(x1 >> 32),
                                             static_cast<uint32_t>(x2 >> 32), static_cast<uint32_t>(x3 >> 32), sh);
                }
#pragma unroll
                for (int p = 0; p < NPL; ++p) {
                    acc[0][p] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a[s2][p], bl, acc[0][p], 0, 0, 0);
                    acc[1][p] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a[s2][p], bh, acc[1][p], 0, 0, 0);
                }
            }
        }
        __builtin_amdgcn_wave_barrier();
    }
    // row sums: register q of half t holds row 8 (q / 4) + 4 g + (q % 4),
    // candidate 64 w + 32 t + (lane & 31); the wavefronts' exact integer
    // partial sums meet in LDS (two's-complement adds, order-free)
    __syncthreads();                               // zeroed buffer visible to every wavefront
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            RT sum = 0;
#pragma unroll
            for (int p = 0; p < NPL; ++p) sum += static_cast<RT>(static_cast<int64_t>(acc[t][p][q])) << (8 * p);
            atomicAdd(&red[t][q][lane], sum);
        }
    __syncthreads();
    if (wave == 0) {
        int cnt[2] = {0, 0};
#pragma unroll
        for (int t = 0; t < 2; ++t)
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                const int row = 8 * (q >> 2) + 4 * g + (q & 3);
                if (row < R) {
                    const int64_t sum = W64 ? static_cast<int64_t>(red[t][q][lane])
                                            : static_cast<int64_t>(static_cast<int32_t>(red[t][q][lane]));
                    const int j = rows[r0 + row];
                    const int64_t bj = rhs[j];
                    cnt[t] += ((j < m1) ? (sum < bj) : (sum != bj)) ? 1 : 0;
                }
            }
        cnt[0] += __shfl_xor(cnt[0], 32);
        cnt[1] += __shfl_xor(cnt[1], 32);
        vpart[static_cast<int64_t>(tile) * K + 64 * w + 32 * g + i] = g ? cnt[1] : cnt[0];
    }
}

void launch_eval_mfma(hipStream_t s, int ntiles, const int *tile_ids, const Tiles &et, int npl, bool acc64,
                      const int *rows, const int64_t *mf_off, const int *mf_c0, const int *mf_span,
                      const int8_t *dig, const int64_t *rhs, int m1, const uint64_t *X, int W,
                      int *vpart, int K) {
    if (!ntiles) return;
    const int64_t blocks = static_cast<int64_t>((ntiles + 7) / 8) * 8 * W;
#define GF_MF(N, B) k_eval_mfma<N, B><<<static_cast<int>(blocks), 256, 0, s>>>(ntiles, W, tile_ids, et.b0, et.b1, rows, mf_off, mf_c0, mf_span, dig, rhs, m1, X, vpart, K)
    if (acc64) {
        if (npl == 1) GF_MF(1, true);
        else if (npl == 2) GF_MF(2, true);
        else GF_MF(3, true);
    } else {
        if (npl == 1) GF_MF(1, false);
        else if (npl == 2) GF_MF(2, false);
        else GF_MF(3, false);
    }
#undef GF_MF
}

void launch_eval_general(hipStream_t s, int ntiles, const int *tile_ids, const Tiles &et,
                         bool acc64, const int *rows, const int *rp, const int *ci,
                         const int *val, const int64_t *rhs, int m1, const uint64_t *X,
                         const uint8_t *xkind, int W, int *vpart, int K, bool long_rows,
                         bool coef24) {
    if (!ntiles) return;
    if (long_rows && W <= 16 && (W & (W - 1)) == 0) {
#define GF_RS(WW, ACCT, M) k_eval_rows_split<WW, ACCT, M><<<ntiles, 256, 0, s>>>(tile_ids, et.b0, et.b1, rows, rp, ci, val, rhs, m1, X, vpart, K)
#define GF_RSW(ACCT, M) switch (W) { case 1: GF_RS(1, ACCT, M); break; case 2: GF_RS(2, ACCT, M); break; \
        case 4: GF_RS(4, ACCT, M); break; case 8: GF_RS(8, ACCT, M); break; default: GF_RS(16, ACCT, M); break; }
        if (acc64) { GF_RSW(int64_t, false) } else if (coef24) { GF_RSW(int32_t, true) } else { GF_RSW(int32_t, false) }
#undef GF_RSW
#undef GF_RS
        return;
    }
    if (W <= 16 && (W & (W - 1)) == 0) {
#define GF_RA(WW, ACCT) k_eval_rows_allw<WW, ACCT><<<ntiles, 256, 0, s>>>(tile_ids, et.b0, et.b1, rows, rp, ci, val, rhs, m1, X, vpart, K)
#define GF_RAW(ACCT) switch (W) { case 1: GF_RA(1, ACCT); break; case 2: GF_RA(2, ACCT); break; \
        case 4: GF_RA(4, ACCT); break; case 8: GF_RA(8, ACCT); break; default: GF_RA(16, ACCT); break; }
        if (acc64) { GF_RAW(int64_t) } else { GF_RAW(int32_t) }
#undef GF_RAW
#undef GF_RA
        return;
    }
    const int NW = W <= 16 ? W : 16;
    if (acc64)
        k_eval_general<int64_t><<<ntiles, NW * 64, 0, s>>>(tile_ids, et.b0, et.b1, rows, rp, ci, val, rhs, m1, X, W, vpart, K);
    else
        k_eval_general<int32_t><<<ntiles, NW * 64, 0, s>>>(tile_ids, et.b0, et.b1, rows, rp, ci, val, rhs, m1, X, W, vpart, K);
}

// ---------------------------------------------------------------------------
// Quadratic objective <x, Q x> per candidate, lane = candidate:
//   sum over the entries (i, k) of a tile's rows of Q_ik [x_i and x_k].
// Four wavefronts per tile, each taking every fourth candidate word.  For a
// word, a wavefront stages, per entry of the tile (up to kQuadStage at a
// time; lane = entry), the AND of the words of x_i and x_k (the entry's row i
// from rowQ) as low / high 32-bit planes plus Q_ik into LDS, then sums the
// staged entries in one flat loop: bit (lane & 31) of the lane's half times
// Q_ik, read as wave-uniform LDS broadcasts (one 24-bit multiply-add into an
// int32 when every entry is below 2^21 in magnitude, so that a staged block's
// sum cannot overflow, else a 64-bit select and an add).  For a symmetric Q
// the entries are those of the upper triangle, off-diagonal ones doubled.
// ---------------------------------------------------------------------------
constexpr int kQuadStage = 1024;

template <bool MAD24>
__global__ void __launch_bounds__(256)
k_eval_quad(const int *__restrict__ tb0, const int *__restrict__ tb1,
            const int *__restrict__ rpQ, const int *__restrict__ rowQ, const int *__restrict__ ciQ,
            const int *__restrict__ valQ, const uint64_t *__restrict__ X, int W,
            int64_t *__restrict__ zq, int K) {
    __shared__ uint32_t stage[4][3][kQuadStage];   // low / high halves of x_i & x_k, Q values
    const int tile = blockIdx.x;
    const int i0 = tb0[tile], i1 = tb1[tile];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x >> 6));   // wave-uniform
    const unsigned sh = lane & 31;
    const int half = lane >> 5;
    const cptr<int> rpQ_c = to_const(rpQ);
    const int E0 = rpQ_c[i0], E1 = rpQ_c[i1];
    const uint32_t *pl = stage[wave][half];
    const int *qv = reinterpret_cast<const int *>(stage[wave][2]);
    for (int w = wave; w < W; w += 4) {
        int64_t z = 0;
        for (int cb = E0; cb < E1; cb += kQuadStage) {
            const int ce = min(E1, cb + kQuadStage);
            __builtin_amdgcn_wave_barrier();
#pragma unroll 4
            for (int t = 0; t < kQuadStage / 64; ++t) {
                const int e = cb + 64 * t + lane;
                if (e < ce) {
                    const uint64_t xw = X[static_cast<int64_t>(ciQ[e]) * W + w] &
                                        X[static_cast<int64_t>(rowQ[e]) * W + w];
                    stage[wave][0][e - cb] = static_cast<uint32_t>(xw);
                    stage[wave][1][e - cb] = static_cast<uint32_t>(xw >> 32);
                    stage[wave][2][e - cb] = static_cast<uint32_t>(valQ[e]);
                }
            }
            __builtin_amdgcn_wave_barrier();
            const int ne = ce - cb;
            if (MAD24) {
                int acc = 0;
#pragma unroll 8
                for (int e = 0; e < ne; ++e)
                    acc += __mul24(qv[e], static_cast<int>(__builtin_amdgcn_ubfe(pl[e], sh, 1u)));
                z += acc;
            } else {
                int64_t acc = 0;
#pragma unroll 8
                for (int e = 0; e < ne; ++e)
                    acc += __builtin_amdgcn_ubfe(pl[e], sh, 1u) ? static_cast<int64_t>(qv[e]) : int64_t(0);
                z += acc;
            }
        }
        zq[static_cast<int64_t>(tile) * K + 64 * w + lane] = z;
    }
}

void launch_eval_quad(hipStream_t s, const Tiles &qt, const int *rpQ, const int *rowQ,
                      const int *ciQ, const int *valQ, const uint64_t *X, int W, int64_t *zqpart,
                      int K, bool q24) {
    if (!qt.count) return;
    if (q24) k_eval_quad<true><<<qt.count, 256, 0, s>>>(qt.b0, qt.b1, rpQ, rowQ, ciQ, valQ, X, W, zqpart, K);
    else k_eval_quad<false><<<qt.count, 256, 0, s>>>(qt.b0, qt.b1, rpQ, rowQ, ciQ, valQ, X, W, zqpart, K);
}

// ---------------------------------------------------------------------------
// Per (instance, candidate): viol = sum of the instance's violation partials,
// z = linear partials (+ quadratic partials).  Two stages with a fixed
// summation order: stage 1 splits each instance's tile range into S slices
// (grid T x K/256 x S), stage 2 adds the S slice sums.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void slice_range(const int *first, int inst, int sl, int S, int &a, int &b) {
    const int t0 = first[inst], t1 = first[inst + 1];
    const int len = (t1 - t0 + S - 1) / S;
    a = min(t1, t0 + sl * len);
    b = min(t1, a + len);
}

__global__ void __launch_bounds__(256)
k_reduce_cand1(int K, int S, const int *__restrict__ efirst, const int *__restrict__ vpart,
               const int *__restrict__ sfirst, const int64_t *__restrict__ zpart,
               const int *__restrict__ qfirst, const int64_t *__restrict__ zqpart, int has_q,
               int32_t *__restrict__ rv, int64_t *__restrict__ rz) {
    const int inst = blockIdx.x;
    const int l = blockIdx.y * 256 + threadIdx.x;
    const int sl = blockIdx.z;
    if (l >= K) return;
    int v = 0;
    int64_t zz = 0;
    int a, b;
    slice_range(efirst, inst, sl, S, a, b);
    for (int t = a; t < b; ++t) v += vpart[static_cast<int64_t>(t) * K + l];
    slice_range(sfirst, inst, sl, S, a, b);
    for (int t = a; t < b; ++t) zz += zpart[static_cast<int64_t>(t) * K + l];
    if (has_q) {
        slice_range(qfirst, inst, sl, S, a, b);
        for (int t = a; t < b; ++t) zz += zqpart[static_cast<int64_t>(t) * K + l];
    }
    const int64_t o = (static_cast<int64_t>(inst) * S + sl) * K + l;
    rv[o] = v;
    rz[o] = zz;
}

__global__ void __launch_bounds__(256)
k_reduce_cand2(int K, int S, const int32_t *__restrict__ rv, const int64_t *__restrict__ rz,
               int32_t *__restrict__ viol, int64_t *__restrict__ z) {
    const int inst = blockIdx.x;
    const int l = blockIdx.y * 256 + threadIdx.x;
    if (l >= K) return;
    int v = 0;
    int64_t zz = 0;
    for (int sl = 0; sl < S; ++sl) {
        const int64_t o = (static_cast<int64_t>(inst) * S + sl) * K + l;
        v += rv[o];
        zz += rz[o];
    }
    viol[static_cast<int64_t>(inst) * K + l] = v;
    z[static_cast<int64_t>(inst) * K + l] = zz;
}

void launch_reduce_cand(hipStream_t s, int T, int K, int S, const Tiles &et, const int *vpart,
                        const Tiles &st, const int64_t *zpart, const Tiles &qt,
                        const int64_t *zqpart, int has_q, int32_t *rv, int64_t *rz,
                        int32_t *viol, int64_t *z) {
    dim3 g1(T, (K + 255) / 256, S);
    k_reduce_cand1<<<g1, 256, 0, s>>>(K, S, et.first, vpart, st.first, zpart,
                                       has_q ? qt.first : st.first, zqpart, has_q, rv, rz);
    dim3 g2(T, (K + 255) / 256);
    k_reduce_cand2<<<g2, 256, 0, s>>>(K, S, rv, rz, viol, z);
}

// ---------------------------------------------------------------------------
// EvalBest: l* = lowest index attaining min{z_l : viol_l = 0}; replace the
// incumbent on strict improvement.  With advance != 0 the trigger counter n
// grows and rho follows UpdatePenalty (Sec. 3):
//   rho_n = min(max(rho_min (1 + n/T)^p, rho_{n-1} + delta), rho_max).
// advance: 0 = final rounding (no round consumed), 1 = sampling trigger (round
// consumed, rho advances), 2 = extra round within a trigger (round consumed,
// rho unchanged).  One block per instance.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256)
k_argmin_update(int K, int W, const int32_t *__restrict__ viol, const int64_t *__restrict__ z,
                DevInst di, DevCounters *__restrict__ ctr, int advance) {
    __shared__ int64_t bz[256];
    __shared__ int bl[256];
    const int inst = blockIdx.x;
    int64_t best = INT64_MAX;
    int bi = 0x7fffffff;
    for (int l = threadIdx.x; l < K; l += 256) {
        const int64_t zl = z[static_cast<int64_t>(inst) * K + l];
        if (viol[static_cast<int64_t>(inst) * K + l] == 0 && (zl < best || (zl == best && l < bi))) {
            best = zl;
            bi = l;
        }
    }
    bz[threadIdx.x] = best;
    bl[threadIdx.x] = bi;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (static_cast<int>(threadIdx.x) < o) {
            const int64_t z2 = bz[threadIdx.x + o];
            const int l2 = bl[threadIdx.x + o];
            if (z2 < bz[threadIdx.x] || (z2 == bz[threadIdx.x] && l2 < bl[threadIdx.x])) {
                bz[threadIdx.x] = z2;
                bl[threadIdx.x] = l2;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const int64_t round = ctr->round;
        int imp = 0;
        if (bl[0] != 0x7fffffff && bz[0] < di.zbest[inst]) {
            di.zbest[inst] = bz[0];
            di.inc_l[inst] = bl[0];
            di.inc_round[inst] = advance ? round : -1;
            di.inc_k[inst] = ctr->k;
            di.inc_W[inst] = W;
            imp = 1;
        }
        di.improved[inst] = imp;
        if (advance) {
            if (round < di.hist_cap) di.hist[static_cast<int64_t>(inst) * di.hist_cap + round] = di.zbest[inst];
        }
        if (advance == 1) {   // a sampling trigger: UpdatePenalty
            const int64_t nn = di.ntrig[inst] + 1;
            di.ntrig[inst] = nn;
            const double rt = di.rho_min[inst] * pow(1.0 + static_cast<double>(nn) / di.rho_T[inst], di.rho_p[inst]);
            const double prev = di.rho[inst];
            di.rho[inst] = fmin(fmax(rt, prev + di.rho_delta[inst]), di.rho_max[inst]);
        }
    }
}

__global__ void k_round_bump(DevCounters *ctr) { ctr->round += 1; }

void launch_argmin_update(hipStream_t s, int T, int K, int W, const int32_t *viol,
                          const int64_t *z, DevInst di, DevCounters *ctr, int advance) {
    k_argmin_update<<<T, 256, 0, s>>>(K, W, viol, z, di, ctr, advance);
    if (advance) k_round_bump<<<1, 1, 0, s>>>(ctr);
}

// x_best of every instance whose incumbent just improved: byte per variable.
__global__ void __launch_bounds__(256)
k_extract_best(int64_t n, int T, const int *__restrict__ var_inst, const uint64_t *__restrict__ X,
               DevInst di, uint8_t *__restrict__ xbest) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int t = T > 1 ? var_inst[i] : 0;
        if (!di.improved[t]) continue;
        const int l = static_cast<int>(di.inc_l[t]);
        const int W = di.inc_W[t];
        const uint64_t word = X[i * W + (l >> 6)];
        xbest[i] = static_cast<uint8_t>((word >> (l & 63)) & 1ull);
    }
}

void launch_extract_best(hipStream_t s, int64_t n, int T, const int *var_inst, const uint64_t *X, DevInst di,
                         uint8_t *xbest) {
    int64_t b = (n + 255) / 256;
    if (b > 8192) b = 8192;
    if (b < 1) b = 1;
    k_extract_best<<<static_cast<int>(b), 256, 0, s>>>(n, T, var_inst, X, di, xbest);
}

}  // namespace gfors
