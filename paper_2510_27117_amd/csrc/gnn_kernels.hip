// Learned sampling proposal: a bipartite message-passing network over the
// constraint graph (variables <-> rows), trained and run on the GPU.  Dense
// 64-wide layers run on MFMA (v_mfma_f32_16x16x16_bf16: BF16 operands, FP32
// accumulation); messages are sparse-times-dense products gathering each
// neighbour's 64 features (one 128-byte line in BF16), with nodes split into
// heavy / medium / short classes by degree.  Network, features and loss are
// defined in gnn.h.
#include "gnn.h"

#include <algorithm>

namespace gfors {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float(static_cast<uint32_t>(b) << 16); }
__device__ __forceinline__ uint16_t f2bf(float f) {
    const uint32_t u = __float_as_uint(f);
    const uint32_t r = u + 0x7FFFu + ((u >> 16) & 1u);   // round to nearest even
    return static_cast<uint16_t>(r >> 16);
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// ------------------------------------------------------------------ features
// Hv0 = relu(Fv Uv + uv), Fv_i = [x_i, 4 x_i (1 - x_i), ct_i / ctmax, 1]
// Hc0 = relu(Fc Uc + uc), Fc_j = [y_j / (1 + |y_j|), rt_j / rtmax, [j >= m1], 1]
// 16 lanes per node (four hidden units each), four nodes per wavefront.
__global__ void __launch_bounds__(256)
k_gnn_embed(int64_t n, int64_t m, int m1, const float *__restrict__ x, const float *__restrict__ y,
            const float *__restrict__ ct, const float *__restrict__ rt, float ictmax, float irtmax,
            const float *__restrict__ theta, uint16_t *__restrict__ Hv, uint16_t *__restrict__ Hc) {
    // 16 lanes per node, lane f = hidden units 4f..4f+3 (one 8-byte store)
    const int f = threadIdx.x & 15;
    float Wv[4][4], Wc[4][4], bv[4], bc[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        bv[t] = theta[kGnnOffuv + 4 * f + t] + theta[kGnnOffUv + 3 * kGnnH + 4 * f + t];
        bc[t] = theta[kGnnOffuc + 4 * f + t] + theta[kGnnOffUc + 3 * kGnnH + 4 * f + t];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            Wv[k][t] = theta[kGnnOffUv + k * kGnnH + 4 * f + t];
            Wc[k][t] = theta[kGnnOffUc + k * kGnnH + 4 * f + t];
        }
    }
    // four nodes per 16-lane group and pass: their inputs are loaded together,
    // so a wavefront keeps 8-12 loads in flight instead of 2-3
    constexpr int NPG = 4;
    const int64_t N = n + m;
    const int64_t ng = (static_cast<int64_t>(gridDim.x) * blockDim.x) >> 4;
    for (int64_t base = (blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x) >> 4; base < N;
         base += NPG * ng) {
        float f0[NPG], f1[NPG], f2[NPG];
#pragma unroll
        for (int q = 0; q < NPG; ++q) {
            const int64_t node = base + q * ng;
            if (node < n) {
                const float xi = x[node];
                f0[q] = xi;
                f1[q] = 4.f * xi * (1.f - xi);
                f2[q] = ct[node] * ictmax;
            } else if (node < N) {
                const int64_t j2 = node - n;
                const float yj = y[j2];
                f0[q] = yj / (1.f + fabsf(yj));
                f1[q] = rt[j2] * irtmax;
                f2[q] = j2 >= m1 ? 1.f : 0.f;
            } else {
                f0[q] = f1[q] = f2[q] = 0.f;
            }
        }
#pragma unroll
        for (int q = 0; q < NPG; ++q) {
            const int64_t node = base + q * ng;
            if (node >= N) break;
            const bool var = node < n;
            float h[4];
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                float z = var ? bv[t] : bc[t];
                z = fmaf(f0[q], var ? Wv[0][t] : Wc[0][t], z);
                z = fmaf(f1[q], var ? Wv[1][t] : Wc[1][t], z);
                z = fmaf(f2[q], var ? Wv[2][t] : Wc[2][t], z);
                h[t] = fmaxf(z, 0.f);
            }
            uint2 w;
            w.x = static_cast<uint32_t>(f2bf(h[0])) | (static_cast<uint32_t>(f2bf(h[1])) << 16);
            w.y = static_cast<uint32_t>(f2bf(h[2])) | (static_cast<uint32_t>(f2bf(h[3])) << 16);
            uint16_t *dst = var ? Hv + node * kGnnH : Hc + (node - n) * kGnnH;
            reinterpret_cast<uint2 *>(dst)[f] = w;
        }
    }
}

// ------------------------------------------------------------------ SpMM
// out_r = sum_e E_e in[col_e] with E_e = val_e * rowinv[row of the entry]:
//   ROWS = true : CSR of [A; B]  (r = constraint row, col = variable, rowinv[r])
//   ROWS = false: CSR of [A; B]^T (r = variable, col = row j,        rowinv[j])
// IN_BF16: input features BF16 (else FP32); OUT: 0 store BF16, 1 store FP32,
// 2 add into FP32.
//
// Nodes come in `order`, longest first, in three classes by entry count:
//   heavy  (>= kGnnHeavy)  a workgroup of 8 wavefronts per node;
//   medium (> kGnnShort)   one wavefront per node;
//   short                  16 lanes per node (four nodes per wavefront).
// In the heavy and medium kernels a lane handles features 4f..4f+3 (f = lane
// & 15) of entry slot q = lane >> 4, so one load instruction gathers four
// neighbours' feature rows; eight such loads are issued before any is used.
// Slots (and wavefronts) are then added in a fixed order.
struct Feat4 {
    float v[4];
};

template <bool IN_BF16>
__device__ __forceinline__ Feat4 load_feat4(const void *__restrict__ in, int64_t row, int f) {
    Feat4 r;
    if (IN_BF16) {
        const uint2 w = reinterpret_cast<const uint2 *>(static_cast<const uint16_t *>(in) + row * kGnnH)[f];
        r.v[0] = __uint_as_float(w.x << 16);
        r.v[1] = __uint_as_float(w.x & 0xFFFF0000u);
        r.v[2] = __uint_as_float(w.y << 16);
        r.v[3] = __uint_as_float(w.y & 0xFFFF0000u);
    } else {
        const float4 w = reinterpret_cast<const float4 *>(static_cast<const float *>(in) + row * kGnnH)[f];
        r.v[0] = w.x;
        r.v[1] = w.y;
        r.v[2] = w.z;
        r.v[3] = w.w;
    }
    return r;
}

template <int OUT>
__device__ __forceinline__ void store_feat4(void *__restrict__ out, int64_t row, int f, const float *a) {
    if (OUT == 0) {
        uint2 w;
        w.x = static_cast<uint32_t>(f2bf(a[0])) | (static_cast<uint32_t>(f2bf(a[1])) << 16);
        w.y = static_cast<uint32_t>(f2bf(a[2])) | (static_cast<uint32_t>(f2bf(a[3])) << 16);
        reinterpret_cast<uint2 *>(static_cast<uint16_t *>(out) + row * kGnnH)[f] = w;
    } else {
        float4 *o = reinterpret_cast<float4 *>(static_cast<float *>(out) + row * kGnnH) + f;
        float4 w = make_float4(a[0], a[1], a[2], a[3]);
        if (OUT == 2) {
            const float4 v = *o;
            w.x += v.x;
            w.y += v.y;
            w.z += v.z;
            w.w += v.w;
        }
        *o = w;
    }
}

// Entries [e0, e1) of node r, slot q of this lane, blocks of 32 entries
// b = b0, b0 + bstep, ...: acc += E_e in[col_e] for e = 32 b + 4 u + q.
template <bool ROWS, bool IN_BF16>
__device__ __forceinline__ void gnn_gather_slots(int64_t r, int e0, int e1, int b0, int bstep, int q,
                                                 int f, const int *__restrict__ ci,
                                                 const int *__restrict__ val,
                                                 const float *__restrict__ rowinv,
                                                 const void *__restrict__ in, float *acc) {
    const float rs = ROWS ? rowinv[r] : 1.f;
    for (int eb = e0 + 32 * b0; eb < e1; eb += 32 * bstep) {
        int c[8];
        float a[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int e = eb + 4 * u + q;
            const bool ok = e < e1;
            const int ee = ok ? e : e0;
            c[u] = ci[ee];
            a[u] = ok ? (val ? static_cast<float>(val[ee]) : 1.f) : 0.f;
        }
        Feat4 h[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            if (!ROWS) a[u] *= rowinv[c[u]];
            h[u] = load_feat4<IN_BF16>(in, c[u], f);
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const float w = ROWS ? a[u] * rs : a[u];
#pragma unroll
            for (int k = 0; k < 4; ++k) acc[k] = fmaf(w, h[u].v[k], acc[k]);
        }
    }
}

template <bool ROWS, bool IN_BF16, int OUT>
__global__ void __launch_bounds__(512)
k_gnn_spmm_heavy(int nheavy, const int *__restrict__ order, const int *__restrict__ rp,
                 const int *__restrict__ ci, const int *__restrict__ val,
                 const float *__restrict__ rowinv, const void *__restrict__ in,
                 void *__restrict__ out) {
    __shared__ float red[8][kGnnH];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int q = lane >> 4, f = lane & 15;
    for (int k = blockIdx.x; k < nheavy; k += gridDim.x) {
        const int64_t r = order[k];
        float acc[4] = {0.f, 0.f, 0.f, 0.f};
        gnn_gather_slots<ROWS, IN_BF16>(r, rp[r], rp[r + 1], wave, 8, q, f, ci, val, rowinv, in, acc);
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            acc[t] += __shfl_xor(acc[t], 16, 64);
            acc[t] += __shfl_xor(acc[t], 32, 64);
        }
        if (q == 0) {
#pragma unroll
            for (int t = 0; t < 4; ++t) red[wave][4 * f + t] = acc[t];
        }
        __syncthreads();
        if (wave == 0 && q == 0) {
            float s4[4];
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                float v = red[0][4 * f + t];
                for (int w = 1; w < 8; ++w) v += red[w][4 * f + t];
                s4[t] = v;
            }
            store_feat4<OUT>(out, r, f, s4);
        }
        __syncthreads();
    }
}

template <bool ROWS, bool IN_BF16, int OUT>
__global__ void __launch_bounds__(256)
k_gnn_spmm_medium(int k0, int k1, const int *__restrict__ order, const int *__restrict__ rp,
                  const int *__restrict__ ci, const int *__restrict__ val,
                  const float *__restrict__ rowinv, const void *__restrict__ in,
                  void *__restrict__ out) {
    const int lane = threadIdx.x & 63;
    const int q = lane >> 4, f = lane & 15;
    const int nw = (gridDim.x * blockDim.x) >> 6;
    for (int k = k0 + static_cast<int>((blockIdx.x * blockDim.x + threadIdx.x) >> 6); k < k1; k += nw) {
        const int64_t r = order[k];
        float acc[4] = {0.f, 0.f, 0.f, 0.f};
        gnn_gather_slots<ROWS, IN_BF16>(r, rp[r], rp[r + 1], 0, 1, q, f, ci, val, rowinv, in, acc);
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            acc[t] += __shfl_xor(acc[t], 16, 64);
            acc[t] += __shfl_xor(acc[t], 32, 64);
        }
        if (q == 0) store_feat4<OUT>(out, r, f, acc);
    }
}

template <bool ROWS, bool IN_BF16, int OUT>
__global__ void __launch_bounds__(256)
k_gnn_spmm_short(int k0, int k1, const int *__restrict__ order, const int *__restrict__ rp,
                 const int *__restrict__ ci, const int *__restrict__ val,
                 const float *__restrict__ rowinv, const void *__restrict__ in,
                 void *__restrict__ out) {
    // two nodes per 16-lane group and pass, their entries walked in lockstep
    // (slots past a node's end add 0 x a finite feature), so a wavefront has
    // twice as many independent gathers in flight
    constexpr int NPG = 2;
    const int f = threadIdx.x & 15;
    const int ng = (gridDim.x * blockDim.x) >> 4;
    for (int kb = k0 + static_cast<int>((blockIdx.x * blockDim.x + threadIdx.x) >> 4); kb < k1; kb += NPG * ng) {
        int64_t r[NPG];
        int e0[NPG], e1[NPG];
        float rs[NPG], acc[NPG][4];
        int len = 0;
#pragma unroll
        for (int q = 0; q < NPG; ++q) {
            const int k = kb + q * ng;
            const bool live = k < k1;
            r[q] = live ? order[k] : -1;
            e0[q] = live ? rp[r[q]] : 0;
            e1[q] = live ? rp[r[q] + 1] : 0;
            rs[q] = (ROWS && live) ? rowinv[r[q]] : 1.f;
            len = max(len, e1[q] - e0[q]);
#pragma unroll
            for (int t = 0; t < 4; ++t) acc[q][t] = 0.f;
        }
        for (int d = 0; d < len; d += 4) {
            int c[NPG][4];
            float a[NPG][4];
#pragma unroll
            for (int q = 0; q < NPG; ++q)
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int e = e0[q] + d + u;
                    const bool ok = e < e1[q];
                    // an entry exists (len > 0), so feature row 0 is a valid stand-in
                    c[q][u] = ok ? ci[e] : 0;
                    a[q][u] = ok ? (val ? static_cast<float>(val[e]) : 1.f) : 0.f;
                }
            Feat4 h[NPG][4];
#pragma unroll
            for (int q = 0; q < NPG; ++q)
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    a[q][u] *= ROWS ? rs[q] : rowinv[c[q][u]];
                    h[q][u] = load_feat4<IN_BF16>(in, c[q][u], f);
                }
#pragma unroll
            for (int q = 0; q < NPG; ++q)
#pragma unroll
                for (int u = 0; u < 4; ++u)
#pragma unroll
                    for (int t = 0; t < 4; ++t) acc[q][t] = fmaf(a[q][u], h[q][u].v[t], acc[q][t]);
        }
#pragma unroll
        for (int q = 0; q < NPG; ++q)
            if (r[q] >= 0) store_feat4<OUT>(out, r[q], f, acc[q]);
    }
}

void launch_gnn_spmm(hipStream_t s, bool rows, bool in_bf16, int out_mode, int64_t nrows,
                     const int *order, int nheavy, int nmedium, const int *rp, const int *ci,
                     const int *val, const float *rowinv, const void *in, void *out) {
    if (nrows <= 0) return;
    const int k1 = nheavy, k2 = nheavy + nmedium, k3 = static_cast<int>(nrows);
    const int bh = std::min(nheavy, 1024);
    int64_t bm = (static_cast<int64_t>(nmedium) * 64 + 255) / 256;
    if (bm > 8192) bm = 8192;
    int64_t bs = (static_cast<int64_t>(k3 - k2) * 16 + 255) / 256;
    if (bs > 16384) bs = 16384;
#define GF_SP(R, IB, O)                                                                                          \
    do {                                                                                                         \
        if (bh > 0) k_gnn_spmm_heavy<R, IB, O><<<bh, 512, 0, s>>>(k1, order, rp, ci, val, rowinv, in, out);      \
        if (bm > 0) k_gnn_spmm_medium<R, IB, O><<<static_cast<int>(bm), 256, 0, s>>>(k1, k2, order, rp, ci, val, rowinv, in, out); \
        if (bs > 0) k_gnn_spmm_short<R, IB, O><<<static_cast<int>(bs), 256, 0, s>>>(k2, k3, order, rp, ci, val, rowinv, in, out); \
    } while (0)
#define GF_SP2(R, IB) if (out_mode == 0) GF_SP(R, IB, 0); else if (out_mode == 1) GF_SP(R, IB, 1); else GF_SP(R, IB, 2)
    if (rows) { if (in_bf16) { GF_SP2(true, true); } else { GF_SP2(true, false); } }
    else { if (in_bf16) { GF_SP2(false, true); } else { GF_SP2(false, false); } }
#undef GF_SP2
#undef GF_SP
}

// ------------------------------------------------------------------ MFMA GEMM
// C[N x NO] = [A1 | A2][N x KD] * B[KD x NO]  (BF16 operands, FP32 accumulate)
// A1 holds columns [0, K1), A2 columns [K1, KD) (row stride 64 each); B is
// given transposed, BT[NO][KD] (BF16), and staged in LDS.  Each wavefront
// owns 16 rows and all NO columns (NO/16 MFMA tiles).  Operand layout of
// v_mfma_f32_16x16x16_bf16: lane l supplies A[l%16][4(l/16)+j] and
// B[4(l/16)+j][l%16], j = 0..3, and receives D[4(l/16)+j][l%16].
// Epilogue: + bias[col] (if bias), relu (if RELU); columns [0,64) go to out1,
// [64,128) to out2, as BF16 (OUTB) or FP32 (store or add).
template <int KD, int NO, bool RELU, int OUTM>
__global__ void __launch_bounds__(256)
k_gnn_gemm(int64_t N, const uint16_t *__restrict__ A1, const uint16_t *__restrict__ A2, int K1,
           const uint16_t *__restrict__ BT, const float *__restrict__ bias, void *__restrict__ out1,
           void *__restrict__ out2) {
    __shared__ uint16_t sB[NO * KD];
    // BF16 output tile of each wavefront (16 rows x 64 columns), so that rows
    // are written with 16-byte stores instead of 2-byte ones
    __shared__ uint16_t sO[4][16 * 64];
    for (int i = threadIdx.x; i < NO * KD / 4; i += blockDim.x)
        reinterpret_cast<uint2 *>(sB)[i] = reinterpret_cast<const uint2 *>(BT)[i];
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int li = lane & 15, lk = 4 * (lane >> 4);
    constexpr int NT = NO / 16;
    for (int64_t row0 = (static_cast<int64_t>(blockIdx.x) * 4 + wave) * 16; row0 < N;
         row0 += static_cast<int64_t>(gridDim.x) * 64) {
        f32x4 acc[NT];
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
        const int64_t ra = row0 + li;
#pragma unroll
        for (int k0 = 0; k0 < KD; k0 += 16) {
            bf16x4 a = bf16x4{0, 0, 0, 0};
            if (ra < N) {
                const int kk = k0 + lk;
                const uint16_t *src = kk < K1 ? A1 + ra * kGnnH + kk : A2 + ra * kGnnH + (kk - K1);
                a = *reinterpret_cast<const bf16x4 *>(src);
            }
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                const bf16x4 b = *reinterpret_cast<const bf16x4 *>(&sB[(t * 16 + li) * KD + k0 + lk]);
                acc[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc[t], 0, 0, 0);
            }
        }
        if (OUTM == 0 && NO == 64) {
            // lane (li, lk) holds rows lk..lk+3 of columns t*16 + li: through
            // LDS, then lane L writes row L/4, columns 16 (L%4) .. +15
            uint16_t *T = sO[wave];
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                const int col = t * 16 + li;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    float v = acc[t][j];
                    if (bias) v += bias[col];
                    if (RELU) v = fmaxf(v, 0.f);
                    T[(lk + j) * 64 + col] = f2bf(v);
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            __builtin_amdgcn_wave_barrier();
            const int rr = lane >> 2, cq = (lane & 3) * 16;
            const int64_t r = row0 + rr;
            if (r < N) {
                const uint4 *src = reinterpret_cast<const uint4 *>(T + rr * 64 + cq);
                uint4 *dst = reinterpret_cast<uint4 *>(static_cast<uint16_t *>(out1) + r * kGnnH + cq);
                dst[0] = src[0];
                dst[1] = src[1];
            }
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            __builtin_amdgcn_wave_barrier();
        } else {
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                const int col = t * 16 + li;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int64_t r = row0 + lk + j;
                    if (r >= N) continue;
                    float v = acc[t][j];
                    if (bias) v += bias[col];
                    if (RELU) v = fmaxf(v, 0.f);
                    void *o = col < 64 ? out1 : out2;
                    const int64_t idx = r * kGnnH + (col & 63);
                    if (OUTM == 0) static_cast<uint16_t *>(o)[idx] = f2bf(v);
                    else if (OUTM == 1) static_cast<float *>(o)[idx] = v;
                    else static_cast<float *>(o)[idx] += v;
                }
            }
        }
    }
}

// Forward dense layer out = relu([H | S] W + bias) over N rows (H, S: BF16
// [N][64]; W as BT[64 out][128 in] in LDS; BF16 out).  A wavefront owns 16
// rows at a time; lane (li, kq) loads 16 bytes of row li four times: H and S
// columns 8 kq .. 8 kq + 7 and 32 + 8 kq .. 32 + 8 kq + 7 (each load fills
// 64-byte segments of 16 rows), and the next 16 rows' loads are issued before
// the current rows' MFMAs.  The contraction order is permuted alike in A and
// B: in the MFMA step that uses half h of load q, lane (li, kq) supplies
// the k indices kb(q) + 8 kq + 4 h + j (j = 0..3) of both operands, with
// kb = 0, 32, 64, 96 for H low, H high, S low, S high.  The result tile goes
// through LDS and is written with 16-byte stores.
__global__ void __launch_bounds__(256)
k_gnn_dense_fwd(int64_t N, const uint16_t *__restrict__ H, const uint16_t *__restrict__ S,
                const uint16_t *__restrict__ BT, const float *__restrict__ bias,
                uint16_t *__restrict__ out) {
    __shared__ uint16_t sB[64 * 128];
    __shared__ uint16_t sO[4][16 * 64];
    for (int i = threadIdx.x; i < 64 * 128 / 4; i += blockDim.x)
        reinterpret_cast<uint2 *>(sB)[i] = reinterpret_cast<const uint2 *>(BT)[i];
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int li = lane & 15, kq = lane >> 4;
    float bcol[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) bcol[t] = bias ? bias[t * 16 + li] : 0.f;
    const int64_t step = static_cast<int64_t>(gridDim.x) * 64;
    auto load = [&](int64_t row0, uint4 *a) {
        const int64_t ra = row0 + li;
        if (ra < N) {
            const uint4 *h = reinterpret_cast<const uint4 *>(H + ra * kGnnH);
            const uint4 *sv = reinterpret_cast<const uint4 *>(S + ra * kGnnH);
            a[0] = h[kq];
            a[1] = h[4 + kq];
            a[2] = sv[kq];
            a[3] = sv[4 + kq];
        } else {
#pragma unroll
            for (int q = 0; q < 4; ++q) a[q] = make_uint4(0u, 0u, 0u, 0u);
        }
    };
    int64_t row0 = (static_cast<int64_t>(blockIdx.x) * 4 + wave) * 16;
    uint4 cur[4];
    if (row0 < N) load(row0, cur);
    for (; row0 < N; row0 += step) {
        uint4 nxt[4];
        if (row0 + step < N) load(row0 + step, nxt);
        f32x4 acc[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int kb = (q >> 1) * 64 + (q & 1) * 32 + 8 * kq;
#pragma unroll
            for (int hf = 0; hf < 2; ++hf) {
                const uint32_t w0 = hf ? cur[q].z : cur[q].x, w1 = hf ? cur[q].w : cur[q].y;
                bf16x4 a;
                a[0] = static_cast<short>(w0 & 0xFFFFu);
                a[1] = static_cast<short>(w0 >> 16);
                a[2] = static_cast<short>(w1 & 0xFFFFu);
                a[3] = static_cast<short>(w1 >> 16);
                const int kk = kb + 4 * hf;
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const bf16x4 b = *reinterpret_cast<const bf16x4 *>(&sB[(t * 16 + li) * 128 + kk]);
                    acc[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc[t], 0, 0, 0);
                }
            }
        }
        uint16_t *T = sO[wave];
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int j = 0; j < 4; ++j)
                T[(4 * kq + j) * 64 + t * 16 + li] = f2bf(fmaxf(acc[t][j] + bcol[t], 0.f));
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        const int rr = lane >> 2, cq = (lane & 3) * 16;
        const int64_t r = row0 + rr;
        if (r < N) {
            const uint4 *src = reinterpret_cast<const uint4 *>(T + rr * 64 + cq);
            uint4 *dst = reinterpret_cast<uint4 *>(out + r * kGnnH + cq);
            dst[0] = src[0];
            dst[1] = src[1];
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int q = 0; q < 4; ++q) cur[q] = nxt[q];
    }
}

static int gemm_grid(int64_t N) {
    int64_t b = (N + 63) / 64;
    if (b > 4096) b = 4096;
    return static_cast<int>(b < 1 ? 1 : b);
}

// Forward dense layer: out = relu([A1|A2] W + bias), W given as BT[64][128].
void launch_gnn_dense_fwd(hipStream_t s, int64_t N, const uint16_t *A1, const uint16_t *A2,
                          const uint16_t *BT, const float *bias, uint16_t *out) {
    if (N <= 0) return;
    k_gnn_dense_fwd<<<gemm_grid(N), 256, 0, s>>>(N, A1, A2, BT, bias, out);
}

// Backward through a dense layer: [dA1 | dA2] (+)= dZ W^T, with W^T given as
// BT = W [128][64]; dA1/dA2 FP32 (add when accumulate != 0).
void launch_gnn_dense_bwd_in(hipStream_t s, int64_t N, const uint16_t *dZ, const uint16_t *Wrm,
                             float *dA1, float *dA2, int accumulate) {
    if (N <= 0) return;
    if (accumulate)
        k_gnn_gemm<64, 128, false, 2><<<gemm_grid(N), 256, 0, s>>>(N, dZ, dZ, 64, Wrm, nullptr, dA1, dA2);
    else
        k_gnn_gemm<64, 128, false, 1><<<gemm_grid(N), 256, 0, s>>>(N, dZ, dZ, 64, Wrm, nullptr, dA1, dA2);
}

// ---------------------------------------------------------------------------
// Weight gradient dW[128 x 64] = [A1 | A2]^T dZ (reduction over N on MFMA).
// Each workgroup walks 64-row chunks (LDS-staged), keeps its 128x64 partial
// in registers (4 waves x 8 tiles) and writes it to part[block]; a second
// kernel adds the partials in a fixed order.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256)
k_gnn_wgrad(int64_t N, const uint16_t *__restrict__ A1, const uint16_t *__restrict__ A2,
            const uint16_t *__restrict__ dZ, float *__restrict__ part) {
    __shared__ uint16_t sA[64 * 128];
    __shared__ uint16_t sZ[64 * 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int li = lane & 15, lk = 4 * (lane >> 4);
    // wave w owns dW rows [32 w, 32 w + 32) (2 m-tiles) x all 64 columns (4 n-tiles)
    f32x4 acc[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int64_t c0 = static_cast<int64_t>(blockIdx.x) * 64; c0 < N; c0 += static_cast<int64_t>(gridDim.x) * 64) {
        __syncthreads();
        for (int i = threadIdx.x; i < 64 * 32; i += 256) {      // A: 64 rows x 128 cols, 4 per thread
            const int r = i >> 5, q = (i & 31) * 4;
            uint2 v = {0u, 0u};
            if (c0 + r < N) {
                const uint16_t *src = q < 64 ? A1 + (c0 + r) * kGnnH + q : A2 + (c0 + r) * kGnnH + (q - 64);
                v = *reinterpret_cast<const uint2 *>(src);
            }
            *reinterpret_cast<uint2 *>(&sA[r * 128 + q]) = v;
        }
        for (int i = threadIdx.x; i < 64 * 16; i += 256) {      // dZ: 64 rows x 64 cols
            const int r = i >> 4, q = (i & 15) * 4;
            uint2 v = {0u, 0u};
            if (c0 + r < N) v = *reinterpret_cast<const uint2 *>(dZ + (c0 + r) * kGnnH + q);
            *reinterpret_cast<uint2 *>(&sZ[r * 64 + q]) = v;
        }
        __syncthreads();
#pragma unroll
        for (int ks = 0; ks < 64; ks += 16) {
            bf16x4 a[2], b[4];
#pragma unroll
            for (int mt = 0; mt < 2; ++mt) {
                const int col = 32 * wave + 16 * mt + li;   // dW row = input feature
#pragma unroll
                for (int j = 0; j < 4; ++j) a[mt][j] = static_cast<short>(sA[(ks + lk + j) * 128 + col]);
            }
#pragma unroll
            for (int nt = 0; nt < 4; ++nt)
#pragma unroll
                for (int j = 0; j < 4; ++j) b[nt][j] = static_cast<short>(sZ[(ks + lk + j) * 64 + 16 * nt + li]);
#pragma unroll
            for (int mt = 0; mt < 2; ++mt)
#pragma unroll
                for (int nt = 0; nt < 4; ++nt)
                    acc[mt * 4 + nt] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[mt], b[nt], acc[mt * 4 + nt], 0, 0, 0);
        }
    }
    float *P = part + static_cast<int64_t>(blockIdx.x) * 128 * 64;
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
        for (int nt = 0; nt < 4; ++nt)
#pragma unroll
            for (int j = 0; j < 4; ++j)
                P[(32 * wave + 16 * mt + lk + j) * 64 + 16 * nt + li] = acc[mt * 4 + nt][j];
}

// out[i] (+)= sum_b part[b][i], i < len; dst split: rows [0,64) -> dst1, [64,128) -> dst2.
__global__ void k_gnn_sum_parts(int nparts, int len, const float *__restrict__ part,
                                float *__restrict__ dst1, float *__restrict__ dst2, int half) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= len) return;
    float s = 0.f;
    for (int b = 0; b < nparts; ++b) s += part[static_cast<int64_t>(b) * len + i];
    if (i < half) dst1[i] = s;
    else dst2[i - half] = s;
}

void launch_gnn_wgrad(hipStream_t s, int64_t N, const uint16_t *A1, const uint16_t *A2,
                      const uint16_t *dZ, float *part, int max_parts, float *dW1, float *dW2) {
    int g = static_cast<int>((N + 63) / 64);
    if (g > max_parts) g = max_parts;
    if (g < 1) g = 1;
    k_gnn_wgrad<<<g, 256, 0, s>>>(N, A1, A2, dZ, part);
    k_gnn_sum_parts<<<(128 * 64 + 255) / 256, 256, 0, s>>>(g, 128 * 64, part, dW1, dW2, 64 * 64);
}

// ---------------------------------------------------------------------------
// dZ = dOut o [Out > 0] (BF16, for MFMA) and column sums of dZ (bias gradient)
// as per-workgroup partials.  One wavefront per row, lane = column.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256)
k_gnn_mask(int64_t N, const float *__restrict__ dOut, const uint16_t *__restrict__ Out,
           uint16_t *__restrict__ dZ, float *__restrict__ part) {
    __shared__ float sh[4][64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    float cs = 0.f;
    const int64_t nw = (static_cast<int64_t>(gridDim.x) * blockDim.x) >> 6;
    for (int64_t r = (blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x) >> 6; r < N; r += nw) {
        const int64_t o = r * kGnnH + lane;
        const float v = (Out[o] != 0 && bf2f(Out[o]) > 0.f) ? dOut[o] : 0.f;
        dZ[o] = f2bf(v);
        cs += v;
    }
    sh[wave][lane] = cs;
    __syncthreads();
    if (wave == 0) part[static_cast<int64_t>(blockIdx.x) * 64 + lane] = sh[0][lane] + sh[1][lane] + sh[2][lane] + sh[3][lane];
}

void launch_gnn_mask(hipStream_t s, int64_t N, const float *dOut, const uint16_t *Out,
                     uint16_t *dZ, float *part, int max_parts, float *db) {
    int g = static_cast<int>((N * 64 + 255) / 256);
    if (g > max_parts) g = max_parts;
    if (g < 1) g = 1;
    k_gnn_mask<<<g, 256, 0, s>>>(N, dOut, Out, dZ, part);
    k_gnn_sum_parts<<<1, 64, 0, s>>>(g, 64, part, db, db, 64);
}

// ---------------------------------------------------------------------------
// Output layer: logit_i = Hv_i . wo + bo; p_i = sigmoid(logit_i).  With a
// target: loss partials (softplus(z) - t z), dlogit = (p - t)/n, dHv = dlogit wo^T
// (FP32), and partials of dwo = sum_i dlogit_i Hv_i, dbo = sum dlogit.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256)
k_gnn_out(int64_t n, const uint16_t *__restrict__ Hv, const float *__restrict__ theta,
          float *__restrict__ logit, float *__restrict__ p, const float *__restrict__ target,
          float *__restrict__ dHv, float *__restrict__ part) {
    // 16 lanes per node, lane f = hidden units 4f..4f+3; the 4 node groups of a
    // wavefront add their contributions separately, in a fixed order at the end
    __shared__ float sh[4][66];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, f = lane & 15;
    float wo[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) wo[t] = theta[kGnnOffwo + 4 * f + t];
    const float bo = theta[kGnnOffbo];
    float gw[4] = {0.f, 0.f, 0.f, 0.f}, gb = 0.f, ls = 0.f;
    const float inv_n = 1.f / static_cast<float>(n);
    const int64_t ng = (static_cast<int64_t>(gridDim.x) * blockDim.x) >> 4;
    // four nodes per group and pass, their feature loads issued together; the
    // nodes are then taken in the order of a one-node loop (same sums)
    constexpr int NPG = 4;
    for (int64_t ib = (blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x) >> 4; ib < n; ib += NPG * ng) {
        uint2 wq[NPG];
#pragma unroll
        for (int u = 0; u < NPG; ++u) {
            const int64_t i = ib + u * ng;
            wq[u] = i < n ? reinterpret_cast<const uint2 *>(Hv + i * kGnnH)[f] : make_uint2(0u, 0u);
        }
#pragma unroll
        for (int u = 0; u < NPG; ++u) {
            const int64_t i = ib + u * ng;
            if (i >= n) break;   // uniform over the node's 16 lanes
            const uint2 w = wq[u];
            const float h[4] = {__uint_as_float(w.x << 16), __uint_as_float(w.x & 0xFFFF0000u),
                                __uint_as_float(w.y << 16), __uint_as_float(w.y & 0xFFFF0000u)};
            float zz = h[0] * wo[0];
            zz = fmaf(h[1], wo[1], zz);
            zz = fmaf(h[2], wo[2], zz);
            zz = fmaf(h[3], wo[3], zz);
#pragma unroll
            for (int o = 8; o > 0; o >>= 1) zz += __shfl_xor(zz, o, 16);
            const float z = zz + bo;
            const float pz = 1.f / (1.f + __expf(-z));
            if (f == 0) {
                if (logit) logit[i] = z;
                if (p) p[i] = pz;
            }
            if (target) {
                const float t = target[i];
                const float dz = (pz - t) * inv_n;
                reinterpret_cast<float4 *>(dHv + i * kGnnH)[f] =
                    make_float4(dz * wo[0], dz * wo[1], dz * wo[2], dz * wo[3]);
#pragma unroll
                for (int q = 0; q < 4; ++q) gw[q] += dz * h[q];
                if (f == 0) {
                    gb += dz;
                    ls += fmaxf(z, 0.f) + log1pf(__expf(-fabsf(z))) - t * z;
                }
            }
        }
    }
    if (!target) return;
    // node groups of the wavefront (lanes f, f+16, f+32, f+48), in order
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        gw[q] += __shfl_down(gw[q], 16, 64);
        gw[q] += __shfl_down(gw[q], 32, 64);
    }
    gb += __shfl_down(gb, 16, 64);
    gb += __shfl_down(gb, 32, 64);
    ls += __shfl_down(ls, 16, 64);
    ls += __shfl_down(ls, 32, 64);
    if (lane < 16) {
#pragma unroll
        for (int q = 0; q < 4; ++q) sh[wave][4 * f + q] = gw[q];
    }
    if (lane == 0) { sh[wave][64] = gb; sh[wave][65] = ls; }
    __syncthreads();
    if (wave == 0) {
        float* P = part + static_cast<int64_t>(blockIdx.x) * 66;
        P[lane] = sh[0][lane] + sh[1][lane] + sh[2][lane] + sh[3][lane];
        if (lane < 2) P[64 + lane] = sh[0][64 + lane] + sh[1][64 + lane] + sh[2][64 + lane] + sh[3][64 + lane];
    }
}

// loss_out[0] = mean loss; grad[wo], grad[bo].
__global__ void k_gnn_out_reduce(int nparts, int64_t n, const float *__restrict__ part,
                                 float *__restrict__ grad, float *__restrict__ loss_out) {
    const int i = threadIdx.x;   // 66 threads
    if (i >= 66) return;
    float s = 0.f;
    for (int b = 0; b < nparts; ++b) s += part[static_cast<int64_t>(b) * 66 + i];
    if (i < 64) grad[kGnnOffwo + i] = s;
    else if (i == 64) grad[kGnnOffbo] = s;
    else loss_out[0] = s / static_cast<float>(n);
}

void launch_gnn_out(hipStream_t s, int64_t n, const uint16_t *Hv, const float *theta, float *logit,
                    float *p, const float *target, float *dHv, float *part, int max_parts,
                    float *grad, float *loss_out) {
    // training keeps one partial per workgroup (max_parts of them); inference
    // needs no partials and takes enough workgroups to fill the device
    int64_t g = (n * 16 + 255) / 256;
    if (g > (target ? max_parts : 8192)) g = target ? max_parts : 8192;
    if (g < 1) g = 1;
    k_gnn_out<<<static_cast<int>(g), 256, 0, s>>>(n, Hv, theta, logit, p, target, dHv, part);
    if (target) k_gnn_out_reduce<<<1, 128, 0, s>>>(static_cast<int>(g), n, part, grad, loss_out);
}

// ---------------------------------------------------------------------------
// Embedding backward: dZ0 = dH o [H0 > 0]; dU[k][h] = sum F[k] dZ0[h], du = sum dZ0.
// part[block][5*64] = {dU rows 0..3, du}.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256)
k_gnn_embed_bwd(int64_t N, int is_var, int m1, const float *__restrict__ xy,
                const float *__restrict__ crt, float iscale, const uint16_t *__restrict__ H0,
                const float *__restrict__ dH, float *__restrict__ part) {
    __shared__ float sh[4][5][64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    float acc[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
    const int64_t nw = (static_cast<int64_t>(gridDim.x) * blockDim.x) >> 6;
    for (int64_t r = (blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x) >> 6; r < N; r += nw) {
        const int64_t o = r * kGnnH + lane;
        const float dz = bf2f(H0[o]) > 0.f ? dH[o] : 0.f;
        float f0, f1, f2;
        if (is_var) {
            const float xi = xy[r];
            f0 = xi; f1 = 4.f * xi * (1.f - xi); f2 = crt[r] * iscale;
        } else {
            const float yj = xy[r];
            f0 = yj / (1.f + fabsf(yj)); f1 = crt[r] * iscale; f2 = r >= m1 ? 1.f : 0.f;
        }
        acc[0] += f0 * dz; acc[1] += f1 * dz; acc[2] += f2 * dz; acc[3] += dz; acc[4] += dz;
    }
    for (int k = 0; k < 5; ++k) sh[wave][k][lane] = acc[k];
    __syncthreads();
    if (wave == 0)
        for (int k = 0; k < 5; ++k)
            part[static_cast<int64_t>(blockIdx.x) * 320 + k * 64 + lane] = sh[0][k][lane] + sh[1][k][lane] + sh[2][k][lane] + sh[3][k][lane];
}

// dU (4x64) then du (64) contiguous in grad: U at offU, u at offu.
__global__ void k_gnn_embed_bwd_reduce(int nparts, const float *__restrict__ part,
                                       float *__restrict__ gU, float *__restrict__ gu) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;   // 320
    if (i >= 320) return;
    float s = 0.f;
    for (int b = 0; b < nparts; ++b) s += part[static_cast<int64_t>(b) * 320 + i];
    if (i < 256) gU[i] = s;
    else gu[i - 256] = s;
}

void launch_gnn_embed_bwd(hipStream_t s, int64_t N, int is_var, int m1, const float *xy,
                          const float *crt, float iscale, const uint16_t *H0, const float *dH,
                          float *part, int max_parts, float *gU, float *gu) {
    if (N <= 0) {   // no nodes of this kind: zero gradient (fill kernel, no memset node)
        k_gnn_sum_parts<<<2, 256, 0, s>>>(0, 320, part, gU, gu, 256);
        return;
    }
    int g = static_cast<int>((N * 64 + 255) / 256);
    if (g > max_parts) g = max_parts;
    if (g < 1) g = 1;
    k_gnn_embed_bwd<<<g, 256, 0, s>>>(N, is_var, m1, xy, crt, iscale, H0, dH, part);
    k_gnn_embed_bwd_reduce<<<2, 256, 0, s>>>(g, part, gU, gu);
}

void launch_gnn_embed(hipStream_t s, int64_t n, int64_t m, int m1, const float *x, const float *y,
                      const float *ct, const float *rt, float ictmax, float irtmax,
                      const float *theta, uint16_t *Hv, uint16_t *Hc) {
    int64_t blocks = ((n + m) * 16 + 255) / 256;
    if (blocks > 16384) blocks = 16384;
    if (blocks > 0)
        k_gnn_embed<<<static_cast<int>(blocks), 256, 0, s>>>(n, m, m1, x, y, ct, rt, ictmax, irtmax, theta, Hv, Hc);
}

// ---------------------------------------------------------------------------
// BF16 operand copies of the layer weights from the FP32 master:
//   fwd[l][side] = W^T [64 out][128 in] (in = [self | message]),
//   bwd[l][side] = W   [128 in][64 out].
// ---------------------------------------------------------------------------
__global__ void k_gnn_pack(const float *__restrict__ theta, uint16_t *__restrict__ wf,
                           uint16_t *__restrict__ wb) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;   // over L*2*128*64
    if (idx >= kGnnL * 2 * 128 * 64) return;
    const int blk = idx / (128 * 64);      // l*2 + side (0 = constraint side, 1 = variable side)
    const int r = idx % (128 * 64);
    const int in = r / 64, o = r % 64;     // W[in][o]
    const int l = blk >> 1, side = blk & 1;
    const float *base = theta + kGnnOffLayer + l * kGnnLayerSize + side * (2 * 64 * 64 + 64);
    const float w = in < 64 ? base[in * 64 + o] : base[64 * 64 + (in - 64) * 64 + o];
    wb[static_cast<int64_t>(blk) * 128 * 64 + in * 64 + o] = f2bf(w);
    wf[static_cast<int64_t>(blk) * 128 * 64 + o * 128 + in] = f2bf(w);
}

void launch_gnn_pack(hipStream_t s, const float *theta, uint16_t *wf, uint16_t *wb) {
    k_gnn_pack<<<(kGnnL * 2 * 128 * 64 + 255) / 256, 256, 0, s>>>(theta, wf, wb);
}

// Adam (Kingma & Ba) on the flat FP32 parameter vector.
__global__ void k_gnn_adam(int np, float *__restrict__ theta, const float *__restrict__ g,
                           float *__restrict__ m, float *__restrict__ v, float lr, float b1,
                           float b2, float eps, float c1, float c2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= np) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    theta[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

void launch_gnn_adam(hipStream_t s, int np, float *theta, const float *g, float *m, float *v,
                     float lr, float b1, float b2, float eps, float c1, float c2) {
    k_gnn_adam<<<(np + 255) / 256, 256, 0, s>>>(np, theta, g, m, v, lr, b1, b2, eps, c1, c2);
}

}  // namespace gfors
