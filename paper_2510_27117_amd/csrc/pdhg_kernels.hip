// PDHG kernels (Algorithm 2), the FP64 power iteration of Preprocess (Sec. 3)
// and the FP64 residuals of Theorem 2 / CheckHalt (Sec. 3), for gfx950.
//
// SpMV mapping: a group of LPR lanes (a power of two, LPR | 64) owns one CSR
// row; the lanes stride through the row so that consecutive lanes read
// consecutive column indices (coalesced), partial sums are combined with
// cross-lane xor-shuffles inside the wavefront.  No atomics anywhere: the
// transposed product K^T y runs over a second CSR holding K^T.
#include "gfors_internal.h"

namespace gfors {

template <int LPR, typename T>
__device__ __forceinline__ T group_sum(T v) {
#pragma unroll
    for (int o = LPR / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, LPR);
    return v;
}

// ---------------------------------------------------------------------------
// Dual step: y_k = Pi( y_{k-1} + tau2 (K~ xbar_{k-1} + r~) ).
// With K~_j = -omega_j a_j and r~_j = omega_j r_j this is
//   t_j = rt_j - omega_j * sum_i a_ji xbar_i,   y_j <- y_j + tau2 t_j,
// projected onto R_+ for inequality rows (j < m1).  Also writes
// wy_j = omega_j y_j, which the primal step multiplies by the integer a_ji.
// ---------------------------------------------------------------------------
template <int LPR, bool UNIT, bool BATCH, typename VT>
__global__ void __launch_bounds__(256)
k_dual(int m, int m1, const int *__restrict__ rp, const int *__restrict__ ci,
       const VT *__restrict__ val, const float *__restrict__ omega,
       const float *__restrict__ rt, const float *__restrict__ xbar,
       const float *__restrict__ y_in, float *__restrict__ y_out, float *__restrict__ wy,
       float tau2, const float *__restrict__ tau2_inst, const int *__restrict__ row_inst,
       int skip_len) {
    const int tid = blockIdx.x * blockDim.x + threadIdx.x;
    const int row = tid / LPR;
    const int sub = tid & (LPR - 1);
    float s = 0.f;
    bool own = row < m;
    if (own) {
        const int e0 = rp[row], e1 = rp[row + 1];
        // rows of skip_len entries or more belong to the workgroup-per-row kernel
        if (skip_len > 0 && e1 - e0 >= skip_len) own = false;
        for (int e = e0 + sub; own && e < e1; e += LPR) {
            const float xv = xbar[ci[e]];
            if (UNIT) s += xv;
            else s = fmaf(static_cast<float>(val[e]), xv, s);
        }
    }
    s = group_sum<LPR>(s);
    if (own && sub == 0) {
        const float om = omega[row];
        const float t = rt[row] - om * s;
        const float ta = BATCH ? tau2_inst[row_inst[row]] : tau2;
        float y = y_in[row] + ta * t;
        if (row < m1) y = fmaxf(y, 0.f);
        y_out[row] = y;
        wy[row] = om * y;
    }
}

// Slot of workgroup b in a list processed one item per workgroup: groups of
// 16 consecutive slots run on one XCD (workgroup b runs on XCD b % 8) and the
// groups are dealt to the XCDs in turn.  Consecutive heavy rows or variables
// often gather neighbouring elements (one cache line serves up to 16 of them),
// which then meet in one L2 instead of eight.  A bijection on [0, 128 k).
__device__ __forceinline__ int xcd_grouped_slot(int b) {
    const int x = b & 7, k = b >> 3;
    return ((((k >> 4) << 3) + x) << 4) + (k & 15);
}

constexpr int kLongUnroll = 4;   // loads in flight per lane in the heavy kernels

// Dual step for long rows: a workgroup of 256 lanes per row (rows taken
// longest first from `order`, so that the longest rows do not trail; slots
// grouped per XCD), lanes strided over the row with four independent loads
// in flight each, partial sums combined by shuffles inside each wavefront and
// then across the four wavefronts in a fixed order.
// Sum of a_e xbar[col_e] over the row's entries by the workgroup's 256 lanes
// (four loads in flight per lane); DENSE: the row's columns are the range
// c0, c0 + 1, ..., so no column index is loaded.
template <bool UNIT, bool DENSE, typename VT>
__device__ __forceinline__ float long_row_sum(int e0, int e1, int c0, const int *__restrict__ ci,
                                              const VT *__restrict__ val, const float *__restrict__ xbar) {
    float s = 0.f;
    for (int eb = e0 + static_cast<int>(threadIdx.x); eb < e1; eb += kLongUnroll * 256) {
        float xv[kLongUnroll];
        int a[kLongUnroll];
#pragma unroll
        for (int u = 0; u < kLongUnroll; ++u) {
            const int e = min(eb + 256 * u, e1 - 1);
            const float v = xbar[DENSE ? c0 + (e - e0) : ci[e]];
            const bool in = eb + 256 * u < e1;
            xv[u] = in ? v : 0.f;
            a[u] = UNIT ? 1 : (in ? static_cast<int>(val[e]) : 0);
        }
#pragma unroll
        for (int u = 0; u < kLongUnroll; ++u) {
            if (UNIT) s += xv[u];
            else s = fmaf(static_cast<float>(a[u]), xv[u], s);
        }
    }
    return s;
}

template <bool UNIT, bool BATCH>
__global__ void __launch_bounds__(256)
k_dual_long(int count, int m1, const int *__restrict__ order, const int *__restrict__ rp,
            const int *__restrict__ rowc0, const int *__restrict__ ci, const int *__restrict__ val,
            const int16_t *__restrict__ val16, const uint8_t *__restrict__ rowunit,
            const float *__restrict__ omega, const float *__restrict__ rt,
            const float *__restrict__ xbar, const float *__restrict__ y_in,
            float *__restrict__ y_out, float *__restrict__ wy, float tau2,
            const float *__restrict__ tau2_inst, const int *__restrict__ row_inst) {
    __shared__ float ws[4];
    const int slot = xcd_grouped_slot(blockIdx.x);
    if (slot >= count) return;                          // uniform per workgroup
    const int row = order[slot];
    const int e0 = rp[row], e1 = rp[row + 1];
    const int c0 = rowc0[row];                          // first column of a dense row, else -1
    // val16: the same coefficients as int16 (all fit), half the stream
    float s;
    if (!UNIT && rowunit && rowunit[row])   // every coefficient of the row is 1: no coefficient stream
        s = c0 >= 0 ? long_row_sum<true, true>(e0, e1, c0, ci, val, xbar)
                    : long_row_sum<true, false>(e0, e1, c0, ci, val, xbar);
    else if (!UNIT && val16)
        s = c0 >= 0 ? long_row_sum<UNIT, true>(e0, e1, c0, ci, val16, xbar)
                    : long_row_sum<UNIT, false>(e0, e1, c0, ci, val16, xbar);
    else
        s = c0 >= 0 ? long_row_sum<UNIT, true>(e0, e1, c0, ci, val, xbar)
                    : long_row_sum<UNIT, false>(e0, e1, c0, ci, val, xbar);
    s = group_sum<64>(s);
    if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        const float tot = ((ws[0] + ws[1]) + ws[2]) + ws[3];
        const float om = omega[row];
        const float t = rt[row] - om * tot;
        const float ta = BATCH ? tau2_inst[row_inst[row]] : tau2;
        float y = y_in[row] + ta * t;
        if (row < m1) y = fmaxf(y, 0.f);
        y_out[row] = y;
        wy[row] = om * y;
    }
}

void launch_dual_long(hipStream_t s, bool unit, bool batched, int m, int m1, const int *order,
                      const int *rp, const int *rowc0, const int *ci, const int *val, const int16_t *val16,
                      const uint8_t *rowunit, const float *omega,
                      const float *rt, const float *xbar, const float *y_in, float *y_out,
                      float *wy, float tau2, const float *tau2_inst, const int *row_inst) {
    if (m <= 0) return;
    const int grid = ((m + 127) / 128) * 128;
#define GF_DL(U, B) k_dual_long<U, B><<<grid, 256, 0, s>>>(m, m1, order, rp, rowc0, ci, val, val16, rowunit, omega, rt, xbar, y_in, y_out, wy, tau2, tau2_inst, row_inst)
    if (unit) { if (batched) GF_DL(true, true); else GF_DL(true, false); }
    else { if (batched) GF_DL(false, true); else GF_DL(false, false); }
#undef GF_DL
}

// Primal step for variables in many rows (no Q): a workgroup per variable,
// taken from `order` (most rows first), same summation structure as
// k_dual_long.  The iteration counter is advanced by the companion kernel.
template <bool UNIT, bool BATCH>
__global__ void __launch_bounds__(256)
k_primal_long(int count, const int *__restrict__ order, const int *__restrict__ rpT,
              const int *__restrict__ ciT, const int *__restrict__ valT,
              const float *__restrict__ wy, const float *__restrict__ x_in,
              float *__restrict__ x_out, float *__restrict__ xbar, const float *__restrict__ ct,
              float tau1, const float *__restrict__ tau1_inst, const double *__restrict__ rho,
              const int *__restrict__ var_inst) {
    __shared__ float ws[4];
    const int slot = xcd_grouped_slot(blockIdx.x);
    if (slot >= count) return;                          // uniform per workgroup
    const int i = order[slot];
    const int e0 = rpT[i], e1 = rpT[i + 1];
    float s = 0.f;
    for (int eb = e0 + static_cast<int>(threadIdx.x); eb < e1; eb += kLongUnroll * 256) {
        float w[kLongUnroll];
        int a[kLongUnroll];
#pragma unroll
        for (int u = 0; u < kLongUnroll; ++u) {
            const int e = min(eb + 256 * u, e1 - 1);
            const float v = wy[ciT[e]];
            const bool in = eb + 256 * u < e1;
            w[u] = in ? v : 0.f;
            a[u] = UNIT ? 1 : (in ? valT[e] : 0);
        }
#pragma unroll
        for (int u = 0; u < kLongUnroll; ++u) {
            if (UNIT) s += w[u];
            else s = fmaf(static_cast<float>(a[u]), w[u], s);
        }
    }
    s = group_sum<64>(s);
    if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        const float tot = ((ws[0] + ws[1]) + ws[2]) + ws[3];
        const int t = BATCH ? var_inst[i] : 0;
        const float xi = x_in[i];
        const float rh = static_cast<float>(rho[t]);
        const float ta = BATCH ? tau1_inst[t] : tau1;
        const float g = ct[i] + rh - tot - 2.f * rh * xi;
        const float xn = fminf(fmaxf(xi - ta * g, 0.f), 1.f);
        x_out[i] = xn;
        xbar[i] = 2.f * xn - xi;
    }
}

void launch_primal_long(hipStream_t s, bool unit, bool batched, int count, const int *order,
                        const int *rpT, const int *ciT, const int *valT, const float *wy,
                        const float *x_in, float *x_out, float *xbar, const float *ct, float tau1,
                        const float *tau1_inst, const double *rho, const int *var_inst) {
    if (count <= 0) return;
    const int grid = ((count + 127) / 128) * 128;
#define GF_PL(U, B) k_primal_long<U, B><<<grid, 256, 0, s>>>(count, order, rpT, ciT, valT, wy, x_in, x_out, xbar, ct, tau1, tau1_inst, rho, var_inst)
    if (unit) { if (batched) GF_PL(true, true); else GF_PL(true, false); }
    else { if (batched) GF_PL(false, true); else GF_PL(false, false); }
#undef GF_PL
}

// ---------------------------------------------------------------------------
// Primal step:
//   delta_i = c~_i + rho - sum_j a_ji wy_j + (2/s_o) sum_k Q_ik x_k - 2 rho x_i
//   x_k = clip(x_{k-1} - tau1 delta, 0, 1),   xbar_k = 2 x_k - x_{k-1}
// (K~^T y = -sum_j a_ji omega_j y_j; Q~ = Q / s_o.)  The gradient uses x_{k-1},
// read from x_in while x_out receives x_k (double buffer).
// KMODE: 0 = no constraint rows, 1 = unit coefficients, 2 = int32 values.
// ---------------------------------------------------------------------------
template <int LPR, int KMODE, bool HASQ, bool BATCH>
__global__ void __launch_bounds__(256)
k_primal(int n, const int *__restrict__ rpT, const int *__restrict__ colT0, const int *__restrict__ ciT,
         const int *__restrict__ valT, const float *__restrict__ wy,
         const int *__restrict__ rpQ, const int *__restrict__ ciQ, const int *__restrict__ valQ,
         const float *__restrict__ x_in, float *__restrict__ x_out, float *__restrict__ xbar,
         const float *__restrict__ ct, float tau1, float two_so,
         const float *__restrict__ tau1_inst, const float *__restrict__ two_so_inst,
         const double *__restrict__ rho, const int *__restrict__ var_inst,
         DevCounters *__restrict__ ctr, int skip_len) {
    const int tid = blockIdx.x * blockDim.x + threadIdx.x;
    const int i = tid / LPR;
    const int sub = tid & (LPR - 1);
    float s1 = 0.f, s2 = 0.f;
    // per-row operands are independent of the gathers: load them first
    float xi = 0.f, cti = 0.f;
    int t = 0;
    bool own = i < n;
    // variables in skip_len or more rows belong to the workgroup-per-variable kernel
    if (own && KMODE != 0 && skip_len > 0 && rpT[i + 1] - rpT[i] >= skip_len) own = false;
    if (own) {
        xi = x_in[i];
        cti = ct[i];
        if (BATCH) t = var_inst[i];
    }
    if (own) {
        if (KMODE != 0) {
            // a variable whose rows are one contiguous range (dense rows of a
            // batched instance) computes its row indices instead of loading them
            const int e0 = rpT[i], e1 = rpT[i + 1];
            const int r0 = colT0 ? colT0[i] : -1;   // null: no variable is a contiguous range
#pragma unroll 4
            for (int e = e0 + sub; e < e1; e += LPR) {
                int j;
                if (r0 >= 0) j = r0 + (e - e0);
                else j = ciT[e];
                const float w = wy[j];
                if (KMODE == 1) s1 += w;
                else s1 = fmaf(static_cast<float>(valT[e]), w, s1);
            }
        }
        if (HASQ) {
            const int e1 = rpQ[i + 1];
            for (int e = rpQ[i] + sub; e < e1; e += LPR)
                s2 = fmaf(static_cast<float>(valQ[e]), x_in[ciQ[e]], s2);
        }
    }
    if (KMODE != 0) s1 = group_sum<LPR>(s1);
    if (HASQ) s2 = group_sum<LPR>(s2);
    if (own && sub == 0) {
        const float rh = static_cast<float>(rho[t]);
        const float ta = BATCH ? tau1_inst[t] : tau1;
        float g = cti + rh;
        if (KMODE != 0) g -= s1;
        if (HASQ) g = fmaf(BATCH ? two_so_inst[t] : two_so, s2, g);
        g -= 2.f * rh * xi;
        const float xn = fminf(fmaxf(xi - ta * g, 0.f), 1.f);
        x_out[i] = xn;
        xbar[i] = 2.f * xn - xi;
    }
    if (tid == 0) ctr->k += 1;
}

template <int LPR>
static void dual_lpr(hipStream_t s, bool unit, bool batched, int m, int m1, const int *rp,
                     const int *ci, const int *val, const int16_t *val16, const float *omega, const float *rt,
                     const float *xbar, const float *y_in, float *y_out, float *wy, float tau2,
                     const float *tau2_inst, const int *row_inst, int skip_len) {
    const int64_t threads = static_cast<int64_t>(m) * LPR;
    const int blocks = static_cast<int>((threads + 255) / 256);
    if (blocks == 0) return;
#define GF_DUAL(U, B, VT, V) \
    k_dual<LPR, U, B, VT><<<blocks, 256, 0, s>>>(m, m1, rp, ci, V, omega, rt, xbar, y_in, y_out, wy, tau2, tau2_inst, row_inst, skip_len)
    if (unit) { if (batched) GF_DUAL(true, true, int, val); else GF_DUAL(true, false, int, val); }
    else if (val16) { if (batched) GF_DUAL(false, true, int16_t, val16); else GF_DUAL(false, false, int16_t, val16); }
    else { if (batched) GF_DUAL(false, true, int, val); else GF_DUAL(false, false, int, val); }
#undef GF_DUAL
}

void launch_dual(hipStream_t s, int lpr, bool unit, bool batched, int m, int m1,
                 const int *rp, const int *ci, const int *val, const int16_t *val16, const float *omega,
                 const float *rt, const float *xbar, const float *y_in, float *y_out,
                 float *wy, float tau2, const float *tau2_inst, const int *row_inst,
                 int skip_len) {
    switch (lpr) {
#define GF_CASE(L) case L: dual_lpr<L>(s, unit, batched, m, m1, rp, ci, val, val16, omega, rt, xbar, y_in, y_out, wy, tau2, tau2_inst, row_inst, skip_len); break;
        GF_CASE(1) GF_CASE(2) GF_CASE(4) GF_CASE(8) GF_CASE(16) GF_CASE(32) GF_CASE(64)
#undef GF_CASE
        default: break;
    }
}

template <int LPR, int KMODE, bool HASQ>
static void primal_k(hipStream_t s, bool batched, int n, const int *rpT, const int *colT0, const int *ciT,
                     const int *valT, const float *wy, const int *rpQ, const int *ciQ,
                     const int *valQ, const float *x_in, float *x_out, float *xbar,
                     const float *ct, float tau1, float two_so, const float *tau1_inst,
                     const float *two_so_inst, const double *rho, const int *var_inst,
                     DevCounters *ctr, int skip_len) {
    const int64_t threads = static_cast<int64_t>(n) * LPR;
    const int blocks = static_cast<int>((threads + 255) / 256);
    if (blocks == 0) return;
    if (batched)
        k_primal<LPR, KMODE, HASQ, true><<<blocks, 256, 0, s>>>(n, rpT, colT0, ciT, valT, wy, rpQ, ciQ, valQ, x_in, x_out, xbar, ct, tau1, two_so, tau1_inst, two_so_inst, rho, var_inst, ctr, skip_len);
    else
        k_primal<LPR, KMODE, HASQ, false><<<blocks, 256, 0, s>>>(n, rpT, colT0, ciT, valT, wy, rpQ, ciQ, valQ, x_in, x_out, xbar, ct, tau1, two_so, tau1_inst, two_so_inst, rho, var_inst, ctr, skip_len);
}

template <int LPR>
static void primal_lpr(hipStream_t s, int kmode, bool hasq, bool batched, int n,
                       const int *rpT, const int *colT0, const int *ciT, const int *valT, const float *wy,
                       const int *rpQ, const int *ciQ, const int *valQ, const float *x_in,
                       float *x_out, float *xbar, const float *ct, float tau1, float two_so,
                       const float *tau1_inst, const float *two_so_inst, const double *rho,
                       const int *var_inst, DevCounters *ctr, int skip_len) {
#define GF_P(KM, HQ) primal_k<LPR, KM, HQ>(s, batched, n, rpT, colT0, ciT, valT, wy, rpQ, ciQ, valQ, x_in, x_out, xbar, ct, tau1, two_so, tau1_inst, two_so_inst, rho, var_inst, ctr, skip_len)
    if (hasq) {
        if (kmode == 0) GF_P(0, true); else if (kmode == 1) GF_P(1, true); else GF_P(2, true);
    } else {
        if (kmode == 0) GF_P(0, false); else if (kmode == 1) GF_P(1, false); else GF_P(2, false);
    }
#undef GF_P
}

void launch_primal(hipStream_t s, int lpr, int kmode, bool hasq, bool batched, int n,
                   const int *rpT, const int *colT0, const int *ciT, const int *valT, const float *wy,
                   const int *rpQ, const int *ciQ, const int *valQ, const float *x_in,
                   float *x_out, float *xbar, const float *ct, float tau1, float two_so,
                   const float *tau1_inst, const float *two_so_inst, const double *rho,
                   const int *var_inst, DevCounters *ctr, int skip_len) {
    switch (lpr) {
#define GF_CASE(L) case L: primal_lpr<L>(s, kmode, hasq, batched, n, rpT, colT0, ciT, valT, wy, rpQ, ciQ, valQ, x_in, x_out, xbar, ct, tau1, two_so, tau1_inst, two_so_inst, rho, var_inst, ctr, skip_len); break;
        GF_CASE(1) GF_CASE(2) GF_CASE(4) GF_CASE(8) GF_CASE(16) GF_CASE(32) GF_CASE(64)
#undef GF_CASE
        default: break;
    }
}

// ---------------------------------------------------------------------------
// XCD-sliced SpMV.  The columns are cut into P slices and the matrix is stored
// as P CSR matrices (slice-major).  Workgroup b works on slice b % P: the
// hardware hands consecutive workgroups to consecutive XCDs, so with P = 8 every
// XCD gathers from one slice of the vector only and that slice stays resident
// in the XCD's own L2.  Each slice writes its partial row sums; the combine
// kernels below add the P partials in a fixed order and apply the PDHG update.
// ---------------------------------------------------------------------------
template <int LPR, bool UNIT>
__global__ void __launch_bounds__(256)
k_spmv_part(int nrows, int P, const int *__restrict__ rpP, const int *__restrict__ ci,
            const int *__restrict__ val, const float *__restrict__ v, float *__restrict__ part) {
    const int sl = blockIdx.x % P;
    const int chunk = blockIdx.x / P;
    const int row = chunk * (256 / LPR) + static_cast<int>(threadIdx.x) / LPR;
    const int sub = threadIdx.x & (LPR - 1);
    const int *rp = rpP + static_cast<int64_t>(sl) * (nrows + 1);
    float acc = 0.f;
    if (row < nrows) {
        const int e1 = rp[row + 1];
        for (int e = rp[row] + sub; e < e1; e += LPR) {
            const int c = __builtin_nontemporal_load(ci + e);
            const float xv = v[c];
            if (UNIT) acc += xv;
            else acc = fmaf(static_cast<float>(__builtin_nontemporal_load(val + e)), xv, acc);
        }
    }
    acc = group_sum<LPR>(acc);
    if (row < nrows && sub == 0) part[static_cast<int64_t>(sl) * nrows + row] = acc;
}

// PP > 0: the slice count as a compile-time constant (all loads in flight).
template <bool BATCH, int PP>
__global__ void __launch_bounds__(256)
k_dual_combine(int m, int m1, int P, const float *__restrict__ part,
               const float *__restrict__ omega, const float *__restrict__ rt,
               const float *__restrict__ y_in, float *__restrict__ y_out, float *__restrict__ wy,
               float tau2, const float *__restrict__ tau2_inst, const int *__restrict__ row_inst,
               uint64_t *__restrict__ wybits) {
    const int row = blockIdx.x * blockDim.x + threadIdx.x;
    float w = 0.f;
    if (row < m) {
        float s = 0.f;
        if (PP > 0) {
            float pv[PP > 0 ? PP : 1];
#pragma unroll
            for (int q = 0; q < PP; ++q) pv[q] = part[static_cast<int64_t>(q) * m + row];
#pragma unroll
            for (int q = 0; q < PP; ++q) s += pv[q];
        } else {
            for (int q = 0; q < P; ++q) s += part[static_cast<int64_t>(q) * m + row];
        }
        const float om = omega[row];
        const float t = rt[row] - om * s;
        const float ta = BATCH ? tau2_inst[row_inst[row]] : tau2;
        float y = y_in[row] + ta * t;
        if (row < m1) y = fmaxf(y, 0.f);
        y_out[row] = y;
        w = om * y;
        wy[row] = w;
    }
    // nonzero bitmap of wy for the next primal step: a wavefront holds 64
    // consecutive rows (64-aligned)
    if (wybits) {
        const uint64_t b = __ballot(row < m && w != 0.f);
        if ((threadIdx.x & 63) == 0 && row < m) wybits[row >> 6] = b;
    }
}

template <bool BATCH>
__global__ void __launch_bounds__(256)
k_primal_combine(int n, int P, const float *__restrict__ part, const float *__restrict__ x_in,
                 float *__restrict__ x_out, float *__restrict__ xbar, const float *__restrict__ ct,
                 float tau1, const float *__restrict__ tau1_inst, const double *__restrict__ rho,
                 const int *__restrict__ var_inst, DevCounters *__restrict__ ctr,
                 uint64_t *__restrict__ xbits) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) ctr->k += 1;
    float xb = 0.f;
    if (i < n) {
        const int t = BATCH ? var_inst[i] : 0;
        const float xi = x_in[i];
        float s1 = 0.f;
        for (int q = 0; q < P; ++q) s1 += part[static_cast<int64_t>(q) * n + i];
        const float rh = static_cast<float>(rho[t]);
        const float ta = BATCH ? tau1_inst[t] : tau1;
        const float g = ct[i] + rh - s1 - 2.f * rh * xi;
        const float xn = fminf(fmaxf(xi - ta * g, 0.f), 1.f);
        x_out[i] = xn;
        xb = 2.f * xn - xi;
        xbar[i] = xb;
    }
    if (xbits) {
        const uint64_t b = __ballot(i < n && xb != 0.f);
        if ((threadIdx.x & 63) == 0 && i < n) xbits[i >> 6] = b;
    }
}

template <int LPR>
static void spmv_part_lpr(hipStream_t s, bool unit, int nrows, int P, const int *rpP,
                          const int *ci, const int *val, const float *v, float *part) {
    const int rows_per_block = 256 / LPR;
    const int64_t chunks = (static_cast<int64_t>(nrows) + rows_per_block - 1) / rows_per_block;
    const int64_t blocks = chunks * P;
    if (blocks == 0) return;
    if (unit) k_spmv_part<LPR, true><<<static_cast<int>(blocks), 256, 0, s>>>(nrows, P, rpP, ci, val, v, part);
    else k_spmv_part<LPR, false><<<static_cast<int>(blocks), 256, 0, s>>>(nrows, P, rpP, ci, val, v, part);
}

void launch_spmv_part(hipStream_t s, int lpr, bool unit, int nrows, int P, const int *rpP,
                      const int *ci, const int *val, const float *v, float *part) {
    switch (lpr) {
#define GF_CASE(L) case L: spmv_part_lpr<L>(s, unit, nrows, P, rpP, ci, val, v, part); break;
        GF_CASE(1) GF_CASE(2) GF_CASE(4) GF_CASE(8) GF_CASE(16) GF_CASE(32) GF_CASE(64)
#undef GF_CASE
        default: break;
    }
}

void launch_dual_combine(hipStream_t s, bool batched, int m, int m1, int P, const float *part,
                         const float *omega, const float *rt, const float *y_in, float *y_out,
                         float *wy, float tau2, const float *tau2_inst, const int *row_inst,
                         uint64_t *wybits) {
    const int blocks = (m + 255) / 256;
    if (!blocks) return;
#define GF_DC(B, PPV) k_dual_combine<B, PPV><<<blocks, 256, 0, s>>>(m, m1, P, part, omega, rt, y_in, y_out, wy, tau2, tau2_inst, row_inst, wybits)
    if (P == kXcdSlices) { if (batched) GF_DC(true, kXcdSlices); else GF_DC(false, kXcdSlices); }
    else { if (batched) GF_DC(true, 0); else GF_DC(false, 0); }
#undef GF_DC
}

void launch_primal_combine(hipStream_t s, bool batched, int n, int P, const float *part,
                           const float *x_in, float *x_out, float *xbar, const float *ct,
                           float tau1, const float *tau1_inst, const double *rho,
                           const int *var_inst, DevCounters *ctr, uint64_t *xbits) {
    const int blocks = (n + 255) / 256;
    if (!blocks) return;
    if (batched) k_primal_combine<true><<<blocks, 256, 0, s>>>(n, P, part, x_in, x_out, xbar, ct, tau1, tau1_inst, rho, var_inst, ctr, xbits);
    else k_primal_combine<false><<<blocks, 256, 0, s>>>(n, P, part, x_in, x_out, xbar, ct, tau1, tau1_inst, rho, var_inst, ctr, xbits);
}

// ---------------------------------------------------------------------------
// SELL-64 (sliced ELLPACK, chunk = one wavefront).  Rows are sorted by length
// inside windows, cut into chunks of 64 rows, and every chunk is padded to its
// longest row and stored column-major: entry k of the chunk's lane-th row sits
// at ptr[c] + 64 k + lane.  Lane = row, so a wavefront issues its column-index
// loads back to back, each one fully coalesced, and the chunk's extent is a
// single uniform (scalar) load.  Padding entries point at a zero element
// placed one past the end of the gathered vector.  row_of maps (chunk, lane)
// to the original row (-1 for an empty slot).  With P > 1 the matrix is cut
// into P column slices (as for k_spmv_part), slice = workgroup index % P.
// MODE 0 writes the slice's partial sums; MODE 1 applies the dual update;
// MODE 2 the primal update (no Q).
// ---------------------------------------------------------------------------
template <bool UNIT, int MODE, bool BATCH>
__global__ void __launch_bounds__(256)
k_sell(int nrows, int P, int nchunk, const int *__restrict__ ptr, const int *__restrict__ ci,
       const int *__restrict__ val, const int16_t *__restrict__ val16, const int *__restrict__ row_of,
       const int *__restrict__ sc0, const int *__restrict__ slen, const float *__restrict__ v,
       float *__restrict__ part,
       // dual epilogue
       int m1, const float *__restrict__ omega, const float *__restrict__ rt,
       const float *__restrict__ y_in, float *__restrict__ y_out, float *__restrict__ wy,
       float tau2, const float *__restrict__ tau2_inst, const int *__restrict__ row_inst,
       // primal epilogue
       const float *__restrict__ x_in, float *__restrict__ x_out, float *__restrict__ xbar,
       const float *__restrict__ ct, float tau1, const float *__restrict__ tau1_inst,
       const double *__restrict__ rho, const int *__restrict__ var_inst,
       DevCounters *__restrict__ ctr) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int sl = blockIdx.x % P;
    const int c = (blockIdx.x / P) * 4 + wave;
    if (MODE == 2 && blockIdx.x == 0 && threadIdx.x == 0) ctr->k += 1;
    if (c >= nchunk) return;
    const int64_t pb = static_cast<int64_t>(sl) * (nchunk + 1);
    const int e0 = ptr[pb + c];
    const int L = (ptr[pb + c + 1] - e0) >> 6;
    const int *cic = ci + e0 + lane;
    float acc = 0.f;
    const int64_t slot = (static_cast<int64_t>(sl) * nchunk + c) * 64 + lane;
    const int cb = sc0 ? sc0[slot] : -1;          // null: no slot is a contiguous range
    if (cb >= 0) {
        // the row's entries here are the columns cb, cb + 1, ...: indices are
        // computed; slots past its length add 0 like the padding entries
        const int ln = slen[slot];
        if (UNIT) {
#pragma unroll 4
            for (int k = 0; k < L; ++k) acc += k < ln ? v[cb + k] : 0.f;
        } else if (val16) {                      // the coefficients as int16 (all fit)
            const int16_t *vc = val16 + e0 + lane;
#pragma unroll 8
            for (int k = 0; k < L; ++k)
                acc = fmaf(static_cast<float>(__builtin_nontemporal_load(vc + 64 * k)), k < ln ? v[cb + k] : 0.f, acc);
        } else {
            const int *vc = val + e0 + lane;
#pragma unroll 4
            for (int k = 0; k < L; ++k)
                acc = fmaf(static_cast<float>(__builtin_nontemporal_load(vc + 64 * k)), k < ln ? v[cb + k] : 0.f, acc);
        }
    } else if (UNIT) {
#pragma unroll 4
        for (int k = 0; k < L; ++k) acc += v[__builtin_nontemporal_load(cic + 64 * k)];
    } else {
        const int *vc = val + e0 + lane;
#pragma unroll 4
        for (int k = 0; k < L; ++k)
            acc = fmaf(static_cast<float>(__builtin_nontemporal_load(vc + 64 * k)),
                       v[__builtin_nontemporal_load(cic + 64 * k)], acc);
    }
    const int row = row_of[(static_cast<int64_t>(sl) * nchunk + c) * 64 + lane];
    if (row < 0) return;
    if (MODE == 0) {
        part[static_cast<int64_t>(sl) * nrows + row] = acc;
    } else if (MODE == 1) {
        const float om = omega[row];
        const float t = rt[row] - om * acc;
        const float ta = BATCH ? tau2_inst[row_inst[row]] : tau2;
        float y = y_in[row] + ta * t;
        if (row < m1) y = fmaxf(y, 0.f);
        y_out[row] = y;
        wy[row] = om * y;
    } else {
        const int t = BATCH ? var_inst[row] : 0;
        const float xi = x_in[row];
        const float rh = static_cast<float>(rho[t]);
        const float ta = BATCH ? tau1_inst[t] : tau1;
        const float g = ct[row] + rh - acc - 2.f * rh * xi;
        const float xn = fminf(fmaxf(xi - ta * g, 0.f), 1.f);
        x_out[row] = xn;
        xbar[row] = 2.f * xn - xi;
    }
}

void launch_sell(hipStream_t s, const SellView &sv, int mode, bool unit, bool batched,
                 const float *v, float *part, int m1, const float *omega, const float *rt,
                 const float *y_in, float *y_out, float *wy, float tau2, const float *tau2_inst,
                 const int *row_inst, const float *x_in, float *x_out, float *xbar,
                 const float *ct, float tau1, const float *tau1_inst, const double *rho,
                 const int *var_inst, DevCounters *ctr) {
    const int64_t blocks = static_cast<int64_t>((sv.nchunk + 3) / 4) * sv.P;
    if (blocks == 0) return;
#define GF_SELL(U, M, B)     k_sell<U, M, B><<<static_cast<int>(blocks), 256, 0, s>>>(sv.nrows, sv.P, sv.nchunk, sv.ptr, sv.ci, sv.val, sv.val16, sv.row_of, sv.c0, sv.len, v, part, m1, omega, rt, y_in, y_out, wy, tau2, tau2_inst, row_inst, x_in, x_out, xbar, ct, tau1, tau1_inst, rho, var_inst, ctr)
#define GF_SELL_M(U, B)     if (mode == 0) GF_SELL(U, 0, B); else if (mode == 1) GF_SELL(U, 1, B); else GF_SELL(U, 2, B)
    if (unit) { if (batched) { GF_SELL_M(true, true); } else { GF_SELL_M(true, false); } }
    else { if (batched) { GF_SELL_M(false, true); } else { GF_SELL_M(false, false); } }
#undef GF_SELL_M
#undef GF_SELL
}

// ---------------------------------------------------------------------------
// Nonzero bitmaps.  PDHG iterates sit on the box bounds for most variables and
// many duals stay at 0, so most gathered operands of the two SpMVs are zeros.
// bits[i/32] bit i%32 = (v_i != 0); the SpMV variants below keep the bitmap of
// their slice in LDS and only issue the gather for set bits (skipping zero
// terms leaves the FP32 sums unchanged).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256)
k_nzbits(const float *__restrict__ v, int64_t n, int64_t nwords64, uint64_t *__restrict__ bits) {
    const int lane = threadIdx.x & 63;
    for (int64_t w = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6; w < nwords64;
         w += (static_cast<int64_t>(gridDim.x) * blockDim.x) >> 6) {
        const int64_t i = w * 64 + lane;
        const bool nz = i < n && v[i] != 0.f;
        const uint64_t mask = __ballot(nz);
        if (lane == 0) bits[w] = mask;
    }
}

void launch_nzbits(hipStream_t s, const float *v, int64_t n, int64_t nwords64, uint64_t *bits) {
    int64_t blocks = (nwords64 * 64 + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    if (blocks > 0) k_nzbits<<<static_cast<int>(blocks), 256, 0, s>>>(v, n, nwords64, bits);
}

// Copy nw bitmap words into LDS: 8 independent loads per thread are issued
// before any of them is waited for (the address of an out-of-range slot is
// clamped to the last word; its value is not stored).
__device__ __forceinline__ void load_bitmap_lds(uint32_t *sb, const uint32_t *__restrict__ src,
                                                int nw) {
    for (int w0 = threadIdx.x; w0 < nw; w0 += 8 * blockDim.x) {
        uint32_t t[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) t[u] = src[min(w0 + u * static_cast<int>(blockDim.x), nw - 1)];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int w = w0 + u * static_cast<int>(blockDim.x);
            if (w < nw) sb[w] = t[u];
        }
    }
}

// Sliced SELL partial SpMV with the slice's bitmap in LDS (persistent: G
// workgroups per slice loop over the slice's chunks).
template <bool UNIT>
__global__ void __launch_bounds__(1024)
k_sell_part_bits(int nrows, int P, int nchunk, int ns, int ncols, int G,
                 const int *__restrict__ ptr, const int *__restrict__ ci,
                 const int *__restrict__ val, const int *__restrict__ row_of,
                 const float *__restrict__ v, const uint32_t *__restrict__ bits,
                 float *__restrict__ part) {
    extern __shared__ uint32_t sb[];
    const int sl = blockIdx.x % P;
    const int gb = blockIdx.x / P;
    const int base = sl * ns;
    const int nw = ns >> 5;
    load_bitmap_lds(sb, bits + (base >> 5), nw);
    __syncthreads();
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int nwv = blockDim.x >> 6;
    const int64_t pb = static_cast<int64_t>(sl) * (nchunk + 1);
    for (int c = gb * nwv + wave; c < nchunk; c += G * nwv) {
        const int e0 = ptr[pb + c];
        const int L = (ptr[pb + c + 1] - e0) >> 6;
        const int *cic = ci + e0 + lane;
        float acc = 0.f;
#pragma unroll 4
        for (int k = 0; k < L; ++k) {
            const int col = __builtin_nontemporal_load(cic + 64 * k);
            if (col < ncols) {
                const int loc = col - base;
                if ((sb[loc >> 5] >> (loc & 31)) & 1u) {
                    if (UNIT) acc += v[col];
                    else acc = fmaf(static_cast<float>(val[e0 + lane + 64 * k]), v[col], acc);
                }
            }
        }
        const int row = row_of[(static_cast<int64_t>(sl) * nchunk + c) * 64 + lane];
        if (row >= 0) part[static_cast<int64_t>(sl) * nrows + row] = acc;
    }
}

void launch_sell_part_bits(hipStream_t s, const SellView &sv, int ns, int ncols, bool unit,
                           const float *v, const uint32_t *bits, float *part) {
    const int G = 64;   // 8 slices x 64 workgroups x 16 wavefronts
    const size_t lds = static_cast<size_t>(ns / 32) * 4;
    if (unit) k_sell_part_bits<true><<<G * sv.P, 1024, lds, s>>>(sv.nrows, sv.P, sv.nchunk, ns, ncols, G, sv.ptr, sv.ci, sv.val, sv.row_of, v, bits, part);
    else k_sell_part_bits<false><<<G * sv.P, 1024, lds, s>>>(sv.nrows, sv.P, sv.nchunk, ns, ncols, G, sv.ptr, sv.ci, sv.val, sv.row_of, v, bits, part);
}

// SELL-64 SpMV that skips zero operands, any epilogue (MODE as in k_sell).
// Persistent: G workgroups per column slice, each holding the slice's nonzero
// bitmap of v in LDS, walk the slice's chunks.  Within a chunk the column
// indices of 8 consecutive entries are loaded together, then their bits are
// looked up, then the gathers of the nonzero operands are issued together, so
// a wavefront keeps up to 16 loads in flight.  The terms are added in the same
// order as k_sell and the skipped terms are zeros, so the sums equal k_sell's.
template <bool UNIT, int MODE, bool BATCH, int NC>
__global__ void __launch_bounds__(512)
k_sell_bits(int nrows, int P, int nchunk, int ns, int ncols, int G, const int *__restrict__ ptr,
            const int *__restrict__ ci, const int *__restrict__ val,
            const int *__restrict__ row_of, const float *__restrict__ v,
            const uint32_t *__restrict__ bits, float *__restrict__ part,
            int m1, const float *__restrict__ omega, const float *__restrict__ rt,
            const float *__restrict__ y_in, float *__restrict__ y_out, float *__restrict__ wy,
            float tau2, const float *__restrict__ tau2_inst, const int *__restrict__ row_inst,
            const float *__restrict__ x_in, float *__restrict__ x_out, float *__restrict__ xbar,
            const float *__restrict__ ct, float tau1, const float *__restrict__ tau1_inst,
            const double *__restrict__ rho, const int *__restrict__ var_inst,
            DevCounters *__restrict__ ctr) {
    extern __shared__ uint32_t sb[];
    const int sl = blockIdx.x % P;
    const int gb = blockIdx.x / P;
    const int base = sl * ns;
    const int nw = ns >> 5;
    load_bitmap_lds(sb, bits + (base >> 5), nw);
    if (MODE == 2 && blockIdx.x == 0 && threadIdx.x == 0) ctr->k += 1;
    __syncthreads();
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int nwv = blockDim.x >> 6;
    const int64_t pb = static_cast<int64_t>(sl) * (nchunk + 1);
    const int stride = G * nwv;
    // NC chunks per pass (c, c + stride, ...), so that a wavefront has NC
    // times as many independent loads in flight.  Each chunk's terms are still
    // added in its own order.  Branch-free: slots past a chunk's end load
    // (clamped) entry L-1 and are masked; the bitmap word is read for every
    // slot (index clamped into the slice); a zero operand gathers the padding
    // element v[ncols] instead, one address shared by the wavefront (one cache
    // line, no extra L2 traffic), and its term is not added.
    for (int c0 = gb * nwv + wave; c0 < nchunk; c0 += NC * stride) {
        int cc[NC], e0[NC], L[NC], row[NC];
        float acc[NC];
#pragma unroll
        for (int h = 0; h < NC; ++h) {
            acc[h] = 0.f;
            cc[h] = c0 + h * stride;
            const bool live = cc[h] < nchunk;
            const int cx = live ? cc[h] : c0;
            e0[h] = ptr[pb + cx];
            L[h] = live ? (ptr[pb + cx + 1] - e0[h]) >> 6 : 0;
            row[h] = live ? row_of[(static_cast<int64_t>(sl) * nchunk + cx) * 64 + lane] : -1;
        }
        int Lm = 0;
#pragma unroll
        for (int h = 0; h < NC; ++h) Lm = max(Lm, L[h]);
        for (int k0 = 0; k0 < Lm; k0 += 8) {
            int col[NC][8];
            int a[NC][8];
#pragma unroll
            for (int h = 0; h < NC; ++h) {
                if (k0 < L[h]) {                   // uniform across the wavefront
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        const int k = min(k0 + u, L[h] - 1);
                        const int cv = ci[e0[h] + lane + 64 * k];
                        col[h][u] = k0 + u < L[h] ? cv : ncols;
                        a[h][u] = UNIT ? 0 : val[e0[h] + lane + 64 * k];
                    }
                } else {
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        col[h][u] = ncols;
                        a[h][u] = 0;
                    }
                }
            }
            bool nz[NC][8];
#pragma unroll
            for (int h = 0; h < NC; ++h) {
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int loc = col[h][u] - base;
                    const bool in = (col[h][u] < ncols) & (static_cast<unsigned>(loc) < static_cast<unsigned>(ns));
                    const int li = in ? loc : 0;
                    const uint32_t word = sb[li >> 5];
                    nz[h][u] = in & (((word >> (li & 31)) & 1u) != 0u);
                }
            }
            float g[NC][8];
#pragma unroll
            for (int h = 0; h < NC; ++h) {
#pragma unroll
                for (int u = 0; u < 8; ++u) g[h][u] = v[nz[h][u] ? col[h][u] : ncols];
            }
#pragma unroll
            for (int h = 0; h < NC; ++h) {
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const float t = UNIT ? acc[h] + g[h][u] : fmaf(static_cast<float>(a[h][u]), g[h][u], acc[h]);
                    acc[h] = nz[h][u] ? t : acc[h];
                }
            }
        }
#pragma unroll
        for (int h = 0; h < NC; ++h) {
            const int r = row[h];
            if (r < 0) continue;
            const float sum = acc[h];
            if (MODE == 0) {
                part[static_cast<int64_t>(sl) * nrows + r] = sum;
            } else if (MODE == 1) {
                const float om = omega[r];
                const float t = rt[r] - om * sum;
                const float ta = BATCH ? tau2_inst[row_inst[r]] : tau2;
                float y = y_in[r] + ta * t;
                if (r < m1) y = fmaxf(y, 0.f);
                y_out[r] = y;
                wy[r] = om * y;
            } else {
                const int t = BATCH ? var_inst[r] : 0;
                const float xi = x_in[r];
                const float rh = static_cast<float>(rho[t]);
                const float ta = BATCH ? tau1_inst[t] : tau1;
                const float gr = ct[r] + rh - sum - 2.f * rh * xi;
                const float xn = fminf(fmaxf(xi - ta * gr, 0.f), 1.f);
                x_out[r] = xn;
                xbar[r] = 2.f * xn - xi;
            }
        }
    }
}

int sell_bits_blocks(const SellView &sv, int nc) {
    // workgroups of 8 wavefronts; per CU as many as the bitmap (LDS) and the
    // resident wavefronts allow (32, or 16 for four chunks per pass, which
    // holds twice the registers); the grid is a multiple of P so that
    // workgroup b (slice b % P) runs on XCD b % 8 when P = 8
    const int64_t bytes = static_cast<int64_t>(sv.ns / 32) * 4 + 1024;
    int per_cu = static_cast<int>((160 * 1024) / bytes);
    const int cap = nc >= 4 ? 2 : 4;
    if (per_cu > cap) per_cu = cap;
    if (per_cu < 1) per_cu = 1;
    int G = 256 * per_cu / sv.P;
    const int need = (sv.nchunk + 8 * nc - 1) / (8 * nc);
    if (G > need) G = need;
    return G < 1 ? 1 : G;
}

void launch_sell_bits(hipStream_t s, const SellView &sv, int mode, bool unit, bool batched,
                      int ncols, const float *v, const uint32_t *bits, float *part, int m1,
                      const float *omega, const float *rt, const float *y_in, float *y_out,
                      float *wy, float tau2, const float *tau2_inst, const int *row_inst,
                      const float *x_in, float *x_out, float *xbar, const float *ct, float tau1,
                      const float *tau1_inst, const double *rho, const int *var_inst,
                      DevCounters *ctr, int nc) {
    if (sv.nchunk <= 0 || sv.P <= 0) return;
    const int G = sell_bits_blocks(sv, nc);
    const size_t lds = static_cast<size_t>(sv.ns / 32) * 4;
    const int blocks = G * sv.P;
#define GF_SB(U, M, B, N) k_sell_bits<U, M, B, N><<<blocks, 512, lds, s>>>(sv.nrows, sv.P, sv.nchunk, sv.ns, ncols, G, sv.ptr, sv.ci, sv.val, sv.row_of, v, bits, part, m1, omega, rt, y_in, y_out, wy, tau2, tau2_inst, row_inst, x_in, x_out, xbar, ct, tau1, tau1_inst, rho, var_inst, ctr)
#define GF_SB_N(U, M, B) if (nc >= 4) GF_SB(U, M, B, 4); else GF_SB(U, M, B, 2)
#define GF_SB_M(U, B) if (mode == 0) { GF_SB_N(U, 0, B); } else if (mode == 1) { GF_SB_N(U, 1, B); } else { GF_SB_N(U, 2, B); }
    if (unit) { if (batched) { GF_SB_M(true, true); } else { GF_SB_M(true, false); } }
    else { if (batched) { GF_SB_M(false, true); } else { GF_SB_M(false, false); } }
#undef GF_SB_M
#undef GF_SB_N
#undef GF_SB
}

// Primal step with the whole dual bitmap in LDS (persistent grid-stride over
// virtual blocks of 256 threads; no Q).
constexpr int kPrimalBatch = 8;   // entries per lane and load stage
template <int LPR, bool UNIT, bool BATCH>
__global__ void __launch_bounds__(1024)
k_primal_bits(int n, int m, int nvb, const int *__restrict__ rpT, const int *__restrict__ ciT,
              const int *__restrict__ valT, const float *__restrict__ wy,
              const uint32_t *__restrict__ bits, const float *__restrict__ x_in,
              float *__restrict__ x_out, float *__restrict__ xbar, const float *__restrict__ ct,
              float tau1, const float *__restrict__ tau1_inst, const double *__restrict__ rho,
              const int *__restrict__ var_inst, DevCounters *__restrict__ ctr,
              uint64_t *__restrict__ xbits, int deg) {
    extern __shared__ uint32_t sb[];
    const int nw = (m + 31) >> 5;
    load_bitmap_lds(sb, bits, nw);
    __syncthreads();
    if (blockIdx.x == 0 && threadIdx.x == 0) ctr->k += 1;
    for (int vb = blockIdx.x; vb < nvb; vb += gridDim.x) {
        const int tid = vb * 1024 + threadIdx.x;
        const int i = tid / LPR;
        const int sub = tid & (LPR - 1);
        float xi = 0.f, cti = 0.f, s1 = 0.f;
        int t = 0;
        if (i < n) {
            xi = x_in[i];
            cti = ct[i];
            if (BATCH) t = var_inst[i];
            // every variable with deg entries: its range is computed, not read
            const int eb0 = deg ? deg * i : rpT[i];
            const int e1 = deg ? eb0 + deg : rpT[i + 1];
            // batches of kPrimalBatch entries per lane, branch-free: row
            // indices first, then their bits, then the gathers of the nonzero
            // operands (a zero operand reads the padding element wy[m], shared
            // by the wavefront); terms are added in entry order
            for (int eb = eb0 + sub; eb < e1; eb += kPrimalBatch * LPR) {
                int j[kPrimalBatch], a[kPrimalBatch];
#pragma unroll
                for (int u = 0; u < kPrimalBatch; ++u) {
                    const int e = eb + u * LPR;
                    const int ec = min(e, e1 - 1);
                    const int jj = ciT[ec];
                    j[u] = e < e1 ? jj : m;
                    a[u] = UNIT ? 1 : valT[ec];
                }
                bool nz[kPrimalBatch];
#pragma unroll
                for (int u = 0; u < kPrimalBatch; ++u) {
                    const int jc = j[u] < m ? j[u] : 0;
                    nz[u] = (j[u] < m) & (((sb[jc >> 5] >> (jc & 31)) & 1u) != 0u);
                }
                float g[kPrimalBatch];
#pragma unroll
                for (int u = 0; u < kPrimalBatch; ++u) g[u] = wy[nz[u] ? j[u] : m];
#pragma unroll
                for (int u = 0; u < kPrimalBatch; ++u) {
                    const float tt = UNIT ? s1 + g[u] : fmaf(static_cast<float>(a[u]), g[u], s1);
                    s1 = nz[u] ? tt : s1;
                }
            }
        }
        s1 = group_sum<LPR>(s1);
        float xb = 0.f;
        if (i < n && sub == 0) {
            const float rh = static_cast<float>(rho[t]);
            const float ta = BATCH ? tau1_inst[t] : tau1;
            const float g = cti + rh - s1 - 2.f * rh * xi;
            const float xn = fminf(fmaxf(xi - ta * g, 0.f), 1.f);
            x_out[i] = xn;
            xb = 2.f * xn - xi;
            xbar[i] = xb;
        }
        // nonzero bitmap of xbar for the next dual step: the wavefront's 64/LPR
        // consecutive variables (variable i0 + l sits in lane l * LPR) become
        // 64/LPR bits, stored as whole bytes at bit offset i0
        if (LPR <= 8 && xbits) {
            constexpr int VW = 64 / LPR;
            const int lane = threadIdx.x & 63;
            const float vv = __shfl(xb, (lane % VW) * LPR, 64);
            const uint64_t bal = __ballot(lane < VW && vv != 0.f);
            const int64_t i0 = (static_cast<int64_t>(vb) * 1024 + (threadIdx.x & ~63)) / LPR;
            if (lane == 0 && i0 < n) {
                uint8_t *dst = reinterpret_cast<uint8_t *>(xbits) + (i0 >> 3);
                if (VW == 64) *reinterpret_cast<uint64_t *>(dst) = bal;
                else if (VW == 32) *reinterpret_cast<uint32_t *>(dst) = static_cast<uint32_t>(bal);
                else if (VW == 16) *reinterpret_cast<uint16_t *>(dst) = static_cast<uint16_t>(bal);
                else *dst = static_cast<uint8_t>(bal);
            }
        }
    }
}

template <int LPR>
static void primal_bits_lpr(hipStream_t s, bool unit, bool batched, int n, int m,
                            const int *rpT, const int *ciT, const int *valT, const float *wy,
                            const uint32_t *bits, const float *x_in, float *x_out, float *xbar,
                            const float *ct, float tau1, const float *tau1_inst,
                            const double *rho, const int *var_inst, DevCounters *ctr,
                            uint64_t *xbits, int deg) {
    const int64_t nvb64 = (static_cast<int64_t>(n) * LPR + 1023) / 1024;
    const int nvb = static_cast<int>(nvb64);
    const int grid = nvb < 512 ? nvb : 512;   // two 16-wave workgroups per CU
    const size_t lds = static_cast<size_t>((m + 31) / 32) * 4;
    if (grid <= 0) return;
#define GF_PB(U, B) k_primal_bits<LPR, U, B><<<grid, 1024, lds, s>>>(n, m, nvb, rpT, ciT, valT, wy, bits, x_in, x_out, xbar, ct, tau1, tau1_inst, rho, var_inst, ctr, xbits, deg)
    if (unit) { if (batched) GF_PB(true, true); else GF_PB(true, false); }
    else { if (batched) GF_PB(false, true); else GF_PB(false, false); }
#undef GF_PB
}

void launch_primal_bits(hipStream_t s, int lpr, bool unit, bool batched, int n, int m,
                        const int *rpT, const int *ciT, const int *valT, const float *wy,
                        const uint32_t *bits, const float *x_in, float *x_out, float *xbar,
                        const float *ct, float tau1, const float *tau1_inst, const double *rho,
                        const int *var_inst, DevCounters *ctr, uint64_t *xbits, int deg) {
    switch (lpr) {
#define GF_CASE(L) case L: primal_bits_lpr<L>(s, unit, batched, n, m, rpT, ciT, valT, wy, bits, x_in, x_out, xbar, ct, tau1, tau1_inst, rho, var_inst, ctr, xbits, deg); break;
        GF_CASE(1) GF_CASE(2) GF_CASE(4) GF_CASE(8) GF_CASE(16) GF_CASE(32) GF_CASE(64)
#undef GF_CASE
        default: break;
    }
}

// ---------------------------------------------------------------------------
// Primal step with the dual vector staged in LDS (unit coefficients, every
// variable in exactly DEG rows, one instance, no Q).  The random gathers of
// wy are the cost of the plain kernels: each is an L1 -> L2 request.  Here a
// workgroup owns VPT x 1024 consecutive variables (thread t: variables
// i0 + 1024 v + t), keeps their DEG row indices in registers (read once from
// an entry-major copy, ell[u n + i]), and walks the rows in slices of SL: the
// slice of wy is loaded into LDS with coalesced 16-byte loads (the next slice
// is in flight while the current one is used: two LDS buffers), and every
// variable consumes its entries that fall in the slice from LDS.  A
// variable's rows are ascending, so its terms are added in entry order, as in
// the plain kernels.  The epilogue is the one of k_primal (box projection,
// extrapolation) plus the nonzero bitmap of xbar for the next dual step.
// ---------------------------------------------------------------------------
template <int VPT, int DEG>
__global__ void __launch_bounds__(1024)
k_primal_lds(int n, int m, int SL, const int *__restrict__ ell, const float *__restrict__ wy,
             const float *__restrict__ x_in, float *__restrict__ x_out, float *__restrict__ xbar,
             const float *__restrict__ ct, float tau1, const double *__restrict__ rho,
             DevCounters *__restrict__ ctr, uint64_t *__restrict__ xbits) {
    extern __shared__ float4 stage4[];
    float *stage = reinterpret_cast<float *>(stage4);
    const int t = static_cast<int>(threadIdx.x);
    const int64_t i0 = static_cast<int64_t>(blockIdx.x) * (VPT * 1024);
    if (blockIdx.x == 0 && t == 0) ctr->k += 1;
    int row[VPT][DEG];
    float sum[VPT];
#pragma unroll
    for (int v = 0; v < VPT; ++v) {
        const int64_t i = i0 + v * 1024 + t;
        sum[v] = 0.f;
#pragma unroll
        for (int u = 0; u < DEG; ++u) row[v][u] = i < n ? ell[static_cast<int64_t>(u) * n + i] : 0x7fffffff;
    }
    const int nslice = (m + SL - 1) / SL;
    const int q4 = SL / 4096;   // float4 loads per thread per slice (SL a multiple of 4096)
    float4 pre[4];
    auto fetch = [&](int sl) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            if (q >= q4) break;
            const int e = sl * SL + (q * 1024 + t) * 4;   // first row of this float4
            if (e + 3 < m) pre[q] = *reinterpret_cast<const float4 *>(wy + e);
            else {
                pre[q].x = e < m ? wy[e] : 0.f;
                pre[q].y = e + 1 < m ? wy[e + 1] : 0.f;
                pre[q].z = e + 2 < m ? wy[e + 2] : 0.f;
                pre[q].w = 0.f;
            }
        }
    };
    auto put = [&](int buf) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            if (q >= q4) break;
            stage4[buf * (SL / 4) + q * 1024 + t] = pre[q];
        }
    };
    fetch(0);
    put(0);
    __syncthreads();
    for (int sl = 0; sl < nslice; ++sl) {
        if (sl + 1 < nslice) fetch(sl + 1);
        const float *cur = stage + (sl & 1) * SL;
        const int lo = sl * SL, hi = lo + SL;
#pragma unroll
        for (int v = 0; v < VPT; ++v) {
#pragma unroll
            for (int u = 0; u < DEG; ++u) {
                if (row[v][0] >= hi) break;
                sum[v] += cur[row[v][0] - lo];
#pragma unroll
                for (int w = 0; w < DEG - 1; ++w) row[v][w] = row[v][w + 1];
                row[v][DEG - 1] = 0x7fffffff;
            }
        }
        if (sl + 1 < nslice) put((sl + 1) & 1);
        __syncthreads();
    }
    const float rh = static_cast<float>(rho[0]);
    const int lane = t & 63;
#pragma unroll
    for (int v = 0; v < VPT; ++v) {
        const int64_t i = i0 + v * 1024 + t;
        float xb = 0.f;
        if (i < n) {
            const float xi = x_in[i];
            const float g = ct[i] + rh - sum[v] - 2.f * rh * xi;
            const float xn = fminf(fmaxf(xi - tau1 * g, 0.f), 1.f);
            x_out[i] = xn;
            xb = 2.f * xn - xi;
            xbar[i] = xb;
        }
        if (xbits) {
            const uint64_t bal = __ballot(i < n && xb != 0.f);
            const int64_t w0 = i0 + v * 1024 + (t & ~63);
            if (lane == 0 && w0 < n) xbits[w0 >> 6] = bal;
        }
    }
}

// Rows per LDS slice of k_primal_lds for a workgroup LDS limit (two buffers).
int primal_lds_slice(size_t lds_limit) {
    if (lds_limit >= 2 * 16384 * sizeof(float)) return 16384;
    if (lds_limit >= 2 * 8192 * sizeof(float)) return 8192;
    return 4096;
}

bool launch_primal_lds(hipStream_t s, int n, int m, int deg, int SL, const int *ell, const float *wy,
                       const float *x_in, float *x_out, float *xbar, const float *ct, float tau1,
                       const double *rho, DevCounters *ctr, uint64_t *xbits) {
    constexpr int VPT = 8;
    const int grid = static_cast<int>((static_cast<int64_t>(n) + VPT * 1024 - 1) / (VPT * 1024));
    const size_t lds = 2 * static_cast<size_t>(SL) * sizeof(float);
    if (grid == 0) return true;
    switch (deg) {
#define GF_PL(D) case D: k_primal_lds<VPT, D><<<grid, 1024, lds, s>>>(n, m, SL, ell, wy, x_in, x_out, xbar, ct, tau1, rho, ctr, xbits); return true;
        GF_PL(1) GF_PL(2) GF_PL(3) GF_PL(4) GF_PL(5) GF_PL(6) GF_PL(7) GF_PL(8)
#undef GF_PL
        default: return false;
    }
}

// ---------------------------------------------------------------------------
// Light part with signed indices (one instance, every |a| = 1, no Q): the rows
// (dual) or variables (primal) with fewer than kHeavyLen entries lie in a
// range [i0, i0 + L) and have D entries each, stored entry-major with the
// coefficient's sign in bit 31 (sidx[u L + k] = index of entry u of item
// i0 + k, negative when a = -1); a heavy item inside the range is a hole
// (sidx[k] = kLightHole) left to its workgroup kernel.  A lane per item loads its D indices with
// coalesced loads and reads neither row pointers nor coefficients; the terms
// are added in entry order (a +-1 product is exact, so the sums equal the CSR
// kernels' with one lane per item).  The heavy items keep their
// workgroup-per-item kernels.
// ---------------------------------------------------------------------------
template <int D>
__global__ void __launch_bounds__(256)
k_dual_light(int i0, int L, int m1, const int *__restrict__ sidx, const float *__restrict__ omega,
             const float *__restrict__ rt, const float *__restrict__ xbar, const float *__restrict__ y_in,
             float *__restrict__ y_out, float *__restrict__ wy, float tau2) {
    const int k = blockIdx.x * 256 + threadIdx.x;
    if (k >= L) return;
    int c[D];
#pragma unroll
    for (int u = 0; u < D; ++u) c[u] = sidx[static_cast<int64_t>(u) * L + k];
    if (c[0] == kLightHole) return;   // a heavy row: its workgroup kernel updates it
    float g[D];
#pragma unroll
    for (int u = 0; u < D; ++u) g[u] = xbar[c[u] & 0x7fffffff];
    float sum = 0.f;
#pragma unroll
    for (int u = 0; u < D; ++u) sum += c[u] < 0 ? -g[u] : g[u];
    const int row = i0 + k;
    const float om = omega[row];
    const float t = rt[row] - om * sum;
    float y = y_in[row] + tau2 * t;
    if (row < m1) y = fmaxf(y, 0.f);
    y_out[row] = y;
    wy[row] = om * y;
}

// xbits (optional, only when the light range is every variable): the nonzero
// bitmap of the new xbar for the zero-skipping dual, one word per wavefront.
template <int D>
__global__ void __launch_bounds__(256)
k_primal_light(int i0, int L, const int *__restrict__ sidx, const float *__restrict__ wy,
               const float *__restrict__ x_in, float *__restrict__ x_out, float *__restrict__ xbar,
               const float *__restrict__ ct, float tau1, const double *__restrict__ rho,
               DevCounters *__restrict__ ctr, uint64_t *__restrict__ xbits) {
    const int k = blockIdx.x * 256 + threadIdx.x;
    if (k == 0) ctr->k += 1;
    float xb = 0.f;
    const bool live = k < L && sidx[k] != kLightHole;   // holes: heavy variables, updated elsewhere
    if (live) {
        const int i = i0 + k;
        const float xi = x_in[i], cti = ct[i];
        int c[D];
#pragma unroll
        for (int u = 0; u < D; ++u) c[u] = sidx[static_cast<int64_t>(u) * L + k];
        float g[D];
#pragma unroll
        for (int u = 0; u < D; ++u) g[u] = wy[c[u] & 0x7fffffff];
        float sum = 0.f;
#pragma unroll
        for (int u = 0; u < D; ++u) sum += c[u] < 0 ? -g[u] : g[u];
        const float rh = static_cast<float>(rho[0]);
        float gr = cti + rh;
        gr -= sum;
        gr -= 2.f * rh * xi;
        const float xn = fminf(fmaxf(xi - tau1 * gr, 0.f), 1.f);
        x_out[i] = xn;
        xb = 2.f * xn - xi;
        xbar[i] = xb;
    }
    if (xbits) {
        const uint64_t bal = __ballot(live && xb != 0.f);
        if ((threadIdx.x & 63) == 0 && k < L) xbits[k >> 6] = bal;
    }
}

// Heavy variables in groups of up to kHgWidth (16) consecutive ones whose
// rows are unit shifts of each other (variable v0 + d has rows r + d for the
// rows r of v0, with the same coefficients: the facilities of a facility
// location, whose link rows are numbered customer-major).  A workgroup takes a
// chunk of a group's entries: 256 / kHgWidth entry slots x kHgWidth
// variables, lane (q, d) adds a_e wy[r_e + d] over its slot's entries of the
// chunk, so the lanes of one entry read consecutive floats (one request
// instead of kHgWidth gathers).  The chunk's slot sums are added in slot order;
// k_primal_hgroup_fin adds a variable's chunk sums in chunk order and applies
// the primal update.
// Workgroup b takes chunk ord[b] (-1: none): the host places the chunks of
// two neighbouring groups, which share the 128-byte lines of wy, eight slots
// apart, so that both run on one XCD (workgroup b runs on XCD b % 8) at about
// the same time and fetch each line into one L2 once.
template <bool UNIT>
__global__ void __launch_bounds__(256)
k_primal_hgroup(const int *__restrict__ ord, const int *__restrict__ ch_g, const int *__restrict__ ch_b,
                const int *__restrict__ ch_e, const int *__restrict__ hg_w, const int *__restrict__ hg_e0,
                const int *__restrict__ ciT, const int *__restrict__ valT, const float *__restrict__ wy,
                float *__restrict__ part) {
    constexpr int NS = 256 / kHgWidth;   // entry slots
    __shared__ float red[NS][kHgWidth + 1];
    const int c = ord[blockIdx.x];
    if (c < 0) return;                   // padding slot (whole workgroup, before any barrier)
    const int g = ch_g[c];
    const int d = threadIdx.x % kHgWidth, q = threadIdx.x / kHgWidth;
    const int w = hg_w[g], base = hg_e0[g];
    const int b1 = ch_e[c];
    float acc = 0.f;
    for (int e = ch_b[c] + q; e < b1; e += NS * kLongUnroll) {
        int r[kLongUnroll], a[kLongUnroll];
#pragma unroll
        for (int u = 0; u < kLongUnroll; ++u) {
            const int ee = e + NS * u;
            const bool in = ee < b1;
            r[u] = in ? ciT[base + ee] : 0;
            a[u] = UNIT ? (in ? 1 : 0) : (in ? valT[base + ee] : 0);
        }
        float v[kLongUnroll];
#pragma unroll
        for (int u = 0; u < kLongUnroll; ++u) v[u] = (a[u] != 0 && d < w) ? wy[r[u] + d] : 0.f;
#pragma unroll
        for (int u = 0; u < kLongUnroll; ++u) acc = fmaf(static_cast<float>(a[u]), v[u], acc);
    }
    red[q][d] = acc;
    __syncthreads();
    if (threadIdx.x < kHgWidth) {
        float sum = 0.f;
#pragma unroll
        for (int k = 0; k < NS; ++k) sum += red[k][threadIdx.x];
        part[static_cast<int64_t>(c) * kHgWidth + threadIdx.x] = sum;
    }
}

__global__ void __launch_bounds__(256)
k_primal_hgroup_fin(int ngroup, const int *__restrict__ hg_var0, const int *__restrict__ hg_w,
                    const int *__restrict__ hg_c0, const float *__restrict__ part,
                    const float *__restrict__ x_in, float *__restrict__ x_out, float *__restrict__ xbar,
                    const float *__restrict__ ct, float tau1, const double *__restrict__ rho) {
    const int tid = blockIdx.x * 256 + threadIdx.x;
    const int g = tid / kHgWidth, d = tid % kHgWidth;
    if (g >= ngroup || d >= hg_w[g]) return;
    const int c0 = hg_c0[g], c1 = hg_c0[g + 1];
    const float *pr = part + static_cast<int64_t>(c0) * kHgWidth + d;
    float tot = 0.f;
    int c = 0;
    for (; c + 8 <= c1 - c0; c += 8) {
        float v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = pr[static_cast<int64_t>(c + u) * kHgWidth];
#pragma unroll
        for (int u = 0; u < 8; ++u) tot += v[u];
    }
    for (; c < c1 - c0; ++c) tot += pr[static_cast<int64_t>(c) * kHgWidth];
    const int i = hg_var0[g] + d;
    const float xi = x_in[i];
    const float rh = static_cast<float>(rho[0]);
    const float gr = ct[i] + rh - tot - 2.f * rh * xi;
    const float xn = fminf(fmaxf(xi - tau1 * gr, 0.f), 1.f);
    x_out[i] = xn;
    xbar[i] = 2.f * xn - xi;
}

void launch_primal_hgroup(hipStream_t s, bool unit, int nslot, int ngroup, const int *ord, const int *ch_g,
                          const int *ch_b, const int *ch_e, const int *hg_var0, const int *hg_w, const int *hg_e0,
                          const int *hg_c0, const int *ciT, const int *valT, const float *wy, float *part,
                          const float *x_in, float *x_out, float *xbar, const float *ct, float tau1,
                          const double *rho) {
    if (nslot <= 0 || ngroup <= 0) return;
    if (unit) k_primal_hgroup<true><<<nslot, 256, 0, s>>>(ord, ch_g, ch_b, ch_e, hg_w, hg_e0, ciT, valT, wy, part);
    else k_primal_hgroup<false><<<nslot, 256, 0, s>>>(ord, ch_g, ch_b, ch_e, hg_w, hg_e0, ciT, valT, wy, part);
    k_primal_hgroup_fin<<<(ngroup * kHgWidth + 255) / 256, 256, 0, s>>>(ngroup, hg_var0, hg_w, hg_c0, part, x_in, x_out,
                                                                   xbar, ct, tau1, rho);
}

void launch_dual_light(hipStream_t s, int D, int i0, int L, int m1, const int *sidx, const float *omega,
                       const float *rt, const float *xbar, const float *y_in, float *y_out, float *wy,
                       float tau2) {
    const int blocks = (L + 255) / 256;
    if (blocks == 0) return;
    switch (D) {
#define GF_DL(DD) case DD: k_dual_light<DD><<<blocks, 256, 0, s>>>(i0, L, m1, sidx, omega, rt, xbar, y_in, y_out, wy, tau2); break;
        GF_DL(1) GF_DL(2) GF_DL(3) GF_DL(4) GF_DL(5) GF_DL(6) GF_DL(7) GF_DL(8)
#undef GF_DL
        default: break;
    }
}

void launch_primal_light(hipStream_t s, int D, int i0, int L, const int *sidx, const float *wy,
                         const float *x_in, float *x_out, float *xbar, const float *ct, float tau1,
                         const double *rho, DevCounters *ctr, uint64_t *xbits) {
    const int blocks = (L + 255) / 256;
    if (blocks == 0) return;
    switch (D) {
#define GF_PLG(DD) case DD: k_primal_light<DD><<<blocks, 256, 0, s>>>(i0, L, sidx, wy, x_in, x_out, xbar, ct, tau1, rho, ctr, xbits); break;
        GF_PLG(1) GF_PLG(2) GF_PLG(3) GF_PLG(4) GF_PLG(5) GF_PLG(6) GF_PLG(7) GF_PLG(8)
#undef GF_PLG
        default: break;
    }
}

// ---------------------------------------------------------------------------
// Dense-block SpMVs for batched instances whose rows are dense over their
// instance's variables (every row of instance t has the columns
// v0_t .. v0_t + n_t - 1 in order, at most 64 rows per instance, no Q): the
// knapsack batch.  A tile is kBlkCols consecutive columns of one instance
// (2,048: tiles of 4,096 and a persistent grid over the tiles were measured
// slower); thread t of its workgroup owns the columns c0 + 256 k + t
// (k < kBlkCols / 256).
//   dual:   per tile, xbar of the tile is loaded once into registers and every
//           row of the instance streams its coefficients over it; the row's
//           tile sum (lanes, then the 4 wavefronts in order) goes to pp; a
//           combine kernel adds a row's tile sums in tile order and applies
//           the dual update.  The row kernels re-read xbar per row instead.
//   primal: per tile, wy of the instance's rows sits in LDS and each column
//           adds a_rc wy_r over the rows in order (the order of the CSR
//           kernels), then the primal update of its 8 columns.
// ---------------------------------------------------------------------------
constexpr int kBlkCols = kBlockCols;
constexpr int kBlkGrid = 1 << 30;   // one tile per workgroup (measured faster than a persistent grid)

// The same two kernels over a padded int16 copy of the coefficients (each
// row of an instance at a multiple of 8 entries, zeros past its end): thread
// t owns the kBlkCols / 256 consecutive columns from c0 + (kBlkCols / 256) t
// and reads their coefficients of a row with aligned 16-byte loads; xbar of
// the tile and the primal's column sums pass through LDS so that the
// global loads and stores stay coalesced.
__device__ __forceinline__ void unpack8(const int4 q, float *a) {
    const uint32_t w[4] = {static_cast<uint32_t>(q.x), static_cast<uint32_t>(q.y), static_cast<uint32_t>(q.z),
                           static_cast<uint32_t>(q.w)};
#pragma unroll
    for (int h = 0; h < 4; ++h) {
        a[2 * h] = static_cast<float>(static_cast<int16_t>(w[h] & 0xffffu));
        a[2 * h + 1] = static_cast<float>(static_cast<int16_t>(w[h] >> 16));
    }
}

__global__ void __launch_bounds__(256)
k_dual_block16(int ntile, const int *__restrict__ tile_inst, const int *__restrict__ tile_c0,
               const int *__restrict__ blk_row0, const int *__restrict__ blk_nrow,
               const int64_t *__restrict__ pbase, const int64_t *__restrict__ inst_var0,
               const int64_t *__restrict__ inst_nvar, const int16_t *__restrict__ pval,
               const float *__restrict__ xbar, float *__restrict__ pp) {
    __shared__ float red[4][64];
    __shared__ float4 xs4[kBlkCols / 4];
    constexpr int CPT = kBlkCols / 256;   // consecutive columns per thread (a multiple of 8)
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    float *xs = reinterpret_cast<float *>(xs4);
    // the launch gives every tile its own workgroup (kBlkGrid); the loop
    // also serves a smaller grid
    for (int g = blockIdx.x; g < ntile; g += gridDim.x) {
        const int t = tile_inst[g];
        const int v0 = static_cast<int>(inst_var0[t]);
        const int c0 = tile_c0[g], c1 = min(c0 + kBlkCols, v0 + static_cast<int>(inst_nvar[t]));
        const int nr = blk_nrow[t], r0 = blk_row0[t];
        // the tile's xbar: coalesced loads into LDS, then CPT consecutive values per thread
#pragma unroll
        for (int k = 0; k < CPT; ++k) {
            const int c = c0 + 256 * k + tid;
            xs[256 * k + tid] = c < c1 ? xbar[c] : 0.f;
        }
        __syncthreads();
        const int cb = c0 + CPT * tid;
        float xv[CPT];
#pragma unroll
        for (int h = 0; h < CPT / 4; ++h) {
            const float4 a = xs4[(CPT / 4) * tid + h];
            xv[4 * h] = a.x; xv[4 * h + 1] = a.y; xv[4 * h + 2] = a.z; xv[4 * h + 3] = a.w;
        }
        const int coff = cb - v0;
#pragma unroll 4
        for (int r = 0; r < nr; ++r) {
            float sacc = 0.f;
            if (cb < c1) {
                const int4 *q4 = reinterpret_cast<const int4 *>(pval + pbase[r0 + r] + coff);
#pragma unroll
                for (int h = 0; h < CPT / 8; ++h) {
                    if (cb + 8 * h >= c1) break;
                    float a[8];
                    unpack8(q4[h], a);
#pragma unroll
                    for (int k = 0; k < 8; ++k) sacc = fmaf(a[k], xv[8 * h + k], sacc);
                }
            }
            sacc = group_sum<64>(sacc);
            if (lane == 0) red[wv][r] = sacc;
        }
        __syncthreads();
        if (tid < nr) pp[static_cast<int64_t>(g) * 64 + tid] = ((red[0][tid] + red[1][tid]) + red[2][tid]) + red[3][tid];
        __syncthreads();   // red and xs are reused by the next tile
    }
}

__global__ void __launch_bounds__(256)
k_primal_block16(int ntile, const int *__restrict__ tile_inst, const int *__restrict__ tile_c0,
                 const int *__restrict__ blk_row0, const int *__restrict__ blk_nrow,
                 const int *__restrict__ blk_rows, const int64_t *__restrict__ pbase,
                 const int64_t *__restrict__ inst_var0, const int64_t *__restrict__ inst_nvar,
                 const int16_t *__restrict__ pval, const float *__restrict__ wy, const float *__restrict__ x_in,
                 float *__restrict__ x_out, float *__restrict__ xbar, const float *__restrict__ ct,
                 const float *__restrict__ tau1_inst, const double *__restrict__ rho,
                 DevCounters *__restrict__ ctr) {
    __shared__ float wys[64];
    __shared__ float4 gs4[kBlkCols / 4];
    constexpr int CPT = kBlkCols / 256;
    const int tid = threadIdx.x;
    if (blockIdx.x == 0 && tid == 0) ctr->k += 1;
    const float *gsum = reinterpret_cast<const float *>(gs4);
    for (int g = blockIdx.x; g < ntile; g += gridDim.x) {
        const int t = tile_inst[g];
        const int v0 = static_cast<int>(inst_var0[t]);
        const int c0 = tile_c0[g], c1 = min(c0 + kBlkCols, v0 + static_cast<int>(inst_nvar[t]));
        const int nr = blk_nrow[t], r0 = blk_row0[t];
        if (tid < nr) wys[tid] = wy[blk_rows[r0 + tid]];
        __syncthreads();
        const int cb = c0 + CPT * tid;
        const int coff = cb - v0;
        float acc[CPT];
#pragma unroll
        for (int k = 0; k < CPT; ++k) acc[k] = 0.f;
        if (cb < c1) {
#pragma unroll 4
            for (int r = 0; r < nr; ++r) {
                const int4 *q4 = reinterpret_cast<const int4 *>(pval + pbase[r0 + r] + coff);
                const float w = wys[r];
#pragma unroll
                for (int h = 0; h < CPT / 8; ++h) {
                    if (cb + 8 * h >= c1) break;
                    float a[8];
                    unpack8(q4[h], a);
#pragma unroll
                    for (int k = 0; k < 8; ++k) acc[8 * h + k] = fmaf(a[k], w, acc[8 * h + k]);
                }
            }
        }
        // through LDS, so that the epilogue's loads and stores are coalesced
#pragma unroll
        for (int h = 0; h < CPT / 4; ++h)
            gs4[(CPT / 4) * tid + h] = make_float4(acc[4 * h], acc[4 * h + 1], acc[4 * h + 2], acc[4 * h + 3]);
        __syncthreads();
        const float rh = static_cast<float>(rho[t]);
        const float ta = tau1_inst[t];
#pragma unroll
        for (int k = 0; k < CPT; ++k) {
            const int c = c0 + 256 * k + tid;
            if (c >= c1) break;
            const float xi = x_in[c];
            float gr = ct[c] + rh;
            gr -= gsum[256 * k + tid];
            gr -= 2.f * rh * xi;
            const float xn = fminf(fmaxf(xi - ta * gr, 0.f), 1.f);
            x_out[c] = xn;
            xbar[c] = 2.f * xn - xi;
        }
        __syncthreads();   // wys and gs4 are reused by the next tile
    }
}

template <typename VT>
__global__ void __launch_bounds__(256)
k_dual_block(const int *__restrict__ tile_inst, const int *__restrict__ tile_c0,
             const int *__restrict__ blk_row0, const int *__restrict__ blk_nrow,
             const int *__restrict__ blk_rows, const int *__restrict__ rp,
             const int64_t *__restrict__ inst_var0, const int64_t *__restrict__ inst_nvar,
             const VT *__restrict__ val, const float *__restrict__ xbar, float *__restrict__ pp) {
    __shared__ float red[4][64];
    __shared__ int rbase[64];
    const int g = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int t = tile_inst[g];
    const int v0 = static_cast<int>(inst_var0[t]);
    const int c0 = tile_c0[g], c1 = min(c0 + kBlkCols, v0 + static_cast<int>(inst_nvar[t]));
    const int nr = blk_nrow[t], r0 = blk_row0[t];
    // the rows' first entries, once: the row loop then issues only coefficient loads
    if (tid < nr) rbase[tid] = rp[blk_rows[r0 + tid]];
    constexpr int CPT = kBlkCols / 256;
    float xv[CPT];
    int off[CPT];
#pragma unroll
    for (int k = 0; k < CPT; ++k) {
        const int c = c0 + 256 * k + tid;
        xv[k] = c < c1 ? xbar[c] : 0.f;
        off[k] = c < c1 ? c - v0 : 0;
    }
    __syncthreads();
#pragma unroll 2
    for (int r = 0; r < nr; ++r) {
        const VT *a = val + rbase[r];
        float sacc = 0.f;
#pragma unroll
        for (int k = 0; k < CPT; ++k) sacc = fmaf(static_cast<float>(a[off[k]]), xv[k], sacc);
        sacc = group_sum<64>(sacc);
        if (lane == 0) red[wv][r] = sacc;
    }
    __syncthreads();
    if (tid < nr) pp[static_cast<int64_t>(g) * 64 + tid] = ((red[0][tid] + red[1][tid]) + red[2][tid]) + red[3][tid];
}

__global__ void __launch_bounds__(256)
k_dual_block_combine(int m, int m1, const int *__restrict__ row_inst, const int *__restrict__ row_rank,
                     const int *__restrict__ inst_tile0, const int *__restrict__ inst_ntile,
                     const float *__restrict__ pp, const float *__restrict__ omega,
                     const float *__restrict__ rt, const float *__restrict__ tau2_inst,
                     const float *__restrict__ y_in, float *__restrict__ y_out, float *__restrict__ wy) {
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= m) return;
    const int t = row_inst[j], rk = row_rank[j];
    const int g0 = inst_tile0[t], ng = inst_ntile[t];
    const float *pr = pp + static_cast<int64_t>(g0) * 64 + rk;
    // the tile sums in tile order; eight loads issued before their adds, so
    // the chain waits on one memory latency per eight tiles, not per tile
    float sacc = 0.f;
    int q = 0;
    for (; q + 8 <= ng; q += 8) {
        float v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = pr[static_cast<int64_t>(q + u) * 64];
#pragma unroll
        for (int u = 0; u < 8; ++u) sacc += v[u];
    }
    for (; q < ng; ++q) sacc += pr[static_cast<int64_t>(q) * 64];
    const float om = omega[j];
    float y = y_in[j] + tau2_inst[t] * (rt[j] - om * sacc);
    if (j < m1) y = fmaxf(y, 0.f);
    y_out[j] = y;
    wy[j] = om * y;
}

template <typename VT>
__global__ void __launch_bounds__(256)
k_primal_block(const int *__restrict__ tile_inst, const int *__restrict__ tile_c0,
               const int *__restrict__ blk_row0, const int *__restrict__ blk_nrow,
               const int *__restrict__ blk_rows, const int *__restrict__ rp,
               const int64_t *__restrict__ inst_var0, const int64_t *__restrict__ inst_nvar,
               const VT *__restrict__ val, const float *__restrict__ wy, const float *__restrict__ x_in,
               float *__restrict__ x_out, float *__restrict__ xbar, const float *__restrict__ ct,
               const float *__restrict__ tau1_inst, const double *__restrict__ rho,
               DevCounters *__restrict__ ctr) {
    __shared__ float wys[64];
    __shared__ int rbase[64];
    const int g = blockIdx.x, tid = threadIdx.x;
    const int t = tile_inst[g];
    const int v0 = static_cast<int>(inst_var0[t]);
    const int c0 = tile_c0[g], c1 = min(c0 + kBlkCols, v0 + static_cast<int>(inst_nvar[t]));
    const int nr = blk_nrow[t], r0 = blk_row0[t];
    if (tid < nr) {
        const int j = blk_rows[r0 + tid];
        wys[tid] = wy[j];
        rbase[tid] = rp[j];
    }
    if (g == 0 && tid == 0) ctr->k += 1;
    __syncthreads();
    constexpr int CPT = kBlkCols / 256;
    float acc[CPT];
    int off[CPT];
#pragma unroll
    for (int k = 0; k < CPT; ++k) {
        const int c = c0 + 256 * k + tid;
        acc[k] = 0.f;
        off[k] = c < c1 ? c - v0 : 0;
    }
#pragma unroll 2
    for (int r = 0; r < nr; ++r) {
        const VT *a = val + rbase[r];
        const float w = wys[r];
#pragma unroll
        for (int k = 0; k < CPT; ++k) acc[k] = fmaf(static_cast<float>(a[off[k]]), w, acc[k]);
    }
    const float rh = static_cast<float>(rho[t]);
    const float ta = tau1_inst[t];
#pragma unroll
    for (int k = 0; k < CPT; ++k) {
        const int c = c0 + 256 * k + tid;
        if (c >= c1) continue;
        const float xi = x_in[c];
        float gr = ct[c] + rh;
        gr -= acc[k];
        gr -= 2.f * rh * xi;
        const float xn = fminf(fmaxf(xi - ta * gr, 0.f), 1.f);
        x_out[c] = xn;
        xbar[c] = 2.f * xn - xi;
    }
}

void launch_dual_block(hipStream_t s, const BlockView &b, int m, int m1, const int *rp, const int *val,
                       const int16_t *val16, const int64_t *inst_var0, const int64_t *inst_nvar,
                       const float *xbar, const float *omega, const float *rt, const float *tau2_inst,
                       const int *row_inst, const float *y_in, float *y_out, float *wy) {
    if (b.ntile <= 0) return;
    if (b.pval)
        k_dual_block16<<<std::min(b.ntile, kBlkGrid), 256, 0, s>>>(b.ntile, b.tile_inst, b.tile_c0, b.row0, b.nrow,
                                                                   b.pbase, inst_var0, inst_nvar, b.pval, xbar, b.pp);
    else if (val16)
        k_dual_block<int16_t><<<b.ntile, 256, 0, s>>>(b.tile_inst, b.tile_c0, b.row0, b.nrow, b.rows, rp, inst_var0,
                                                       inst_nvar, val16, xbar, b.pp);
    else
        k_dual_block<int><<<b.ntile, 256, 0, s>>>(b.tile_inst, b.tile_c0, b.row0, b.nrow, b.rows, rp, inst_var0,
                                                   inst_nvar, val, xbar, b.pp);
    k_dual_block_combine<<<(m + 255) / 256, 256, 0, s>>>(m, m1, row_inst, b.row_rank, b.inst_tile0, b.inst_ntile,
                                                         b.pp, omega, rt, tau2_inst, y_in, y_out, wy);
}

void launch_primal_block(hipStream_t s, const BlockView &b, const int *rp, const int *val, const int16_t *val16,
                         const int64_t *inst_var0, const int64_t *inst_nvar, const float *wy,
                         const float *x_in, float *x_out, float *xbar, const float *ct, const float *tau1_inst,
                         const double *rho, DevCounters *ctr) {
    if (b.ntile <= 0) return;
    if (b.pval)
        k_primal_block16<<<std::min(b.ntile, kBlkGrid), 256, 0, s>>>(b.ntile, b.tile_inst, b.tile_c0, b.row0, b.nrow,
                                                                     b.rows, b.pbase, inst_var0, inst_nvar, b.pval, wy,
                                                                     x_in, x_out, xbar, ct, tau1_inst, rho, ctr);
    else if (val16)
        k_primal_block<int16_t><<<b.ntile, 256, 0, s>>>(b.tile_inst, b.tile_c0, b.row0, b.nrow, b.rows, rp, inst_var0,
                                                         inst_nvar, val16, wy, x_in, x_out, xbar, ct, tau1_inst, rho,
                                                         ctr);
    else
        k_primal_block<int><<<b.ntile, 256, 0, s>>>(b.tile_inst, b.tile_c0, b.row0, b.nrow, b.rows, rp, inst_var0,
                                                     inst_nvar, val, wy, x_in, x_out, xbar, ct, tau1_inst, rho, ctr);
}

// ------------------------------------------------------------ small helpers
__global__ void k_copy_f32(float *__restrict__ d, const float *__restrict__ s, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        d[i] = s[i];
}
__global__ void k_fill_f32(float *__restrict__ d, float v, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        d[i] = v;
}
__global__ void k_set_xbar(int64_t n, const float *__restrict__ x, const float *__restrict__ xp,
                           float *__restrict__ xbar) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        xbar[i] = 2.f * x[i] - xp[i];
}
static int grid_for(int64_t n) {
    int64_t b = (n + 255) / 256;
    if (b > 4096) b = 4096;
    return static_cast<int>(b < 1 ? 1 : b);
}
void launch_copy_f32(hipStream_t s, float *dst, const float *src, int64_t n) {
    if (n > 0) k_copy_f32<<<grid_for(n), 256, 0, s>>>(dst, src, n);
}
void launch_fill_f32(hipStream_t s, float *dst, float v, int64_t n) {
    if (n > 0) k_fill_f32<<<grid_for(n), 256, 0, s>>>(dst, v, n);
}
void launch_set_xbar(hipStream_t s, int64_t n, const float *x, const float *xp, float *xbar) {
    if (n > 0) k_set_xbar<<<grid_for(n), 256, 0, s>>>(n, x, xp, xbar);
}

// ---------------------------------------------------------------------------
// FP64 pieces of Preprocess: w_r = rowscale_r * sum_e val_e v[col_e]
// (rowscale NULL = 1), one wavefront per row.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256)
k_spmv64(int nrows, const int *__restrict__ rp, const int *__restrict__ ci,
         const int *__restrict__ val, const double *__restrict__ rowscale,
         const double *__restrict__ v, double *__restrict__ w) {
    const int row = (blockIdx.x * blockDim.x + threadIdx.x) >> 4;
    const int sub = threadIdx.x & 15;
    double s = 0.0;
    if (row < nrows) {
        const int e1 = rp[row + 1];
        for (int e = rp[row] + sub; e < e1; e += 16)
            s += (val ? static_cast<double>(val[e]) : 1.0) * v[ci[e]];
    }
    s = group_sum<16>(s);
    if (row < nrows && sub == 0) w[row] = rowscale ? rowscale[row] * s : s;
}
void launch_spmv64(hipStream_t s, int nrows, const int *rp, const int *ci, const int *val,
                   const double *rowscale, const double *v, double *w) {
    const int64_t threads = static_cast<int64_t>(nrows) * 16;
    const int blocks = static_cast<int>((threads + 255) / 256);
    if (blocks) k_spmv64<<<blocks, 256, 0, s>>>(nrows, rp, ci, val, rowscale, v, w);
}

__global__ void k_scale64(int64_t n, double *__restrict__ x, const double *__restrict__ a,
                          double sign) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        x[i] = sign * a[i] * x[i];
}
void launch_scale64(hipStream_t s, int64_t n, double *x, const double *a, double sign) {
    if (n > 0) k_scale64<<<grid_for(n), 256, 0, s>>>(n, x, a, sign);
}
__global__ void k_fill64(double *__restrict__ x, double v, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        x[i] = v;
}
void launch_fill64(hipStream_t s, double *x, double v, int64_t n) {
    if (n > 0) k_fill64<<<grid_for(n), 256, 0, s>>>(x, v, n);
}

// Block reduction of a double over 256 threads.
__device__ __forceinline__ double block_sum256(double v, double *sh) {
    v = group_sum<64>(v);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) sh[wv] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0) r = sh[0] + sh[1] + sh[2] + sh[3];
    __syncthreads();
    return r;
}

// Sum of squares over each tile's contiguous range [b0, b1): part[tile].
__global__ void __launch_bounds__(256)
k_tile_sumsq(const int *__restrict__ b0, const int *__restrict__ b1,
             const double *__restrict__ x, double *__restrict__ part) {
    __shared__ double sh[4];
    const int t = blockIdx.x;
    double acc = 0.0;
    for (int i = b0[t] + threadIdx.x; i < b1[t]; i += 256) acc += x[i] * x[i];
    acc = block_sum256(acc, sh);
    if (threadIdx.x == 0) part[t] = acc;
}
void launch_tile_sumsq(hipStream_t s, const Tiles &t, const double *x, double *part) {
    if (t.count) k_tile_sumsq<<<t.count, 256, 0, s>>>(t.b0, t.b1, x, part);
}

// out[inst*out_stride] = sum over the instance's tiles of part[tile*stride + comp]
// (square-rooted if take_sqrt).  Fixed summation order: deterministic.
__global__ void __launch_bounds__(256)
k_inst_sum(const int *__restrict__ first, const double *__restrict__ part, int stride,
           int comp, double *__restrict__ out, int out_stride, int take_sqrt) {
    __shared__ double sh[4];
    const int inst = blockIdx.x;
    double acc = 0.0;
    for (int t = first[inst] + threadIdx.x; t < first[inst + 1]; t += 256)
        acc += part[(int64_t)t * stride + comp];
    acc = block_sum256(acc, sh);
    if (threadIdx.x == 0) out[(int64_t)inst * out_stride] = take_sqrt ? sqrt(acc) : acc;
}
void launch_inst_sum(hipStream_t s, int T, const Tiles &t, const double *part, int stride,
                     int comp, double *out, int out_stride, bool take_sqrt) {
    if (T) k_inst_sum<<<T, 256, 0, s>>>(t.first, part, stride, comp, out, out_stride, take_sqrt ? 1 : 0);
}

// x[i] /= nrm[inst(tile)] for each tile's range; a zero norm leaves x untouched.
__global__ void __launch_bounds__(256)
k_tile_scale_inv(const int *__restrict__ inst, const int *__restrict__ b0,
                 const int *__restrict__ b1, double *__restrict__ x,
                 const double *__restrict__ nrm) {
    const int t = blockIdx.x;
    const double v = nrm[inst[t]];
    if (v == 0.0) return;
    for (int i = b0[t] + threadIdx.x; i < b1[t]; i += 256) x[i] = x[i] / v;
}
void launch_tile_scale_inv(hipStream_t s, const Tiles &t, double *x, const double *nrm) {
    if (t.count) k_tile_scale_inv<<<t.count, 256, 0, s>>>(t.inst, t.b0, t.b1, x, nrm);
}

// ---------------------------------------------------------------------------
// FP64 residuals (Theorem 2; CheckHalt of Sec. 3), per row tile:
//   s^y_j   = (y_{k-1} - y_k)_j / tau2 + K~_j (xbar_{k-1} - x_k)
//   gap_j   = (K~ x_k + r~)_j, positive part on inequality rows
// part[tile*2 + {0,1}] = {sum (s^y)^2, sum gap^2}.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256)
k_res_rows(const int *__restrict__ tinst, const int *__restrict__ tb0,
           const int *__restrict__ tb1, int m1, const int *__restrict__ rp,
           const int *__restrict__ ci, const int *__restrict__ val,
           const double *__restrict__ omega64, const int64_t *__restrict__ rhs,
           const float *__restrict__ xsave, const float *__restrict__ x,
           const float *__restrict__ y_prev, const float *__restrict__ y,
           const double *__restrict__ tau2d, double *__restrict__ part) {
    __shared__ double sh[4];
    const int t = blockIdx.x;
    const double tau2 = tau2d[tinst[t]];
    const int sub = threadIdx.x & 15, grp = threadIdx.x >> 4;
    double a1 = 0.0, a2 = 0.0;
    for (int j0 = tb0[t]; j0 < tb1[t]; j0 += 16) {
        const int j = j0 + grp;
        double d1 = 0.0, d2 = 0.0;
        if (j < tb1[t]) {
            const int e1 = rp[j + 1];
            for (int e = rp[j] + sub; e < e1; e += 16) {
                const double a = val ? static_cast<double>(val[e]) : 1.0;
                const int c = ci[e];
                d1 += a * (static_cast<double>(xsave[c]) - static_cast<double>(x[c]));
                d2 += a * static_cast<double>(x[c]);
            }
        }
        d1 = group_sum<16>(d1);
        d2 = group_sum<16>(d2);
        if (j < tb1[t] && sub == 0) {
            const double om = omega64[j];
            const double sy = (static_cast<double>(y_prev[j]) - static_cast<double>(y[j])) / tau2 - om * d1;
            double g = om * (static_cast<double>(rhs[j]) - d2);
            if (j < m1 && g < 0.0) g = 0.0;
            a1 += sy * sy;
            a2 += g * g;
        }
    }
    a1 = block_sum256(a1, sh);
    a2 = block_sum256(a2, sh);
    if (threadIdx.x == 0) { part[2 * t] = a1; part[2 * t + 1] = a2; }
}
void launch_res_rows(hipStream_t s, const Tiles &rt, int m1, const int *rp, const int *ci,
                     const int *val, const double *omega64, const int64_t *rhs,
                     const float *xsave, const float *x, const float *y_prev,
                     const float *y, const double *tau2d, double *part) {
    if (rt.count)
        k_res_rows<<<rt.count, 256, 0, s>>>(rt.inst, rt.b0, rt.b1, m1, rp, ci, val, omega64, rhs,
                                             xsave, x, y_prev, y, tau2d, part);
}

// Per variable tile:  s^x_i = -dx_i/tau1 - 2 rho dx_i + (2/s_o) (Q dx)_i, dx = x_k - x_{k-1};
// binary gap x_i (1 - x_i).  part[tile*2 + {0,1}] = {sum (s^x)^2, sum x(1-x)}.
__global__ void __launch_bounds__(256)
k_res_vars(const int *__restrict__ tinst, const int *__restrict__ tb0,
           const int *__restrict__ tb1, const int *__restrict__ rpQ,
           const int *__restrict__ ciQ, const int *__restrict__ valQ,
           const float *__restrict__ x, const float *__restrict__ xp,
           const double *__restrict__ rho, const double *__restrict__ tau1d,
           const double *__restrict__ two_sod, double *__restrict__ part) {
    __shared__ double sh[4];
    const int t = blockIdx.x;
    const int inst = tinst[t];
    const double r = rho[inst], tau1 = tau1d[inst], tso = two_sod[inst];
    double a1 = 0.0, a2 = 0.0;
    for (int i = tb0[t] + threadIdx.x; i < tb1[t]; i += 256) {
        const double xi = x[i];
        const double dx = xi - static_cast<double>(xp[i]);
        double sx = -dx / tau1 - 2.0 * r * dx;
        if (rpQ) {
            double q = 0.0;
            for (int e = rpQ[i]; e < rpQ[i + 1]; ++e) {
                const int c = ciQ[e];
                q += static_cast<double>(valQ[e]) * (static_cast<double>(x[c]) - static_cast<double>(xp[c]));
            }
            sx += tso * q;
        }
        a1 += sx * sx;
        a2 += xi * (1.0 - xi);
    }
    a1 = block_sum256(a1, sh);
    a2 = block_sum256(a2, sh);
    if (threadIdx.x == 0) { part[2 * t] = a1; part[2 * t + 1] = a2; }
}
void launch_res_vars(hipStream_t s, const Tiles &vt, const int *rpQ, const int *ciQ,
                     const int *valQ, const float *x, const float *xp, const double *rho,
                     const double *tau1d, const double *two_sod, double *part) {
    if (vt.count)
        k_res_vars<<<vt.count, 256, 0, s>>>(vt.inst, vt.b0, vt.b1, rpQ, ciQ, valQ, x, xp, rho,
                                             tau1d, two_sod, part);
}

}  // namespace gfors
