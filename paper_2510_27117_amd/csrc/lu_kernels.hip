// Kernels of the factorised TU reformulation (Theorem and Remark of Sec. 2.4.1)
// for gfx950.  The reformulated matrix is never stored: its rows are the
// original rows on the lifted vector z = (xbar, t) with t = S xbar, and
//     t        = M^{-1} (-B_JIbar xbar)          (lift)
//     S^T v    = -B_JIbar^T (M^{-T} v)           (projection of the pivot part)
// where M = L U is the pivot block in elimination order (entries of L and U in
// {-1, 0, 1}, unit diagonal of L, +-1 diagonal of U).
//
// Triangular solves run in place on one vector, level by level (a row reads
// only rows of earlier levels).  Runs of narrow levels go to one workgroup
// that keeps the vector in LDS and separates the levels with barriers; a wide
// level is one launch over its rows.  The candidates' exact lift solves the
// same systems in int32 for 64 candidates per wavefront (one lane per
// candidate: the systems of different candidates never interact).
#include "gfors_internal.h"

namespace gfors {

namespace {

template <int L>
__device__ __forceinline__ float lu_group_sum(float v) {
#pragma unroll
    for (int o = L / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, L);
    return v;
}
template <int L>
__device__ __forceinline__ double lu_group_sum(double v) {
#pragma unroll
    for (int o = L / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, L);
    return v;
}

__device__ __forceinline__ double lu_block_sum256(double v, double *sh) {
    v = lu_group_sum<64>(v);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0) t = ((sh[0] + sh[1]) + sh[2]) + sh[3];
    __syncthreads();
    return t;
}

// One row of an in-place solve: x_k = d_k (x_k - sum_e a_e x_{c_e}), a_e and d_k = +-1.
template <typename T>
__device__ __forceinline__ void trsv_row(int p, const int *__restrict__ row, const int *__restrict__ ptr,
                                         const int *__restrict__ ent, T *x) {
    const int rk = row[p];
    const int k = rk >> 1;
    T acc = x[k];
    const int e1 = ptr[p + 1];
    for (int e = ptr[p]; e < e1; ++e) {
        const int c = ent[e];
        const T v = x[c >> 1];
        acc = (c & 1) ? acc + v : acc - v;
    }
    x[k] = (rk & 1) ? -acc : acc;
}

}  // namespace

// Levels [l0, l1) of a solve in one workgroup.  LDSX: the whole vector (r
// entries) and the run's rows and entries are staged in LDS first (their
// loads are independent of each other), so that each level costs LDS reads
// and a barrier only; the vector is written back at the end, and with xbar
// given also xbar[k] = 2 x[k] - xold[k] (the lifted part of xbar, fused into
// the last run of a lift).
template <typename T, bool LDSX>
__global__ void __launch_bounds__(256)
k_lu_trsv_seg(const int *__restrict__ row, const int *__restrict__ ptr, const int *__restrict__ ent,
              const int *__restrict__ lvl, int l0, int l1, T *__restrict__ x, int r,
              const T *__restrict__ xold, T *__restrict__ xbar) {
    extern __shared__ __align__(16) unsigned char lu_lds[];
    if (!LDSX) {
        for (int l = l0; l < l1; ++l) {
            const int p1 = lvl[l + 1];
            for (int p = lvl[l] + static_cast<int>(threadIdx.x); p < p1; p += 256) trsv_row(p, row, ptr, ent, x);
            __syncthreads();
        }
        return;
    }
    const int pb = lvl[l0], pe = lvl[l1];
    const int np = pe - pb, eb = ptr[pb], ne = ptr[pe] - eb;
    T *xs = reinterpret_cast<T *>(lu_lds);
    int *srow = reinterpret_cast<int *>(xs + r);
    int *sptr = srow + np;          // np + 1 entries, relative to eb
    int *sent = sptr + np + 1;
    for (int i = threadIdx.x; i < r; i += 256) xs[i] = x[i];
    for (int i = threadIdx.x; i < np; i += 256) srow[i] = row[pb + i];
    for (int i = threadIdx.x; i <= np; i += 256) sptr[i] = ptr[pb + i] - eb;
    for (int i = threadIdx.x; i < ne; i += 256) sent[i] = ent[eb + i];
    __syncthreads();
    for (int l = l0; l < l1; ++l) {
        const int p1 = lvl[l + 1] - pb;
        for (int p = lvl[l] - pb + static_cast<int>(threadIdx.x); p < p1; p += 256) trsv_row(p, srow, sptr, sent, xs);
        __syncthreads();
    }
    for (int i = threadIdx.x; i < r; i += 256) {
        const T v = xs[i];
        x[i] = v;
        if (xbar) xbar[i] = static_cast<T>(2) * v - xold[i];
    }
}

// One wide level: rows [p0, p1) of the level order, one thread each.
template <typename T>
__global__ void __launch_bounds__(256)
k_lu_trsv_level(const int *__restrict__ row, const int *__restrict__ ptr, const int *__restrict__ ent,
                int p0, int p1, T *__restrict__ x) {
    const int p = p0 + static_cast<int>(blockIdx.x * 256 + threadIdx.x);
    if (p < p1) trsv_row(p, row, ptr, ent, x);
}

// xbar[k] = 2 x[k] - xold[k], k < r (when it could not ride on the last run).
template <typename T>
__global__ void k_lu_xbar(int r, const T *__restrict__ x, const T *__restrict__ xold, T *__restrict__ xbar) {
    const int k = blockIdx.x * 256 + threadIdx.x;
    if (k < r) xbar[k] = static_cast<T>(2) * x[k] - xold[k];
}

// LDS bytes of a staged run (vector, rows, pointers, entries).
size_t lu_seg_lds_bytes(const LuSolve &sv, const LuSeg &sg, size_t tsize) {
    const int np = sv.hlvl[sg.b] - sv.hlvl[sg.a];
    const int ne = sv.hptr_at_lvl[sg.b] - sv.hptr_at_lvl[sg.a];
    return static_cast<size_t>(sv.r) * tsize + 4u * static_cast<size_t>(2 * np + 1 + ne);
}

template <typename T>
void launch_lu_trsv(hipStream_t s, const LuSolve &sv, T *x, const T *xold, T *xbar) {
    const int r = sv.r;
    bool fused = false;
    for (int g = 0; g < sv.nseg; ++g) {
        const LuSeg &sg = sv.seg[g];
        const bool last = g == sv.nseg - 1;
        if (sg.wide) {
            const int p0 = sg.a, p1 = sg.b;
            k_lu_trsv_level<T><<<(p1 - p0 + 255) / 256, 256, 0, s>>>(sv.row, sv.ptr, sv.ent, p0, p1, x);
            continue;
        }
        const size_t lds = lu_seg_lds_bytes(sv, sg, sizeof(T));
        if (sv.use_lds && lds <= kLuLdsBytes) {
            const bool f = last && xbar != nullptr;
            k_lu_trsv_seg<T, true><<<1, 256, lds, s>>>(sv.row, sv.ptr, sv.ent, sv.lvl, sg.a, sg.b, x, r,
                                                        f ? xold : nullptr, f ? xbar : nullptr);
            fused = fused || f;
        } else {
            k_lu_trsv_seg<T, false><<<1, 256, 0, s>>>(sv.row, sv.ptr, sv.ent, sv.lvl, sg.a, sg.b, x, r, nullptr,
                                                       nullptr);
        }
    }
    if (xbar && !fused && r > 0) k_lu_xbar<T><<<(r + 255) / 256, 256, 0, s>>>(r, x, xold, xbar);
}
template void launch_lu_trsv<float>(hipStream_t, const LuSolve &, float *, const float *, float *);
template void launch_lu_trsv<double>(hipStream_t, const LuSolve &, double *, const double *, double *);

// y[i] (+)= sgn * sum_e val_e x[col_e] over rows [0, nrows), LPR lanes per row.
template <int LPR, typename TI, typename TO, bool ACC>
__global__ void __launch_bounds__(256)
k_lu_mv(int nrows, const int *__restrict__ rp, const int *__restrict__ ci, const int *__restrict__ val,
        const TI *__restrict__ x, TO *__restrict__ y, TO sgn) {
    const int tid = blockIdx.x * 256 + threadIdx.x;
    const int i = tid / LPR, sub = tid & (LPR - 1);
    TO acc = 0;
    if (i < nrows) {
        const int e1 = rp[i + 1];
        for (int e = rp[i] + sub; e < e1; e += LPR) acc += static_cast<TO>(val[e]) * static_cast<TO>(x[ci[e]]);
    }
    if (LPR > 1) acc = lu_group_sum<LPR>(acc);
    if (i < nrows && sub == 0) y[i] = ACC ? y[i] + sgn * acc : sgn * acc;
}

template <typename TI, typename TO, bool ACC>
static void mv_lpr(hipStream_t s, int lpr, int nrows, const int *rp, const int *ci, const int *val,
                   const TI *x, TO *y, TO sgn) {
    if (nrows <= 0) return;
    const int blocks = static_cast<int>((static_cast<int64_t>(nrows) * lpr + 255) / 256);
    switch (lpr) {
        case 1: k_lu_mv<1, TI, TO, ACC><<<blocks, 256, 0, s>>>(nrows, rp, ci, val, x, y, sgn); break;
        case 4: k_lu_mv<4, TI, TO, ACC><<<blocks, 256, 0, s>>>(nrows, rp, ci, val, x, y, sgn); break;
        case 16: k_lu_mv<16, TI, TO, ACC><<<blocks, 256, 0, s>>>(nrows, rp, ci, val, x, y, sgn); break;
        default: k_lu_mv<64, TI, TO, ACC><<<blocks, 256, 0, s>>>(nrows, rp, ci, val, x, y, sgn); break;
    }
}
void launch_lu_mv_f32(hipStream_t s, int lpr, int nrows, const int *rp, const int *ci, const int *val,
                      const float *x, float *y, float sgn) {
    mv_lpr<float, float, false>(s, lpr, nrows, rp, ci, val, x, y, sgn);
}
void launch_lu_mv_f64(hipStream_t s, int lpr, int nrows, const int *rp, const int *ci, const int *val,
                      const double *x, double *y, double sgn, bool accumulate) {
    if (accumulate) mv_lpr<double, double, true>(s, lpr, nrows, rp, ci, val, x, y, sgn);
    else mv_lpr<double, double, false>(s, lpr, nrows, rp, ci, val, x, y, sgn);
}

// Pivot part of the primal gradient, position k:
//   v_k = -sum_{j} a_{j, nk+k} wy_j + (2/s_o) sum_i Q_{nk+k, i} x_i
// (column nk + k of the lifted rows, row nk + k of the lifted Q; x lifted).
template <int LPR, bool HASQ>
__global__ void __launch_bounds__(256)
k_lu_tail_grad(int r, int nk, const int *__restrict__ rpT, const int *__restrict__ ciT,
               const int *__restrict__ valT, const float *__restrict__ wy, const int *__restrict__ rpQ,
               const int *__restrict__ ciQ, const int *__restrict__ valQ, const float *__restrict__ x,
               const float *__restrict__ two_so, float *__restrict__ v) {
    const int tid = blockIdx.x * 256 + threadIdx.x;
    const int k = tid / LPR, sub = tid & (LPR - 1);
    float s1 = 0.f, s2 = 0.f;
    if (k < r) {
        const int i = nk + k;
        for (int e = rpT[i] + sub; e < rpT[i + 1]; e += LPR) s1 = fmaf(static_cast<float>(valT[e]), wy[ciT[e]], s1);
        if (HASQ)
            for (int e = rpQ[i] + sub; e < rpQ[i + 1]; e += LPR) s2 = fmaf(static_cast<float>(valQ[e]), x[ciQ[e]], s2);
    }
    s1 = lu_group_sum<LPR>(s1);
    if (HASQ) s2 = lu_group_sum<LPR>(s2);
    if (k < r && sub == 0) v[k] = HASQ ? fmaf(two_so[0], s2, -s1) : -s1;
}

// Primal step of the kept variables (Algorithm 2) with the pivot part of the
// gradient: g_i = c~_i + rho - sum_j a_ji wy_j + (2/s_o) (Q z)_i
//               - sum_k (B_JIbar)_{k i} u_k - 2 rho x_i,   u = M^{-T} v.
template <int LPR, bool HASQ>
__global__ void __launch_bounds__(256)
k_lu_primal(int nk, const int *__restrict__ rpT, const int *__restrict__ ciT, const int *__restrict__ valT,
            const float *__restrict__ wy, const int *__restrict__ rpQ, const int *__restrict__ ciQ,
            const int *__restrict__ valQ, const int *__restrict__ rpB, const int *__restrict__ ciB,
            const int *__restrict__ valB, const float *__restrict__ u, const float *__restrict__ x_in,
            float *__restrict__ x_out, float *__restrict__ xbar, const float *__restrict__ ct,
            const float *__restrict__ tau1, const float *__restrict__ two_so,
            const double *__restrict__ rho, DevCounters *__restrict__ ctr) {
    const int tid = blockIdx.x * 256 + threadIdx.x;
    const int i = tid / LPR, sub = tid & (LPR - 1);
    float s1 = 0.f, s2 = 0.f, s3 = 0.f;
    if (i < nk) {
        for (int e = rpT[i] + sub; e < rpT[i + 1]; e += LPR) s1 = fmaf(static_cast<float>(valT[e]), wy[ciT[e]], s1);
        if (HASQ)
            for (int e = rpQ[i] + sub; e < rpQ[i + 1]; e += LPR) s2 = fmaf(static_cast<float>(valQ[e]), x_in[ciQ[e]], s2);
        for (int e = rpB[i] + sub; e < rpB[i + 1]; e += LPR) s3 = fmaf(static_cast<float>(valB[e]), u[ciB[e]], s3);
    }
    s1 = lu_group_sum<LPR>(s1);
    if (HASQ) s2 = lu_group_sum<LPR>(s2);
    s3 = lu_group_sum<LPR>(s3);
    if (i < nk && sub == 0) {
        const float rh = static_cast<float>(rho[0]);
        const float xi = x_in[i];
        float g = ct[i] + rh - s1;
        if (HASQ) g = fmaf(two_so[0], s2, g);
        g -= s3;
        g -= 2.f * rh * xi;
        const float xn = fminf(fmaxf(xi - tau1[0] * g, 0.f), 1.f);
        x_out[i] = xn;
        xbar[i] = 2.f * xn - xi;
    }
    if (tid == 0) ctr->k += 1;
}

// Dual step of the long lifted rows (kHeavyLen+ entries), cut into chunks
// spread over the device: k_lu_rowpart sums a_e xbar_{c_e} of one chunk per
// workgroup; k_lu_heavy_combine adds a row's chunk sums in order and applies
//   y_j = Pi(y_j + tau2 (rt_j - omega_j s_j)),  wy_j = omega_j y_j.
__global__ void __launch_bounds__(256)
k_lu_rowpart(const int *__restrict__ ch_row, const int *__restrict__ ch_e0, const int *__restrict__ ch_e1,
             const int *__restrict__ rowc0, const int *__restrict__ rp, const int *__restrict__ ci,
             const int *__restrict__ val, const float *__restrict__ xbar, float *__restrict__ part) {
    __shared__ float ws[4];
    const int c = blockIdx.x;
    const int j = ch_row[c], e0 = ch_e0[c], e1 = ch_e1[c];
    const int c0 = rowc0[j], b0 = rp[j];
    float s = 0.f;
#pragma unroll 4
    for (int e = e0 + static_cast<int>(threadIdx.x); e < e1; e += 256) {
        const int col = c0 >= 0 ? c0 + (e - b0) : ci[e];
        s = fmaf(static_cast<float>(val[e]), xbar[col], s);
    }
    s = lu_group_sum<64>(s);
    if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) part[c] = ((ws[0] + ws[1]) + ws[2]) + ws[3];
}
__global__ void k_lu_heavy_combine(int nheavy, int m1, const int *__restrict__ order,
                                   const int *__restrict__ first, const float *__restrict__ part,
                                   const float *__restrict__ omega, const float *__restrict__ rt, float tau2,
                                   const float *__restrict__ y_in, float *__restrict__ y_out,
                                   float *__restrict__ wy) {
    const int h = blockIdx.x * 64 + threadIdx.x;
    if (h >= nheavy) return;
    const int j = order[h];
    float sum = 0.f;
    for (int c = first[h]; c < first[h + 1]; ++c) sum += part[c];
    const float om = omega[j];
    float y = y_in[j] + tau2 * (rt[j] - om * sum);
    if (j < m1) y = fmaxf(y, 0.f);
    y_out[j] = y;
    wy[j] = om * y;
}
void launch_lu_dual_heavy(hipStream_t s, int nchunk, int nheavy, int m1, const int *ch_row, const int *ch_e0,
                          const int *ch_e1, const int *first, const int *order, const int *rowc0, const int *rp,
                          const int *ci, const int *val, const float *xbar, float *part, const float *omega,
                          const float *rt, float tau2, const float *y_in, float *y_out, float *wy) {
    if (nchunk <= 0) return;
    k_lu_rowpart<<<nchunk, 256, 0, s>>>(ch_row, ch_e0, ch_e1, rowc0, rp, ci, val, xbar, part);
    k_lu_heavy_combine<<<(nheavy + 63) / 64, 64, 0, s>>>(nheavy, m1, order, first, part, omega, rt, tau2, y_in,
                                                         y_out, wy);
}

// xbar's lifted part: t(xbar_k) = 2 t(x_k) - t(x_{k-1}) (the lift is linear).
__global__ void k_lu_xbar_tail(int r, int nk, const float *__restrict__ x_new, const float *__restrict__ x_old,
                               float *__restrict__ xbar) {
    const int k = blockIdx.x * 256 + threadIdx.x;
    if (k < r) xbar[nk + k] = 2.f * x_new[nk + k] - x_old[nk + k];
}

void launch_lu_tail_grad(hipStream_t s, int lpr, bool hasq, int r, int nk, const int *rpT, const int *ciT,
                         const int *valT, const float *wy, const int *rpQ, const int *ciQ, const int *valQ,
                         const float *x, const float *two_so, float *v) {
    if (r <= 0) return;
    const int blocks = static_cast<int>((static_cast<int64_t>(r) * lpr + 255) / 256);
#define GF_TG(L) \
    do { if (hasq) k_lu_tail_grad<L, true><<<blocks, 256, 0, s>>>(r, nk, rpT, ciT, valT, wy, rpQ, ciQ, valQ, x, two_so, v); \
         else k_lu_tail_grad<L, false><<<blocks, 256, 0, s>>>(r, nk, rpT, ciT, valT, wy, rpQ, ciQ, valQ, x, two_so, v); } while (0)
    switch (lpr) {
        case 1: GF_TG(1); break;
        case 4: GF_TG(4); break;
        case 16: GF_TG(16); break;
        default: GF_TG(64); break;
    }
#undef GF_TG
}

void launch_lu_primal(hipStream_t s, int lpr, bool hasq, int nk, const int *rpT, const int *ciT,
                      const int *valT, const float *wy, const int *rpQ, const int *ciQ, const int *valQ,
                      const int *rpB, const int *ciB, const int *valB, const float *u, const float *x_in,
                      float *x_out, float *xbar, const float *ct, const float *tau1, const float *two_so,
                      const double *rho, DevCounters *ctr) {
    const int blocks = static_cast<int>((static_cast<int64_t>(nk) * lpr + 255) / 256);
#define GF_PR(L) \
    do { if (hasq) k_lu_primal<L, true><<<blocks, 256, 0, s>>>(nk, rpT, ciT, valT, wy, rpQ, ciQ, valQ, rpB, ciB, valB, u, x_in, x_out, xbar, ct, tau1, two_so, rho, ctr); \
         else k_lu_primal<L, false><<<blocks, 256, 0, s>>>(nk, rpT, ciT, valT, wy, rpQ, ciQ, valQ, rpB, ciB, valB, u, x_in, x_out, xbar, ct, tau1, two_so, rho, ctr); } while (0)
    switch (lpr) {
        case 1: GF_PR(1); break;
        case 4: GF_PR(4); break;
        case 16: GF_PR(16); break;
        default: GF_PR(64); break;
    }
#undef GF_PR
}

void launch_lu_xbar_tail(hipStream_t s, int r, int nk, const float *x_new, const float *x_old, float *xbar) {
    if (r > 0) k_lu_xbar_tail<<<(r + 255) / 256, 256, 0, s>>>(r, nk, x_new, x_old, xbar);
}

// d[i] = a[i] - b[i] in FP64 (FP32 operands), i < n.
__global__ void k_lu_diff64(int n, const float *__restrict__ a, const float *__restrict__ b, double *__restrict__ d) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < n) d[i] = b ? static_cast<double>(a[i]) - static_cast<double>(b[i]) : static_cast<double>(a[i]);
}
void launch_lu_diff64(hipStream_t s, int n, const float *a, const float *b, double *d) {
    if (n > 0) k_lu_diff64<<<(n + 255) / 256, 256, 0, s>>>(n, a, b, d);
}

// FP64 residual rows on lifted FP64 vectors (Theorem 2, CheckHalt of Sec. 3):
//   s^y_j = (y_{k-1} - y_k)_j / tau2 - omega_j (row_j . d1),  d1 = lift(xbar_{k-1} - x_k)
//   gap_j = omega_j (r_j - row_j . d2), positive part on inequality rows, d2 = lift(x_k)
__global__ void __launch_bounds__(256)
k_lu_res_rows(const int *__restrict__ tb0, const int *__restrict__ tb1, int m1, const int *__restrict__ rp,
              const int *__restrict__ ci, const int *__restrict__ val, const double *__restrict__ omega64,
              const int64_t *__restrict__ rhs, const double *__restrict__ d1, const double *__restrict__ d2,
              const float *__restrict__ y_prev, const float *__restrict__ y, const double *__restrict__ tau2d,
              double *__restrict__ part) {
    __shared__ double sh[4];
    const int t = blockIdx.x;
    const double tau2 = tau2d[0];
    const int sub = threadIdx.x & 15, grp = threadIdx.x >> 4;
    double a1 = 0.0, a2 = 0.0;
    for (int j0 = tb0[t]; j0 < tb1[t]; j0 += 16) {
        const int j = j0 + grp;
        double s1 = 0.0, s2 = 0.0;
        if (j < tb1[t])
            for (int e = rp[j] + sub; e < rp[j + 1]; e += 16) {
                const double a = static_cast<double>(val[e]);
                s1 += a * d1[ci[e]];
                s2 += a * d2[ci[e]];
            }
        s1 = lu_group_sum<16>(s1);
        s2 = lu_group_sum<16>(s2);
        if (j < tb1[t] && sub == 0) {
            const double om = omega64[j];
            const double sy = (static_cast<double>(y_prev[j]) - static_cast<double>(y[j])) / tau2 - om * s1;
            double g = om * (static_cast<double>(rhs[j]) - s2);
            if (j < m1 && g < 0.0) g = 0.0;
            a1 += sy * sy;
            a2 += g * g;
        }
    }
    a1 = lu_block_sum256(a1, sh);
    a2 = lu_block_sum256(a2, sh);
    if (threadIdx.x == 0) { part[2 * t] = a1; part[2 * t + 1] = a2; }
}
void launch_lu_res_rows(hipStream_t s, const Tiles &rt, int m1, const int *rp, const int *ci, const int *val,
                        const double *omega64, const int64_t *rhs, const double *d1, const double *d2,
                        const float *y_prev, const float *y, const double *tau2d, double *part) {
    if (rt.count)
        k_lu_res_rows<<<rt.count, 256, 0, s>>>(rt.b0, rt.b1, m1, rp, ci, val, omega64, rhs, d1, d2, y_prev, y,
                                                tau2d, part);
}

// FP64 residual of the kept variables:  s^x_i = -dx_i/tau1 - 2 rho dx_i + (2/s_o) (Q' dx)_i
// with (Q' dx) given (null without Q); binary gap x_i (1 - x_i).
__global__ void __launch_bounds__(256)
k_lu_res_vars(const int *__restrict__ tb0, const int *__restrict__ tb1, const double *__restrict__ qd,
              const float *__restrict__ x, const float *__restrict__ xp, const double *__restrict__ rho,
              const double *__restrict__ tau1d, const double *__restrict__ two_sod, double *__restrict__ part) {
    __shared__ double sh[4];
    const int t = blockIdx.x;
    const double r = rho[0], tau1 = tau1d[0], tso = two_sod[0];
    double a1 = 0.0, a2 = 0.0;
    for (int i = tb0[t] + threadIdx.x; i < tb1[t]; i += 256) {
        const double xi = x[i];
        const double dx = xi - static_cast<double>(xp[i]);
        double sx = -dx / tau1 - 2.0 * r * dx;
        if (qd) sx += tso * qd[i];
        a1 += sx * sx;
        a2 += xi * (1.0 - xi);
    }
    a1 = lu_block_sum256(a1, sh);
    a2 = lu_block_sum256(a2, sh);
    if (threadIdx.x == 0) { part[2 * t] = a1; part[2 * t + 1] = a2; }
}
void launch_lu_res_vars(hipStream_t s, const Tiles &vt, const double *qd, const float *x, const float *xp,
                        const double *rho, const double *tau1d, const double *two_sod, double *part) {
    if (vt.count) k_lu_res_vars<<<vt.count, 256, 0, s>>>(vt.b0, vt.b1, qd, x, xp, rho, tau1d, two_sod, part);
}

// ---------------------------------------------------------------------------
// Exact lift of the candidates (EvalBest on the reformulated model).
// XI[k][l] (int32, candidate-minor with stride K) first receives
//   d_{J_{a_k}} - (B_JIbar x_l)_k,
// then the in-place solves L forward, U backward turn it into x_{I_{b_k}} of
// candidate l (its value s + S x_l, any integer).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256)
k_lu_eval_rhs(int r, int W, int K, const int *__restrict__ rp, const int *__restrict__ ci,
              const int *__restrict__ val, const int64_t *__restrict__ dJ, const uint64_t *__restrict__ X,
              int *__restrict__ XI) {
    const int g = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (g >= r * W) return;
    const int k = g / W, w = g - k * W;
    int acc = static_cast<int>(dJ[k]);
    // 64 entries at a time: lane j loads entry j's column, coefficient and
    // candidate word (one gather for all 64), then every lane walks them in
    // entry order through lane reads (integer sums: the order is free anyway)
    const int e0 = rp[k], e1 = rp[k + 1];
    for (int eb = e0; eb < e1; eb += 64) {
        const int e = eb + lane;
        const bool in = e < e1;
        const int vl = in ? val[e] : 0;
        const uint64_t wl = in ? X[static_cast<int64_t>(ci[e]) * W + w] : 0ull;
        const uint32_t wlo = static_cast<uint32_t>(wl), whi = static_cast<uint32_t>(wl >> 32);
        const int cnt = min(64, e1 - eb);
        for (int j = 0; j < cnt; ++j) {
            const int vj = __builtin_amdgcn_readlane(vl, j);
            const uint32_t lo = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(wlo), j));
            const uint32_t hi = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(whi), j));
            const uint32_t half = lane < 32 ? lo : hi;
            if ((half >> (lane & 31)) & 1u) acc -= vj;
        }
    }
    XI[static_cast<int64_t>(k) * K + 64 * w + lane] = acc;
}

__device__ __forceinline__ void trsm_row(int p, const int *__restrict__ row, const int *__restrict__ ptr,
                                         const int *__restrict__ ent, int *__restrict__ XI, int K, int l) {
    const int rk = row[p];
    const int k = rk >> 1;
    int acc = XI[static_cast<int64_t>(k) * K + l];
    for (int e = ptr[p]; e < ptr[p + 1]; ++e) {
        const int c = ent[e];
        const int v = XI[static_cast<int64_t>(c >> 1) * K + l];
        acc = (c & 1) ? acc + v : acc - v;
    }
    XI[static_cast<int64_t>(k) * K + l] = (rk & 1) ? -acc : acc;
}

// Narrow levels [l0, l1): workgroup w owns candidates 64w .. 64w+63; its four
// wavefronts split the rows of a level.
__global__ void __launch_bounds__(256)
k_lu_trsm_seg(const int *__restrict__ row, const int *__restrict__ ptr, const int *__restrict__ ent,
              const int *__restrict__ lvl, int l0, int l1, int *__restrict__ XI, int K) {
    const int l = 64 * blockIdx.x + (threadIdx.x & 63);
    const int wv = threadIdx.x >> 6;
    for (int lv = l0; lv < l1; ++lv) {
        const int p1 = lvl[lv + 1];
        for (int p = lvl[lv] + wv; p < p1; p += 4) trsm_row(p, row, ptr, ent, XI, K, l);
        __syncthreads();
    }
}
// A wide level: rows [p0, p1), four per workgroup, 64 candidates per wavefront.
__global__ void __launch_bounds__(256)
k_lu_trsm_level(const int *__restrict__ row, const int *__restrict__ ptr, const int *__restrict__ ent,
                int p0, int p1, int *__restrict__ XI, int K) {
    const int p = p0 + 4 * static_cast<int>(blockIdx.x) + (threadIdx.x >> 6);
    const int l = 64 * blockIdx.y + (threadIdx.x & 63);
    if (p < p1) trsm_row(p, row, ptr, ent, XI, K, l);
}

void launch_lu_trsm(hipStream_t s, const LuSolve &sv, int *XI, int K) {
    const int W = K / 64;
    for (int g = 0; g < sv.nseg; ++g) {
        const LuSeg &sg = sv.seg[g];
        if (sg.wide) {
            dim3 grid((sg.b - sg.a + 3) / 4, W);
            k_lu_trsm_level<<<grid, 256, 0, s>>>(sv.row, sv.ptr, sv.ent, sg.a, sg.b, XI, K);
        } else {
            k_lu_trsm_seg<<<W, 256, 0, s>>>(sv.row, sv.ptr, sv.ent, sv.lvl, sg.a, sg.b, XI, K);
        }
    }
}

void launch_lu_eval_rhs(hipStream_t s, int r, int K, const int *rp, const int *ci, const int *val,
                        const int64_t *dJ, const uint64_t *X, int *XI) {
    const int W = K / 64;
    const int64_t waves = static_cast<int64_t>(r) * W;
    if (waves > 0) k_lu_eval_rhs<<<static_cast<int>((waves + 3) / 4), 256, 0, s>>>(r, W, K, rp, ci, val, dJ, X, XI);
}

// Value of lifted column c for candidate l (lane) of word w: a kept variable's
// bit, or the lifted integer of position c - nk.
__device__ __forceinline__ int64_t lifted_val(int c, int nk, const uint64_t *__restrict__ X, int W, int w,
                                              int lane, const int *__restrict__ XI, int K) {
    if (c < nk) return static_cast<int64_t>((X[static_cast<int64_t>(c) * W + w] >> lane) & 1ull);
    return static_cast<int64_t>(XI[static_cast<int64_t>(c - nk) * K + 64 * w + lane]);
}

// Rows of the reformulated model on the lifted integer point, one wavefront
// per (row chunk, candidate word).  A row in one chunk is decided at once
// (violation: lhs < rhs on an inequality row, lhs != rhs on an equality row:
// one count for its candidate); a row in several chunks adds its partial sums
// into rsum[slot] and is decided by k_lu_eval_multi.
__global__ void __launch_bounds__(256)
k_lu_eval_rows(int nch, int W, int K, int nk, int m1, const int *__restrict__ ch_row,
               const int *__restrict__ ch_e0, const int *__restrict__ ch_e1, const int *__restrict__ ch_slot,
               const int *__restrict__ ci, const int *__restrict__ val, const int64_t *__restrict__ rhs,
               const uint64_t *__restrict__ X, const int *__restrict__ XI, int *__restrict__ vcnt,
               unsigned long long *__restrict__ rsum) {
    const int g = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (g >= nch * W) return;
    const int c = g / W, w = g - c * W;
    const int j = ch_row[c];
    int64_t acc = 0;
    // 64 entries at a time: lane q loads entry q's column and coefficient and,
    // for a kept variable, its candidate word (one gather for all 64); every
    // lane then walks them in entry order through lane reads, loading only the
    // lifted integers (one coalesced load per lifted entry)
    const int e0 = ch_e0[c], e1 = ch_e1[c];
    for (int eb = e0; eb < e1; eb += 64) {
        const int e = eb + lane;
        const bool in = e < e1;
        const int cl = in ? ci[e] : 0;
        const int vl = in ? val[e] : 0;
        const uint64_t wl = (in && cl < nk) ? X[static_cast<int64_t>(cl) * W + w] : 0ull;
        const uint32_t wlo = static_cast<uint32_t>(wl), whi = static_cast<uint32_t>(wl >> 32);
        const int cnt = min(64, e1 - eb);
        for (int q = 0; q < cnt; ++q) {
            const int cq = __builtin_amdgcn_readlane(cl, q);
            const int vq = __builtin_amdgcn_readlane(vl, q);
            int64_t xv;
            if (cq < nk) {   // uniform over the wavefront
                const uint32_t lo = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(wlo), q));
                const uint32_t hi = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(whi), q));
                xv = static_cast<int64_t>(((lane < 32 ? lo : hi) >> (lane & 31)) & 1u);
            } else {
                xv = static_cast<int64_t>(XI[static_cast<int64_t>(cq - nk) * K + 64 * w + lane]);
            }
            acc += static_cast<int64_t>(vq) * xv;
        }
    }
    const int slot = ch_slot[c];
    const int l = 64 * w + lane;
    if (slot < 0) {
        const bool bad = j < m1 ? acc < rhs[j] : acc != rhs[j];
        if (bad) atomicAdd(&vcnt[l], 1);
    } else {
        atomicAdd(&rsum[static_cast<int64_t>(slot) * K + l], static_cast<unsigned long long>(acc));
    }
}
__global__ void __launch_bounds__(256)
k_lu_eval_multi(int nslot, int K, int m1, const int *__restrict__ slot_row, const int64_t *__restrict__ rhs,
                const unsigned long long *__restrict__ rsum, int *__restrict__ vcnt) {
    const int64_t t = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    if (t >= static_cast<int64_t>(nslot) * K) return;
    const int sl = static_cast<int>(t / K), l = static_cast<int>(t - static_cast<int64_t>(sl) * K);
    const int j = slot_row[sl];
    const int64_t acc = static_cast<int64_t>(rsum[t]);
    const bool bad = j < m1 ? acc < rhs[j] : acc != rhs[j];
    if (bad) atomicAdd(&vcnt[l], 1);
}

// Objective beyond the sampler's sum over kept variables: per candidate
//   zx_l = -c'_0 + sum_k c_{I_{b_k}} x_{I_{b_k}}   (k_lu_eval_lin, also the initialiser)
//        + <z_l, Q z_l>                               (k_lu_eval_quad, Q rows in chunks)
// on the lifted integer point z_l, so that the total is the reformulated
// objective <x', Q' x'> + <c', x'> = f(x) - c'_0.
__global__ void __launch_bounds__(512)
k_lu_eval_lin(int r, int K, const int64_t *__restrict__ c_tail, int64_t c0, const int *__restrict__ XI,
              int64_t *__restrict__ zx) {
    // workgroup = 64 candidates; its 8 wavefronts split the positions k
    __shared__ int64_t part[8][64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int l = 64 * blockIdx.x + lane;
    int64_t acc = 0;
#pragma unroll 4
    for (int k = wv; k < r; k += 8) acc += c_tail[k] * static_cast<int64_t>(XI[static_cast<int64_t>(k) * K + l]);
    part[wv][lane] = acc;
    __syncthreads();
    if (wv == 0) {
        int64_t t = -c0;
        for (int j = 0; j < 8; ++j) t += part[j][lane];
        zx[l] = t;
    }
}
__global__ void __launch_bounds__(256)
k_lu_eval_quad(int nch, int W, int K, int nk, const int *__restrict__ ch_row, const int *__restrict__ ch_e0,
               const int *__restrict__ ch_e1, const int *__restrict__ ciQ, const int *__restrict__ valQ,
               const uint64_t *__restrict__ X, const int *__restrict__ XI, unsigned long long *__restrict__ zx) {
    const int g = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (g >= nch * W) return;
    const int c = g / W, w = g - c * W;
    const int a = ch_row[c];
    const int64_t va = lifted_val(a, nk, X, W, w, lane, XI, K);
    if (__ballot(va != 0) == 0) return;   // no candidate of the word has x_a != 0 (uniform)
    int64_t acc = 0;
    // 64 entries at a time, as in k_lu_eval_rows (every lane of the wavefront
    // takes part in the lane reads; lanes with x_a = 0 add nothing at the end)
    const int e0 = ch_e0[c], e1 = ch_e1[c];
    for (int eb = e0; eb < e1; eb += 64) {
        const int e = eb + lane;
        const bool in = e < e1;
        const int cl = in ? ciQ[e] : 0;
        const int vl = in ? valQ[e] : 0;
        const uint64_t wl = (in && cl < nk) ? X[static_cast<int64_t>(cl) * W + w] : 0ull;
        const uint32_t wlo = static_cast<uint32_t>(wl), whi = static_cast<uint32_t>(wl >> 32);
        const int cnt = min(64, e1 - eb);
        for (int q = 0; q < cnt; ++q) {
            const int cq = __builtin_amdgcn_readlane(cl, q);
            const int vq = __builtin_amdgcn_readlane(vl, q);
            int64_t xv;
            if (cq < nk) {   // uniform over the wavefront
                const uint32_t lo = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(wlo), q));
                const uint32_t hi = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(whi), q));
                xv = static_cast<int64_t>(((lane < 32 ? lo : hi) >> (lane & 31)) & 1u);
            } else {
                xv = static_cast<int64_t>(XI[static_cast<int64_t>(cq - nk) * K + 64 * w + lane]);
            }
            acc += static_cast<int64_t>(vq) * xv;
        }
    }
    if (va != 0 && acc) atomicAdd(&zx[64 * w + lane], static_cast<unsigned long long>(acc * va));
}

void launch_lu_eval_rows(hipStream_t s, int nch, int K, int nk, int m1, const int *ch_row, const int *ch_e0,
                         const int *ch_e1, const int *ch_slot, const int *ci, const int *val, const int64_t *rhs,
                         const uint64_t *X, const int *XI, int *vcnt, int64_t *rsum) {
    const int W = K / 64;
    const int64_t waves = static_cast<int64_t>(nch) * W;
    if (waves > 0)
        k_lu_eval_rows<<<static_cast<int>((waves + 3) / 4), 256, 0, s>>>(
            nch, W, K, nk, m1, ch_row, ch_e0, ch_e1, ch_slot, ci, val, rhs, X, XI, vcnt,
            reinterpret_cast<unsigned long long *>(rsum));
}
void launch_lu_eval_multi(hipStream_t s, int nslot, int K, int m1, const int *slot_row, const int64_t *rhs,
                          const int64_t *rsum, int *vcnt) {
    const int64_t t = static_cast<int64_t>(nslot) * K;
    if (t > 0)
        k_lu_eval_multi<<<static_cast<int>((t + 255) / 256), 256, 0, s>>>(
            nslot, K, m1, slot_row, rhs, reinterpret_cast<const unsigned long long *>(rsum), vcnt);
}
void launch_lu_eval_obj(hipStream_t s, int r, int K, const int64_t *c_tail, int64_t c0, const int *XI,
                        int nqch, int nk, const int *qch_row, const int *qch_e0, const int *qch_e1,
                        const int *ciQ, const int *valQ, const uint64_t *X, int64_t *zx) {
    k_lu_eval_lin<<<K / 64, 512, 0, s>>>(r, K, c_tail, c0, XI, zx);
    const int W = K / 64;
    const int64_t waves = static_cast<int64_t>(nqch) * W;
    if (waves > 0)
        k_lu_eval_quad<<<static_cast<int>((waves + 3) / 4), 256, 0, s>>>(
            nqch, W, K, nk, qch_row, qch_e0, qch_e1, ciQ, valQ, X, XI, reinterpret_cast<unsigned long long *>(zx));
}

// Fill of int32 / int64 arrays (no memset nodes in captured graphs).
__global__ void k_lu_fill_i64(int64_t *__restrict__ p, int64_t v, int64_t n) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    if (i < n) p[i] = v;
}
void launch_lu_fill_i64(hipStream_t s, int64_t *p, int64_t v, int64_t n) {
    if (n > 0) k_lu_fill_i64<<<static_cast<int>((n + 255) / 256), 256, 0, s>>>(p, v, n);
}
__global__ void k_lu_fill_i32(int *__restrict__ p, int v, int64_t n) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    if (i < n) p[i] = v;
}
void launch_lu_fill_i32(hipStream_t s, int *p, int v, int64_t n) {
    if (n > 0) k_lu_fill_i32<<<static_cast<int>((n + 255) / 256), 256, 0, s>>>(p, v, n);
}

}  // namespace gfors
