// Internal declarations shared by the gfors host code and its HIP kernels.
// Device data layout (all carved from the caller's workspace):
//   constraint rows  : CSR of the ORIGINAL integer coefficients of [A; B]
//                      (inequality rows first), int32 row_ptr / col / val
//                      (val absent when every coefficient is 1); its
//                      transpose (one row per variable) for K^T y without
//                      atomics; Q in full symmetric CSR.
//   PDHG vectors     : x double-buffered (x_{k-1}, x_k), xbar, y double-
//                      buffered, wy = omega o y, FP32; omega_j = 1/(||a_j|| s_K)
//                      and rt_j = r_j omega_j per row; ct = c / s_o per variable.
//   candidates       : bit-packed, variable-major uint64 [n][K/64].
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace gfors {

// Philox4x32-10 constants (Salmon et al., SC'11).
constexpr uint32_t kPhiloxM0 = 0xD2511F53u;
constexpr uint32_t kPhiloxM1 = 0xCD9E8D57u;
constexpr uint32_t kPhiloxW0 = 0x9E3779B9u;
constexpr uint32_t kPhiloxW1 = 0xBB67AE85u;

// Per-problem scalars that kernels read from device memory (so that captured
// graphs stay valid as the loop advances).
struct DevCounters {
    int64_t k;       // PDHG iterations done
    int64_t round;   // Philox sampling rounds done
    int64_t pad[6];
};

// Per-instance device arrays.
struct DevInst {
    double *rho;          // current penalty rho_n
    int64_t *ntrig;       // triggers so far (n of UpdatePenalty)
    int64_t *zbest;       // incumbent objective (INT64_MAX = none)
    int64_t *inc_k, *inc_round, *inc_l;
    int32_t *improved;    // set by the last incumbent update
    int32_t *inc_W;       // words-per-variable of the round that produced the incumbent
    double *rho_min, *rho_max, *rho_T, *rho_p, *rho_delta;
    float *tau1, *tau2, *two_so;   // per-instance FP32 scalars (batched kernels)
    double *tau1d, *tau2d, *two_sod;
    int64_t *hist;        // [T][hist_cap] incumbent after each round
    int32_t hist_cap;
};

// Tile tables.  A tile is a piece of work that never crosses an instance.
struct Tiles {
    int32_t count = 0;
    int32_t *inst = nullptr;   // instance of each tile
    int32_t *b0 = nullptr;     // begin (quad / list position / row / var)
    int32_t *b1 = nullptr;     // end
    int32_t *first = nullptr;  // [T+1] first tile of each instance (tiles sorted by instance)
};

// Launch shapes picked per problem (heuristic or timed by the autotuner).
// slices: 1 = fused CSR kernel; > 1 = XCD-sliced partial SpMV + combine.
struct LaunchCfg {
    int lpr_dual = 16;     // lanes per row for the dual SpMV
    int lpr_primal = 4;    // lanes per row for the transposed SpMV (+Q)
    int slices_dual = 1;
    int slices_primal = 1;
    int sell_dual = 0;     // 1: SELL-64 layout (lane = row) instead of CSR
    int sell_primal = 0;
    int bits_dual = 0;     // 1: skip zero operands through an LDS bitmap
    int bits_primal = 0;
};

constexpr int64_t kMaxLdsBitmapBytes = 64 * 1024;

// A SELL-64 matrix (possibly cut into P column slices, each with nchunk chunks).
struct SellView {
    int nrows = 0, P = 1, nchunk = 0, ns = 0;   // ns: columns per slice (multiple of 64)
    const int *ptr = nullptr, *ci = nullptr, *val = nullptr, *row_of = nullptr;
    // per slot: first column of a row whose entries in the slice are one
    // contiguous range (else -1) and the row's entry count in the slice
    const int *c0 = nullptr, *len = nullptr;
    const int16_t *val16 = nullptr;   // the coefficients as int16 when all fit (else null)
};

constexpr int kXcdSlices = 8;   // XCDs per MI355X
// Evaluation kinds of rows whose violation is a bitwise function of the
// candidate words (per-row byte: kind << 4 | truth table of pair rows).
constexpr int kEvalCover = 0;        // inequality, coefficients 1, rhs 1:  violated iff none set
constexpr int kEvalAtMostOne = 1;    // inequality, coefficients -1, rhs -1: violated iff >= 2 set
constexpr int kEvalExactlyOne = 2;   // equality, coefficients +-1, rhs +-1: violated iff != 1 set
constexpr int kEvalPair = 3;         // one or two entries: truth table over (x_p, x_q)
constexpr int kLprBlock = 256;  // launch shape "a workgroup of 256 lanes per row"; 256 + L:
                                // rows of kHeavyLen+ entries a workgroup each, others L lanes
constexpr int kHeavyLen = 256;
constexpr int kLightHole = 0x7fffffff;   // signed-index slot of a heavy item inside the light range
constexpr int kHgChunk = 512;   // entries per workgroup of the heavy shift-group primal
constexpr int kHgWidth = 16;    // variables per shift group (32 measured slower: fewer entries in flight)

// ------------------------------------------------------------------ PDHG
// val16: the coefficients as int16 when every |a| <= 32767 (else null)
void launch_dual(hipStream_t s, int lpr, bool unit, bool batched, int m, int m1,
                 const int *rp, const int *ci, const int *val, const int16_t *val16, const float *omega,
                 const float *rt, const float *xbar, const float *y_in, float *y_out,
                 float *wy, float tau2, const float *tau2_inst, const int *row_inst,
                 int skip_len);

void launch_primal(hipStream_t s, int lpr, int kmode, bool hasq, bool batched, int n,
                   const int *rpT, const int *colT0, const int *ciT, const int *valT, const float *wy,
                   const int *rpQ, const int *ciQ, const int *valQ, const float *x_in,
                   float *x_out, float *xbar, const float *ct, float tau1, float two_so,
                   const float *tau1_inst, const float *two_so_inst, const double *rho,
                   const int *var_inst, DevCounters *ctr, int skip_len);
void launch_primal_long(hipStream_t s, bool unit, bool batched, int count, const int *order,
                        const int *rpT, const int *ciT, const int *valT, const float *wy,
                        const float *x_in, float *x_out, float *xbar, const float *ct, float tau1,
                        const float *tau1_inst, const double *rho, const int *var_inst);

void launch_spmv_part(hipStream_t s, int lpr, bool unit, int nrows, int P, const int *rpP,
                      const int *ci, const int *val, const float *v, float *part);
void launch_dual_combine(hipStream_t s, bool batched, int m, int m1, int P, const float *part,
                         const float *omega, const float *rt, const float *y_in, float *y_out,
                         float *wy, float tau2, const float *tau2_inst, const int *row_inst,
                         uint64_t *wybits);
void launch_primal_combine(hipStream_t s, bool batched, int n, int P, const float *part,
                           const float *x_in, float *x_out, float *xbar, const float *ct,
                           float tau1, const float *tau1_inst, const double *rho,
                           const int *var_inst, DevCounters *ctr, uint64_t *xbits);

void launch_sell(hipStream_t s, const SellView &sv, int mode, bool unit, bool batched,
                 const float *v, float *part, int m1, const float *omega, const float *rt,
                 const float *y_in, float *y_out, float *wy, float tau2, const float *tau2_inst,
                 const int *row_inst, const float *x_in, float *x_out, float *xbar,
                 const float *ct, float tau1, const float *tau1_inst, const double *rho,
                 const int *var_inst, DevCounters *ctr);

void launch_nzbits(hipStream_t s, const float *v, int64_t n, int64_t nwords64, uint64_t *bits);
void launch_dual_long(hipStream_t s, bool unit, bool batched, int m, int m1, const int *order,
                      const int *rp, const int *rowc0, const int *ci, const int *val,
                      const int16_t *val16, const uint8_t *rowunit, const float *omega,
                      const float *rt, const float *xbar, const float *y_in, float *y_out,
                      float *wy, float tau2, const float *tau2_inst, const int *row_inst);
void launch_sell_bits(hipStream_t s, const SellView &sv, int mode, bool unit, bool batched,
                      int ncols, const float *v, const uint32_t *bits, float *part, int m1,
                      const float *omega, const float *rt, const float *y_in, float *y_out,
                      float *wy, float tau2, const float *tau2_inst, const int *row_inst,
                      const float *x_in, float *x_out, float *xbar, const float *ct, float tau1,
                      const float *tau1_inst, const double *rho, const int *var_inst,
                      DevCounters *ctr, int nc);
int sell_bits_blocks(const SellView &sv, int nc);
void launch_sell_part_bits(hipStream_t s, const SellView &sv, int ns, int ncols, bool unit,
                           const float *v, const uint32_t *bits, float *part);
void launch_primal_bits(hipStream_t s, int lpr, bool unit, bool batched, int n, int m,
                        const int *rpT, const int *ciT, const int *valT, const float *wy,
                        const uint32_t *bits, const float *x_in, float *x_out, float *xbar,
                        const float *ct, float tau1, const float *tau1_inst, const double *rho,
                        const int *var_inst, DevCounters *ctr, uint64_t *xbits, int deg);

// Dense-block SpMVs of batched instances whose rows are dense over their
// instance's variables (at most 64 rows per instance, no Q).
struct BlockView {
    int ntile = 0;
    const int *tile_inst = nullptr, *tile_c0 = nullptr;   // per tile: instance, first column
    const int *row0 = nullptr, *nrow = nullptr;            // per instance: its rows in `rows`
    const int *rows = nullptr;                             // rows of each instance, in order
    const int *row_rank = nullptr;                         // per row: index within its instance
    const int *inst_tile0 = nullptr, *inst_ntile = nullptr;   // per instance: its tiles
    float *pp = nullptr;                                   // per tile: 64 row sums
    // padded int16 copy (each row of an instance at a multiple of 8 entries,
    // zero past its end; null when absent) and the first entry of every row
    // of `rows` in it
    const int16_t *pval = nullptr;
    const int64_t *pbase = nullptr;
};
constexpr int kBlockCols = 2048;   // columns per tile of the dense-block SpMVs (256 threads x 8)
void launch_dual_block(hipStream_t s, const BlockView &b, int m, int m1, const int *rp, const int *val,
                       const int16_t *val16, const int64_t *inst_var0, const int64_t *inst_nvar,
                       const float *xbar, const float *omega, const float *rt, const float *tau2_inst,
                       const int *row_inst, const float *y_in, float *y_out, float *wy);
void launch_primal_block(hipStream_t s, const BlockView &b, const int *rp, const int *val, const int16_t *val16,
                         const int64_t *inst_var0, const int64_t *inst_nvar, const float *wy,
                         const float *x_in, float *x_out, float *xbar, const float *ct, const float *tau1_inst,
                         const double *rho, DevCounters *ctr);

// Primal step with wy staged in LDS slices of SL rows (unit coefficients,
// every variable in deg <= 8 rows, one instance, no Q); ell[u n + i] = the
// u-th row of variable i (ascending).  Returns false for an unsupported deg.
int primal_lds_slice(size_t lds_limit);
// Light rows / variables [i0, i0 + L) of D <= 8 entries each, indices entry-major
// with the coefficient's sign (|a| = 1) in bit 31; one instance, no Q.  xbits:
// nonzero bitmap of xbar (only when the range is every variable), or null.
void launch_dual_light(hipStream_t s, int D, int i0, int L, int m1, const int *sidx, const float *omega,
                       const float *rt, const float *xbar, const float *y_in, float *y_out, float *wy,
                       float tau2);
void launch_primal_light(hipStream_t s, int D, int i0, int L, const int *sidx, const float *wy,
                         const float *x_in, float *x_out, float *xbar, const float *ct, float tau1,
                         const double *rho, DevCounters *ctr, uint64_t *xbits);
// Heavy variables in groups of <= kHgWidth whose rows are unit shifts of the first
// one's (one instance, no Q): chunk partials, then the per-variable update.
void launch_primal_hgroup(hipStream_t s, bool unit, int nslot, int ngroup, const int *ord, const int *ch_g,
                          const int *ch_b, const int *ch_e, const int *hg_var0, const int *hg_w, const int *hg_e0,
                          const int *hg_c0, const int *ciT, const int *valT, const float *wy, float *part,
                          const float *x_in, float *x_out, float *xbar, const float *ct, float tau1,
                          const double *rho);
bool launch_primal_lds(hipStream_t s, int n, int m, int deg, int SL, const int *ell, const float *wy,
                       const float *x_in, float *x_out, float *xbar, const float *ct, float tau1,
                       const double *rho, DevCounters *ctr, uint64_t *xbits);

void launch_copy_f32(hipStream_t s, float *dst, const float *src, int64_t n);
void launch_set_xbar(hipStream_t s, int64_t n, const float *x, const float *xp, float *xbar);
void launch_fill_f32(hipStream_t s, float *dst, float v, int64_t n);

// ------------------------------------------------- FP64 (Preprocess, residuals)
void launch_spmv64(hipStream_t s, int nrows, const int *rp, const int *ci, const int *val,
                   const double *rowscale, const double *v, double *w);
void launch_scale64(hipStream_t s, int64_t n, double *x, const double *a, double sign);
void launch_fill64(hipStream_t s, double *x, double v, int64_t n);
void launch_tile_sumsq(hipStream_t s, const Tiles &t, const double *x, double *part);
void launch_inst_sum(hipStream_t s, int T, const Tiles &t, const double *part, int stride,
                     int comp, double *out, int out_stride, bool take_sqrt);
void launch_tile_scale_inv(hipStream_t s, const Tiles &t, double *x, const double *nrm);

void launch_res_rows(hipStream_t s, const Tiles &rt, int m1, const int *rp, const int *ci,
                     const int *val, const double *omega64, const int64_t *rhs,
                     const float *xsave, const float *x, const float *y_prev,
                     const float *y, const double *tau2d, double *part);
void launch_res_vars(hipStream_t s, const Tiles &vt, const int *rpQ, const int *ciQ,
                     const int *valQ, const float *x, const float *xp, const double *rho,
                     const double *tau1d, const double *two_sod, double *part);

// --------------------------------------------------------- sampling / eval
void launch_philox_peak(hipStream_t s, int blocks, int iters, uint32_t *sink);
void launch_read_peak(hipStream_t s, int blocks, const void *p, int64_t n16, uint32_t *sink);
// Monotone relaxation repair (Sec. 2.4) of the sampled candidates: in each of
// the nrows relaxed set-partitioning rows (variables var[rp[r]..rp[r+1]) in
// (cost, index) order) only the first set variable of every candidate stays
// set; cleared costs are taken off the candidates' objectives in zpart[0..K).
void launch_mono_repair(hipStream_t s, int nrows, int W, int K, const int *rp, const int *var,
                        const int64_t *cost, uint64_t *X, uint8_t *xkind, int64_t *zpart);
// Customized 3D-assignment sampler (Algorithm 4): candidates of an n x n x n
// assignment from p into X (cleared first, with zpart[0, nzpart) and xkind),
// objectives into zpart[0 .. K); part: int[2 n] scratch.
constexpr int kA3MaxN = 1024;     // largest n
constexpr int kA3MaxTop = 4096;   // largest gamma n
void launch_a3(hipStream_t s, const float *p, int n, int m, int K, int L, uint32_t key0,
               uint32_t key1, const DevCounters *ctr, const int64_t *cost, int *part, uint64_t *X,
               int W, int64_t *zpart, int64_t nzpart, uint8_t *xkind);
void launch_sample(hipStream_t s, int W, bool obj64, const float *p, const int64_t *cost,
                   uint64_t *X, const Tiles &st, const int64_t *inst_var0,
                   const int64_t *inst_nvar, int64_t *zpart, int K, uint32_t key0,
                   uint32_t key1, const DevCounters *ctr, int threshold_mode, uint8_t *xkind);

void launch_eval_cover(hipStream_t s, int ntiles, const int *tile_ids, const Tiles &et,
                       const int *rows, const uint8_t *rkind, const int *rp, const int *ci,
                       const uint64_t *X, const uint8_t *xkind, int W, int *vpart, int K,
                       bool pair_rows);   // most rows of two entries: four rows in flight per group
void launch_eval_general(hipStream_t s, int ntiles, const int *tile_ids, const Tiles &et,
                         bool acc64, const int *rows, const int *rp, const int *ci,
                         const int *val, const int64_t *rhs, int m1, const uint64_t *X,
                         const uint8_t *xkind, int W, int *vpart, int K, bool long_rows,
                         bool coef24);
// Tiles of <= 32 general rows densified as int8 digit planes (npl in 1..3);
// acc64: some row's sum of |a| reaches 2^31.
void launch_eval_mfma(hipStream_t s, int ntiles, const int *tile_ids, const Tiles &et, int npl, bool acc64,
                      const int *rows, const int64_t *mf_off, const int *mf_c0, const int *mf_span,
                      const int8_t *dig, const int64_t *rhs, int m1, const uint64_t *X, int W,
                      int *vpart, int K);
void launch_eval_quad(hipStream_t s, const Tiles &qt, const int *rpQ, const int *rowQ,
                      const int *ciQ, const int *valQ, const uint64_t *X, int W, int64_t *zqpart,
                      int K, bool q24);
void launch_reduce_cand(hipStream_t s, int T, int K, int S, const Tiles &et, const int *vpart,
                        const Tiles &st, const int64_t *zpart, const Tiles &qt,
                        const int64_t *zqpart, int has_q, int32_t *rv, int64_t *rz,
                        int32_t *viol, int64_t *z);
void launch_argmin_update(hipStream_t s, int T, int K, int W, const int32_t *viol,
                          const int64_t *z, DevInst di, DevCounters *ctr, int advance);
void launch_extract_best(hipStream_t s, int64_t n, int T, const int *var_inst, const uint64_t *X,
                         DevInst di, uint8_t *xbest);

// ---------------------------------------------------------------------------
// Factorised TU reformulation (lu_kernels.hip)
// ---------------------------------------------------------------------------
// A run of a level-scheduled in-place triangular solve: levels [a, b) in one
// workgroup (wide = 0), or positions [a, b) of one wide level (wide = 1).
struct LuSeg {
    int wide, a, b;
};
// Device arrays of one solve (positions in level order) and its launch plan
// (host array).
struct LuSolve {
    int r = 0, nseg = 0;
    int use_lds = 1;   // stage the vector and the run in LDS for one-workgroup runs when they fit
    const int *row = nullptr, *ptr = nullptr, *ent = nullptr, *lvl = nullptr;
    const LuSeg *seg = nullptr;
    // host copies: first position of each level, first entry of each level's first position
    const int *hlvl = nullptr, *hptr_at_lvl = nullptr;
};
// LDS that a one-workgroup run may stage the solved vector in.
constexpr size_t kLuLdsBytes = 64 * 1024;

// In-place solve; with xbar given, xbar[k] = 2 x[k] - xold[k] afterwards.
template <typename T>
void launch_lu_trsv(hipStream_t s, const LuSolve &sv, T *x, const T *xold = nullptr, T *xbar = nullptr);
void launch_lu_mv_f32(hipStream_t s, int lpr, int nrows, const int *rp, const int *ci, const int *val,
                      const float *x, float *y, float sgn);
void launch_lu_mv_f64(hipStream_t s, int lpr, int nrows, const int *rp, const int *ci, const int *val,
                      const double *x, double *y, double sgn, bool accumulate);
void launch_lu_tail_grad(hipStream_t s, int lpr, bool hasq, int r, int nk, const int *rpT, const int *ciT,
                         const int *valT, const float *wy, const int *rpQ, const int *ciQ, const int *valQ,
                         const float *x, const float *two_so, float *v);
void launch_lu_primal(hipStream_t s, int lpr, bool hasq, int nk, const int *rpT, const int *ciT,
                      const int *valT, const float *wy, const int *rpQ, const int *ciQ, const int *valQ,
                      const int *rpB, const int *ciB, const int *valB, const float *u, const float *x_in,
                      float *x_out, float *xbar, const float *ct, const float *tau1, const float *two_so,
                      const double *rho, DevCounters *ctr);
void launch_lu_dual_heavy(hipStream_t s, int nchunk, int nheavy, int m1, const int *ch_row, const int *ch_e0,
                          const int *ch_e1, const int *first, const int *order, const int *rowc0, const int *rp,
                          const int *ci, const int *val, const float *xbar, float *part, const float *omega,
                          const float *rt, float tau2, const float *y_in, float *y_out, float *wy);
void launch_lu_xbar_tail(hipStream_t s, int r, int nk, const float *x_new, const float *x_old, float *xbar);
void launch_lu_diff64(hipStream_t s, int n, const float *a, const float *b, double *d);
void launch_lu_res_rows(hipStream_t s, const Tiles &rt, int m1, const int *rp, const int *ci, const int *val,
                        const double *omega64, const int64_t *rhs, const double *d1, const double *d2,
                        const float *y_prev, const float *y, const double *tau2d, double *part);
void launch_lu_res_vars(hipStream_t s, const Tiles &vt, const double *qd, const float *x, const float *xp,
                        const double *rho, const double *tau1d, const double *two_sod, double *part);
void launch_lu_trsm(hipStream_t s, const LuSolve &sv, int *XI, int K);
void launch_lu_eval_rhs(hipStream_t s, int r, int K, const int *rp, const int *ci, const int *val,
                        const int64_t *dJ, const uint64_t *X, int *XI);
void launch_lu_eval_rows(hipStream_t s, int nch, int K, int nk, int m1, const int *ch_row, const int *ch_e0,
                         const int *ch_e1, const int *ch_slot, const int *ci, const int *val, const int64_t *rhs,
                         const uint64_t *X, const int *XI, int *vcnt, int64_t *rsum);
void launch_lu_eval_multi(hipStream_t s, int nslot, int K, int m1, const int *slot_row, const int64_t *rhs,
                          const int64_t *rsum, int *vcnt);
void launch_lu_eval_obj(hipStream_t s, int r, int K, const int64_t *c_tail, int64_t c0, const int *XI,
                        int nqch, int nk, const int *qch_row, const int *qch_e0, const int *qch_e1,
                        const int *ciQ, const int *valQ, const uint64_t *X, int64_t *zx);
void launch_lu_fill_i64(hipStream_t s, int64_t *p, int64_t v, int64_t n);
void launch_lu_fill_i32(hipStream_t s, int *p, int v, int64_t n);

}  // namespace gfors
