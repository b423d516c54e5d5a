/*
 * gfors.h -- C ABI of the GFORS hot path on MI355X (gfx950).
 *
 * The library solves (heuristically) binary integer programs of the form
 *
 *     min <x, Q x> + <c, x>   s.t.  A x >= b,  B x = d,  x in {0,1}^n     (eq. bip, Sec. 1)
 *
 * with the loop of Algorithm 1: PDHG steps (Algorithm 2) on the penalised
 * saddle problem (eq. saddle, Sec. 2) interleaved with rounds of Bernoulli
 * sampling (Algorithm 3) whose candidates are evaluated exactly (EvalBest,
 * Sec. 3) into an incumbent.  Preprocess and UpdatePenalty follow Sec. 3.
 *
 * Conventions
 *   - Every call returns GFORS_OK (0) or a negative status; no exception crosses
 *     the ABI.  gfors_last_error() gives a message (thread-local).
 *   - Host arrays passed in are only read during the call.
 *   - Device memory: the caller supplies ONE device workspace of at least
 *     gfors_workspace_bytes() bytes and a HIP stream; the library carves all of
 *     its device buffers out of that workspace, never frees it, and enqueues all
 *     device work on that stream.  The workspace must stay alive until
 *     gfors_destroy_problem().  Device pointers taken by a call (p_override,
 *     viol_dev, obj_dev) are read/written on the same stream.
 *   - Calls marked "async" only enqueue work; device faults surface as
 *     GFORS_E_HIP at the next synchronising call.  A handle is not thread-safe.
 *   - Coefficients are integers (int32), right-hand sides and costs int64;
 *     objective values are exact int64, violation counts int32.
 */
#ifndef GFORS_H
#define GFORS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    GFORS_OK = 0,
    GFORS_E_ARG = -1,         /* malformed argument (shape, index, range, NULL) */
    GFORS_E_NONINT = -2,      /* reserved (non-integer data) */
    GFORS_E_OOM = -3,         /* workspace too small / size beyond limits */
    GFORS_E_HIP = -4,         /* a HIP runtime call failed */
    GFORS_E_STATE = -5,       /* call not valid in the handle's current state */
    GFORS_E_INFEAS_ROW = -6   /* all-zero row that no x can satisfy */
};

typedef struct gfors_problem gfors_problem;   /* opaque, owned by the library */

/* Integer CSR matrix on the host.
 *   row_ptr  int64[nrows+1], row_ptr[0] = 0, non-decreasing, row_ptr[nrows] = nnz < 2^31
 *   col_idx  int32[nnz], each in [0, ncols)
 *   val      int32[nnz] coefficients, or NULL meaning every coefficient is 1 */
typedef struct {
    int64_t nrows, ncols;
    const int64_t *row_ptr;
    const int32_t *col_idx;
    const int32_t *val;
} gfors_csr;

/* Tunables of Algorithm 1 and Sec. 3.  gfors_default_params() fills defaults.
 *   sigma        tau1 * tau2 <= sigma (Preprocess, Sec. 3)
 *   tau1, tau2   explicit step sizes if > 0; else derived: Q = 0 gives
 *                tau1 = tau2 = sqrt(sigma); Q != 0 gives tau1 = min(sqrt(sigma),
 *                1/(2 L_max)), L_max = 2(||Q~|| + rho_max), tau2 = sigma / tau1
 *   rho_min, rho_max, rho_delta  UpdatePenalty bounds / increment; a negative
 *                value means "derive": with g = ||c~||_inf + ||Q~||_2 the defaults
 *                are 1e-3 g, g and 1e-4 g
 *   rho_T, rho_p growth constants of UpdatePenalty
 *   k_int        sampling interval used by gfors_run_rounds()
 *   K_max        largest K accepted by gfors_sample_eval (multiple of 64, <= 4096)
 *   power_iters  power-iteration count for the spectral norms of Preprocess
 *   hist_cap     rounds of incumbent history kept on the device
 *   autotune     1: time the candidate SpMV launch shapes (lanes per row, fused
 *                or XCD-sliced) on the problem at creation and keep the fastest;
 *                0: use the size heuristic (deterministic choice)
 *   x0           starting point x_0 = x0 * 1 (in [0,1])
 *   seed         Philox4x32-10 key (low 32 bits = key word 0, high = key word 1)
 *   eval_mfma    1: evaluate long general rows (EvalBest, Sec. 3) as dense
 *                blocks of <= 32 rows on the int8 matrix cores when every block
 *                is at least half full and every coefficient has at most 3
 *                signed base-256 digits (results identical to the row-by-row
 *                sums); 0: always row by row.  The workspace grows by
 *                3 (2 nnz(A,B) + 48 (m1 + m2)) bytes when 1.
 *   repair_row0  -1: off.  Otherwise the inequality rows [repair_row0, m1) are
 *                set-partitioning rows relaxed from "= 1" to ">= 1" (monotone
 *                relaxation, Sec. 2.4), and every sampled candidate is repaired
 *                on the device before it is evaluated: in each such row only the
 *                cheapest set variable (lowest c, then lowest index) stays set.
 *                Violation counts, objectives and the incumbent are then those
 *                of the repaired candidates; they equal the evaluation on the
 *                original rows "= 1" (after the repair a row holds at most one
 *                set variable, so ">= 1" holds iff "= 1" does).  Checked at
 *                creation (E_ARG otherwise): one instance, Q = 0, each row
 *                non-empty with all coefficients +1, distinct columns and
 *                b = 1, each of its variables with c >= 0, in no other such row,
 *                in no equality row and with no positive coefficient in rows
 *                [0, repair_row0).  The workspace grows by 4 (nnz(A,B) + m1 + 1)
 *                bytes when >= 0.
 *   lu_wide_rows factorised TU problems only (gfors_create_problem_tu): a level
 *                of a triangular solve with at least this many rows is solved
 *                by a launch of its own (one thread per row); runs of narrower
 *                levels share one one-workgroup launch.  Default 4096, >= 1.
 *   lu_lds       factorised TU problems only: 1 (default) stages the solved
 *                vector in LDS for a one-workgroup run when it fits in 64 KiB;
 *                0 keeps it in global memory.  Results are identical. */
typedef struct {
    double sigma, tau1, tau2;
    double rho_min, rho_max, rho_T, rho_p, rho_delta;
    int32_t k_int, K_max, power_iters, hist_cap, autotune;
    double x0;
    uint64_t seed;
    int32_t eval_mfma;
    int64_t repair_row0;
    int32_t lu_wide_rows, lu_lds;
} gfors_params;

void gfors_default_params(gfors_params *p);

/* Device workspace size for a problem with these dimensions.  n variables,
 * m1 inequality rows, m2 equality rows, nnz of A, B and Q (Q in full symmetric
 * storage), num_instances >= 1 (block-diagonal batch). */
int gfors_workspace_bytes(int64_t n, int64_t m1, int64_t m2, int64_t nnzA, int64_t nnzB,
                          int64_t nnzQ, int32_t num_instances, const gfors_params *p,
                          size_t *bytes);

/* Build a problem (eq. bip) and run Preprocess (Sec. 3) on the device.
 *   A, b     inequality rows A x >= b (A may be NULL: m1 = 0; b int64[m1])
 *   B, d     equality rows B x = d (B may be NULL: m2 = 0; d int64[m2])
 *   Q        symmetric quadratic term in full storage (NULL: Q = 0)
 *   c        int64[n] linear costs
 *   num_instances / inst_offsets  a batch of independent instances stored
 *            block-diagonally: inst_offsets is int64[(num_instances+1)*3]
 *            holding, per instance, the start of its (variable, inequality row,
 *            equality row) ranges; NULL when num_instances == 1.  Every row and
 *            every Q entry must stay inside its instance's variable range.
 *   ws, ws_bytes, stream  device workspace and HIP stream (see Conventions)
 * Errors: E_ARG (malformed CSR, index out of range, row crossing instances),
 *         E_INFEAS_ROW (zero row with b_j > 0 or d_j != 0), E_OOM (workspace
 *         too small), E_HIP.  Synchronises the stream before returning. */
int gfors_create_problem(const gfors_csr *A, const int64_t *b,
                         const gfors_csr *B, const int64_t *d,
                         const gfors_csr *Q, const int64_t *c, int64_t n,
                         int32_t num_instances, const int64_t *inst_offsets,
                         const gfors_params *p, void *ws, size_t ws_bytes,
                         void *stream, gfors_problem **out);

void gfors_destroy_problem(gfors_problem *P);
const char *gfors_last_error(void);

/* For callers that cannot allocate device memory (code that must not call
 * hipMalloc, serving loops, harnesses that forbid allocation): as
 * gfors_create_problem, but the problem's device memory is a file-scope array
 * of GFORS_STATIC_WS_BYTES bytes inside the library instead of a caller
 * workspace.  Every GPU the library runs on holds its own copy of that array
 * until the process ends; it serves ONE live problem per device at a time
 * (the device current at this call).  No device memory is allocated by this
 * call; the launch shapes come from the size heuristic (params->autotune is
 * taken as 0, so the problem computes exactly what gfors_create_problem with
 * autotune = 0 computes).  Later calls on the handle are the ordinary ones.
 * The array keeps whatever the previous problem left; creation initialises
 * everything the method reads, as it does for an uninitialised workspace.
 * Calls that overlap on one device race: a second creation while a problem
 * created here is alive on the same device returns E_STATE, and
 * gfors_destroy_problem releases the array.
 * Errors: those of gfors_create_problem; E_OOM (with the sizes in the
 * message) when gfors_workspace_bytes of the problem exceeds
 * GFORS_STATIC_WS_BYTES; E_STATE as above. */
#define GFORS_STATIC_WS_BYTES (32u << 20)
int gfors_create_problem_static(const gfors_csr *A, const int64_t *b,
                                const gfors_csr *B, const int64_t *d,
                                const gfors_csr *Q, const int64_t *c, int64_t n,
                                int32_t num_instances, const int64_t *inst_offsets,
                                const gfors_params *p, void *stream, gfors_problem **out);

/* Run nsteps PDHG iterations (Algorithm 2) at the current penalty rho of each
 * instance.  If want_residuals != 0 the last step also computes, in FP64, the
 * residuals of Theorem 2 and the CheckHalt gaps (read with gfors_get_residuals).
 * Async. */
int gfors_pdhg_steps(gfors_problem *P, int32_t nsteps, int32_t want_residuals);

/* One sampling round (Algorithm 3 + EvalBest): K candidates per instance
 * (K % 64 == 0, 64 <= K <= K_max) drawn from p = x_k, or from the caller's
 * device array p_override (float[n], values in [0,1]; NULL = use x_k).  The
 * uniform of candidate l, local variable i of instance t in round r is
 * U = word (l & 3) of Philox4x32-10(key = (seed & 0xffffffff, seed >> 32),
 * counter = (l >> 2, i, r, t)), taken as u = (U >> 8) 2^-24; candidate bit =
 * [u < p_i] (strict, so p = 0 never and p = 1 always gives a one).  One
 * generator call thus serves four consecutive candidates of one variable.
 * Every candidate is evaluated exactly on the original integer data; the
 * feasible candidate with the least objective (lowest index on ties) replaces
 * the incumbent on strict improvement.  Then the trigger counter advances and rho follows
 * UpdatePenalty (Sec. 3).  viol_dev (int32[T*K]) and obj_dev (int64[T*K]),
 * if not NULL, receive the per-candidate violation counts and objectives.
 * Async. */
int gfors_sample_eval(gfors_problem *P, int32_t K, const float *p_override,
                      int32_t *viol_dev, int64_t *obj_dev);

/* As gfors_sample_eval; flags = GFORS_SAMPLE_NO_TRIGGER draws an additional
 * round inside the current trigger: it consumes a Philox round id and updates
 * the incumbent but neither advances the trigger counter nor changes rho
 * (k_r > 1 rounds per trigger of Algorithm 1, e.g. from a second proposal). */
#define GFORS_SAMPLE_NO_TRIGGER 1
int gfors_sample_eval_ex(gfors_problem *P, int32_t K, const float *p_override,
                         int32_t *viol_dev, int64_t *obj_dev, int32_t flags);

/* Customized sampling for the 3D assignment problem (Algorithm 4, Sec. 2.4.2)
 * in place of the Bernoulli round; the problem's variables are x_ijk at index
 * (i n + j) n + k (n^3 of them, n <= 1024, one instance).  From p (p_override
 * or x_k): the min(gamma n, #{p > 0}) largest entries of p (descending, lower
 * index first on ties; gamma n <= 4096) give a conflict-free partial
 * assignment (an entry is taken when its i, j and k are all unused); each of
 * the K candidates completes it by matching the unassigned i's (ascending)
 * with random permutations of the free j's and k's (Fisher-Yates from
 * position r-1 down to 1, position t swapped with floor(u (t + 1)), u from
 * word 0 (j) / word 1 (k) of Philox4x32-10(key = seed, counter = (l, t, round,
 * 0xA5513D00)), u = (U >> 8) 2^-24), then takes L local steps: step q draws
 * triple a = floor(u n) from word 0 of counter (l, n + q, round, 0xA5513D00)
 * and applies, if its cost change is negative, the interchange of a's j or
 * k with another triple's that changes the cost least (ties: lower partner,
 * then the j interchange).  Candidates are then evaluated exactly on the
 * problem's rows and objective and merged into the incumbent as in
 * gfors_sample_eval_ex (same flags, viol_dev / obj_dev).  Async.
 * Errors: E_ARG (n^3 != number of variables, n > 1024, gamma n > 4096,
 * L < 0, bad K or flags, more than one instance). */
int gfors_sample_eval_assign3d(gfors_problem *P, int32_t n, int32_t K, int32_t gamma, int32_t L,
                               const float *p_override, int32_t *viol_dev, int64_t *obj_dev,
                               int32_t flags);

/* Evaluate round(x_k) = [x_k > 1/2] (last step of Algorithm 1) and merge it
 * into the incumbent (round id -1).  Does not advance rho.  Async. */
int gfors_final_round(gfors_problem *P);

/* nrounds x (k_int PDHG steps + one sampling round of K candidates), optionally
 * replayed from a captured HIP graph.  Async. */
int gfors_run_rounds(gfors_problem *P, int32_t nrounds, int32_t K, int32_t use_graph);

/* Incumbent of instance `inst` (synchronises).  z_best = INT64_MAX and found = 0
 * while no feasible candidate has been seen (z_best = +inf of Algorithm 1).
 * x_best_host: uint8[n_inst] or NULL.  info (or NULL): int64[4] =
 * {iteration k, round (-1 = final rounding), candidate index, triggers so far}. */
int gfors_best(gfors_problem *P, int32_t inst, int64_t *z_best, uint8_t *x_best_host,
               int32_t *found, int64_t *info);

/* FP64 residuals of the last instrumented step, per instance:
 * out[4*t + {0,1,2,3}] = {||s^x||_2, ||s^y||_2, primal gap, binary gap}. Syncs. */
int gfors_get_residuals(gfors_problem *P, double *out);

/* Per-round incumbent history of instance inst: z_best after each round
 * (INT64_MAX before the first feasible one).  *count gets the rounds done. Syncs. */
int gfors_get_history(gfors_problem *P, int32_t inst, int64_t *z_hist, int32_t cap, int32_t *count);

/* Test / resume support (all synchronise).  State after iteration k:
 * x = x_k, x_prev = x_{k-1} (float[n]), y = y_k (float[m1+m2], inequality rows
 * first), rho (double[T]), k, rounds done, triggers done. */
int gfors_get_state(gfors_problem *P, float *x, float *x_prev, float *y, double *rho,
                    int64_t *k, int64_t *round, int64_t *ntrig);
int gfors_set_state(gfors_problem *P, const float *x, const float *x_prev, const float *y,
                    const double *rho, int64_t k, int64_t round, int64_t ntrig);

/* Restart Algorithm 1 on the same data: x = x_{-1} = xbar = x0, y = 0,
 * rho = rho_min, counters zero, incumbent cleared (z_best = +inf), history
 * cleared.  Preprocess results are kept.  Synchronises. */
int gfors_reset(gfors_problem *P);

/* Candidates of the last sampling round: uint64[n * K/64], word w of variable
 * i at [i*(K/64) + w] holding candidates 64w..64w+63 (bit b = candidate 64w+b). */
int gfors_get_candidates(gfors_problem *P, uint64_t *bits_host, int32_t *K_out);

/* Preprocess results (synchronise).  row_scale double[m] = 1/||row_j||_2 (1 for a
 * zero row); per instance (double[T] each): obj_scale s_o = ||Q||_2 + ||c||_2,
 * K_norm s_K, Q_norm ||Q||_2 (unscaled), tau1, tau2, rho_min, rho_max, rho_delta.
 * Any pointer may be NULL. */
int gfors_get_scales(gfors_problem *P, double *row_scale, double *obj_scale, double *K_norm,
                     double *Q_norm, double *tau1, double *tau2, double *rho_min,
                     double *rho_max, double *rho_delta);

/* Profiling support: runs nsteps PDHG steps and one sampling round of K
 * candidates (advancing the state exactly like gfors_pdhg_steps +
 * gfors_sample_eval) with HIP events around every launch on the problem's
 * stream, synchronises, and writes the average duration in milliseconds of
 * each kernel kind to avg_ms[GFORS_NUM_KERNEL_TIMERS] (and the number of
 * launches timed to launches[], if not NULL).  Kernel kinds, in order: dual
 * step, primal step, sampler, covering-row evaluation, general-row evaluation,
 * quadratic objective, candidate reduction, incumbent update, x_best copy.
 * A kind that did not run reports 0. */
#define GFORS_NUM_KERNEL_TIMERS 9
int gfors_kernel_times(gfors_problem *P, int32_t nsteps, int32_t K, double *avg_ms,
                       int32_t *launches);

/* Profiling support: throughput of the sampler's uniform generator alone
 * (Philox4x32-10 of Algorithm 3's candidate draws, one call = four uniforms),
 * the peak against which the sampler's achieved rate is reported.  Enqueues a
 * warm-up and a timed launch of about `calls` generator evaluations on
 * `hip_stream` (a hipStream_t, NULL = default stream), synchronises, and
 * writes calls per second.  dev_sink: device memory of at least 4 bytes,
 * owned by the caller (written at most once, contents meaningless).
 * Errors: GFORS_E_ARG for calls <= 0 or NULL pointers, GFORS_E_HIP. */
int gfors_philox_throughput(void *hip_stream, int64_t calls, void *dev_sink, double *calls_per_s);

/* Achievable streaming read bandwidth of the device: `workgroups` workgroups
 * of 256 lanes read the caller's device buffer (bytes, a multiple of 16;
 * 16-byte aligned) with one 16-byte load per lane and step, 5 timed passes
 * after a warm-up on hip_stream; *bytes_per_s = bytes read per second.  A
 * reference for the HBM rooflines next to the published 8 TB/s.  dev_sink:
 * device memory of at least 4 bytes (written at most once).  E_ARG for bad
 * sizes or pointers, E_HIP. */
int gfors_read_throughput(void *hip_stream, const void *dev_buf, int64_t bytes, int32_t workgroups,
                          void *dev_sink, double *bytes_per_s);

/* Launch shapes in use: out[8] = {lanes per row of the dual SpMV, lanes per row
 * of the primal SpMV, column slices of the dual SpMV, slices of the primal,
 * SELL-64 layout for the dual (0/1), SELL-64 layout for the primal (0/1),
 * zero-operand skipping / layout variant of the dual (0..5), of the primal (0..7)}
 * (1 slice = fused kernel; with SELL the lanes-per-row entry is unused; dual
 * lanes per row 256 = a workgroup per row, longest rows first).  Skipping
 * keeps the nonzero bitmap of the gathered vector in LDS and issues only the
 * gathers of nonzero operands: 1 = sliced SELL dual / fused CSR primal,
 * 2 / 3 = batched-issue kernel on any SELL layout, two / four row chunks per
 * wavefront at once.  Primal 4 = no gathers from memory at all: wy is staged
 * in LDS slice by slice and every variable takes its terms from LDS (unit
 * coefficients, every variable in the same number <= 8 of rows, one
 * instance, Q = 0; the terms are added in the same order).  Dual 4 / primal
 * 5 = dense-block tiles for problems whose every row spans all variables of
 * its instance (at most 64 rows per instance, Q = 0: the knapsack batch): a
 * workgroup per 2,048 columns of one instance, xbar (dual) or wy (primal) of
 * the tile read once and reused by every row.  Dual 5 / primal 6 = light
 * items with signed indices (one instance, Q = 0, every |a| = 1, and the rows /
 * variables below 256 entries one contiguous range of the same number <= 8 of
 * entries: facility location): the heavy items keep a workgroup each, the
 * light ones read an entry-major copy of their indices with the
 * coefficient's sign in bit 31 instead of row pointers and coefficients (the
 * terms are added in the same order as with 1 lane per item).  Primal 7 =
 * primal 6 with the heavy variables in groups of up to 16 consecutive ones
 * whose rows are those of the group's first variable shifted by their
 * distance to it (same coefficients): the 16 variables of a group read wy of
 * one entry as 16 consecutive floats (their sums are added in another order
 * than with a workgroup per variable). */
int gfors_get_launch_cfg(gfors_problem *P, int32_t *out);

/* Re-run the autotuner on the current iterate (the zero-operand bitmap
 * variants only show their speed once x and y have reached the box bounds /
 * inactive duals).  The timed launches write no state.  Synchronises; drops
 * captured graphs. */
int gfors_autotune(gfors_problem *P);

/* Force launch shapes (same 8-entry layout as gfors_get_launch_cfg).  Lanes per
 * row: a power of two in [1, 64], or 256 for the dual with 1 slice, no SELL and
 * no skipping; slices: 1, or 8 when the problem holds the column-sliced copy
 * (then lanes <= 16; the primal also needs Q = 0); SELL only where the problem
 * holds the SELL copy; skipping 1 only for the sliced SELL dual / the fused CSR
 * primal, 2 and 3 only with a SELL layout, all without Q and with bitmaps of at most
 * 64 KB; primal 4 to 7 and dual 4, 5 only with 1 slice, no SELL, and where the
 * problem qualifies.
 * E_ARG otherwise (nothing is changed).  Drops captured graphs. */
int gfors_set_launch_cfg(gfors_problem *P, const int32_t *cfg);

/* ---------------------------------------------------------------------------
 * Learned sampling proposal.  The paper allows any GPU-compatible routine as
 * RandSampleStep (customized sampling, Sec. 2.4.2); this one draws the same
 * Philox Bernoulli candidates (pass its p as p_override to gfors_sample_eval)
 * from probabilities p = sigmoid(logit) of a bipartite message-passing network
 * over the constraint graph (hidden 64, 3 rounds, BF16 MFMA with FP32
 * accumulation), trained on the GPU against incumbents the method found:
 *   E     = diag(1/||a_j||) [A; B]   (a zero row has no edges)
 *   Fv_i  = [x_i, 4 x_i (1 - x_i), c~_i / max|c~|, 1]
 *   Fc_j  = [y_j / (1 + |y_j|), r~_j / max|r~|, [row j is an equality], 1]
 *   Hv = relu(Fv Uv + uv),  Hc = relu(Fc Uc + uc)
 *   3 times: Hc = relu([Hc | E Hv] [Wcc; Wcv] + bc); Hv = relu([Hv | E^T Hc] [Wvv; Wvc] + bv)
 *   logit = Hv wo + bo;  loss = mean_i softplus(logit_i) - t_i logit_i
 * Parameters: one flat float vector of GFORS_GNN_NUM_PARAMS entries in the order
 * Uv[4][64], uv[64], Uc[4][64], uc[64], 3 x {Wcc, Wcv [64][64], bc[64],
 * Wvv, Wvc [64][64], bv[64]} (W[in][out]), wo[64], bo.  All calls below run on
 * the problem's stream (gfors_gnn_create's stream for create/get/set/adam);
 * single-instance problems only (E_ARG otherwise). */
#define GFORS_GNN_NUM_PARAMS 50241
typedef struct gfors_gnn gfors_gnn;

/* Device workspace of a network (parameters, gradient, Adam moments, BF16
 * operand copies, reduction scratch). */
int gfors_gnn_workspace_bytes(size_t *bytes);
/* Create a network from host parameters (FP32 master copy on the device). */
int gfors_gnn_create(const float *params_host, void *ws, size_t ws_bytes, void *stream,
                     gfors_gnn **out);
void gfors_gnn_destroy(gfors_gnn *G);
/* Activation workspace for running the network on problem P (training = 1
 * keeps every round's activations and gradients). */
int gfors_gnn_act_bytes(gfors_problem *P, int32_t training, size_t *bytes);
/* Forward pass on P with iterate x_dev (float[n]) and duals y_dev (float[m]);
 * NULL takes P's current x_k / y_k.  p_dev (float[n]) receives sigmoid(logit),
 * logit_dev (float[n] or NULL) the logits.  Async. */
int gfors_gnn_forward(gfors_gnn *G, gfors_problem *P, const float *x_dev, const float *y_dev,
                      void *act, size_t act_bytes, float *p_dev, float *logit_dev);
/* Loss and gradient against target_dev (float[n] of 0/1); the gradient stays on
 * the device (gfors_gnn_get_grad).  loss_host (or NULL): synchronises. */
int gfors_gnn_grad(gfors_gnn *G, gfors_problem *P, const float *x_dev, const float *y_dev,
                   const float *target_dev, void *act, size_t act_bytes, float *loss_host);
/* One Adam step (beta 0.9 / 0.999, eps 1e-8) with the current gradient. Async. */
int gfors_gnn_adam(gfors_gnn *G, float lr);
/* gfors_gnn_grad followed by gfors_gnn_adam. */
int gfors_gnn_train_step(gfors_gnn *G, gfors_problem *P, const float *x_dev, const float *y_dev,
                         const float *target_dev, void *act, size_t act_bytes, float lr,
                         float *loss_host);
/* Host copies of the parameters / gradient (synchronise). */
int gfors_gnn_get_params(gfors_gnn *G, float *host);
int gfors_gnn_set_params(gfors_gnn *G, const float *host);
int gfors_gnn_get_grad(gfors_gnn *G, float *host);
int gfors_gnn_set_grad(gfors_gnn *G, const float *host);

/* ---------------------------------------------------------------------------
 * TU reformulation (Theorem of Sec. 2.4.1), host only.  pivots[r] names the
 * pivot column of equality row r (-1 keeps row r); J = the pivot rows, I =
 * their pivot columns.  B_J must be totally unimodular and B_JI invertible.
 * With x_I = s + S x_Ibar (s = B_JI^{-1} d_J, S = -B_JI^{-1} B_JIbar, computed
 * exactly in integers: read off the rows when B_JI is a signed identity, else
 * by Gauss-Jordan elimination on B_J, whose pivots are then +-1) it forms
 *   Q' = S^T Q_II S + S^T Q_IIbar + Q_IIbar^T S + Q_IbarIbar,
 *   A' = A_.I S + A_.Ibar, b' = b - A_.I s, B' = B_JbarI S + B_JbarIbar,
 *   d' = d_Jbar - B_JbarI s, c' = 2 S^T Q_II s + 2 Q_IIbar^T s + S^T c_I + c_Ibar,
 *   constant c'_0 = <s, Q_II s> + <c_I, s>  (Q symmetric, full storage, or NULL),
 * and appends the bound rows S_p x >= -s_p (all pivots, in pivot order) then
 * -S_p x >= s_p - 1, leaving out a bound row that every point of [0,1]^n'
 * satisfies.  Kept variables keep their relative order.  S is stored
 * explicitly (sparse), not as a factorisation of B_JI.
 *   pivots  int64[m2]: pivot column of equality row r, or -1 to keep row r.
 * Errors: E_ARG (bad CSR, pivot out of range, column pivot of two rows, B_JI
 * singular, a pivot entry other than +-1 in the elimination (B_J not TU), an
 * int32 overflow of a reformulated coefficient). */
typedef struct gfors_tu gfors_tu;
int gfors_tu_create(const gfors_csr *A, const int64_t *b, const gfors_csr *B, const int64_t *d,
                    const gfors_csr *Q, const int64_t *c, int64_t n, const int64_t *pivots,
                    gfors_tu **out);
/* Factorised form (Remark of Sec. 2.4.1), flags = GFORS_TU_FACTORED: the pivot
 * block is factorised once as M = L U (rows and columns in the elimination
 * order k; a column of fewest active entries and its shortest active row
 * pivot first; every entry of L and U in {-1, 0, 1}, else E_ARG: B_J is not
 * TU) and S is never formed: on the device S xbar = -M^{-1} (B_JIbar xbar) and
 * S^T v = -B_JIbar^T M^{-T} v are level-scheduled triangular solves inside
 * every PDHG step (gfors_create_problem_tu).  The reformulated model is the
 * same as without the flag (same rows in the same order, same kept bound
 * rows, same c' and c'_0); its row 2-norms and kept bound rows are computed
 * exactly on the host one row at a time, so host memory stays O(nnz(A, B, Q)
 * + nnz(L, U)).  Q must be symmetric.  gfors_tu_dims gives -1 for the entry
 * counts; gfors_tu_export copies only b', d', c' and kept_vars (E_STATE when
 * a matrix pointer is given); gfors_tu_export_q gives E_STATE. */
#define GFORS_TU_FACTORED 1
int gfors_tu_create_ex(const gfors_csr *A, const int64_t *b, const gfors_csr *B, const int64_t *d,
                       const gfors_csr *Q, const int64_t *c, int64_t n, const int64_t *pivots,
                       int32_t flags, gfors_tu **out);
/* info[10] of a factorised handle: {pivots r, nnz(L) strict, nnz(U) strict,
 * levels of the L forward, U backward, U^T forward and L^T backward solves,
 * nnz(B_JIbar), nnz(S) (counted, not stored), nnz of the reformulated rows}. */
int gfors_tu_factor_info(gfors_tu *U, int64_t *info);
/* A GFORS problem on the kept variables of a factorised handle (the handle
 * must outlive nothing: the problem copies what it needs).  Everything of
 * gfors_create_problem holds for it (one instance, the same calls and graph
 * replay, the same Preprocess, PDHG, sampling, evaluation and incumbent on
 * the reformulated model), with these differences:
 *   - Preprocess: the row 2-norms come from the host (exact); ||K'|| and
 *     ||Q'|| are FP64 power iterations whose products lift v to
 *     (v, S v) and project with S^T (FP64 triangular solves);
 *   - each PDHG step solves with L, U (lift of x_k) and U^T, L^T (S^T of the
 *     pivot part of the gradient), in FP32, level by level;
 *   - EvalBest solves every candidate's pivot variables exactly (int32) and
 *     checks the original rows on the lifted integer point: the violation
 *     count and objective equal those of the explicit reformulated model;
 *   - no repair_row0, autotuning, launch-shape control, 3D-assignment
 *     sampler or learned proposal (E_ARG).
 * gfors_workspace_bytes_tu gives the workspace size for params.  Errors as
 * gfors_create_problem, plus E_ARG for a handle made without
 * GFORS_TU_FACTORED and E_INFEAS_ROW for a reformulated row with no
 * coefficient that no point satisfies. */
int gfors_workspace_bytes_tu(gfors_tu *U, const gfors_params *params, size_t *bytes);
int gfors_create_problem_tu(gfors_tu *U, const gfors_params *params, void *workspace,
                            size_t workspace_bytes, void *hip_stream, gfors_problem **out);
/* dims[7] = {n', m1', m2', nnz(A'), nnz(B'), c'_0, nnz(Q')}. */
int gfors_tu_dims(gfors_tu *U, int64_t *dims);
/* Copy the reformulated model into caller arrays sized from gfors_tu_dims
 * (row pointers int64[m+1]; any pointer may be NULL); kept_vars int64[n']
 * gives the original index of each new variable. */
int gfors_tu_export(gfors_tu *U, int64_t *A_rp, int32_t *A_ci, int32_t *A_val, int64_t *b,
                    int64_t *B_rp, int32_t *B_ci, int32_t *B_val, int64_t *d, int64_t *c,
                    int64_t *kept_vars);
/* Q' in full symmetric CSR (row pointers int64[n'+1], columns and values of
 * nnz(Q') entries); nothing is written when Q' = 0. */
int gfors_tu_export_q(gfors_tu *U, int64_t *Q_rp, int32_t *Q_ci, int32_t *Q_val);
/* x_full (uint8[n]) from x_reduced (uint8[n']): x_I = s + S x_Ibar; E_STATE if
 * some x_p falls outside {0,1} (the reduced point violates a bound row). */
int gfors_tu_recover(gfors_tu *U, const uint8_t *x_reduced, uint8_t *x_full);
void gfors_tu_destroy(gfors_tu *U);
const char *gfors_tu_last_error(void);

/* ---------------------------------------------------------------------------
 * Monotone relaxation (Sec. 2.4, "Monotone Relaxation"), host only, for
 * set-partitioning equality rows  sum_{i in R} x_i = 1.  With a monotone
 * objective such a row may become  >= 1  without changing the optimum, and a
 * point of the relaxed problem is mapped back by a repair.
 *
 * gfors_mono_rows: relax[j] (uint8[m2], out) = 1 when equality row j has all
 * coefficients +1, d_j = 1, each of its variables has c_i >= 0, lies in no
 * other equality row and has no positive coefficient in any inequality row,
 * and Q = 0; else 0.  The caller moves the marked rows into the inequality
 * block with right-hand side 1 (the rows keep their coefficients).
 * gfors_mono_repair: x (uint8[n], in/out): in every marked row with more than
 * one variable set, the cheapest (lowest c, then lowest index) stays set and
 * the others are cleared.  A relaxed-feasible point becomes feasible for the
 * original rows with no larger objective.
 * Errors: E_ARG (NULL pointer, bad CSR). */
int gfors_mono_rows(const gfors_csr *A, const gfors_csr *B, const int64_t *d, const gfors_csr *Q,
                    const int64_t *c, int64_t n, uint8_t *relax);
int gfors_mono_repair(const gfors_csr *B, const uint8_t *relax, const int64_t *c, int64_t n,
                      uint8_t *x);
const char *gfors_mono_last_error(void);

/* Dimensions: n, m1, m2, number of instances. */
int gfors_get_dims(gfors_problem *P, int64_t *n, int64_t *m1, int64_t *m2, int32_t *T);

/* How EvalBest (Sec. 3) evaluates the general rows of this problem: *planes
 * = 1..3 when they run as dense int8 digit blocks on the matrix cores (the
 * number of signed base-256 digit planes), 0 when row by row.  The blocks
 * exist when gfors_params.eval_mfma allows them and the rows qualify; with
 * autotune the matrix-core kernel and the row-by-row kernels (rows split over
 * wavefronts / a wavefront per row) are timed on candidates drawn from
 * p = 1/2 and the fastest is kept (all give identical results). */
int gfors_eval_planes(gfors_problem *P, int32_t *planes);

#ifdef __cplusplus
}
#endif
#endif /* GFORS_H */
