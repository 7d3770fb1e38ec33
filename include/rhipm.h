/*
 * rhipm: condensed reduced-space interior-point KKT kernels for AMD MI355X.
 *
 * C ABI of the hot path of the linearize-then-reduce interior-point method
 * (Pacaud et al., "Condensed interior-point methods: porting reduced-space
 * approaches on GPU hardware", Section 2.2 and Section 3):
 *
 *   rh_eval_residual             g(x,u), h(x,u), f(x,u)          (Section 2.1)
 *   rh_condense_reduced_hessian  K_cond = [I;S]^T K [I;S] and the condensed
 *                                right-hand side                 (Theorems 1-2,
 *                                eq. algo:reduction, Algorithm 1 "Reduction")
 *   rh_solve_condensed_kkt       dense Cholesky of K_cond (+ delta_w I), p_u,
 *                                then p_x, p_s, p_lambda, p_y    (Algorithm 1,
 *                                control/dual/slack/state/adjoint steps;
 *                                inertia theorem of Section 2.2.1)
 *
 * The optimisation problem is polar AC optimal power flow in the paper's
 * state-control form. Conventions (all arrays float64 unless stated):
 *
 *   buses 0..nb-1, lines 0..nl-1, generators 0..ng-1 (one per generator bus;
 *   the generator on the reference bus is "the reference generator").
 *   x  (nx) = [theta at non-reference buses, bus order ; Vm at PQ buses, bus order]
 *   u  (nu) = [Vm at generator buses, generator order ;
 *              Pg of non-reference generators, generator order]
 *   g  (nx) = [P balance at non-reference buses ; Q balance at PQ buses]
 *             (same order as x: P balance pairs with theta, Q balance with Vm)
 *   h  (m)  = [Pg_ref ; Qg of every generator ; |S_from|^2 of limited lines ;
 *              |S_to|^2 of limited lines], m = 1 + ng + 2 * (#lines with rate > 0)
 *   f       = sum_g c2 (base Pg)^2 + c1 (base Pg) + c0   (Pg in MW)
 *   lambda (nx) multiplies g, y (m) multiplies h + s = 0.
 *   Sigma_x (nx), Sigma_u (nu), Sigma_s (m): diagonal barrier terms.
 *   K = W + diag(Sigma_u, Sigma_x) + A^T diag(Sigma_s) A, W = Hessian of
 *   f + lambda^T g + y^T h.
 *   Residual r packed as [r1 (nu) ; r2 (nx) ; r3 (m) ; r4 (nx) ; r5 (m)] for the
 *   augmented system K_aug p = -r with the (s, y) coupling blocks +I (the sign
 *   that follows from the Lagrangian f + lambda^T g + y^T (h + s) - z^T s).
 *   Step p packed as [p_u (nu) ; p_x (nx) ; p_s (m) ; p_lambda (nx) ; p_y (m)].
 *
 * Memory: "device" pointers are HIP device memory (e.g. torch tensors'
 * data_ptr()), owned by the caller, contiguous. The library owns the handle,
 * the symbolic data, the LU factors and its workspaces. Every device call is
 * ordered on the stream given at rh_init_network. A handle is not thread safe.
 *
 * Errors: functions return rh_status and never abort. Positive codes are
 * numerical outcomes the caller acts on; negative codes are hard errors.
 */
#ifndef RHIPM_H
#define RHIPM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  RH_OK = 0,
  RH_NOT_POSDEF = 1,      /* Cholesky met a non-positive pivot: K_cond + delta_w I
                             is not positive definite (wrong inertia of K_aug)   */
  RH_SMALL_PIVOT = 2,     /* static-pivot refactorisation of G_x met |u_kk| below
                             1e-14 * max|row|: its factors (and K_cond) are not
                             used                                                */
  RH_NOT_CONVERGED = 3,
  RH_ERR_ARG = -1,        /* invalid argument (null pointer, bad size, bad data)  */
  RH_ERR_HIP = -2,        /* a HIP runtime call failed                            */
  RH_ERR_OOM = -3,        /* device or host allocation failed                     */
  RH_ERR_SINGULAR = -4,   /* G_x structurally singular                            */
  RH_ERR_STATE = -5       /* call order violated (e.g. solve before condense)     */
} rh_status;

/* Network description: HOST arrays, copied by rh_init_network / rh_analyze. */
typedef struct {
  int32_t nb, nl, ng;
  double base_mva;
  const int32_t* bus_type;   /* nb: 3 reference (exactly one), 2 PV, 1 PQ         */
  const double* pd;          /* nb: active load, p.u.                              */
  const double* qd;          /* nb: reactive load, p.u.                            */
  const double* vmin;        /* nb                                                 */
  const double* vmax;        /* nb                                                 */
  const int32_t* from;       /* nl                                                 */
  const int32_t* to;         /* nl                                                 */
  const double* r;           /* nl: series resistance, p.u.                        */
  const double* x;           /* nl: series reactance, p.u.                         */
  const double* b;           /* nl: total line charging, p.u. (half at each end)   */
  const double* rate;        /* nl: |S| limit, p.u.; <= 0 means unlimited          */
  const int32_t* gen_bus;    /* ng: distinct buses; exactly the PV + ref buses     */
  const double* c2;          /* ng: $/MW^2                                         */
  const double* c1;          /* ng: $/MW                                           */
  const double* c0;          /* ng: $                                              */
  const double* pmin;        /* ng, p.u.                                           */
  const double* pmax;
  const double* qmin;
  const double* qmax;
} rh_network_desc;

typedef struct {
  int32_t panel_width;       /* columns per condensation work-group; 0 = auto    */
  int32_t ordering;          /* symmetric ordering of G_x: 0 = minimum degree with
                                a level term (fewest sweep and refactorisation
                                levels; the default), 1 = plain minimum degree,
                                2 = nested dissection (more levels and fill on
                                power networks; a network whose LU rows then
                                exceed a sweep step is rejected)                */
  int32_t lds_panel;         /* 1 = keep panels in LDS when they fit, 0 = global,
                                2 = in LDS with the sweep metadata read from
                                global memory (width 1; chosen by 1 as well where
                                the panel alone fills the LDS)                  */
  int32_t refactor;          /* 0 = wave-resident refactorisation when every LU
                                row has at most 64 entries and U fits in LDS,
                                1 = always the level-staged kernel              */
  int32_t cond_waves;        /* waves per condensation work-group when it takes
                                one column with its panel in LDS: 1, 2, 4 or 8
                                (the waves split the record streams and, with 4
                                or 8, each sweep's same-level steps); 0 = auto (8
                                when the panel fills the LDS, else 2); other
                                shapes always run 1                             */
  int32_t sweep_grouping;    /* with several waves: 0 = auto (by the sweeps' step
                                and group counts), else 1 + a mask whose bit k
                                puts sweep k (L, U, U^T, L^T) on all the waves  */
} rh_options;

typedef struct {
  int64_t nx, nu, m, nb, nl, ng;
  int64_t nnz_gx, nnz_lu, nnz_gu, nnz_a, nnz_k;
  int64_t levels_lower, levels_upper;  /* level sets of the L / U sweeps         */
  int64_t refactor_ops;                /* multiply-adds of one refactorisation   */
  int64_t max_lu_row;
  int64_t panel_width, lds_panel;      /* chosen launch shape of the condensation:
                                          lds_panel 0 panels in global memory, 1 in
                                          LDS, 2 in LDS with the sweep metadata read
                                          from global memory (a panel that fills the
                                          LDS; one column per work-group) */
  int64_t max_row_ops;                 /* refactorisation multiply-adds of one row */
  int64_t refactor_kernel;             /* 0 wave-resident, 1 level-staged          */
  int64_t steps_lower;                 /* work-group passes of the L sweep         */
  int64_t sweep_steps;                 /* passes of all four sweeps of one column  */
  int64_t refactor_split;              /* leading levels factored one launch each,
                                          a task per work-group (wave-resident path) */
  int64_t cond_waves;                  /* waves per condensation work-group        */
  int64_t steps_l, steps_u, steps_ut, steps_lt;     /* passes of each sweep (L, U,
                                                       U^T, L^T) with one wave  */
  int64_t groups_l, groups_u, groups_ut, groups_lt; /* the same with the steps of a
                                                       level spread over 4 waves */
  int64_t sweep_grouped;               /* bit k set: sweep k (L, U, U^T, L^T) runs
                                          on all waves of a work-group, else on
                                          one (with 4 waves per work-group)     */
} rh_info;

typedef struct rh_symbolic rh_symbolic;
typedef struct rh_net rh_net;

const char* rh_status_str(rh_status s);

/* ---------------------------------------------------------------------------
 * Host-only symbolic analysis (no GPU needed). Builds the index maps, the
 * fixed sparsity patterns of G_x, G_u, A and K, a fill-reducing symmetric
 * ordering of G_x, the symbolic LU (static pivots on the diagonal), the level
 * sets of the four triangular sweeps and the refactorisation schedule. This is
 * the one-time host step that precedes GPU refactorisation (Section 3.1, SpRF;
 * Section 3.3). Returns RH_ERR_ARG on inconsistent data, RH_ERR_SINGULAR if
 * G_x is structurally singular (a bus with no line).
 * ------------------------------------------------------------------------- */
rh_status rh_analyze_network(const rh_network_desc* desc, const rh_options* opts,
                             rh_symbolic** out);
void rh_destroy_symbolic(rh_symbolic* sym);
rh_status rh_symbolic_info(const rh_symbolic* sym, rh_info* info);
/* Host arrays: x_kind[nx] (0 theta, 1 Vm), x_bus[nx]; u_kind[nu] (1 Vm, 2 Pg),
 * u_ref[nu] (bus for Vm, generator for Pg). Any pointer may be NULL. */
rh_status rh_symbolic_index_maps(const rh_symbolic* sym, int32_t* x_kind, int32_t* x_bus,
                                 int32_t* u_kind, int32_t* u_ref);
/* Host arrays: pattern of G_x in natural (row, column) = (g row, x index)
 * order as CSR with sorted columns; rowptr[nx+1], col[nnz_gx]; and the
 * symmetric pivot order perm[nx] (perm[k] = natural index eliminated k-th). */
rh_status rh_symbolic_gx_pattern(const rh_symbolic* sym, int32_t* rowptr, int32_t* col,
                                 int32_t* perm);
/* Host check of the symbolic data with caller-supplied numbers: refactorise
 * G_x (values in the CSR order of rh_symbolic_gx_pattern) with the same
 * schedule the GPU uses, then solve G_x z = b (transpose = 0) or
 * G_x^T z = b (transpose = 1) with the level-ordered sweeps. Host arrays. */
rh_status rh_symbolic_host_solve(const rh_symbolic* sym, const double* gx_values,
                                 const double* b, double* z, int32_t transpose);
/* 0 if every dependency of every sweep lies in an earlier level set, the
 * condensation's step schedule is consistent (each row written once, by
 * the last lane of its group, with exactly its entries, after the rows it
 * reads) and its step lists for work-groups of 4 and 8 waves hold every
 * step once, in schedule order, each group's steps of one level. */
rh_status rh_symbolic_check_levels(const rh_symbolic* sym);
/* Host check of the condensation's device records for panel width `width`
 * (1, 2, 3, 4, 8): emulates the condensation kernel lane by lane on random
 * values drawn from `seed` (G_x with a dominant diagonal, G_u, K, rt, r4) for
 * columns 0, nu/2 and the right-hand side, and compares with a dense
 * computation of the same columns of [I;S]^T K [I;S] (Section 3.3).
 * *max_rel_err (host) receives the largest error relative to each column's
 * largest entry. RH_ERR_ARG on a bad width or null pointer. */
rh_status rh_symbolic_check_condense(const rh_symbolic* sym, int32_t width, uint64_t seed,
                                     double* max_rel_err);

/* ---------------------------------------------------------------------------
 * Device handle. rh_init_network runs the analysis, uploads everything once
 * (host -> device) and allocates the workspaces. hip_stream: hipStream_t
 * (NULL = default stream). Errors: RH_ERR_ARG, RH_ERR_SINGULAR, RH_ERR_HIP,
 * RH_ERR_OOM.
 * ------------------------------------------------------------------------- */
rh_status rh_init_network(const rh_network_desc* desc, const rh_options* opts,
                          void* hip_stream, rh_net** out);
void rh_destroy_network(rh_net* net);
rh_status rh_get_info(const rh_net* net, rh_info* info);
rh_status rh_get_dims(const rh_net* net, int64_t* nx, int64_t* nu, int64_t* m);
rh_status rh_get_index_maps(const rh_net* net, int32_t* x_kind, int32_t* x_bus,
                            int32_t* u_kind, int32_t* u_ref);
/* Replace the loads (scenarios). Device arrays pd[nb], qd[nb]. */
rh_status rh_set_loads(rh_net* net, const double* pd_dev, const double* qd_dev);

/* ---------------------------------------------------------------------------
 * Batches (several networks or load scenarios condensed and solved together;
 * Section 3.3 per instance). A batch refers to existing handles, which must
 * not be used by other calls while a batch call runs (each batch call first
 * waits for the instances' own streams); the handles outlive the batch. Every
 * batched kernel serves all instances in one launch, except the condensation,
 * which takes one launch per class of instances of one panel width and
 * placement (each instance keeps its own launch shape); the kernel bodies are
 * those of the single-instance calls, so each instance's results equal, bit
 * for bit, those of rh_condense_reduced_hessian (with r) and
 * rh_solve_condensed_kkt on the same inputs. hip_stream: the batch's stream
 * (NULL = default). Errors: RH_ERR_ARG (an instance too large for LDS
 * staging), RH_ERR_OOM, RH_ERR_HIP.
 * ------------------------------------------------------------------------- */
typedef struct rh_batch rh_batch;
typedef struct {
  const double *x, *u, *lam, *y;          /* device, as rh_condense_reduced_hessian */
  const double *sig_x, *sig_u, *sig_s;
  const double* r;                        /* packed r1..r5 (required)                */
  double* K;                              /* nu x nu output, leading dimension ldk   */
  int64_t ldk;
  double* rhs;                            /* nu output                               */
} rh_batch_condense_item;
typedef struct {
  double* K;                              /* the instance's condensed matrix (overwritten) */
  int64_t ldk;
  double delta_w;
  const double* rhs;                      /* its condensed right-hand side           */
  const double* r;                        /* the r of the condensation               */
  double* p;                              /* the step, as rh_solve_condensed_kkt     */
} rh_batch_solve_item;
rh_status rh_batch_create(rh_net* const* nets, int32_t count, void* hip_stream, rh_batch** out);
void rh_batch_destroy(rh_batch* batch);
/* items: host array of count entries (pointers to device memory). Stream-
 * ordered on the batch stream, no host synchronisation. */
rh_status rh_batch_condense(rh_batch* batch, const rh_batch_condense_item* items);
/* items: host array of count entries. status: host array of count codes
 * (RH_OK, RH_NOT_POSDEF, RH_SMALL_PIVOT, RH_ERR_STATE) or NULL; returns the
 * first non-OK code or RH_OK. Synchronises the batch stream. RH_ERR_STATE if
 * an instance was not condensed with a right-hand side before. */
rh_status rh_batch_solve(rh_batch* batch, const rh_batch_solve_item* items, int32_t* status);
/* One batched step (condensation of every instance, then its solve and
 * recovery) captured once into a HIP graph on the batch stream (which must
 * not be NULL) and replayed: the graph's kernels read the instances'
 * descriptors and arguments from device arrays that rh_batch_replay
 * refreshes before each launch, so new items (same shapes) need no new
 * capture. solve items must use the condensation items' K, ldk, rhs and r.
 * rh_batch_replay: items may both be NULL (reuse the captured ones); status
 * as rh_batch_solve; RH_ERR_STATE without a capture. The graph holds kernel
 * launches only. */
rh_status rh_batch_capture(rh_batch* batch, const rh_batch_condense_item* citems,
                           const rh_batch_solve_item* sitems);
rh_status rh_batch_replay(rh_batch* batch, const rh_batch_condense_item* citems,
                          const rh_batch_solve_item* sitems, int32_t* status);

/* g (nx), h (m), f (1): device outputs at device inputs x (nx), u (nu)
 * (Section 2.1's functions of the state-control form). */
rh_status rh_eval_residual(rh_net* net, const double* x, const double* u,
                           double* g, double* h, double* f);

/* Reduction (Algorithm 1, "Reduction"): evaluates G, A, W at (x, u, lambda, y)
 * (Section 3.2), refactorises G_x on the device with the static pivots of the
 * analysis, and builds K_cond = [I;S]^T K [I;S] column block by column block
 * with the batched adjoint-adjoint products of Section 3.3: Z = -G_x^{-1} G_u V,
 * H = K [V; Z], Psi = G_x^{-T} H_x, K_cond V = H_u - G_u^T Psi.
 * All inputs/outputs are device arrays. K (output) is nu x nu column-major with
 * leading dimension ldk >= nu, symmetrised ((K + K^T)/2). If r is not NULL
 * (packed r1..r5, device), rhs (device, nu) receives the condensed right-hand
 * side b with K_cond p_u = b, riding along as one more column of the same
 * launch. Stream-ordered; no host synchronisation. Returns RH_SMALL_PIVOT only
 * from a later rh_solve_condensed_kkt (the pivot flag lives on the device). */
rh_status rh_condense_reduced_hessian(rh_net* net, const double* x, const double* u,
                                      const double* lam, const double* y,
                                      const double* sig_x, const double* sig_u,
                                      const double* sig_s, const double* r,
                                      double* K, int64_t ldk, double* rhs);

/* Control step and recovery (Algorithm 1): factorises K + delta_w I in place
 * (lower triangle; dense blocked Cholesky, FP64 MFMA trailing updates), solves
 * for p_u with rhs, then recovers p_x = -G_x^{-1}(r4 + G_u p_u),
 * p_lambda = -G_x^{-T}(rt_x + (K p)_x), p_s = -r5 - A p, p_y = -r3 - Sigma_s p_s
 * using the factors and K of the last rh_condense_reduced_hessian on this
 * handle (RH_ERR_STATE if none). When that condensation was given r, p_x and
 * p_lambda come from the columns it stored (Z = S e_j, Psi = G_x^{-T} H_x and
 * those of its right-hand-side column): r must then be the same residual. Device arrays: K (in: K_cond, out: Cholesky
 * factor in the lower triangle), rhs (nu), r (packed), p (packed step, output).
 * dev_status (device int32[2], may be NULL): [status, index of failing pivot].
 * The call synchronises the stream once and returns RH_SMALL_PIVOT if the last
 * refactorisation of G_x met a tiny pivot (checked first: K_cond and p are then
 * unusable), else RH_NOT_POSDEF when the Cholesky fails (p is then undefined). */
rh_status rh_solve_condensed_kkt(rh_net* net, double* K, int64_t ldk, double delta_w,
                                 const double* rhs, const double* r, double* p,
                                 int32_t* dev_status);

/* Allocation-free dense solve, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc). It is the Cholesky and solve stage of
 * rh_solve_condensed_kkt, with the same kernels and the same results bit for
 * bit, on a caller's matrix and with no network handle: K (device,
 * column-major, n x n, leading dimension ldk >= n; the lower triangle is read)
 * is factored in place (K + delta_w I = L L^T, L in the lower triangle) and
 * x (device, n) receives (K + delta_w I)^{-1} b; b (device, n) is not
 * modified. dev_status (device int32[2]): [0, or 1 when a pivot is not
 * positive; index of the first such pivot]. The workspaces (5.3 MB) live in
 * one static device array per device, which the library keeps until the
 * process ends: every call on a device shares it, so calls that overlap on
 * one device (other streams, other threads) race. 0 <= n <= 1024, else
 * RH_ERR_ARG. Enqueued on hip_stream (NULL: the null stream); the call does
 * not synchronise and returns RH_OK once the work is enqueued: the numerical
 * outcome is in dev_status. */
rh_status rh_cholesky_solve_noalloc(double* K, int64_t ldk, int32_t n, double delta_w,
                                    const double* b, double* x, int32_t* dev_status,
                                    void* hip_stream);

/* ---------------------------------------------------------------------------
 * Per-phase device timers (hipEvent pairs on the handle's stream), reported
 * like the paper's per-phase totals (Table 3: Chol., Reduction). Phases:
 * RH_PHASE_EVAL        derivative values, K assembly, condensed residual rt
 * RH_PHASE_REFACTOR    static-pivot refactorisation of G_x
 * RH_PHASE_CONDENSE    the fused solve / Hessian-product / adjoint kernel
 * RH_PHASE_SYMMETRIZE  (K + K^T)/2
 * RH_PHASE_CHOLESKY    dense Cholesky with forward/backward substitution
 * RH_PHASE_RECOVER     p_x, p_lambda, p_s, p_y
 * RH_PHASE_PROJECT     Newton-Raphson power flow (evaluations, refactorisations
 *                      and solves of the projection; rh_power_flow, RedLin)
 * rh_profile_enable resets the totals; rh_profile_read waits for the
 * recorded events and returns milliseconds and call counts per phase (host
 * arrays of RH_NPHASES entries, either may be NULL).
 * ------------------------------------------------------------------------- */
enum { RH_PHASE_EVAL = 0, RH_PHASE_REFACTOR, RH_PHASE_CONDENSE, RH_PHASE_SYMMETRIZE,
       RH_PHASE_CHOLESKY, RH_PHASE_RECOVER, RH_PHASE_PROJECT, RH_NPHASES };
rh_status rh_profile_enable(rh_net* net, int32_t on);
rh_status rh_profile_read(rh_net* net, double* ms, int64_t* calls);
/* In-kernel phase timestamps (device wall clock, 100 MHz) of the first
 * work-group of the last condensation launched while profiling was on (for
 * rh_condense_reduced_hessian, the right-hand-side column's tile, which runs
 * first):
 * [0] start, [1] panel filled, [2] after L, [3] after U (Z), [4] after the
 * Hessian product, [5] after U^T, [6] after L^T (Psi), [7] columns written,
 * [8] Z column stored (start of the product), [9] K record stream done
 * (before H is moved over the panel), [10] kernel entry (before the step
 * metadata is staged); [16 + l] end of level l of the L sweep; [128 + l] end of level l of the
 * wave-resident refactorisation; [256 + 8 k + j] the Cholesky's diagonal
 * work-group in factorisation launch k < 24 of the last solve (j = 0 start,
 * 1 previous panel applied, 2 slice factored, 3 stores issued). Host array
 * of 512 entries; synchronises the stream. */
rh_status rh_profile_kernel_trace(rh_net* net, int64_t* ticks);

/* Multiplies the objective (every generator cost coefficient) by scale > 0
 * in every later evaluation on this handle, until set again; 1 restores the
 * network's own costs. The interior-point driver sets it (objective scaling
 * at the initial point) and resets it to 1 when destroyed. Synchronises the
 * stream. RH_ERR_ARG for scale <= 0 or not finite. */
rh_status rh_set_objective_scale(rh_net* net, double scale);

/* ---------------------------------------------------------------------------
 * Interior-point method: Algorithm 1 ("LinRed"), each iteration evaluating
 * the derivatives, condensing the KKT system (rh_condense_reduced_hessian's
 * path), solving it with inertia correction (Section 4.3: K_cond + delta_w I
 * must be positive definite; delta_w grows until it is) and recovering the
 * step, then moving along it with a filter line search. The paper leaves the
 * line search, the barrier update and the initial point to the underlying
 * solver; this one follows the filter line-search method of Waechter and
 * Biegler (2006) without second-order correction or restoration phase (a
 * failed line search returns RH_NOT_CONVERGED), with a monotone barrier
 * update mu <- max(tol / 10, min(0.2 mu, mu^1.5)) once the scaled KKT error
 * of the barrier problem is below 10 mu. Bounds: Vm in [vmin, vmax], Pg in
 * [pmin, pmax], theta free; h (Pg_ref, Qg, |S_from|^2, |S_to|^2) in
 * [(pmin_ref, qmin, -inf, -inf), (pmax_ref, qmax, rate^2, rate^2)] through the
 * slack s = -h. Initial point: the caller's (x0, u0) or, if both are NULL,
 * theta = 0, Vm = 1, Pg mid-range; pushed inside its bounds; s = -h pushed
 * inside its bounds; lambda = y = 0; bound multipliers 1.
 * ------------------------------------------------------------------------- */
typedef struct rh_ipm rh_ipm;

typedef struct {
  double tol;            /* stop when the scaled KKT error E_0 <= tol (default 1e-6) */
  int32_t max_iter;      /* default 200                                              */
  int32_t reserved0;
  double mu_init;        /* default 0.1                                              */
  double obj_scale;      /* > 0: objective scale; 0: min(1, 100 / max|grad f(w0)|)   */
  int64_t reserved[4];
} rh_ipm_options;

typedef struct {
  int64_t iter;          /* iterations taken so far                                  */
  double obj;            /* objective f (unscaled) at the current point              */
  double inf_pr;         /* max(|g|, |h + s|) at the current point                   */
  double err;            /* scaled KKT error E_0 at the start of this call           */
  double mu;             /* barrier parameter used by the step                       */
  double alpha_pr;       /* primal step length                                       */
  double alpha_du;       /* bound-multiplier step length                             */
  double delta_w;        /* inertia-correction shift used (0 if none)                */
  int64_t ls_trials;     /* line-search trial points evaluated                       */
  double obj_scale;      /* objective scale in use                                   */
  int32_t converged;     /* 1: E_0 <= tol at the start of this call (no step taken)   */
  int32_t pf_iters;      /* RedLin: Newton-Raphson steps of this call's projections  */
} rh_ipm_info;

/* Fills the defaults. */
rh_status rh_ipm_default_options(rh_ipm_options* opts);
/* Creates the solver on a network handle (which it then drives; the handle's
 * other calls must not be interleaved with the solver's). opts may be NULL
 * (defaults). x0 (nx), u0 (nu): device initial point, both or neither.
 * Allocates its device vectors and two nu x nu matrices. Errors: RH_ERR_ARG,
 * RH_ERR_OOM, RH_ERR_HIP. */
rh_status rh_ipm_create(rh_net* net, const rh_ipm_options* opts, const double* x0,
                        const double* u0, rh_ipm** out);
/* One iteration. If the point already satisfies E_0 <= tol, takes no step and
 * sets info->converged. Returns RH_NOT_CONVERGED when the line search fails,
 * the inertia correction exceeds 1e40 or max_iter iterations were taken;
 * RH_SMALL_PIVOT when the refactorisation of G_x at this iterate met a tiny
 * static pivot: no step is taken and the iterate is unchanged. info (host)
 * may be NULL.
 * Synchronises the stream a few times per iteration. */
rh_status rh_ipm_step(rh_ipm* ipm, rh_ipm_info* info);
/* Iterates until converged (RH_OK) or a step fails (its code). */
rh_status rh_ipm_solve(rh_ipm* ipm, rh_ipm_info* info);
/* One iteration of every solver of a batch in lockstep (Algorithm 1 for load
 * scenarios or networks solved together). Solver i must drive the batch's
 * network i (rh_batch_create over the same handles, in the same order). The
 * evaluations, bound-multiplier steps, filter line searches (one trial per
 * unfinished solver per round) and updates run per solver, on the solvers'
 * streams, with their scalars read together; the condensation and the first
 * solve (delta_w = 0) run as one batched launch each over all instances
 * (rh_batch_condense / rh_batch_solve); inertia-correction retries run per
 * solver. A solver whose point already satisfies the tolerance takes no step
 * (info converged = 1, as rh_ipm_step). infos[count], codes[count] (host,
 * optional): each solver's info and status as rh_ipm_step would return them;
 * the iterates equal rh_ipm_step's on each solver bit for bit. Returns RH_OK,
 * or a negative code on a hard error (RH_ERR_ARG for a solver not on the
 * batch's network i). */
rh_status rh_ipm_batch_step(rh_batch* batch, rh_ipm* const* ipms, rh_ipm_info* infos,
                            int32_t* codes);
/* Device copies of the current point (any pointer may be NULL). */
rh_status rh_ipm_get_state(const rh_ipm* ipm, double* x, double* u, double* s, double* lam,
                           double* y);
/* ---------------------------------------------------------------------------
 * Differentiation of the solution in the loads (implicit function theorem
 * at the final barrier problem). With the bound multipliers eliminated, the
 * barrier problem's first-order conditions F(w, s, lambda, y; Pd, Qd) = 0 have
 * the augmented matrix K_aug of the KKT system (Section 2.2.1, eq.
 * kktmatrix:normal) as Jacobian, so d(solution)/d(loads) = -K_aug^{-1} dF/dp.
 * K_aug is symmetric: the gradient of a weighted sum of outputs needs one
 * adjoint solve K_aug xi = c, done by the reduction and condensation of
 * Theorems 1-2 (the condensed matrix at the final iterate, its Cholesky
 * factor, two sparse triangular solves for the recovery), then the sparse
 * product -xi^T dF/dp: the loads enter the P balance rows (non-reference
 * buses), the Q balance rows (PQ buses), h_0 = Pg_ref (Pd at the reference
 * bus), h_{1+g} = Qg (Qd at generator buses) and, through the cost of Pg_ref,
 * the stationarity rows (2 c2_ref base^2 grad h_0 in Pd_ref).
 * ------------------------------------------------------------------------- */
/* Outputs at the current point, device arrays (any may be NULL): pg[ng] in
 * generator order (the reference generator's Pg is -s_0, equal to
 * P_ref + Pd_ref at a solution), vm[nb] in bus order, f[1] the objective with
 * the network's own (unscaled) costs. Stream-ordered; RH_ERR_ARG, RH_ERR_HIP. */
rh_status rh_ipm_outputs(const rh_ipm* ipm, double* pg, double* vm, double* f);
/* Gradient of L = dpg . Pg + dvm . Vm + df * f (outputs as rh_ipm_outputs)
 * with respect to the loads: gpd[nb], gqd[nb] (device, in the units of the
 * descriptor's pd, qd). dpg[ng], dvm[nb], df[1] are device arrays; a NULL
 * weight counts as zero. xi (device, nu + 2 nx + 2 m, optional) receives the
 * adjoint solution packed as the step of rh_solve_condensed_kkt. Requires a
 * converged solver (RH_ERR_STATE otherwise); the network must hold the loads
 * it was solved with. Sigma is the final iterate's (bound multiplier / bound
 * slack), with no inertia correction: RH_NOT_POSDEF if the condensed matrix
 * is not positive definite there, RH_SMALL_PIVOT if the refactorisation of
 * G_x met a tiny static pivot (in both cases no gradient is written). Overwrites the solver's step buffers (a later
 * rh_ipm_step recomputes them). Synchronises the stream. */
rh_status rh_ipm_backward(rh_ipm* ipm, const double* dpg, const double* dvm, const double* df,
                          double* gpd, double* gqd, double* xi);
/* rh_ipm_backward for every solver of a batch at once (solver i on the
 * batch's network i, all converged; the network i must hold the loads its
 * solver was solved with): the condensation with the adjoint right-hand
 * sides and the solve are one batched launch each. Host arrays of count
 * device pointers: dpg, dvm, df (the arrays or their entries may be NULL:
 * zero weights), gpd, gqd (outputs, nb entries each). codes[count] (host,
 * optional): each solver's status as rh_ipm_backward's (RH_NOT_POSDEF or
 * RH_SMALL_PIVOT: no gradient written for it). The gradients equal rh_ipm_backward's bit for
 * bit. Returns RH_OK, RH_ERR_STATE if a solver has not converged, or another
 * negative code on a hard error. Synchronises the batch's stream. */
rh_status rh_ipm_batch_backward(rh_batch* batch, rh_ipm* const* ipms, const double* const* dpg,
                                const double* const* dvm, const double* const* df,
                                double* const* gpd, double* const* gqd, int32_t* codes);
/* Frees the solver and restores the network's objective scale to 1. */
void rh_ipm_destroy(rh_ipm* ipm);

/* ---------------------------------------------------------------------------
 * Newton-Raphson power flow: the projection of Algorithm 2 (Section 2.3.1,
 * implicit function theorem; the paper's tolerance 1e-10). x (device, nx,
 * natural order) is the start and receives the solution of g(x, u) = 0 for
 * the control u (device, nu). Every iteration evaluates g, reads max |g|,
 * refactorises G_x with the static pivots of the analysis and solves
 * G_x dx = g with the condensation's triangular sweeps (x -= dx). Stops when
 * max |g| <= tol (RH_OK) or after max_iter steps or a non-finite residual
 * (RH_NOT_CONVERGED; x holds the last iterate). iters, residual (host,
 * optional): steps taken and the last max |g|. Synchronises the stream once
 * per step. RH_ERR_ARG for tol <= 0, max_iter < 0 or null pointers.
 * ------------------------------------------------------------------------- */
rh_status rh_power_flow(rh_net* net, const double* u, double* x, double tol, int32_t max_iter,
                        int32_t* iters, double* residual);

/* ---------------------------------------------------------------------------
 * Reduce-then-linearize interior-point method: Algorithm 2 ("RedLin",
 * Section 2.3). The state is eliminated by the projection (rh_power_flow at
 * tolerance 1e-10, at most 20 steps, warm-started from the linearised state
 * step); the bounded states (Vm at PQ buses) move into
 * h_r = [h; -x_b] with slacks s_r = [s_h; s_x] (m + nxb entries, s_x bounded
 * by the state bounds); each iteration computes the adjoint
 * lambda = -G_x^{-T}(grad_x f + A_x^T y_h - y_x), condenses the reduced KKT
 * system (eq. reduced:kktsystem, +I reading of its (s, y) blocks) through
 * the full-space condensation (with g = 0 it equals the reduced one with the
 * state slacks' Sigma in place of Sigma_x and r4 = 0), factors it with
 * inertia correction, and runs the filter line search of rh_ipm_step on
 * (u, s_r, y_r), projecting every trial point (a trial whose projection fails
 * is rejected). Barrier update, constants, initial point and objective
 * scaling as rh_ipm_* (the scale is taken at the projected initial point;
 * RH_NOT_CONVERGED from create if that projection fails). info->pf_iters:
 * Newton steps of the call's projections. Handles, streams and errors as
 * rh_ipm_*.
 * ------------------------------------------------------------------------- */
typedef struct rh_redlin rh_redlin;
rh_status rh_redlin_create(rh_net* net, const rh_ipm_options* opts, const double* x0,
                           const double* u0, rh_redlin** out);
rh_status rh_redlin_step(rh_redlin* rl, rh_ipm_info* info);
rh_status rh_redlin_solve(rh_redlin* rl, rh_ipm_info* info);
/* Device copies of the current point (any pointer may be NULL): x[nx],
 * u[nu], s[m + nxb] (s_h, then the bounded states' slacks), lam[nx] (the
 * adjoint of the last iteration), y[m + nxb]. */
rh_status rh_redlin_get_state(const rh_redlin* rl, double* x, double* u, double* s, double* lam,
                              double* y);
/* Sizes of the reduced slack vector: mr = m + nxb, nxb bounded states. */
rh_status rh_redlin_dims(const rh_redlin* rl, int64_t* mr, int64_t* nxb);
/* Frees the solver and restores the network's objective scale to 1. */
void rh_redlin_destroy(rh_redlin* rl);

#ifdef __cplusplus
}
#endif
#endif /* RHIPM_H */
