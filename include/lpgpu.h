/*
 * lpgpu: dense revised simplex with an explicit basis inverse on one MI355X (gfx950).
 *
 * The LP is the standard form of Raeisi Gahrouei & Ghatee, "Effective Implementation
 * of GPU-based Revised Simplex algorithm applying new memory management and cycle
 * avoidance strategies" (arXiv 1803.04378), Section 2.1:
 *
 *     optimise  c^T x   s.t.  A' x + s = b,  x >= 0,  s >= 0,  b >= 0,
 *
 * with A' an m x n dense matrix and s the m slack variables, so that A = (A', I_m).
 * Variables are numbered 0..n-1 (structural) and n..n+m-1 (slack of row i is n+i).
 * The solver starts from the slack basis (feasible because b >= 0) and runs the
 * iteration of Section 2.1, Steps 3-8, with the Dantzig entering rule, the tabu
 * rule of Sections 2.2/3.4, and the tableau update of Section 3.1 applied to an
 * explicitly stored B^-1 that lives in device memory for the whole solve (the
 * "Case 1" memory layout of Section 3).
 *
 * lp_create_general adds the two-phase start of Section 3.4 (finding the initial
 * feasible solution): rows of type <=, >= or =, and b of any sign.
 *
 * All functions are thread-compatible, not thread-safe: one handle must not be used
 * from two threads at once.  No function aborts or throws; failures are reported as
 * negative return codes, and lp_error_string() describes the most recent failure of
 * the calling thread.
 */
#ifndef LPGPU_H
#define LPGPU_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- return codes (negative = error) ---- */
#define LP_OK 0
#define LP_ERR_ARG (-1)     /* NULL pointer, m <= 0, n < 0, non-finite data, m above LP_MAX_ROWS */
#define LP_ERR_NEG_RHS (-2) /* lp_create / lp_create_device: some b_i < 0, so the slack basis is infeasible
                               (lp_create_general accepts such LPs: it runs the two-phase start) */
#define LP_ERR_NOMEM (-3)   /* device, pinned or ordinary host memory could not be allocated; no
                               host exception leaves an entry point: it becomes this code, and a
                               handle under construction is released */
#define LP_ERR_DEVICE (-4)  /* a HIP runtime call failed (no GPU, bad stream, launch failure) */
#define LP_ERR_STATE (-5)   /* the handle is not in a state that allows the call */

/* ---- solve status ---- */
#define LP_RUNNING 0
#define LP_OPTIMAL 1    /* no nonbasic reduced cost below -eps_d (Step 4) */
#define LP_UNBOUNDED 2  /* the entering column has no entry alpha_i > eps_p (Step 5) */
#define LP_ITER_LIMIT 3 /* max_iter pivots done and the basis is not optimal; lp_solve resumes */
#define LP_NUMERICAL 4  /* the entering column Y_k had a non-finite entry, or the minimum ratio
                           overflowed: the solve stopped before that pivot */
#define LP_INFEASIBLE 5 /* lp_create_general: phase 1 ended with the sum of the artificial
                           variables above eps_f = 1e-9 (1 + max_i |b_i|): no x satisfies the rows */

/* ---- pivot-log flags ---- */
#define LP_PIVOT_DEGENERATE 1 /* step length theta == 0 */
#define LP_PIVOT_TIE 2        /* several rows reach zero (within eps_t) at the minimum step (Step 6) */
#define LP_PIVOT_ASPIRATION 4 /* every improving variable was tabu; chosen among all of them */
#define LP_PIVOT_LCLEAR 8     /* the tabu list of the entering variable excluded every tied row */
#define LP_PIVOT_DRIVEOUT 16  /* phase switch: a pivot with step 0 that replaced an artificial
                                 variable left basic at zero by phase 1 */

/* ---- row types of lp_create_general ---- */
#define LP_ROW_LE 0 /* a_i x <= b_i */
#define LP_ROW_GE 1 /* a_i x >= b_i */
#define LP_ROW_EQ 2 /* a_i x  = b_i */

#define LP_MIN 0
#define LP_MAX 1

/* ---- arithmetic of the pricing step ---- */
#define LP_FP64 0  /* every step in FP64 */
#define LP_MIXED 1 /* FP32 screening of the reduced costs, shortlist re-priced in FP64 */

/* Largest m the library accepts: the update kernel stages the pivot row rho and the entering
 * column a_q (8 bytes per row each) and the sparse-column index list (ld/8 int32) in the
 * 160 KB of LDS of one CU, next to 2.2 KB of its own: 16.5 * 9792 + 2256 <= 163840.  The
 * batched form has its own, smaller limit (LP_ERR_ARG from lp_batch_create). */
#define LP_MAX_ROWS 9792

typedef struct lp_options {
  int32_t sense;          /* LP_MIN or LP_MAX (default LP_MAX) */
  int32_t tabu_tenure;    /* a leaving variable may not re-enter for this many pivots (default 5; 0 = off) */
  int32_t leaving_list;   /* 1 = tie rows are broken by the entering variable's tabu list (default 1) */
  int32_t iters_per_sync; /* iterations issued per status read-back (default 16) */
  int64_t max_iter;       /* pivot limit for lp_solve (default 0 = 10*(m+n)) */
  double eps_d;           /* optimality tolerance on reduced costs (default 1e-9) */
  double eps_p;           /* pivot tolerance: rows with alpha_i > eps_p are ratio candidates (1e-9) */
  double eps_z;           /* after each pivot |x_B,i| < eps_z is set to 0 (default 1e-9) */
  double eps_t;           /* a row is tied in the ratio test when its value at the minimum step is
                             <= eps_t, i.e. it reaches zero with the leaving row (default 1e-9) */
  int32_t record_pivots;  /* 1 = keep the pivot log readable by lp_get_pivots (default 1) */
  int32_t profile;        /* 1 = time every kernel of the iteration with HIP event nodes in the
                             iteration graph (each time includes the launch gap before the
                             kernel); 2 = launch the kernels directly on the stream, each with
                             start and stop events bound to its own execution (no graph, no
                             gap); 0 = off (default) */
  int32_t batch_small_m;  /* batched solver: LPs with m <= this get one wavefront each, larger ones a
                             whole workgroup; -1 = chosen per m-bucket by timing (default) */
  void *stream;           /* hipStream_t to run on; NULL = a stream owned by the handle */
  int32_t precision;      /* LP_FP64 (default) or LP_MIXED: the reduced costs are first computed in
                             FP32 from an FP32 copy of A'; the shortlist_k smallest over nonbasic
                             non-tabu columns are re-priced in FP64 and the entering variable is the
                             best improving one among them.  When none of them improves, every
                             column is priced in FP64 (the plain Step 4), so optimality and the
                             aspiration case are always decided in FP64.  FTRAN, the ratio test
                             and the update stay FP64.  Every |A'_ij| must then be at most
                             FLT_MAX (else LP_ERR_ARG). */
  int32_t shortlist_k;    /* LP_MIXED: candidates re-priced in FP64, 1..16 (default 16) */
  int32_t reinv_period;   /* recompute B^-1, x_B, W and z from the basis (FP64 LU on the GPU) after
                             every this many pivots; 0 = never; -1 = default: 64 for LP_MIXED,
                             never for LP_FP64.  Takes effect at status read-backs, so it runs
                             exactly every reinv_period pivots when iters_per_sync divides it. */
  int32_t batch_binv_lds_m; /* batched solver: wide LPs with m <= this keep B^-1 in LDS (run by a
                             second persistent launch); 0 = never; -1 = the threshold is chosen by
                             timing the whole batch on its first solve (default) */
  int64_t device_budget;  /* bytes of device memory the LP may use (Section 3, Figure 2): 0 = the free
                             memory hipMemGetInfo reports (default); > 0 = at most this much.  The
                             whole tableau must fit (Case 1): an LP whose A', B^-1 and vectors
                             exceed the budget is rejected with LP_ERR_NOMEM.  (The row-panel
                             streaming of B^-1 from host memory, Case 2, is switched off in this
                             build: it has not been validated on the device.) */
} lp_options;

typedef struct lp_stats {
  int64_t iterations;       /* pivots done */
  int64_t degenerate;       /* pivots with theta == 0 */
  int64_t ties;             /* pivots with a tie in the ratio test */
  int64_t aspirations;      /* pivots whose entering variable was tabu */
  int64_t list_clears;      /* tabu lists cleared because they excluded every tied row */
  int64_t syncs;            /* status read-backs (one per batch of iters_per_sync iterations) */
  double solve_ms;          /* host wall time spent inside lp_solve calls */
  int64_t price_launches;   /* FP64 pricing kernels timed (profile = 1 or 2; LP_FP64 only, the mixed
                               form times its screening as price32_ms) */
  double price_ms;          /* their summed duration */
  int64_t update_launches;  /* update kernels timed (profile = 1 or 2) */
  double update_ms;         /* their summed duration */
  double price_bytes;       /* algorithmic bytes of those pricing launches: 8*m per priced column */
  double update_bytes;      /* algorithmic bytes of those update launches.  Dense mode: 8*m*m read, plus
                               16 per element pair written back (pairs whose pivot-row entries are
                               both zero are unchanged and not written).  With ld >= 1024 and while
                               at most ld/8 columns of B^-1 can differ from unit vectors (those of
                               slacks that left the basis since the last reinversion), only those
                               columns are read and updated: 8 per entry read or written, plus one
                               unit entry per row */
  int64_t finish_launches;  /* ratio-test finishing kernels timed (profile = 1 or 2) */
  double finish_ms;         /* their summed duration */
  int64_t ray;              /* after LP_UNBOUNDED: the entering variable with no positive alpha_i; else -1 */
  int64_t price32_launches; /* LP_MIXED: FP32 screening passes run */
  int64_t full_prices;      /* LP_MIXED: FP64 passes: after an iteration whose shortlist held no improving
                               column (it ends without a pivot), the next one prices every column in
                               FP64 (and is not counted in price32_launches), so that
                               every column was priced in FP64 */
  int64_t reinversions;     /* reinversions installed */
  int64_t reinv_failed;     /* reinversions abandoned because the basis block had a zero pivot
                               column (the updated B^-1 is then kept) */
  double reinv_ms;          /* device time of all reinversions */
  double price32_ms;        /* profile = 1 or 2, LP_MIXED: summed duration of the FP32 screening */
  double shortlist_ms;      /* profile = 1 or 2, LP_MIXED: summed duration of merge + FP64 re-price */
  double price32_bytes;     /* their algorithmic bytes: 4*m per nonbasic structural column */
  int64_t phase1_iterations; /* lp_create_general: pivots of phase 1 (the rest are phase 2 and
                                drive-outs); -1 while phase 1 runs or when it was not needed */
  int64_t drive_outs;       /* pivots flagged LP_PIVOT_DRIVEOUT */
  double phase_switch_ms;   /* host wall time of the switch (drive-outs and re-pricing) */
  int64_t memory_case;      /* 1: the tableau is in device memory (Section 3, Case 1; the only case
                               this build runs) */
  int64_t panel_rows;       /* 0 (Case 2 row panels are switched off) */
  int64_t panels;           /* 0 (Case 2 row panels are switched off) */
  int64_t price_fin_launches; /* FP64 form: pricing passes that also finished the previous iteration's
                                 ratio test (k_price_fin; counted in price_launches too) */
  double price_fin_ms;      /* their share of price_ms */
} lp_stats;

typedef struct lp_problem lp_problem;

/* Fills *opt with the defaults listed above.  Returns LP_OK or LP_ERR_ARG (opt NULL). */
int lp_default_options(lp_options *opt);

/*
 * Creates a problem from host arrays (Section 2.1 statement).
 *   A_colmajor: m*n doubles, entry (i,j) at A_colmajor[i + j*m]; b: m doubles (all >= 0);
 *   c: n doubles; opt: NULL for defaults.  The arrays are copied to device memory owned
 *   by the handle; the caller keeps ownership of its arrays.
 * Errors: LP_ERR_ARG, LP_ERR_NEG_RHS (checked before any device call), LP_ERR_NOMEM,
 * LP_ERR_DEVICE.  On error *out is set to NULL and nothing is leaked.
 */
int lp_create(lp_problem **out, int32_t m, int32_t n, const double *A_colmajor, const double *b,
              const double *c, const lp_options *opt);

/*
 * Creates an LP whose rows have types and whose right-hand sides have any sign:
 *   optimise c^T x  s.t.  row i of A' x  (<=, >=, =)  b_i,  x >= 0,
 * row_type[i] one of LP_ROW_LE, LP_ROW_GE, LP_ROW_EQ (row_type NULL = all LP_ROW_LE);
 * host arrays as in lp_create.  lp_solve runs the two-phase method (Section 3.4):
 *   - a row with b_i < 0 is multiplied by -1 (its type flips between <= and >=);
 *   - a <= row keeps its slack as the unit column; a >= row gets a surplus column -e_i,
 *     appended after the n given columns in ascending row order; a >= or = row gets an
 *     artificial variable as its unit column;
 *   - phase 1 minimises the sum of the artificial variables with the iteration of
 *     lp_solve; an artificial variable that leaves the basis never enters again;
 *   - its optimum above eps_f (LP_INFEASIBLE) stops the solve; else each artificial
 *     variable still basic (at zero) is replaced by a step-0 pivot on the largest |entry|
 *     of its row of the tableau (LP_PIVOT_DRIVEOUT; lowest column on equal magnitude,
 *     none above eps_p: the row is redundant and keeps it), the costs of the LP are
 *     restored, W = chat_B^T B^-1 and z = chat_B^T x_B are recomputed, and phase 2 runs.
 * When every row is <= after the sign change, no phase 1 runs.  Variable numbers in
 * pivot logs and bases: 0..n-1 the given columns, n..n+ns-1 the surplus columns, then
 * the unit column of row i.  lp_get_solution reports x (n values) and the objective of
 * the given LP, and y_i for the given row i (negated where the row was multiplied by -1).
 * LP_MIXED skips reinversions while phase 1 runs.  Not available in the batched form.
 * Errors: LP_ERR_ARG (also an unknown row type), LP_ERR_NOMEM, LP_ERR_DEVICE.
 */
int lp_create_general(lp_problem **out, int32_t m, int32_t n, const double *A_colmajor, const double *b,
                      const double *c, const int32_t *row_type, const lp_options *opt);

/*
 * Same as lp_create, but A_colmajor, b and c are device pointers of the current device
 * (for example the data of torch tensors).  The library copies them into its own
 * padded device layout before returning and never frees them; the caller may release
 * them once the call has returned.  Non-finite values and b_i < 0 are detected on the
 * device and reported as LP_ERR_ARG / LP_ERR_NEG_RHS.
 */
int lp_create_device(lp_problem **out, int32_t m, int32_t n, const double *A_colmajor, const double *b,
                     const double *c, const lp_options *opt);

/* Runs Steps 3-8 until OPTIMAL, UNBOUNDED, or opt.max_iter pivots in total.  *status_out
 * receives the LP_* status.  After LP_ITER_LIMIT a further call continues from the
 * device state.  Returns LP_OK or an error code. */
int lp_solve(lp_problem *p, int32_t *status_out);

/* As lp_solve, with the total pivot limit given by iter_cap instead of opt.max_iter.  At
 * the cap one more pricing pass decides between LP_OPTIMAL and LP_ITER_LIMIT (Step 4 runs
 * before the limit is checked). */
int lp_solve_until(lp_problem *p, int64_t iter_cap, int32_t *status_out);

/* Runs exactly `count` further iterations of Steps 3-8 (pivots; in the LP_MIXED form an
 * iteration whose shortlist held no improving column does not count), or fewer if a
 * terminal status comes first, and stops without pricing the next one: *status_out is then
 * LP_RUNNING.  A later lp_iterate or lp_solve continues from the device state; the result
 * is the same as one uninterrupted solve.  Returns LP_OK or an error code (LP_ERR_ARG for
 * count < 0). */
int lp_iterate(lp_problem *p, int64_t count, int32_t *status_out);

/* Returns the problem to the slack basis and clears the pivot log and statistics
 * (the LP data are kept). */
int lp_reset(lp_problem *p);

/*
 * Copies the current solution to host buffers (any may be NULL):
 *   objective: sum of c_j x_j over structural basics (user's sense);
 *   x: n structural values; y: m row duals in the user's sense (y = c_B^T B^-1);
 *   basis: m variable ids (basis[i] is basic in row i); iterations: pivots done.
 */
int lp_get_solution(const lp_problem *p, double *objective, double *x, double *y, int32_t *basis,
                    int64_t *iterations);

/* Copies up to `capacity` pivot-log entries (oldest first) into the host arrays (any may
 * be NULL) and stores the number of entries in *count. */
int lp_get_pivots(const lp_problem *p, int32_t *entering, int32_t *leaving_row, int32_t *leaving_var,
                  int32_t *flags, int64_t capacity, int64_t *count);

/* Copies the revised tableau of Figure 1: Binv (m*m, row-major), x_B (m), W = chat_B^T B^-1
 * (m, minimisation form), z = chat_B^T x_B.  Any pointer may be NULL. */
int lp_get_tableau(const lp_problem *p, double *Binv, double *xB, double *W, double *z);

int lp_get_stats(const lp_problem *p, lp_stats *s);

/*
 * Reinversion: recomputes B^-1 from the current basis list and A' in FP64 on the GPU,
 * then x_B = B^-1 b, W = chat_B^T B^-1 and z, discarding the rounding that the
 * product-form updates of Section 3.1 have accumulated.  Only the block of B formed by
 * the structural basic columns and the rows whose slack is nonbasic is factorised (LU
 * with partial pivoting); the slack columns are unit vectors.  lp_solve calls it every
 * opt.reinv_period pivots; it may also be called directly at any time (a pivot left
 * pending by an interrupted solve is absorbed).  If that block is numerically singular
 * (a zero pivot column) the state is left unchanged and lp_stats.reinv_failed counts it.
 * During phase 1 of lp_create_general's two-phase start (where lp_solve does not
 * reinvert on its own), W and z are afterwards recomputed from their definitions with
 * the phase-1 costs.
 * Blocks until the basis has been read back; the rest runs on the handle's stream.
 * Returns LP_OK or LP_ERR_NOMEM / LP_ERR_DEVICE.
 */
int lp_reinvert(lp_problem *p);

/* Frees every device and host resource of the handle.  NULL-safe. */
void lp_destroy(lp_problem *p);

/*
 * For callers that cannot allocate device memory (code under HIP stream capture, tight
 * serving loops, harnesses that forbid hipMalloc): lp_create_device + lp_solve +
 * lp_get_solution + lp_destroy in one call that allocates nothing.  Every buffer of the
 * solve lives in one fixed 128 MiB array of device memory per GPU, which each GPU the
 * library runs on holds until the process ends; no graph, stream or event is created.
 *   A_colmajor (m*n, lda = m), b (m), c (n): device pointers of the current device, read only;
 *   x (n), y (m duals in the user's sense), objective (1): device pointers, any may be NULL;
 *   status, iterations: host pointers, any may be NULL.
 * Runs on opt->stream (NULL = the null stream) and returns when the results are written.
 * Only the FP64 form without reinversion and without profiling is available (LP_ERR_ARG
 * otherwise).  An LP whose buffers (about 8*ld*(n+m) bytes plus 28 bytes per pivot of
 * max_iter, ld = m rounded up to 8) exceed the array is rejected with LP_ERR_ARG before
 * any device work; non-finite data give LP_ERR_ARG and some b_i < 0 LP_ERR_NEG_RHS.
 * The pivots, x, y and objective equal those of lp_create_device + lp_solve (same
 * kernels, same order of operations).  All calls on one GPU share its array, so calls
 * that overlap on one GPU (from two threads, or on two streams) race and must not be made.
 */
int lp_solve_device_noalloc(int32_t m, int32_t n, const double *A_colmajor, const double *b, const double *c,
                            const lp_options *opt, double *x, double *y, double *objective, int32_t *status,
                            int64_t *iterations);

/* ---- batched form: many independent LPs in persistent kernel launches (one, or two when
 *      some LPs keep B^-1 in LDS) ---- */

typedef struct lp_batch lp_batch;

typedef struct lp_batch_stats {
  int64_t count;              /* LPs in the batch */
  int64_t narrow_lps;         /* LPs solved by one wavefront each in the last solve */
  int64_t wide_lps;           /* LPs solved by a whole workgroup */
  int64_t work_items;         /* queue entries of the last solve (both launches) */
  int64_t workgroups;         /* persistent workgroups of the launch that keeps B^-1 in HBM */
  int64_t lds_bytes;          /* LDS per workgroup of that launch */
  int64_t narrow_bucket_mask; /* bit k: m in (16k, 16k+16] was tuned to one wavefront per LP */
  double solve_ms;            /* device time of the last lp_batch_solve (both launches) */
  double tune_ms;             /* host time spent by the autotuner */
  int64_t binv_lds_lps;       /* LPs that kept B^-1 in LDS in the last solve */
  int64_t binv_lds_m;         /* the threshold in effect (option or tuned) */
  int64_t tuned_from_table;   /* m-buckets whose mode came from a tune table (not timed) */
} lp_batch_stats;

/*
 * Creates a batch of `count` LPs, each given as in lp_create (host arrays: A[i] is m[i]*n[i]
 * doubles column-major, b[i] m[i] doubles >= 0, c[i] n[i] doubles); all LPs share *opt
 * (NULL = defaults).  Data are copied to device memory owned by the handle.  Every LP of
 * the batch follows exactly the iteration of lp_solve and gives bit-identical results.
 * Errors: LP_ERR_ARG (sizes, NULL, non-finite data, an LP too large for the solver's LDS
 * budget), LP_ERR_NEG_RHS, LP_ERR_NOMEM, LP_ERR_DEVICE.
 */
int lp_batch_create(lp_batch **out, int32_t count, const int32_t *m, const int32_t *n, const double *const *A,
                    const double *const *b, const double *const *c, const lp_options *opt);

/*
 * A batch of `count` seeded synthetic LPs generated in device memory, for benchmarks and
 * tests (no host arrays and no upload: the device writes every A', b and c itself).  With
 * the counter-based hash h(s, k, i) = mix(mix(mix(s) ^ k) ^ i), mix the SplitMix64
 * finaliser (Steele, Lea & Flood, OOPSLA 2014), u = (h >> 11) 2^-53 and U(a,b) = a + (b-a) u:
 * LP i has m_i = m_lo + (h(seed, 6, i) mod (m_hi - m_lo + 1)) rows and n_i = 2 m_i columns,
 * and with s_i = h(seed, 7, i), the dense law A'_rj = U(0,1) drawn at (s_i, 1, j m_i + r),
 * b_r = U(1,10) at (s_i, 2, r), c_j = U(1,10) at (s_i, 3, j); maximised by default (*opt as
 * in lp_batch_create).  The same bits as host arrays built by that definition.
 * Errors: LP_ERR_ARG (count <= 0, m_lo < 1, m_hi < m_lo, an LP too large for the solver's
 * LDS budget), LP_ERR_NOMEM, LP_ERR_DEVICE.
 */
int lp_batch_create_dense(lp_batch **out, int32_t count, uint64_t seed, int32_t m_lo, int32_t m_hi,
                          const lp_options *opt);

/* Solves every LP of the batch from its slack basis: one persistent launch for the LPs
 * whose B^-1 stays in HBM, then one for those that keep it in LDS (none by default on
 * mixed batches; see batch_binv_lds_m).  The first call with batch_small_m = -1 first times
 * both execution modes per m-bucket, and with batch_binv_lds_m = -1 then times each
 * threshold in {0, 48, 96, 128} that moves some LP to LDS on the whole batch. */
int lp_batch_solve(lp_batch *bt);

/* Per-LP status, objective (user's sense) and pivot count; arrays of `count` entries, any
 * may be NULL.  LP_ERR_STATE before the first lp_batch_solve. */
int lp_batch_results(const lp_batch *bt, int32_t *status, double *objective, int64_t *iterations);

/* LP i: structural x (n[i]), basis (m[i]), and up to `capacity` pivot-log entries; any
 * pointer may be NULL; *count receives the number of logged pivots. */
int lp_batch_get(const lp_batch *bt, int32_t i, double *x, int32_t *basis, int32_t *entering, int32_t *leaving_row,
                 int32_t *flags, int64_t capacity, int64_t *count);

int lp_batch_get_stats(const lp_batch *bt, lp_batch_stats *s);

/* The batch's sizes: m[i] rows and n[i] columns of LP i, arrays of `count` entries, either
 * may be NULL (the sizes lp_batch_create_dense drew). */
int lp_batch_get_sizes(const lp_batch *bt, int32_t *m, int32_t *n);

/* NULL-safe. */
void lp_batch_destroy(lp_batch *bt);

/*
 * The autotuner's table (Section 3.3's block-size choice, made by timing): the mode chosen
 * for each m-bucket (one wavefront or one workgroup per LP; m in (16k, 16k+16]) and the
 * B^-1-in-LDS threshold, keyed by the device's architecture name and the precision, in a
 * JSON file of one record per line.  lp_batch_tune_load, before the first lp_batch_solve,
 * takes the records of this device's architecture: those buckets are not timed again, and a
 * recorded threshold is used.  lp_batch_tune_save merges the batch's tuned buckets and
 * threshold into the file (created if missing; the other records are kept).  With the
 * environment variable LPGPU_BATCH_TUNE naming a file, lp_batch_create loads it and every
 * lp_batch_solve that tuned something saves it.  A missing or unreadable file is an empty
 * table.  Errors: LP_ERR_ARG (NULL argument, a file that cannot be written).
 */
int lp_batch_tune_load(lp_batch *bt, const char *path);
int lp_batch_tune_save(const lp_batch *bt, const char *path);

/* lp_batch_create + lp_batch_solve + lp_batch_results + lp_batch_destroy. */
int lp_solve_batch(int32_t count, const int32_t *m, const int32_t *n, const double *const *A, const double *const *b,
                   const double *const *c, const lp_options *opt, int32_t *status, double *objective,
                   int64_t *iterations);

/* Text for a return code; for an error returned by the calling thread's most recent
 * call, the text also names the failing step.  The pointer stays valid until the next
 * lpgpu call on this thread. */
const char *lp_error_string(int code);

#ifdef __cplusplus
}
#endif

#endif /* LPGPU_H */
