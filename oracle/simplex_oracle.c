/*
 * Plain FP64 revised simplex: the oracle of the GPU path.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU-baseline
 * leg of the benchmark may load this library.  It shares no code with the HIP
 * library and includes none of its headers.
 *
 * What it computes (paper, Section 2.1 "Revised Simplex algorithm", Steps 1-8 and
 * Figure 1; Section 3.1 "Tableau updating"; Sections 2.2/3.4 "Tabu rule"):
 *
 *   min  chat^T X   s.t.  (A', I_m) X = b,  b >= 0,  X >= 0,
 *   chat_j = s*c_j for structural j (s = +1 min, -1 max), chat_{n+i} = 0 for slacks.
 *
 * It keeps the revised tableau of Figure 1 as separate arrays:
 *   W      (1 x m)  = chat_B^T B^-1         top-left block
 *   z      scalar   = chat_B^T B^-1 b       top-middle  (Step 2, read as C_B b-bar)
 *   Binv   (m x m)  = B^-1, row-major       body
 *   xB     (m)      = B^-1 b = b-bar        body, middle column
 * and pivots it on y_rk as Step 8 prescribes, every iteration, never refactorising.
 *
 * Readings of points the paper leaves open:
 *   - m = rows (constraints), n = structural columns.          (Section 2.1)
 *   - ratio-test index runs over the m rows.                    (Step 6)
 *   - optimality: no nonbasic d_j = chat_j - W a_j < -eps_d;
 *     the paper's z_j - c_j equals -d_j.                        (Steps 3-4)
 *   - Y_k <= 0 read as "no alpha_i > eps_p".                    (Steps 5-6)
 *   - entering ties: lowest variable index (slacks after structurals).
 *   - ratio_i = max(xB_i, 0) / alpha_i (IEEE division), theta = min ratio_i.
 *     "No unique leaving element" (Sections 2.2, 3.4) means several rows reach zero
 *     at the step theta.  In FP64 rounding splits such ties, so a row is tied when
 *     the value it takes at that step, fma(-alpha_i, theta, max(xB_i, 0)), is at most
 *     eps_t; this tolerance is in the units of x and is not magnified by a large
 *     alpha_i.  Every tied row gives the same objective change, so the paper's "most
 *     noticeable improvement" cannot separate them; the tie is broken by the lowest
 *     row whose basic variable is not in the tabu list L[q] of the entering variable
 *     q, and that leaving variable is then appended to L[q].  If L[q] excludes every
 *     tied row, L[q] is cleared and the lowest tied row is taken.  The step is theta
 *     for whichever tied row leaves.
 *   - entering mask: a variable that leaves at iteration t may not enter at
 *     iterations t+1 .. t+tenure; if every improving variable is masked, the
 *     choice is made among all improving variables (aspiration).
 *   - update rounding: row r := B^-1[r,:] / alpha_r (correctly rounded division);
 *     rows i != r: fma(-alpha_i, rho_j, B^-1[i,j]); W_j := fma(d_q, rho_j, W_j);
 *     xB_i := fma(-alpha_i, theta, xB_i), xB_r := theta; z := fma(d_q, theta, z);
 *     afterwards every |xB_i| < eps_z is set to 0.            (Section 3.1)
 *   - the iteration limit is checked after pricing: a basis that prices out optimal
 *     is reported OPTIMAL even at the limit.
 *   - non-finite arithmetic (the paper assumes none): if Y_k has a non-finite entry,
 *     or the minimum ratio over the candidate rows overflows, the solve stops with
 *     status NUMERICAL before the pivot; "no candidate row" stays UNBOUNDED.
 *
 * Two-phase start (Section 3.4, "Finding the initial feasible solution"; the textbook
 * two-phase method it refers to), for LPs given with row types (<=, >=, =) and b of any
 * sign, oracle_create_general:
 *   - a row with b_i < 0 is multiplied by -1 (its type flips between <= and >=), so that
 *     b >= 0;
 *   - a <= row keeps its slack as the unit column n+i, basic at the start;
 *   - a >= row gets a surplus column -e_i, appended after the caller's n columns in
 *     ascending row order, and its unit column n+i is an artificial variable;
 *   - an = row has no slack; its unit column n+i is an artificial variable.
 *   Phase 1 minimises the sum of the artificial variables from the basis of the unit
 *   columns (W and z from their definitions).  An artificial variable that leaves the
 *   basis never enters again, in either phase.  At the phase-1 optimum:
 *   - a sum above eps_f = 1e-9 (1 + max_i |b_i|) means the LP is INFEASIBLE;
 *   - otherwise, for each row r in ascending order whose basic variable is still an
 *     artificial one, the nonbasic non-artificial column j with the largest |entry| of
 *     row r of the tableau, B^-1[r,:] a_j (lowest j on equal magnitude; only entries
 *     above eps_p count), replaces it by a pivot with step 0 (x_B[r] := 0, flag
 *     FLAG_DRIVEOUT); a row with no such column is redundant and keeps its artificial
 *     variable, basic at zero;
 *   - phase 2 then restores the costs of the LP and recomputes W = chat_B^T B^-1 and
 *     z = chat_B^T x_B from their definitions (ascending sums over the rows whose basic
 *     variable has a nonzero cost), and the iteration continues.
 *   The tabu state and the pivot count carry over from phase 1.  Reported duals refer
 *   to the caller's rows: y_i = s W_i, negated for rows that were multiplied by -1.
 *
 * Dot products are plain ascending-index fma chains.  Build with
 * -ffp-contract=off so that no other operation is fused.
 *
 * Built with -fopenmp, the loops over independent columns (pricing) and rows (FTRAN,
 * the pivot) are shared among threads.  Each dot product and each element is still
 * computed by one thread in the same order, and every choice is made afterwards by a
 * sequential scan, so the results are bit-identical to the sequential build.
 *
 * oracle_basis_inverse, at the end, gives B^-1 of any basis list by its definition:
 * the reference for the GPU reinversion (parity unpinned by the paper, which does not
 * refactorise; pinned by the tests against closed forms and a library inverse).
 */
#include <math.h>
#include <stdint.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include <stdlib.h>
#include <string.h>

#define OR_RUNNING 0
#define OR_OPTIMAL 1
#define OR_UNBOUNDED 2
#define OR_ITER_LIMIT 3
#define OR_NUMERICAL 4
#define OR_INFEASIBLE 5

#define ROW_LE 0
#define ROW_GE 1
#define ROW_EQ 2

#define FLAG_DEGENERATE 1  /* theta == 0 */
#define FLAG_TIE 2         /* more than one row reaches zero (within eps_t) at the step */
#define FLAG_ASPIRATION 4  /* every improving variable was masked */
#define FLAG_LCLEAR 8      /* L[q] excluded every tied row and was cleared */
#define FLAG_DRIVEOUT 16   /* phase switch: an artificial variable at zero level replaced */

/* pos[v] of an artificial variable that has left the basis: it never enters again. */
#define POS_BARRED (-2)

typedef struct {
  int32_t m, n, sense, tenure, use_llist;
  double eps_d, eps_p, eps_z, eps_t;
  double *A;    /* m x n column-major: A[i + j*m] */
  double *b, *c, *chat;
  double *Binv; /* m x m row-major: Binv[i*m + j] */
  double *xB, *W, *d, *alpha, *rho, *ratio;
  double z;
  int32_t *basis; /* basis[i] = variable basic in row i */
  int32_t *pos;   /* pos[v] = row of basic variable v, -1 if nonbasic */
  int64_t *tabu_until;
  int32_t **L;    /* L[q]: leaving variables chosen on ties while q entered */
  int32_t *L_len, *L_cap;
  int64_t t;
  int32_t status, ray;
  int64_t n_degenerate, n_tie, n_aspiration, n_lclear;
  int32_t *log_enter, *log_row, *log_leave, *log_flags;
  double *log_margin; /* per pivot: how close its closest decision came to its threshold */
  int64_t log_len, log_cap;
  /* Two-phase start (NULL / 0 for an LP created by oracle_create). */
  int32_t phase;   /* 0: one phase; 1: phase 1 running; 2: phase 2 */
  int32_t n_user;  /* the caller's structural columns; n_user..n-1 are surplus columns */
  int8_t *art;     /* art[i] = 1: the unit column n+i is the artificial variable of row i */
  double *rsign;   /* -1 for rows multiplied by -1, else +1 */
  double *chat2;   /* the LP's own costs, restored for phase 2 */
  double eps_f;
} oracle_lp;

void oracle_destroy(oracle_lp *p);

/* Returns NULL if arguments are invalid or memory runs out. */
oracle_lp *oracle_create(int32_t m, int32_t n, const double *A_colmajor, const double *b, const double *c,
                         int32_t sense, int32_t tenure, int32_t use_llist, double eps_d, double eps_p,
                         double eps_z, double eps_t) {
  if (m <= 0 || n < 0 || !A_colmajor || !b || !c) return NULL;
  for (int32_t i = 0; i < m; ++i)
    if (!(b[i] >= 0.0) || !isfinite(b[i])) return NULL;
  oracle_lp *p = (oracle_lp *)calloc(1, sizeof(oracle_lp));
  if (!p) return NULL;
  int32_t N = n + m;
  p->m = m; p->n = n; p->sense = sense; p->tenure = tenure; p->use_llist = use_llist;
  p->eps_d = eps_d; p->eps_p = eps_p; p->eps_z = eps_z; p->eps_t = eps_t;
  p->A = (double *)malloc(sizeof(double) * (size_t)m * (n > 0 ? n : 1));
  p->b = (double *)malloc(sizeof(double) * m);
  p->c = (double *)malloc(sizeof(double) * (n > 0 ? n : 1));
  p->chat = (double *)malloc(sizeof(double) * N);
  p->Binv = (double *)calloc((size_t)m * m, sizeof(double));
  p->xB = (double *)malloc(sizeof(double) * m);
  p->W = (double *)calloc(m, sizeof(double));
  p->d = (double *)malloc(sizeof(double) * N);
  p->alpha = (double *)malloc(sizeof(double) * m);
  p->rho = (double *)malloc(sizeof(double) * m);
  p->ratio = (double *)malloc(sizeof(double) * m);
  p->basis = (int32_t *)malloc(sizeof(int32_t) * m);
  p->pos = (int32_t *)malloc(sizeof(int32_t) * N);
  p->tabu_until = (int64_t *)malloc(sizeof(int64_t) * N);
  p->L = (int32_t **)calloc(N, sizeof(int32_t *));
  p->L_len = (int32_t *)calloc(N, sizeof(int32_t));
  p->L_cap = (int32_t *)calloc(N, sizeof(int32_t));
  if (!p->A || !p->b || !p->c || !p->chat || !p->Binv || !p->xB || !p->W || !p->d || !p->alpha || !p->rho ||
      !p->ratio || !p->basis || !p->pos || !p->tabu_until || !p->L || !p->L_len || !p->L_cap) {
    oracle_destroy(p);
    return NULL;
  }
  memcpy(p->A, A_colmajor, sizeof(double) * (size_t)m * n);
  memcpy(p->b, b, sizeof(double) * m);
  memcpy(p->c, c, sizeof(double) * n);
  double s = sense ? -1.0 : 1.0; /* sense 1 = max: minimise -c^T x */
  for (int32_t j = 0; j < n; ++j) p->chat[j] = s * c[j];
  for (int32_t i = 0; i < m; ++i) p->chat[n + i] = 0.0;
  /* Step 1: the slack columns form B = I, feasible because b >= 0. */
  for (int32_t i = 0; i < m; ++i) {
    p->basis[i] = n + i;
    p->Binv[(size_t)i * m + i] = 1.0;
    p->xB[i] = b[i];
  }
  for (int32_t v = 0; v < N; ++v) { p->pos[v] = -1; p->tabu_until[v] = -1; }
  for (int32_t i = 0; i < m; ++i) p->pos[n + i] = i;
  p->z = 0.0;
  p->t = 0;
  p->status = OR_RUNNING;
  p->ray = -1;
  p->n_user = n;
  return p;
}

void oracle_destroy(oracle_lp *p) {
  if (!p) return;
  if (p->L)
    for (int32_t v = 0; v < p->n + p->m; ++v) free(p->L[v]);
  free(p->L); free(p->L_len); free(p->L_cap);
  free(p->A); free(p->b); free(p->c); free(p->chat); free(p->Binv); free(p->xB); free(p->W);
  free(p->d); free(p->alpha); free(p->rho); free(p->ratio); free(p->basis); free(p->pos);
  free(p->tabu_until); free(p->log_enter); free(p->log_row); free(p->log_leave); free(p->log_flags); free(p->log_margin);
  free(p->art); free(p->rsign); free(p->chat2);
  free(p);
}

static int log_push(oracle_lp *p, int32_t q, int32_t r, int32_t l, int32_t flags, double margin) {
  if (p->log_len == p->log_cap) {
    int64_t cap = p->log_cap ? 2 * p->log_cap : 1024;
    int32_t *a = (int32_t *)realloc(p->log_enter, sizeof(int32_t) * cap);
    if (!a) return -1;
    p->log_enter = a;
    a = (int32_t *)realloc(p->log_row, sizeof(int32_t) * cap);
    if (!a) return -1;
    p->log_row = a;
    a = (int32_t *)realloc(p->log_leave, sizeof(int32_t) * cap);
    if (!a) return -1;
    p->log_leave = a;
    a = (int32_t *)realloc(p->log_flags, sizeof(int32_t) * cap);
    if (!a) return -1;
    p->log_flags = a;
    double *g = (double *)realloc(p->log_margin, sizeof(double) * cap);
    if (!g) return -1;
    p->log_margin = g;
    p->log_cap = cap;
  }
  p->log_enter[p->log_len] = q;
  p->log_row[p->log_len] = r;
  p->log_leave[p->log_len] = l;
  p->log_flags[p->log_len] = flags;
  p->log_margin[p->log_len] = margin;
  p->log_len++;
  return 0;
}

static int in_list(const oracle_lp *p, int32_t q, int32_t v) {
  for (int32_t k = 0; k < p->L_len[q]; ++k)
    if (p->L[q][k] == v) return 1;
  return 0;
}

static int list_add(oracle_lp *p, int32_t q, int32_t v) {
  if (p->L_len[q] == p->L_cap[q]) {
    int32_t cap = p->L_cap[q] ? 2 * p->L_cap[q] : 4;
    int32_t *a = (int32_t *)realloc(p->L[q], sizeof(int32_t) * cap);
    if (!a) return -1;
    p->L[q] = a;
    p->L_cap[q] = cap;
  }
  p->L[q][p->L_len[q]++] = v;
  return 0;
}

/* Step 5: Y_k = B^-1 a_q into alpha (a slack's column is a column of B^-1). */
static void ftran(oracle_lp *p, int32_t q) {
  const int32_t m = p->m, n = p->n;
#pragma omp parallel for schedule(static)
  for (int32_t i = 0; i < m; ++i) {
    const double *row = p->Binv + (size_t)i * m;
    if (q < n) {
      const double *a = p->A + (size_t)q * m;
      double s = 0.0;
      for (int32_t k = 0; k < m; ++k) s = fma(row[k], a[k], s);
      p->alpha[i] = s;
    } else {
      p->alpha[i] = row[q - n];
    }
  }
}

/* Step 8 / Section 3.1 on the body of the tableau: rho = B^-1[r,:] / alpha_r becomes
 * row r, every other row i gets fma(-alpha_i, rho_j, B^-1[i,j]). */
static void pivot_inverse(oracle_lp *p, int32_t r) {
  const int32_t m = p->m;
  const double ar = p->alpha[r];
  double *rowr = p->Binv + (size_t)r * m;
  for (int32_t j = 0; j < m; ++j) p->rho[j] = rowr[j] / ar;
#pragma omp parallel for schedule(static)
  for (int32_t i = 0; i < m; ++i) {
    double *row = p->Binv + (size_t)i * m;
    if (i == r) {
      for (int32_t j = 0; j < m; ++j) row[j] = p->rho[j];
    } else {
      const double na = -p->alpha[i];
      for (int32_t j = 0; j < m; ++j) row[j] = fma(na, p->rho[j], row[j]);
    }
  }
}

/* One iteration (Steps 3-8).  Returns the status after it. */
static int32_t iterate(oracle_lp *p, int64_t max_iter) {
  const int32_t m = p->m, n = p->n, N = n + m;

  /* Step 3: reduced costs d_j = chat_j - W a_j of every nonbasic variable (barred
   * artificial variables are not candidates). */
#pragma omp parallel for schedule(static)
  for (int32_t j = 0; j < N; ++j) {
    if (p->pos[j] != -1) continue;
    if (j < n) {
      const double *a = p->A + (size_t)j * m;
      double s = 0.0;
      for (int32_t i = 0; i < m; ++i) s = fma(p->W[i], a[i], s);
      p->d[j] = p->chat[j] - s;
    } else {
      p->d[j] = p->chat[j] - p->W[j - n]; /* a_{n+i} = e_i */
    }
  }

  /* Step 4: Dantzig choice, most negative d_j, with the entering mask. */
  int32_t q_all = -1, q_free = -1;
  for (int32_t j = 0; j < N; ++j) {
    if (p->pos[j] != -1 || !(p->d[j] < -p->eps_d)) continue;
    if (q_all < 0 || p->d[j] < p->d[q_all]) q_all = j; /* strict: lowest index wins ties */
    if (p->tabu_until[j] < p->t && (q_free < 0 || p->d[j] < p->d[q_free])) q_free = j;
  }
  if (q_all < 0) return OR_OPTIMAL;
  if (p->t >= max_iter) return OR_ITER_LIMIT;
  int32_t flags = 0;
  int32_t q = q_free;
  if (q < 0) { q = q_all; flags |= FLAG_ASPIRATION; p->n_aspiration++; }
  const double dq = p->d[q];

  /* Decision margin of this pivot (reported only, never used in a decision): the
   * smallest distance of a value that a threshold or a comparison decided from that
   * threshold or from its rival.  A threshold test counts only for values at least half
   * the threshold in magnitude: smaller ones (rounding residues of exact zeros) would need
   * an error as large as the threshold to cross it.  Pricing: |d_j + eps_d|, and the gap
   * between d_q and the other values of the set q was chosen from. */
  double margin = INFINITY;
  for (int32_t j = 0; j < N; ++j) {
    if (p->pos[j] != -1) continue;
    if (fabs(p->d[j]) >= 0.5 * p->eps_d) margin = fmin(margin, fabs(p->d[j] + p->eps_d));
    const int in_set = p->d[j] < -p->eps_d && (q == q_all || p->tabu_until[j] < p->t);
    if (in_set && j != q) margin = fmin(margin, fabs(p->d[j] - dq));
  }

  /* Step 5: FTRAN, Y_k = B^-1 a_q. */
  ftran(p, q);

  /* A non-finite entry of Y_k (overflow of the product-form B^-1) stops the solve. */
  for (int32_t i = 0; i < m; ++i)
    if (!isfinite(p->alpha[i])) return OR_NUMERICAL;

  /* Step 6: ratio test over rows with alpha_i > eps_p. */
  double theta_min = INFINITY;
  int32_t nR = 0;
  for (int32_t i = 0; i < m; ++i) {
    if (!(p->alpha[i] > p->eps_p)) continue;
    nR++;
    p->ratio[i] = fmax(p->xB[i], 0.0) / p->alpha[i];
    if (p->ratio[i] < theta_min) theta_min = p->ratio[i];
  }
  if (nR == 0) { p->ray = q; return OR_UNBOUNDED; } /* Step 5: Y_k <= 0 */
  if (!isfinite(theta_min)) return OR_NUMERICAL;     /* the step overflowed */
  int32_t nT = 0, r_low = -1, r_free = -1;
  for (int32_t i = 0; i < m; ++i) {
    if (!(p->alpha[i] > p->eps_p)) continue;
    if (!(fma(-p->alpha[i], theta_min, fmax(p->xB[i], 0.0)) <= p->eps_t)) continue; /* not tied */
    nT++;
    if (r_low < 0) r_low = i;
    if (r_free < 0 && !(p->use_llist && in_list(p, q, p->basis[i]))) r_free = i;
  }
  /* Ratio test margins: |alpha_i - eps_p| and, over the candidate rows, the distance of
   * the value a row reaches at the step from eps_t. */
  for (int32_t i = 0; i < m; ++i) {
    if (fabs(p->alpha[i]) >= 0.5 * p->eps_p) margin = fmin(margin, fabs(p->alpha[i] - p->eps_p));
    if (!(p->alpha[i] > p->eps_p)) continue;
    const double v = fma(-p->alpha[i], theta_min, fmax(p->xB[i], 0.0));
    if (fabs(v) >= 0.5 * p->eps_t) margin = fmin(margin, fabs(v - p->eps_t));
  }
  int32_t r = r_low;
  if (nT >= 2) {
    flags |= FLAG_TIE;
    p->n_tie++;
    if (p->use_llist) {
      if (r_free < 0) { p->L_len[q] = 0; flags |= FLAG_LCLEAR; p->n_lclear++; }
      else r = r_free;
      if (list_add(p, q, p->basis[r])) return -1;
    }
  }
  const double theta = theta_min;
  if (theta == 0.0) { flags |= FLAG_DEGENERATE; p->n_degenerate++; }

  /* Step 7 and the tabu mask: the leaving variable may not re-enter for `tenure` iterations. */
  const int32_t leave = p->basis[r];
  if (p->tenure > 0) p->tabu_until[leave] = p->t + p->tenure;

  /* Step 8 / Section 3.1: pivot the revised tableau on alpha_r. */
  pivot_inverse(p, r);
  for (int32_t j = 0; j < m; ++j) p->W[j] = fma(dq, p->rho[j], p->W[j]);
  for (int32_t i = 0; i < m; ++i) p->xB[i] = (i == r) ? theta : fma(-p->alpha[i], theta, p->xB[i]);
  for (int32_t i = 0; i < m; ++i) {
    if (fabs(p->xB[i]) >= 0.5 * p->eps_z) margin = fmin(margin, fabs(fabs(p->xB[i]) - p->eps_z)); /* the snap */
    if (fabs(p->xB[i]) < p->eps_z) p->xB[i] = 0.0;
  }
  p->z = fma(dq, theta, p->z);
  p->basis[r] = q;
  p->pos[q] = r;
  p->pos[leave] = (p->art && leave >= n && p->art[leave - n]) ? POS_BARRED : -1;
  if (log_push(p, q, r, leave, flags, margin)) return -1;
  p->t++;
  return OR_RUNNING;
}

/* W = chat_B^T B^-1 and z = chat_B^T x_B by their definitions: ascending fma sums over
 * the rows whose basic variable has a nonzero cost. */
static void reprice(oracle_lp *p) {
  const int32_t m = p->m;
  for (int32_t j = 0; j < m; ++j) {
    double s = 0.0;
    for (int32_t i = 0; i < m; ++i) {
      const double cb = p->chat[p->basis[i]];
      if (cb != 0.0) s = fma(cb, p->Binv[(size_t)i * m + j], s);
    }
    p->W[j] = s;
  }
  double z = 0.0;
  for (int32_t i = 0; i < m; ++i) {
    const double cb = p->chat[p->basis[i]];
    if (cb != 0.0) z = fma(cb, p->xB[i], z);
  }
  p->z = z;
}

/* A pivot on (q, r) with step 0: B^-1 as in Step 8, x_B[r] := 0, the other x_B unchanged;
 * W and z are left for reprice.  The leaving variable is an artificial one: barred. */
static int drive_out(oracle_lp *p, int32_t q, int32_t r) {
  ftran(p, q);
  pivot_inverse(p, r);
  const int32_t leave = p->basis[r];
  p->xB[r] = 0.0;
  p->basis[r] = q;
  p->pos[q] = r;
  p->pos[leave] = POS_BARRED;
  if (log_push(p, q, r, leave, FLAG_DRIVEOUT, INFINITY)) return -1;
  p->t++;
  return 0;
}

/* The end of phase 1 (its optimum has been reached): INFEASIBLE, or the start of phase 2. */
static int32_t phase_switch(oracle_lp *p) {
  const int32_t m = p->m, n = p->n, N = n + m;
  if (p->z > p->eps_f) return OR_INFEASIBLE;
  for (int32_t r = 0; r < m; ++r) {
    const int32_t v = p->basis[r];
    if (v < n || !p->art[v - n]) continue;
    const double *row = p->Binv + (size_t)r * m;
    int32_t best = -1;
    double bt = 0.0;
    for (int32_t j = 0; j < N; ++j) {
      if (p->pos[j] != -1 || (j >= n && p->art[j - n])) continue;
      double t;
      if (j < n) {
        const double *a = p->A + (size_t)j * m;
        double s = 0.0;
        for (int32_t k = 0; k < m; ++k) s = fma(a[k], row[k], s);  /* row r of B^-1 times a_j */
        t = s;
      } else {
        t = row[j - n];
      }
      if (fabs(t) > p->eps_p && fabs(t) > fabs(bt)) { best = j; bt = t; }
    }
    if (best >= 0 && drive_out(p, best, r)) return -1;
  }
  memcpy(p->chat, p->chat2, sizeof(double) * N);
  reprice(p);
  p->phase = 2;
  return OR_RUNNING;
}

/* Iterate until a terminal status or until the pivot count reaches max_iter.
 * A handle stopped at the limit resumes from its state on the next call. */
int32_t oracle_run(oracle_lp *p, int64_t max_iter) {
  if (!p) return -1;
  if (p->status == OR_ITER_LIMIT) p->status = OR_RUNNING;
  while (p->status == OR_RUNNING) {
    int32_t s = iterate(p, max_iter);
    if (s == OR_OPTIMAL && p->phase == 1) s = phase_switch(p);
    if (s < 0) return -1;
    p->status = s;
  }
  return p->status;
}

/*
 * An LP with row types (ROW_LE, ROW_GE, ROW_EQ; NULL = all ROW_LE) and b of any sign,
 * solved by the two-phase method described at the top.  The handle's columns are the
 * caller's n followed by one surplus column per >= row (after the sign change); pivot
 * logs and basis lists use that numbering.  Returns NULL on invalid input.
 */
oracle_lp *oracle_create_general(int32_t m, int32_t n, const double *A_colmajor, const double *b, const double *c,
                                 const int32_t *row_type, int32_t sense, int32_t tenure, int32_t use_llist,
                                 double eps_d, double eps_p, double eps_z, double eps_t) {
  if (m <= 0 || n < 0 || !A_colmajor || !b || !c) return NULL;
  double *sg = (double *)malloc(sizeof(double) * m);
  int8_t *ge = (int8_t *)malloc((size_t)m);
  int8_t *art = (int8_t *)calloc((size_t)m, 1);
  if (!sg || !ge || !art) { free(sg); free(ge); free(art); return NULL; }
  int32_t ns = 0, na = 0;
  double bmax = 0.0;
  for (int32_t i = 0; i < m; ++i) {
    const int32_t ty = row_type ? row_type[i] : ROW_LE;
    if (!isfinite(b[i]) || ty < ROW_LE || ty > ROW_EQ) { free(sg); free(ge); free(art); return NULL; }
    sg[i] = b[i] < 0.0 ? -1.0 : 1.0;
    int32_t t2 = ty;
    if (sg[i] < 0.0 && ty != ROW_EQ) t2 = ty == ROW_LE ? ROW_GE : ROW_LE;
    ge[i] = t2 == ROW_GE;
    art[i] = t2 != ROW_LE;
    ns += ge[i];
    na += art[i];
    if (fabs(b[i]) > bmax) bmax = fabs(b[i]);
  }
  const int32_t n2 = n + ns;
  double *A2 = (double *)calloc((size_t)m * (n2 > 0 ? n2 : 1), sizeof(double));
  double *b2 = (double *)malloc(sizeof(double) * m);
  double *c2 = (double *)calloc(n2 > 0 ? n2 : 1, sizeof(double));
  if (!A2 || !b2 || !c2) { free(sg); free(ge); free(art); free(A2); free(b2); free(c2); return NULL; }
  for (int32_t j = 0; j < n; ++j)
    for (int32_t i = 0; i < m; ++i) A2[(size_t)j * m + i] = sg[i] * A_colmajor[(size_t)j * m + i];
  for (int32_t i = 0, k = n; i < m; ++i)
    if (ge[i]) A2[(size_t)(k++) * m + i] = -1.0;
  for (int32_t i = 0; i < m; ++i) b2[i] = sg[i] * b[i];
  for (int32_t j = 0; j < n; ++j) c2[j] = c[j];
  oracle_lp *p = oracle_create(m, n2, A2, b2, c2, sense, tenure, use_llist, eps_d, eps_p, eps_z, eps_t);
  free(A2); free(b2); free(c2); free(ge);
  if (!p) { free(sg); free(art); return NULL; }
  p->n_user = n;
  p->rsign = sg;
  p->art = art;
  p->eps_f = 1e-9 * (1.0 + bmax);
  if (na > 0) {
    const int32_t N = n2 + m;
    p->chat2 = (double *)malloc(sizeof(double) * N);
    if (!p->chat2) { oracle_destroy(p); return NULL; }
    memcpy(p->chat2, p->chat, sizeof(double) * N);
    for (int32_t v = 0; v < N; ++v) p->chat[v] = (v >= n2 && art[v - n2]) ? 1.0 : 0.0;
    reprice(p);
    p->phase = 1;
  }
  return p;
}

/* Threads of the -fopenmp build (n <= 0: leave the default); returns the number in use,
 * 1 for the sequential build. */
int32_t oracle_set_threads(int32_t n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
  return omp_get_max_threads();
#else
  (void)n;
  return 1;
#endif
}

int32_t oracle_phase(const oracle_lp *p) { return p->phase; }
int32_t oracle_columns(const oracle_lp *p) { return p->n; }

int64_t oracle_iterations(const oracle_lp *p) { return p->t; }
int32_t oracle_status(const oracle_lp *p) { return p->status; }
int32_t oracle_ray(const oracle_lp *p) { return p->ray; }

/* Objective in the user's sense: sum over structural basics of c_j x_j, ascending j. */
double oracle_objective(const oracle_lp *p) {
  double s = 0.0;
  for (int32_t j = 0; j < p->n; ++j)
    if (p->pos[j] >= 0) s += p->c[j] * p->xB[p->pos[j]];
  return s;
}

/* x (n values, the handle's columns), y (m duals in the user's sense: y = s*W, negated for rows
 * multiplied by -1), basis (m). Any may be NULL. */
void oracle_solution(const oracle_lp *p, double *x, double *y, int32_t *basis) {
  const double s = p->sense ? -1.0 : 1.0;
  if (x)
    for (int32_t j = 0; j < p->n; ++j) x[j] = p->pos[j] >= 0 ? p->xB[p->pos[j]] : 0.0;
  if (y)
    for (int32_t i = 0; i < p->m; ++i) y[i] = s * p->W[i] * (p->rsign ? p->rsign[i] : 1.0);
  if (basis) memcpy(basis, p->basis, sizeof(int32_t) * p->m);
}

/* Tableau state: Binv (m*m row-major), xB (m), W (m), z (min form). Any may be NULL. */
void oracle_state(const oracle_lp *p, double *Binv, double *xB, double *W, double *z) {
  if (Binv) memcpy(Binv, p->Binv, sizeof(double) * (size_t)p->m * p->m);
  if (xB) memcpy(xB, p->xB, sizeof(double) * p->m);
  if (W) memcpy(W, p->W, sizeof(double) * p->m);
  if (z) *z = p->z;
}

/* Copies up to cap log entries; returns the total number logged. */
/* The decision margin of each logged pivot (INFINITY for a drive-out); returns the count. */
int64_t oracle_margins(const oracle_lp *p, double *out, int64_t cap) {
  int64_t k = p->log_len < cap ? p->log_len : cap;
  if (out) memcpy(out, p->log_margin, sizeof(double) * k);
  return p->log_len;
}

int64_t oracle_pivots(const oracle_lp *p, int32_t *enter, int32_t *row, int32_t *leave, int32_t *flags,
                      int64_t cap) {
  int64_t k = p->log_len < cap ? p->log_len : cap;
  if (enter) memcpy(enter, p->log_enter, sizeof(int32_t) * k);
  if (row) memcpy(row, p->log_row, sizeof(int32_t) * k);
  if (leave) memcpy(leave, p->log_leave, sizeof(int32_t) * k);
  if (flags) memcpy(flags, p->log_flags, sizeof(int32_t) * k);
  return p->log_len;
}

/* counts[0..3] = degenerate pivots, tie pivots, aspiration events, L[q] clears. */
void oracle_counts(const oracle_lp *p, int64_t *counts) {
  counts[0] = p->n_degenerate;
  counts[1] = p->n_tie;
  counts[2] = p->n_aspiration;
  counts[3] = p->n_lclear;
}

/*
 * The basis inverse by its plain definition: B has column p equal to column basis[p] of
 * (A', I_m), and Binv (m x m, row-major) receives B^-1, computed by Gauss-Jordan
 * elimination with partial pivoting on the augmented matrix (B | I).  Returns 0, or -1
 * when a pivot column is entirely zero (B singular) or memory runs out.  This is the
 * reference of the GPU reinversion (which instead factorises only the block of B that
 * is not a slack column).
 */
int32_t oracle_basis_inverse(int32_t m, int32_t n, const double *A_colmajor, const int32_t *basis, double *Binv) {
  const int32_t w = 2 * m;
  double *T = (double *)calloc((size_t)m * w, sizeof(double));
  if (!T) return -1;
  for (int32_t p = 0; p < m; ++p) {
    const int32_t v = basis[p];
    for (int32_t i = 0; i < m; ++i)
      T[(size_t)i * w + p] = v < n ? A_colmajor[(size_t)i + (size_t)v * m] : (i == v - n ? 1.0 : 0.0);
    T[(size_t)p * w + m + p] = 1.0;
  }
  for (int32_t c = 0; c < m; ++c) {
    int32_t piv = c;
    for (int32_t i = c + 1; i < m; ++i)
      if (fabs(T[(size_t)i * w + c]) > fabs(T[(size_t)piv * w + c])) piv = i;
    if (T[(size_t)piv * w + c] == 0.0) {
      free(T);
      return -1;
    }
    if (piv != c)
      for (int32_t j = 0; j < w; ++j) {
        const double tmp = T[(size_t)c * w + j];
        T[(size_t)c * w + j] = T[(size_t)piv * w + j];
        T[(size_t)piv * w + j] = tmp;
      }
    const double pv = T[(size_t)c * w + c];
    for (int32_t j = 0; j < w; ++j) T[(size_t)c * w + j] /= pv;
    for (int32_t i = 0; i < m; ++i) {
      if (i == c) continue;
      const double f = T[(size_t)i * w + c];
      if (f == 0.0) continue;
      for (int32_t j = 0; j < w; ++j) T[(size_t)i * w + j] -= f * T[(size_t)c * w + j];
    }
  }
  for (int32_t i = 0; i < m; ++i)
    for (int32_t j = 0; j < m; ++j) Binv[(size_t)i * m + j] = T[(size_t)i * w + m + j];
  free(T);
  return 0;
}
