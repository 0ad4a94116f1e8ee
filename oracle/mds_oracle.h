/*
 * Plain FP64 CPU oracle for the mixed dense-sparse (MDS) interior-point
 * Newton step.  TEST INFRASTRUCTURE ONLY: the product library never links,
 * loads or calls anything declared here; only the test suite, the smoke check
 * and the CPU-baseline leg of the benchmark do.
 *
 * Everything is written as slow, obviously correct loops in double precision,
 * compiled without floating-point contraction (-ffp-contract=off) so that each
 * expression rounds exactly as written.  Each function names the passage of
 * the paper (Peles et al., "Porting the Nonlinear Optimization Library HiOp to
 * Accelerator-Based Hardware Architectures") or the textbook method it follows.
 *
 * Storage conventions: dense matrices are column-major (element (i,j) of an
 * r-row matrix at [i + j*r]); the sparse Jacobian block J_s is CSR with
 * strictly increasing column indices inside each row.
 */
#ifndef MDS_ORACLE_H
#define MDS_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Quadratic MDS test problem (the objective/constraint class of Sec. 2, with
 * constant Hessian blocks):  min 0.5 x_d'H x_d + c'x_d + sum(0.5 w x_s^2 + g x_s)
 * s.t. (J x)_r = b_r for the first m_E = m - m_I rows (eq. (coneq)),
 *      hl_r <= (J x)_r <= hu_r for the last m_I rows (eq. (ineq)),
 *      xl <= x <= xu  (x = [x_d; x_s], J = [J_d J_s], bounds may be +-INFINITY).
 *
 * The IPM works on the slack form of Sec. 2.1's reformulation: every
 * inequality row becomes (J x)_r - d_r = 0 with a slack d_r bounded by
 * [hl_r, hu_r].  Its primal vector has nx = n + m_I entries (x, then d), and
 * so do its bound multipliers. */
typedef struct {
  int32_t n_d, n_s, m;
  const double *H;      /* n_d x n_d, symmetric                     */
  const double *c;      /* n_d                                       */
  const double *w;      /* n_s, >= 0 (assumption A2)                 */
  const double *g;      /* n_s                                       */
  const double *Jd;     /* m x n_d                                   */
  const int32_t *rp;    /* m+1 CSR row pointers of J_s               */
  const int32_t *ci;    /* nnz column indices                        */
  const double *v;      /* nnz values                                */
  const double *b;      /* m                                         */
  const double *xl;     /* n                                         */
  const double *xu;     /* n                                         */
  int32_t m_I;          /* inequality rows (the last m_I of m)       */
  const double *hl;     /* m_I, may be -INFINITY                     */
  const double *hu;     /* m_I, may be +INFINITY                     */
  /* Optional coupling blocks of the sparse Hessian (assumption A2 in its
   * general form: a pattern that is cheap to solve with).  nblk = 0: none.
   * Otherwise bp (nblk + 1, bp[0] = 0 < bp[1] < ... < bp[nblk] = n_s)
   * splits the sparse variables into consecutive blocks and Wb holds each
   * block's symmetric positive semidefinite s x s matrix (s = bp[b+1] -
   * bp[b]), column-major, one block after the other.  The sparse block of
   * the Hessian is then diag(w) + blockdiag(Wb). */
  int32_t nblk;
  const int32_t *bp;
  const double *Wb;
} orq_problem;

/* ---- condensation (Sec. 2.2, eq. (compressed), 2x2-block form) ---------- */
/* Q_{x_s} = diag(dsbase) + dw I (+ blockdiag(Wb) when P has blocks), with
 * dsbase = w + Sigma_s.  Without blocks: inv_d = 1/(dsbase+dw).  With
 * blocks, every block of Q_{x_s} is factored L Delta L' (unit lower L, no
 * pivoting): lblk holds the blocks' L in Wb's layout (strictly lower part
 * written) and inv_d = 1/Delta; the condensation then works on the
 * transformed Jacobian J_s L^{-T}, whose rows fill the blocks they touch.
 * M is N x N (N = n_d + m), full symmetric, column-major.  lblk may be NULL
 * when P has no blocks. */
void or_condense_dcv(const orq_problem *P, const double *sigma_d, const double *dsbase,
                     double dw, double dc, const double *dcv, double *M, double *inv_d,
                     double *lblk);
void or_condense(const orq_problem *P, const double *sigma_d, const double *dsbase,
                 double dw, double dc, double *M, double *inv_d, double *lblk);
/* rhat = r_y - J_s Q_{x_s}^{-1} r_s */
void or_rhs_condense(const orq_problem *P, const double *inv_d, const double *lblk,
                     const double *r_s, const double *r_y, double *rhat);
/* dx_s = Q_{x_s}^{-1} (r_s - J_s' dy) */
void or_backsub(const orq_problem *P, const double *inv_d, const double *lblk,
                const double *r_s, const double *dy, double *dx_s);
/* doubles of the blocks' storage (sum of s^2), 0 without blocks */
int64_t or_blk_words(const orq_problem *P);

/* ---- Bunch-Kaufman LDL' (Sec. 2.3; Bunch & Kaufman 1977) --------------- */
/* A: N x N column-major, lower triangle read.  On exit the strictly lower
 * triangle holds unit-lower L with P'AP = L D L' (all interchanges applied to
 * every column: "standard form"); dd/ds hold D's diagonal / sub-diagonal;
 * ipiv is LAPACK's 1-based lower encoding.  Returns info (0, or 1-based index
 * of the first exactly-zero 1x1 pivot).  If kind != NULL, kind[k] records the
 * branch taken at pivot step k (0 zero column, 1 plain 1x1, 2 1x1 after the
 * second test, 3 1x1 with swap, 4 2x2). */
int or_bk(int32_t N, double *A, int32_t *ipiv, double *dd, double *ds, int32_t *kind);
/* or_bk stopped after the pivot columns 0 .. kstop-1 (a 2x2 pivot may end
 * one column later): a bounded sample of the factorization's work. */
int or_bk_partial(int32_t N, double *A, int32_t *ipiv, double *dd, double *ds, int32_t kstop);
/* Threads of the elimination (default 1); results are bit-identical for
 * every count. */
void or_set_threads(int32_t n);
/* inertia (npos, nzero, nneg) from D */
void or_inertia(int32_t N, const int32_t *ipiv, const double *dd, const double *ds,
                int32_t out[3]);
/* b <- (P L D L' P')^{-1} b.  Returns 0, or 1 if D has a zero 1x1 pivot. */
int or_ldl_solve(int32_t N, const double *L, const int32_t *ipiv, const double *dd,
                 const double *ds, double *b);

/* ---- full (uncondensed) KKT operator (eq. (linsys4x4)) ------------------- */
/* out = K * [dx_d; dx_s; dy] with
 * K = [[H+diag(sigma_d)+dw I, 0, Jd'], [0, diag(dsbase)+dw I (+ blockdiag(Wb)), Js'],
 *      [Jd, Js, -dc I - diag(dcv)]]
 * (dcv: the (4,4) block -D_h^{-1} of the inequality rows, NULL for none). */
void or_kkt_matvec_dcv(const orq_problem *P, const double *sigma_d, const double *dsbase,
                       double dw, double dc, const double *dcv, const double *dx_d,
                       const double *dx_s, const double *dy, double *o_d, double *o_s,
                       double *o_y);
double or_kkt_norm_inf_dcv(const orq_problem *P, const double *sigma_d, const double *dsbase,
                           double dw, double dc, const double *dcv);
void or_kkt_matvec(const orq_problem *P, const double *sigma_d, const double *dsbase,
                   double dw, double dc, const double *dx_d, const double *dx_s,
                   const double *dy, double *o_d, double *o_s, double *o_y);
double or_kkt_norm_inf(const orq_problem *P, const double *sigma_d, const double *dsbase,
                       double dw, double dc);

/* ---- a factored Newton system with its regularisation -------------------- */
typedef struct {
  int32_t N;
  double dw, dc;
  double *L;        /* N*N */
  double *dd, *ds;  /* N each */
  int32_t *ipiv;    /* N */
  double *inv_d;    /* n_s */
  double *lblk;     /* factors of Q_{x_s}'s blocks (or_blk_words doubles) */
  int32_t inertia[3];
  int32_t info;
  int32_t trials;   /* factorizations done by the last correction loop */
  double *dcv;      /* m: (4,4) diagonal of the current system (0 on equality rows) */
  const double *sig_h; /* m_I: slack barrier diagonal, or NULL (no (4,4) block) */
} or_factor;

/* The (4,4) block of eq. (linsys4x4) once the slack step is eliminated
 * (Sec. 2.1 with the slack reformulation): D_h = Sigma_h + dw on the
 * inequality rows; dcv[r] = 1 / D_h for r >= m_E, 0 for equality rows. */
void or_ineq_dcv(const orq_problem *P, const double *sig_h, double dw, double *dcv);
/* Attach (or detach with NULL) the slack barrier diagonal that every later
 * condensation of F turns into its (4,4) block. */
void or_factor_set_slack(or_factor *F, const double *sig_h);

or_factor *or_factor_new(const orq_problem *P);
void or_factor_free(or_factor *F);
/* Condense + factor once with the given shifts. */
void or_factor_once(const orq_problem *P, const double *sigma_d, const double *dsbase,
                    double dw, double dc, or_factor *F);
/* Inertia-correction loop (Sec. 2.1; Algorithm IC of Waechter & Biegler 2006).
 * *dw_last is read and updated.  Returns 0 when In(M) = (n_d, 0, m), 2 when the
 * shift exceeds dw_max. */
int or_factor_inertia(const orq_problem *P, const double *sigma_d, const double *dsbase,
                      double mu, double *dw_last, double dw_max, or_factor *F);
/* Solve the factored Newton system for one right-hand side (condense the rhs,
 * LDL' solve, back-substitute).  Returns 0 or 1 (zero pivot). */
int or_newton_solve(const orq_problem *P, const or_factor *F, const double *r_d,
                    const double *r_s, const double *r_y, double *dx_d, double *dx_s,
                    double *dy);
/* Solve + classic FP64 iterative refinement on the full KKT residual.
 * eta_out: normwise backward error at exit; returns steps taken. */
int or_newton_refine(const orq_problem *P, const or_factor *F, const double *sigma_d,
                     const double *dsbase, const double *r_d, const double *r_s,
                     const double *r_y, double *dx_d, double *dx_s, double *dy,
                     int32_t max_steps, double eta_tol, double *eta_out);

/* ---- IPM vector quantities (Sec. 2.1, kernels K1/K2) --------------------- */
/* Over the primal vector x = [x; d] (nx entries) and its bounds [xl; hl],
 * [xu; hu]: Sigma = zl/(x-l) + zu/(u-x); r = -(grad L - mu/(x-l) + mu/(u-x))
 * with grad L = [grad f + J'y; -y_h]; r_y = -c with c = [J_g x - b; J_h x - d].
 * Infinite bounds contribute nothing.  sigma (nx), r_x (nx), r_y (m). */
void or_sigma_rhs(const orq_problem *P, const double *x, const double *y, const double *zl,
                  const double *zu, double mu, double *sigma, double *r_x, double *r_y);
/* Largest alpha in (0,1] with v + alpha dv >= (1-tau) v for all entries with dv < 0. */
double or_ftb(int64_t n, const double *v, const double *dv, double tau);
/* Scaled optimality error E_mu (components returned in parts[4]: dual inf,
 * primal inf, lower compl., upper compl.; scaling in parts[4..5]). */
double or_opt_error(const orq_problem *P, const double *x, const double *y,
                    const double *zl, const double *zu, double mu, double parts[6]);
/* objective f, barrier function phi_mu, constraint violation theta = ||Jx-b||_1 */
double or_objective(const orq_problem *P, const double *x);
double or_barrier(const orq_problem *P, const double *x, double mu);
double or_theta(const orq_problem *P, const double *x);

/* Newton direction of the barrier problem at (x, y, zl, zu) exactly as one
 * IPM iteration computes it: Sigma and rhs, the inertia-correction loop from
 * delta_w^last = 0, the condensed solve with refine_steps refinement steps,
 * the slack step and the bound-multiplier steps.  dx, dzl, dzu (nx), dy (m).
 * Returns the correction loop's status (0, or 2 when it failed). */
int or_newton_direction(const orq_problem *P, const double *x, const double *y, const double *zl,
                        const double *zu, double mu, int32_t refine_steps, double *dx,
                        double *dy, double *dzl, double *dzu);

/* ---- filter line-search IPM (Sec. 2.1; Waechter & Biegler 2006) ---------- */
typedef struct {
  double tol;          /* stop when E_0 <= tol              (1e-8) */
  double mu0;          /* initial barrier parameter         (0.1)  */
  int32_t max_iter;    /* (200) */
  int32_t refine_steps;/* IR steps per Newton solve         (2)    */
  double dw_max;       /* (1e20) */
} or_ipm_opts;

typedef struct {       /* one row per iteration */
  double mu, E0, theta, phi, alpha_pr, alpha_du, dw, dc;
  int32_t inertia[3];
  int32_t trials, backtracks;
  int32_t soc;         /* general NLP: a second-order correction was accepted  */
  int32_t resto;       /* general NLP: restoration iterations (-1: failed)     */
  int32_t pad;
} or_ipm_trace;

/* x, zl, zu (nx = n + m_I: variables then slacks) and y (m) are outputs
 * (start point computed inside).
 * Returns 4 converged, 5 line-search failure, 6 max iterations, 2 inertia
 * failure, 7 non-finite values.  *iters: iterations done.  trace may be NULL
 * or hold max_iter rows. */
int or_ipm(const orq_problem *P, const or_ipm_opts *o, double *x, double *y, double *zl,
           double *zu, int32_t *iters, or_ipm_trace *trace);
/* The same IPM from a warm start: proposed x_d (n_d), y (m) and barrier
 * parameter mu0 (see warm_point in mds_oracle.c for the completed point).
 * Returns 8 (not defined) when P has coupling blocks. */
int or_ipm_warm(const orq_problem *P, const or_ipm_opts *o, const double *xd0, const double *y0,
                double mu0, double *x, double *y, double *zl, double *zu, int32_t *iters,
                or_ipm_trace *trace);

/* ---- general NLP through an external model -------------------------------- */
/* The model objects of the problem class (Sec. 2, A1/A2 hold): objective,
 * its gradient over x (n), the constraint values over the m rows (c_r(x),
 * target 0, for the first m_E rows; h_r(x), bounded by [hl, hu], for the
 * rest), the Jacobian values (J_d: m x n_d column-major; J_s: in P's CSR
 * pattern) and the Hessian of the Lagrangian f + y'c at (x, y) (H: n_d x n_d
 * dense; w: the diagonal of the sparse block, >= 0). */
typedef struct {
  void *ctx;
  double (*objective)(void *ctx, const double *x);
  void (*gradient)(void *ctx, const double *x, double *g);
  void (*constraints)(void *ctx, const double *x, double *c);
  void (*jacobian)(void *ctx, const double *x, double *Jd, double *v);
  void (*hessian)(void *ctx, const double *x, const double *y, double *H, double *w);
} or_nlp_model;

typedef struct {
  int32_t soc_trials, soc_accepted, resto_iters, resto_calls;
} or_nlp_stats;

/* The filter line-search IPM of or_ipm on a general NLP: the model is
 * evaluated at every iterate, a rejected first trial point whose constraint
 * violation did not drop gets up to four second-order corrections (the
 * Newton system solved again with c_soc = alpha c(x) + c(x_trial), then
 * c_soc = alpha_soc c_soc + c(x_soc)), and a line search that fails enters
 * the feasibility restoration described at nlp_restore (force_resto >= 0
 * also enters it at that iteration).  P supplies dimensions, the J_s pattern
 * and the bounds.  Returns or_ipm's codes, and 9 when the model's sparse
 * Hessian diagonal is negative. */
int or_nlp_ipm(const orq_problem *P, const or_nlp_model *M, const or_ipm_opts *o,
               int32_t force_resto, double *x, double *y, double *zl, double *zu,
               int32_t *iters, or_ipm_trace *trace, or_nlp_stats *stats);
/* or_nlp_ipm on the separable nonlinear test family built on P's data:
 * f = P's quadratic + sum_k e_k (exp(x_s,k) - x_s,k); rows (J x)_r +
 * sum_j Q_rj x_d,j^2 (- b_r on equality rows); Q is m x n_d column-major. */
int or_nlp_test_ipm(const orq_problem *P, const double *Q, const double *e,
                    const or_ipm_opts *o, int32_t force_resto, double *x, double *y,
                    double *zl, double *zu, int32_t *iters, or_ipm_trace *trace,
                    or_nlp_stats *stats);
double or_nlp_test_eval(const orq_problem *P, const double *Q, const double *e, const double *x,
                        const double *y, double *g, double *c, double *Jd, double *v,
                        double *H, double *w);

#ifdef __cplusplus
}
#endif
#endif
