/*
 * mdsipm — MI355X (gfx950) library for the Newton-step hot path of the
 * mixed dense-sparse (MDS) interior-point method of Peles et al., "Porting the
 * Nonlinear Optimization Library HiOp to Accelerator-Based Hardware
 * Architectures".
 *
 * Problem class (Sec. 2, eqs. (obj)-(bounds), with linear constraints):
 *     min  0.5 x_d'H x_d + c'x_d + sum_i (0.5 w_i x_s,i^2 + g_i x_s,i)
 *     s.t. (J x)_r = b_r          for the first m_E = m - m_I rows (eq. (coneq)),
 *          hl_r <= (J x)_r <= hu_r for the last m_I rows (eq. (ineq)),
 *          xl <= x <= xu,   x = [x_d; x_s],   J = [J_d J_s].
 * Assumption A1 (no cross Hessian) and A2 (diagonal, nonnegative Hessian of
 * the sparse block: w >= 0) hold by construction of this class.
 *
 * Newton system (Sec. 2.1, eq. (linsys4x4); the equality and inequality rows
 * of J are kept in one block y = [y_g; y_h]):
 *     [[H + Sigma_d + dw I, 0,               J_d'],   [dx_d]   [r_d]
 *      [0,                  D_s,             J_s'],   [dx_s] = [r_s]
 *      [J_d,                J_s,     -dc I - Dh ]]   [dy  ]   [r_y]
 * with D_s = w + Sigma_s + dw (diagonal, positive) and Dh = diag(dcv) the
 * (4,4) block -D_h^{-1} of the inequality rows (zero on equality rows).
 * Eliminating dx_s (Sec. 2.2, eq. (compressed)) leaves the dense symmetric
 * indefinite
 *     M = [[H + Sigma_d + dw I, J_d'], [J_d, -J_s D_s^{-1} J_s' - dc I - Dh]]
 * of size N = n_d + m, factored by Bunch-Kaufman LDL' (Sec. 2.3); its inertia
 * plus In(D_s) = (n_s,0,0) is the inertia of the full system (Haynsworth).
 * The IPM turns the inequality rows into equalities (J x)_r - d_r = 0 with a
 * bounded slack d (hl <= d <= hu) and eliminates the slack step: with Sigma_h
 * the slack's barrier diagonal, D_h = Sigma_h + dw and dcv = 1 / D_h.
 *
 * Conventions
 *  - All array pointers are DEVICE pointers (hipMalloc'd or framework-owned
 *    device memory) unless the parameter name ends in _host.  The caller owns
 *    every array, including the workspace; the library owns only the handle.
 *  - Dense matrices are column-major.  J_s is CSR with strictly increasing
 *    column indices in each row (validated).
 *  - Calls are asynchronous on the handle's stream unless documented as
 *    synchronizing (those that return host results synchronize that stream
 *    only).  One handle per host thread.
 *  - Return value: 0 = success; < 0 = usage or system error (outputs
 *    untouched, message in mds_last_error); > 0 = numerical outcome (outputs
 *    valid).  No C++ exception crosses this interface.
 *  - Zero sizes are legal: n_s = 0 (no Schur term), m = 0 (M = H + Sigma_d +
 *    dw I), n_d = 0 (M = -J_s D_s^{-1} J_s' - dc I).
 */
#ifndef MDSIPM_H
#define MDSIPM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mds_handle mds_handle;

enum {
  MDS_OK = 0,
  /* usage / system errors (< 0) */
  MDS_EINVAL = -1,          /* bad argument value                          */
  MDS_ENULL = -2,           /* required pointer is NULL                    */
  MDS_EDIMS = -3,           /* negative or inconsistent dimensions         */
  MDS_EWORKSPACE = -4,      /* workspace too small or misaligned           */
  MDS_ESTATE = -5,          /* call order violated (e.g. solve before factor) */
  MDS_EHIP = -6,            /* HIP runtime error                           */
  MDS_ENONFINITE_INPUT = -7,/* NaN/Inf in problem data                     */
  MDS_EDS_NONPOS = -8,      /* w < 0, xl >= xu, or D_s <= 0                */
  MDS_EPATTERN = -9,        /* CSR pattern invalid (unsorted, out of range) */
  MDS_EMODEL = -10,         /* a model callback reported a failure          */
  /* numerical outcomes (> 0) */
  MDS_ZERO_PIVOT = 1,       /* D has an exactly zero 1x1 pivot             */
  MDS_INERTIA_FAIL = 2,     /* correction shift exceeded dw_max            */
  MDS_REFINE_NOCONV = 3,    /* refinement stopped above its tolerance      */
  MDS_IPM_CONVERGED = 4,
  MDS_IPM_LS_FAIL = 5,      /* line search step below alpha_min            */
  MDS_IPM_MAXITER = 6,
  MDS_IPM_NONFINITE = 7
};

typedef struct {
  int32_t n_d, n_s, m; /* N = n_d + m is the condensed size, N <= 20480 */
  int32_t m_I;         /* inequality rows: the last m_I of the m rows of J
                          (0 <= m_I <= m; 0: equality constraints only)  */
  int64_t nnz_s;       /* nonzeros of J_s */
} mds_dims;

/* Precision of the trailing updates of the factorization.  MDS_FP64: every
 * step in FP64.  MDS_FP32 / MDS_BF16 / MDS_BF16X3: the trailing matrix is
 * stored in FP32 and its rank-w updates run on FP32 MFMA, on BF16 MFMA with
 * FP32 accumulation, or on three BF16 MFMAs per product with each operand
 * split into a BF16 high part and a BF16 residual (FP32 accumulation);
 * pivot search, L, the 1x1/2x2 D blocks and the solves stay
 * FP64, and mds_refine runs GMRES-based iterative refinement in FP64 on the
 * full Newton system, preconditioned by the low-precision factorization.
 * The low-precision factorization is of the equilibrated S M S with
 * S = diag(1 / sqrt(max_j |M_ij|)) (same inertia as M); mds_get_factor
 * returns that factor.  The mixed modes need a register-resident panel
 * (panel 2 or 3). */
enum { MDS_FP64 = 0, MDS_FP32 = 1, MDS_BF16 = 2, MDS_BF16X3 = 3 };

typedef struct {
  int32_t nb;          /* panel width of the blocked factorization (0: default) */
  int32_t panel;       /* 0: automatic (register-resident panel when its tile
                          allows nb >= 16, i.e. N <= 2048; above that the
                          cooperative panel, which hands over to the
                          one-workgroup register panel once at most 1024
                          rows remain),
                          1: panel kept in device memory (FP64 only),
                          2: register-resident panel, one workgroup (N <= 4096),
                          3: register-resident panel over ceil(N / 1024)
                             cooperating workgroups, nb <= 32 (any N); its
                             workgroups exchange pivot data through the
                             workspace and must run concurrently: when an
                             exchange wait expires (~0.7 s) the matrix is
                             condensed again and factored by the memory
                             panel in FP64 (the factor then is an FP64 one
                             in every precision mode; mds_get_fallbacks
                             counts these),
                          4: unblocked factorization of the whole M held in
                             one workgroup's LDS (FP64, N <= 199; the
                             interchanges are applied to whole rows, so the
                             factor is in standard form at once)            */
  int32_t precision;   /* MDS_FP64 (default), MDS_FP32, MDS_BF16, MDS_BF16X3   */
  int32_t panel_threads; /* register panel workgroup: 64, 128, 256, 512 or
                            1024 (0: 128 up to N = 128, 256 up to N = 256,
                            else 512); the cooperative panel uses 512; the
                            LDS factorization 256 or 512 (0: 512)           */
  int32_t nlp;         /* 1: the workspace also holds the model objects of a
                          general NLP (mds_set_nlp)                         */
  int32_t sblk_max;    /* 0: the sparse Hessian block is diag(w).  1..16: the
                          workspace also holds coupling blocks of at most
                          this many sparse variables (mds_set_sparse_blocks)
                          and the transformed Jacobian they induce (up to
                          sblk_max * nnz_s entries)                          */
  int32_t lookahead;   /* cooperative factorization: 0 automatic (on for
                          N >= 8192), 1 on, 2 off.  With look-ahead, panel
                          b + 1 and the update of the 64-column strip ahead
                          of it run on a few reserved compute units (4 per
                          XCD, at least the panel's workgroups) while the
                          rest of panel b's trailing update runs on the
                          others (two CU-masked streams the handle creates;
                          the handle's stream waits for both).  Panel b + 1
                          computes the entries it needs outside the strip
                          from panel b's input and multipliers, so its
                          pivots are those of the sequential order (up to
                          the rounding of those entries).  It applies to
                          every precision mode.  Off, or not applicable
                          (another panel, the memory-panel fallback, a
                          device whose CUs are not 8 equal XCDs): the
                          launches of one factorization are sequential on
                          the handle's stream.                              */
  int32_t reserved[1];
} mds_options;

/* Problem data, all device pointers, caller-owned, must stay valid and
 * unmodified while the handle uses them (until the next mds_set_problem or
 * mds_destroy). */
typedef struct {
  const double *H;        /* n_d x n_d, symmetric (both triangles read)     */
  const double *c;        /* n_d                                             */
  const double *w;        /* n_s, >= 0                                       */
  const double *g;        /* n_s                                             */
  const double *J_d;      /* m x n_d                                         */
  const int32_t *Js_rowptr; /* m+1                                           */
  const int32_t *Js_col;  /* nnz_s                                           */
  const double *Js_val;   /* nnz_s                                           */
  const double *b;        /* m_E = m - m_I: right-hand side of the equality
                             rows (the entries of inequality rows are not
                             read)                                           */
  const double *xl, *xu;  /* n = n_d + n_s; +-INFINITY allowed, xl < xu      */
  const double *hl, *hu;  /* m_I: bounds of the inequality rows, +-INFINITY
                             allowed, hl < hu, at least one finite (eq.
                             (ineq)); may be NULL when m_I = 0               */
} mds_problem;

typedef struct {
  int32_t npos, nzero, nneg; /* inertia of M                               */
  int32_t n2x2;              /* number of 2x2 pivot blocks                  */
  int32_t info;              /* 0, or 1-based index of the first zero pivot */
} mds_inertia;

/* Inertia-correction state (Sec. 2.1; Algorithm IC of Waechter & Biegler).
 * delta_w_last is read and written; the other fields are outputs. */
typedef struct {
  double delta_w_last;
  double delta_w, delta_c;  /* shifts of the accepted factorization          */
  double delta_w_max;       /* cap; 0 selects 1e20                           */
  int32_t trials;           /* factorizations performed                      */
  int32_t pad;
} mds_reg;

typedef struct {
  double eta;               /* normwise backward error on the full system    */
  double rel_residual;      /* ||r - K d||_inf / ||r||_inf                   */
  int32_t steps;            /* refinement corrections applied                */
  int32_t pad;
} mds_refine_info;

/* IPM iterate.  x, zl, zu are device arrays of n + m_I entries: the n
 * variables followed by the m_I inequality slacks d (x[n + r] is the slack
 * of inequality row m_E + r, hl_r <= d_r <= hu_r) and their bound
 * multipliers; y (m) holds the multipliers of all rows.  The scalars are host
 * values that mds_ipm_init sets and mds_ipm_step updates. */
typedef struct {
  double *x, *y, *zl, *zu;
  double mu, tau;
  int32_t iter;
  int32_t pad;
} mds_iterate;

typedef struct {
  double tol;          /* stop when E_0 <= tol (1e-8)                        */
  double mu0;          /* initial barrier parameter (0.1)                    */
  int32_t max_iter;    /* (200)                                              */
  int32_t refine_steps;/* refinement steps per Newton solve (2)              */
  double dw_max;       /* correction cap (1e20)                              */
  int32_t gmres_max;   /* mixed precision: GMRES iterations per Newton solve
                          (0: 60); a solve that stops above backward error
                          1e-14 is redone from an FP64 factorization         */
  int32_t pad;
} mds_ipm_opts;

typedef struct {       /* one IPM iteration (host) */
  double mu, E0, theta, phi, alpha_pr, alpha_du, delta_w, delta_c, eta;
  int32_t inertia[3];
  int32_t trials;      /* factorizations (inertia-correction trials)          */
  int32_t solves;      /* LDL' solves (1 + refinement corrections)            */
  int32_t backtracks, status;
  int32_t fallback;    /* bit 0: the mixed-precision refinement stopped above
                          its tolerance and the step was recomputed from an
                          FP64 factorization of the same Newton system;
                          bit 1: a cooperative panel's exchange wait expired
                          and the memory panel refactored the matrix        */
  int32_t nlp_event;   /* NLP mode (mds_set_nlp): 1 the accepted point came
                          from a second-order correction; 2 the iteration
                          ended in a feasibility restoration phase (x, z are
                          its end point, y is kept; the phase's steps are in
                          mds_get_nlp_stats); 0 otherwise                    */
} mds_step_info;

/* Per-kernel-class device time, accumulated while timing is enabled
 * (hipEvents recorded around each launch on the stream it runs on).  PERMUTE
 * is the conversion of a new factor to standard form before its first solve;
 * SOLVE is one triangular-solve sequence (permute, L, D, L', permute);
 * PANEL_TAIL holds the register-panel launches that finish a cooperative
 * factorization (PANEL then holds only the cooperative ones).  FACTOR is
 * each whole factorization on the handle's stream (with look-ahead its
 * classes overlap, so their sum exceeds it); NEAR the look-ahead's strip
 * updates (TRAILING then holds the rest of each trailing update). */
enum { MDS_T_CONDENSE = 0, MDS_T_PANEL = 1, MDS_T_TRAILING = 2, MDS_T_SOLVE = 3,
       MDS_T_PERMUTE = 4, MDS_T_PANEL_TAIL = 5, MDS_T_FACTOR = 6, MDS_T_NEAR = 7,
       MDS_T_CLASSES = 8 };
typedef struct {
  double ms[MDS_T_CLASSES];     /* summed kernel time per class            */
  int64_t launches[MDS_T_CLASSES];
} mds_timings;

/* ---- lifetime ----------------------------------------------------------- */

/* Bytes of device workspace for these dimensions (256-byte aligned start
 * required).  Dominated by the N x N matrix (8 N^2 bytes). */
size_t mds_workspace_bytes(const mds_dims *dims, const mds_options *opts);

/* Create a handle bound to the current HIP device, the given stream (a
 * hipStream_t; NULL = default stream) and a caller-owned device workspace of
 * at least mds_workspace_bytes() bytes.  opts may be NULL. */
int mds_create(mds_handle **out, const mds_dims *dims, const mds_options *opts,
               void *stream, void *workspace, size_t workspace_bytes);
void mds_destroy(mds_handle *h);

/* Attach problem data; validates it (finite values, w >= 0, xl < xu, sorted
 * in-range CSR) and builds the column-compressed copy of J_s in the
 * workspace.  Leaves NLP mode (mds_set_nlp).  Synchronizes the stream. */
int mds_set_problem(mds_handle *h, const mds_problem *p);

/* ---- Newton-step hot path ------------------------------------------------ */

/* Assemble M (Sec. 2.2, eq. (compressed); kernel class K3) and
 * D_s^{-1} = 1/(dsbase + delta_w) into the workspace.  sigma_d (n_d) and
 * dsbase = w + Sigma_s (n_s, > 0) are device arrays that must remain valid
 * until the next mds_condense (the correction loop re-condenses with them).
 * The (2,2) block is accumulated over the shared columns of each row pair in
 * ascending column order, so M is bitwise reproducible.  Async. */
int mds_condense(mds_handle *h, const double *sigma_d, const double *dsbase,
                 double delta_w, double delta_c);

/* Optional per-row diagonal of the (2,2) block: every later condensation
 * subtracts dcv[r] from M22(r, r) after delta_c, and the full Newton system
 * used by refinement and the backward error carries -delta_c - dcv[r] in its
 * (y, y) block.  This is how the inverse barrier diagonal of inequality rows
 * (-D_h^{-1}) enters the compressed form of Sec. 2.2 when the constraints
 * include inequalities.  dcv: device array (m), caller-owned, finite and
 * >= 0 (checked: MDS_EINVAL otherwise, nothing changes), valid while set;
 * NULL clears it, and so does mds_set_problem.  The IPM computes this block
 * itself from its inequality slacks, so mds_ipm_init and mds_ipm_init_warm
 * return MDS_ESTATE while a caller's diagonal is set.  Invalidates the
 * current M and factor.  Synchronizes. */
int mds_set_m22_diag(mds_handle *h, const double *dcv);

/* ---- general NLP: model objects from an external modeling layer ----------
 * The problem class of Sec. 2 with nonlinear f and rows (A1/A2 hold: no
 * cross Hessian between x_d and x_s, a nonnegative diagonal Hessian of the
 * sparse block); the model objects are supplied by the modeling layer (the
 * end of Sec. 2.3).  Every callback runs on the calling host thread with
 * device arrays and must have finished, or be ordered on the handle's
 * stream, when it returns; 0 means success (any other value ends the IPM
 * step with MDS_EMODEL).  x has n = n_d + n_s entries, y has m. */
typedef struct {
  void *ctx;
  int (*objective)(void *ctx, const double *x, double *f_host);       /* f(x)        */
  int (*gradient)(void *ctx, const double *x, double *g);             /* grad f: n   */
  /* the m rows at x: c_r(x) (target 0) on the first m_E, h_r(x) (bounded by
   * [hl, hu] of mds_problem) on the last m_I */
  int (*constraints)(void *ctx, const double *x, double *c);
  /* Jacobian values at x: J_d (m x n_d, column-major), J_s in the CSR
   * pattern of mds_problem (nnz_s values) */
  int (*jacobian)(void *ctx, const double *x, double *J_d, double *Js_val);
  /* Hessian of the Lagrangian f + y'c at (x, y): H (n_d x n_d, symmetric,
   * column-major) and the diagonal w of the sparse block (n_s, >= 0) */
  int (*hessian)(void *ctx, const double *x, const double *y, double *H, double *w);
} mds_nlp_model;

/* Switch the handle's IPM (mds_ipm_init / mds_ipm_step / mds_ipm_solve) to
 * the general NLP given by `model` (NULL: back to the quadratic problem of
 * mds_set_problem, whose J_s pattern, bounds and inequality bounds the NLP
 * keeps).  Needs a workspace created with options.nlp = 1 (the model's H,
 * J_d, J_s values, w and gradient live there).  In NLP mode the filter line
 * search adds the second-order correction (a rejected first trial whose
 * constraint violation did not drop: up to four re-solves with
 * c_soc = alpha c(x) + c(x_trial), then alpha_soc c_soc + c(x_soc)) and a
 * feasibility restoration when the line search fails (Gauss-Newton-type
 * barrier steps on min zeta/2 ||D_R (x - x_R)||^2 s.t. c(x) = 0, zeta =
 * sqrt(mu), D_R = diag(min(1, 1/|x_R|)), until theta <= 0.9 theta(x_R) and
 * the point is acceptable to the filter; at most 30 steps); a line search
 * takes at most 200 backtracks.  The model's w must stay >= 0 (else the
 * step returns MDS_EDS_NONPOS).  The warm start and coupling blocks are not
 * available in NLP mode (MDS_ESTATE).  The Newton-system calls
 * (mds_condense, mds_sigma_rhs, ...) see the model's values from its last
 * evaluation (the quadratic problem's values right after this call).
 * Synchronizes.  Errors: MDS_ESTATE, MDS_ENULL, MDS_EHIP. */
int mds_set_nlp(mds_handle *h, const mds_nlp_model *model);
/* Statistics of NLP mode since mds_ipm_init: second-order corrections tried
 * and accepted, restoration phases entered and their steps. */
typedef struct { int32_t soc_trials, soc_accepted, resto_calls, resto_iters; } mds_nlp_stats;
int mds_get_nlp_stats(const mds_handle *h, mds_nlp_stats *out_host);

/* A built-in model of that interface, the separable nonlinear family on an
 * MDS problem's data (for tests and benchmarks):
 *   f(x)  = 0.5 x_d'H x_d + c'x_d + sum_k (0.5 w_k x_s,k^2 + g_k x_s,k
 *           + e_k (exp(x_s,k) - x_s,k)),
 *   row r = (J_d x_d)_r + (J_s x_s)_r + sum_j Q_rj x_d,j^2, minus b_r on the
 *           equality rows;
 * Q (m x n_d, column-major) and e (n_s, >= 0) on the device; p's arrays are
 * read by the callbacks (caller-owned, must outlive the model).  The model
 * works on `stream` and needs mds_sep_model_workspace_bytes() of device
 * workspace (256-byte aligned).  model_out receives the callbacks. */
typedef struct mds_sep_model mds_sep_model;
size_t mds_sep_model_workspace_bytes(void);
int mds_sep_model_create(mds_sep_model **out, const mds_dims *dims, const mds_problem *p,
                         const double *Q, const double *e, void *stream, void *workspace,
                         size_t workspace_bytes, mds_nlp_model *model_out);
void mds_sep_model_destroy(mds_sep_model *M);

/* Coupling blocks of the sparse Hessian (assumption A2 of Sec. 2 in its
 * general form: a pattern that makes solves with Q_{x_s} cheap).  The sparse
 * block of the Hessian becomes diag(w) + blockdiag(Wb): bp_host (HOST,
 * nblk + 1 entries, 0 = bp[0] < bp[1] < ... < bp[nblk] = n_s) splits the
 * sparse variables into consecutive blocks of 1 .. options.sblk_max
 * variables; Wb (device, sum of the blocks' s^2 doubles) holds each block's
 * s x s matrix column-major, one after another; only lower triangles are
 * read, but each block must be exactly symmetric, finite and positive
 * semidefinite (checked here, with a copy to the host).  Caller-owned; must
 * stay valid while set.  Condensation then factors every block of
 * Q_{x_s} = blockdiag(Wb) + diag(dsbase) + dw I as L Delta L' and works on
 * J_s L^{-T} with the middle factor 1/Delta (mds_get_inv_ds returns 1/Delta);
 * the solve, the full-system products and norms used by refinement, the
 * objective and its gradient all carry the blocks.  nblk = 0 removes them;
 * mds_set_problem removes them too.  The warm start (mds_ipm_init_warm)
 * returns MDS_ESTATE while blocks are set.  Synchronizes.  Errors: MDS_ESTATE
 * (sblk_max = 0 or no problem), MDS_EDIMS, MDS_EINVAL (layout, sizes,
 * symmetry), MDS_EDS_NONPOS (a block not positive semidefinite),
 * MDS_ENONFINITE_INPUT. */
int mds_set_sparse_blocks(mds_handle *h, int32_t nblk, const int32_t *bp_host, const double *Wb);

/* Bunch-Kaufman LDL' of the condensed M with its inertia (Sec. 2.3, kernel
 * class K4).  reg == NULL: factor M as last condensed.  reg != NULL: run the
 * inertia-correction loop (Sec. 2.1): factor with zero shifts, then re-condense
 * and refactor with growing delta_w (and delta_c = 1e-8 mu^(1/4) if M is
 * singular) until In(M) = (n_d, 0, m).  Synchronizes the stream.
 * Returns 0, MDS_ZERO_PIVOT (reg == NULL and an exact zero pivot) or
 * MDS_INERTIA_FAIL. */
int mds_factor_inertia(mds_handle *h, mds_reg *reg, double mu, mds_inertia *out_host);

/* Solve the factored Newton system for one right-hand side: condense the rhs
 * (r_hat = r_y - J_s D_s^{-1} r_s), LDL' solve for [dx_d; dy], back-substitute
 * dx_s = D_s^{-1} (r_s - J_s' dy).  The first solve after a factorization
 * first brings the factor to standard form in place.  Inputs and outputs are
 * device arrays and must not alias.  Async; a failure of the solve kernels'
 * bounded dependency waits is reported (MDS_EHIP) by the next mds_refine. */
int mds_solve(mds_handle *h, const double *r_d, const double *r_s, const double *r_y,
              double *dx_d, double *dx_s, double *dy);

/* mds_solve followed by FP64 iterative refinement on the residual of the full
 * (uncondensed) system, evaluated matrix-free.  FP64 factorization: classic
 * refinement, which stops when the normwise backward error eta <= eta_tol,
 * when it stops decreasing (the best iterate is kept) or after max_steps
 * corrections.  Mixed-precision factorization: restarted GMRES(20) in FP64
 * with the low-precision LDL' solve as right preconditioner, until
 * eta <= eta_tol or max_steps GMRES iterations; info->steps counts GMRES
 * iterations.  Synchronizes the stream. */
int mds_refine(mds_handle *h, const double *r_d, const double *r_s, const double *r_y,
               double *dx_d, double *dx_s, double *dy, int32_t max_steps, double eta_tol,
               mds_refine_info *info_host);

/* ---- IPM vector kernels (Sec. 2.1, kernel classes K1/K2) ------------------ */

/* Barrier diagonal and Newton right-hand side at an iterate (layout of
 * mds_iterate: x, zl, zu, sigma and r_x have n + m_I entries, the slacks
 * d after the variables).  sigma = zl/(x-xl) + zu/(xu-x);
 * r_x = -(grad L - mu/(x-xl) + mu/(xu-x)) with grad L = [grad f + J'y; -y_h]
 * (the slack entries get y_h + barrier terms); r_y = -c with
 * c = [J_g x - b; J_h x - d].  Infinite bounds contribute nothing.  Async. */
int mds_sigma_rhs(mds_handle *h, const double *x, const double *y, const double *zl,
                  const double *zu, double mu, double *sigma, double *r_x, double *r_y);

/* Fraction to the boundary: largest alpha in (0,1] with
 * v + alpha dv >= (1 - tau) v wherever dv < 0.  Synchronizes. */
int mds_ftb(mds_handle *h, int64_t n, const double *v, const double *dv, double tau,
            double *alpha_host);

/* Allocation-free variant of mds_ftb, for callers that cannot allocate
 * device memory or create a handle (code under stream capture, tight serving
 * loops, harnesses that forbid allocation).  Same step as mds_ftb, written to
 * the DEVICE pointer alpha (one double) on `stream` (a hipStream_t; NULL is
 * the null stream); asynchronous, no host synchronization, no allocation.
 * v, dv: n device doubles; 0 < tau <= 1; n = 0 gives alpha = 1.  The
 * reduction's partial records live in a fixed device array of
 * mds_ftb_noalloc_scratch_bytes() bytes (64 KiB + 64 B) that each GPU holds
 * until the process ends; its need is the same for every n, so no n exceeds
 * it.  Calls on one GPU share that array: calls that overlap on one GPU
 * (several streams or host threads) race.  Errors: MDS_ENULL, MDS_EDIMS
 * (n < 0), MDS_EINVAL (tau), MDS_EHIP. */
int mds_ftb_noalloc(int64_t n, const double *v, const double *dv, double tau, double *alpha,
                    void *stream);
size_t mds_ftb_noalloc_scratch_bytes(void);

/* Scaled optimality error E_mu; parts_host (may be NULL) receives
 * {dual inf, primal inf, lower compl, upper compl, s_d, s_c}.  Synchronizes. */
int mds_opt_error(mds_handle *h, const double *x, const double *y, const double *zl,
                  const double *zu, double mu, double *E_host, double *parts_host);

/* Objective f, barrier function phi_mu (log-barrier over every finite bound
 * of the variables and the slacks) and theta = ||c(x, d)||_1.  x has n + m_I
 * entries.  Synchronizes. */
int mds_merit(mds_handle *h, const double *x, double mu, double *f_host, double *phi_host,
              double *theta_host);

/* ---- filter line-search IPM (Sec. 2.1) ------------------------------------ */

/* Set the start point (x = 0 pushed inside its bounds, each slack d_r the
 * row value (J x)_r pushed inside [hl_r, hu_r] by the same rule, y = 0,
 * z = 1 on finite bounds) and reset the filter and correction state.  opts
 * may be NULL.  MDS_ESTATE while a caller's (2,2) diagonal is set
 * (mds_set_m22_diag). */
int mds_ipm_init(mds_handle *h, mds_iterate *it, const mds_ipm_opts *opts);

/* mds_ipm_init from a proposed start (the learned warm start): x_d0 (n_d)
 * and y0 (m) device arrays, barrier parameter mu0 > 0.  x_s is completed from
 * the sparse block's stationarity, -(g + J_s' y0) / w where w > 0 (else 0);
 * every x_i is pushed into the interior of its bounds by the cold start's
 * rule; y = y0; z = mu0 / slack on finite bounds, plus the part of the dual
 * residual r = grad f(x) + J' y0 the bound can carry (r > 0 added to z_l,
 * -r > 0 to z_u), so that the start is near-stationary when the proposal is
 * near a solution.  Slacks: d = (J x)_h pushed inside [hl, hu], their
 * multipliers mu0 / slack plus the part of -y_h they can carry. */
int mds_ipm_init_warm(mds_handle *h, mds_iterate *it, const mds_ipm_opts *opts,
                      const double *x_d0, const double *y0, double mu0);

/* One IPM iteration: convergence test, barrier update, Newton step with
 * inertia correction and refinement, fraction to the boundary, filter
 * backtracking line search, update with the bound-multiplier safeguard.
 * Returns 0 (step taken), MDS_IPM_CONVERGED (no step taken), or a failure
 * code.  Synchronizes. */
int mds_ipm_step(mds_handle *h, mds_iterate *it, mds_step_info *info_host);

/* mds_ipm_init followed by mds_ipm_step until it returns nonzero.  trace_host
 * (may be NULL) receives one row per call of mds_ipm_step, at most trace_cap
 * rows; *iters_host the number of steps taken.  Returns the final status
 * (MDS_IPM_CONVERGED on success).  Synchronizes. */
int mds_ipm_solve(mds_handle *h, mds_iterate *it, const mds_ipm_opts *opts,
                  mds_step_info *trace_host, int32_t trace_cap, int32_t *iters_host);

/* ---- diagnostics ----------------------------------------------------------- */

/* Copy the assembled M (before factorization) to host (N*N doubles). */
int mds_get_matrix(mds_handle *h, double *M_host);
/* Copy the factor to host in standard form: P'MP = L D L' with L unit lower
 * (N*N column-major, strictly lower part), D diagonal/sub-diagonal (N each)
 * and LAPACK-style 1-based ipiv (lower).  Any pointer may be NULL. */
int mds_get_factor(mds_handle *h, double *L_host, double *dd_host, double *ds_host,
                   int32_t *ipiv_host);
/* Copy the pivot sequence (N, LAPACK-style 1-based, lower: k+1 for a 1x1
 * pivot without interchange, q+1 after interchanging k and q, -(q+1) on both
 * rows of a 2x2 pivot) to host.  Synchronizes. */
int mds_get_pivots(mds_handle *h, int32_t *ipiv_host);
/* Copy D^{-1}_s (n_s) to host. */
int mds_get_inv_ds(mds_handle *h, double *inv_d_host);

/* Configuration chosen at mds_create (host). */
typedef struct {
  int32_t nb;           /* panel width limit                                  */
  int32_t min_width;    /* fewest columns a panel factors (except the last)   */
  int32_t panel;        /* 0: register-resident panel, 1: panel in memory,
                           2: cooperative register-resident panel,
                           3: whole M in one workgroup's LDS                 */
  int32_t precision;    /* MDS_FP64, MDS_FP32, MDS_BF16 or MDS_BF16X3          */
  int32_t panel_threads; /* workgroup size of the panel kernel                */
  int32_t lookahead_cus; /* look-ahead: compute units reserved for the panel
                            and the near update (0: no look-ahead)           */
  int64_t workspace_bytes;
} mds_info;
int mds_get_info(const mds_handle *h, mds_info *out_host);

/* Robustness counters since mds_create (host): coop_aborts = cooperative
 * factorizations whose exchange wait expired and which the memory panel
 * redid; fp64_refactors = mixed-precision Newton solves of mds_ipm_step that
 * were redone from an FP64 factorization. */
typedef struct {
  int64_t coop_aborts, fp64_refactors;
} mds_fallbacks;
int mds_get_fallbacks(const mds_handle *h, mds_fallbacks *out_host);

/* Pivot statistics of the last factorization (host): panels, steps of the
 * cooperative panel and how many of them took its second exchange (the
 * candidate column, when the first Bunch-Kaufman test of Sec. 2.3 fails),
 * and 2x2 pivots.  Synchronizes. */
typedef struct {
  int32_t panels, coop_steps, coop_second, n2x2;
} mds_panel_stats;
int mds_get_panel_stats(mds_handle *h, mds_panel_stats *out_host);

/* Latency probe of the cooperative panel's exchange (the floor of its
 * per-pivot chain): P workgroups (1..32) of 512 threads run `rounds`
 * exchanges in which every workgroup publishes `words` tagged 64-bit words
 * (1..512, P * words <= 2048) and reads every workgroup's words in one
 * round trip, with no other work.  *us_per_round_host receives the wall
 * time per round.  Uses the handle's exchange buffer: do not overlap it with
 * a factorization on another stream.  The P workgroups must be resident at
 * once (else MDS_EHIP after the bounded wait).  Synchronizes. */
int mds_probe_exchange(mds_handle *h, int32_t P, int32_t rounds, int32_t words,
                       double *us_per_round_host);

/* Test hook for the failure paths, in the spirit of fault injection from the
 * host: flag MDS_DEBUG_COOP_ABORT makes every later cooperative panel launch
 * report an expired exchange wait at once (each workgroup leaves before its
 * first exchange, so every kernel still ends normally), which exercises the
 * memory-panel refactorization.  Flag MDS_DEBUG_FORCE_RESTO makes the next
 * IPM step in NLP mode enter the feasibility restoration after its line
 * search, whether or not the search accepted a point (the step consumes the
 * flag).  0 clears the flags.  Synchronizes. */
enum { MDS_DEBUG_COOP_ABORT = 1, MDS_DEBUG_FORCE_RESTO = 2 };
int mds_set_debug(mds_handle *h, int32_t flags);

/* Enable (1) or disable (0) per-launch timing; enabling clears the totals. */
int mds_set_timing(mds_handle *h, int enable);
/* Synchronize the stream and return the accumulated totals. */
int mds_get_timings(mds_handle *h, mds_timings *out_host);

const char *mds_status_string(int status);
const char *mds_last_error(const mds_handle *h);

/* ---- batched Newton solves (many scenario problems of uneven size) -------- */

/* One problem of a batch: the data of one regularised Newton system (Sec. 2.2,
 * eq. (compressed)) and its right-hand side.  All pointers are device
 * pointers, caller-owned, valid for the batch's lifetime; outputs are
 * written by every mds_batch_run.  Layouts as in mds_problem.  Condensed size
 * N = n_d + m must satisfy 1 <= N <= 2048. */
typedef struct {
  int32_t n_d, n_s, m, pad;
  int64_t nnz_s;
  const double *H, *J_d;                  /* n_d x n_d, m x n_d column-major   */
  const int32_t *Js_rowptr, *Js_col;      /* CSR of J_s (m x n_s), sorted rows */
  const double *Js_val;
  const double *sigma_d, *dsbase;         /* Sigma_d (n_d), w + Sigma_s (n_s)  */
  const double *r_d, *r_s, *r_y;          /* right-hand side                   */
  double *dx_d, *dx_s, *dy;               /* solution                          */
} mds_batch_problem;

/* Per-problem outcome (host).  Times are wall-clock ticks (100 MHz) since
 * the first workgroup of the launch started. */
typedef struct {
  int32_t npos, nzero, nneg, trials;      /* final inertia of M, factorizations */
  double delta_w, delta_c;                /* shifts of the accepted factor      */
  int64_t t_start, t_done;
  int32_t status;                         /* 0 or MDS_INERTIA_FAIL              */
  int32_t slot;                           /* workgroup that solved it           */
  int32_t refine_steps, pad;              /* FP64 refinement steps (MDS_FP32)   */
  double residual;                        /* max|r - Kx| / max|r| before the last
                                             refinement step (MDS_FP32)          */
} mds_batch_result;

typedef struct {
  int32_t nb;         /* panel width, 2..16 (0: 16)                              */
  int32_t grid;       /* persistent workgroups = scratch slots (0: min(count, 256)) */
  int32_t use_graph;  /* 0: plain launches; otherwise replay a captured hipGraph */
  int32_t precision;  /* MDS_FP64 (0, default) or MDS_FP32: equilibrated S M S
                         stored in FP32, trailing tiles on FP32 MFMA (panel
                         decisions, L and D in FP64), then FP64 iterative
                         refinement on the full Newton system,
                         x += K^-1 (r - K x) through the FP32 factor          */
  int32_t refine_steps; /* MDS_FP32: refinement steps at most (0: 10); a step
                         whose correction is below 1e-15 max|x| ends it       */
  int32_t ipm_max_iter; /* 0: Newton systems only.  > 0 (at most 1000): the
                         workspace also holds, per slot, the vectors of a whole
                         IPM and, per problem, a trace of ipm_max_iter + 1
                         iterations (mds_batch_ipm); the Newton-system arrays
                         of mds_batch_problem may then be NULL (mds_batch_run
                         needs them)                                          */
  int32_t reserved[2];
} mds_batch_opts;

typedef struct mds_batch mds_batch;

/* Bytes of device workspace for a batch (0: invalid sizes). */
size_t mds_batch_workspace_bytes(const mds_batch_problem *probs_host, int32_t count,
                                 const mds_batch_opts *opts);
/* Build the batch: column-compressed copies of every J_s, the problem table
 * (largest N first) and one scratch slot per persistent workgroup.
 * Synchronizes the stream. */
int mds_batch_create(mds_batch **out, const mds_batch_problem *probs_host, int32_t count,
                     const mds_batch_opts *opts, void *stream, void *workspace,
                     size_t workspace_bytes);
/* Solve every problem: for each, condense, factor with the inertia
 * correction loop (delta_c = 1e-8 mu^(1/4) on a singular M), solve and
 * back-substitute (MDS_FP32: then refine in FP64), in one persistent kernel
 * (hipGraph replay on the batch's own stream, after the caller's stream has
 * drained).  results_host (may be NULL) receives count entries.
 * Synchronizes. */
int mds_batch_run(mds_batch *b, double mu, mds_batch_result *results_host);
/* Whole-IPM data of one batched problem (each problem of the scenario batch
 * an IPM of Sec. 2.1 on its own, equality constraints J x = b): objective
 * c (n_d), w (n_s, >= 0), g (n_s); b (m); bounds xl, xu (n = n_d + n_s,
 * +-INFINITY allowed, xl < xu); outputs: the final iterate x (n), y (m),
 * zl, zu (n).  Device arrays, caller-owned. */
typedef struct {
  const double *c, *w, *g, *b, *xl, *xu;
  double *x, *y, *zl, *zu;
} mds_batch_ipm_problem;

typedef struct {
  int32_t status;          /* MDS_IPM_CONVERGED, MDS_IPM_LS_FAIL,
                              MDS_IPM_MAXITER, MDS_INERTIA_FAIL or
                              MDS_IPM_NONFINITE                               */
  int32_t iters;           /* iterations (Newton steps) taken                */
  double mu, E0;           /* barrier parameter and optimality error at exit */
  int64_t t_start, t_done; /* 100 MHz ticks since the launch's first workgroup */
  int32_t slot;            /* workgroup that solved it                       */
  int32_t factorizations;  /* over all iterations (correction trials)       */
} mds_batch_ipm_result;

typedef struct {           /* one iteration of one problem */
  double mu, alpha_pr, delta_w;
  int32_t inertia[3];      /* of the accepted M                             */
  int32_t trials, backtracks, pad;
} mds_batch_ipm_iter;

/* Whole IPMs of every problem of the batch (Sec. 1's scenario motivation; the
 * filter line-search IPM of Sec. 2.1 with mds_ipm_step's start point,
 * constants and tests, FP64): one persistent kernel, each workgroup running
 * complete IPMs of the problems it takes from the queue (largest first),
 * every reduction inside the workgroup; Newton systems through the batch's
 * condense / blocked Bunch-Kaufman / inertia correction (delta_w^last kept
 * per problem) / solve, then FP64 iterative refinement on the full system
 * (<= opts.refine_steps, stop at backward error 1e-14 or no decrease).
 * Needs a batch created with ipm_max_iter >= opts.max_iter and precision
 * MDS_FP64 (else MDS_ESTATE).  ipm_host: count entries.  results_host and
 * trace_host (count x (ipm_max_iter + 1) rows, problem-major; rows past a
 * problem's last iteration are unspecified) may be NULL.  Synchronizes. */
int mds_batch_ipm(mds_batch *b, const mds_batch_ipm_problem *ipm_host, const mds_ipm_opts *opts,
                  mds_batch_ipm_result *results_host, mds_batch_ipm_iter *trace_host);
/* Time each candidate (panel width x grid) once and keep the fastest;
 * chosen_host (may be NULL) receives it.  Runs the batch several times. */
int mds_batch_autotune(mds_batch *b, double mu, mds_batch_opts *chosen_host);
int mds_batch_get_config(const mds_batch *b, mds_batch_opts *out_host);
/* Text of the last HIP failure of a batch call. */
const char *mds_batch_last_error(const mds_batch *b);
void mds_batch_destroy(mds_batch *b);

/* ---- learned warm start: the multilayer perceptron ------------------------ */

/* MLP dims[0] -> dims[1] -> dims[2] -> dims[3] with GELU (erf form) after the
 * two hidden layers and a linear skip path from the input to the output
 * (Y = H2 W2 + b2 + X Ws), trained by mean-squared error with Adam (beta 0.9 /
 * 0.999, eps 1e-8) in FP32 on FP32 MFMA; inference in FP32 or on BF16 MFMA
 * with FP32 accumulation.  Parameters are one FP32 vector: W0 (dims[0] x
 * dims[1], row-major), b0, W1, b1, W2, b2, Ws (dims[0] x dims[3]).
 * Activations are row-major (batch x features) device arrays. */
typedef struct mds_mlp mds_mlp;
size_t mds_mlp_workspace_bytes(const int32_t dims[4], int32_t max_batch);
int mds_mlp_create(mds_mlp **out, const int32_t dims[4], int32_t max_batch, void *stream,
                   void *workspace, size_t workspace_bytes);
void mds_mlp_destroy(mds_mlp *M);
int32_t mds_mlp_param_count(const mds_mlp *M);
/* Host copies of the parameters; set resets the Adam state.  Synchronize. */
int mds_mlp_set_params(mds_mlp *M, const float *params_host);
int mds_mlp_get_params(const mds_mlp *M, float *params_host);
/* Gradient of the last training step (host).  Synchronizes. */
int mds_mlp_get_grad(const mds_mlp *M, float *grad_host);
/* Y = MLP(X), precision MDS_FP32 or MDS_BF16.  Async. */
int mds_mlp_forward(mds_mlp *M, const float *X, int32_t batch, int32_t precision, float *Y);
/* One Adam step on mean((MLP(X) - T)^2); *loss_host (may be NULL) gets the
 * loss before the step.  Synchronizes. */
int mds_mlp_train_step(mds_mlp *M, const float *X, const float *T, int32_t batch, float lr,
                       double *loss_host);

#ifdef __cplusplus
}
#endif
#endif
