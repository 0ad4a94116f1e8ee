// Internal declarations of the mdsipm library (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <utility>
#include <vector>

#include "mdsipm.h"

namespace mds {

constexpr int kPanelThreads = 1024;  // one workgroup factors a panel
constexpr int kMaxNb = 64;           // largest supported panel width
constexpr int kRedBlocks = 1024;     // partial-reduction slots
constexpr int kDotBlocks = 64;       // blocks per column of a Krylov dot product
constexpr int kGmresRestart = 20;    // GMRES restart length of the mixed-precision refinement
constexpr int kCoopMaxP = 32;        // cooperative panel: most workgroups
constexpr int kCoopSlotWords = 512;  // cooperative panel: 64-bit exchange words per workgroup and parity
constexpr int kSBlkMax = 16;         // largest coupling block of the sparse Hessian

// Coupling blocks of the sparse Hessian (sblock.hip) and the transformed
// Jacobian Jh = J_s L^{-T} they induce (device pointers into the workspace;
// Wb is the caller's).
struct SBlk {
  int nblk = 0;
  int64_t nnz = 0;                     // entries of Jh
  const int32_t *bp = nullptr;         // nblk + 1 block starts
  const int32_t *boff = nullptr;       // nblk offsets of the blocks in Wb / lblk
  const int32_t *kblk = nullptr;       // n_s: block of each sparse variable
  const double *Wb = nullptr;          // the blocks (caller's), column-major
  double *lblk = nullptr;              // their unit lower factors, same layout
  int32_t *hrp = nullptr, *hci = nullptr, *hsrc = nullptr;  // Jh CSR; source entry of J_s or -1
  double *hval = nullptr;
  int32_t *hcptr = nullptr, *hcrow = nullptr, *hcmap = nullptr;  // Jh CSC; CSC -> CSR entry
  double *hcval = nullptr;
  double *tmp = nullptr, *tmp2 = nullptr;  // n_s scratch
};

// Device-side factorization progress, written by the panel kernel.
struct FacState {
  int32_t k;       // first unfactored index (start of the next panel)
  int32_t npanel;  // panels completed
  int32_t info;    // 1-based index of the first exact zero pivot, or 0
  int32_t npos, nzero, nneg, n2x2;
  uint32_t xtag;  // cooperative panel: launch counter behind its exchange tags (never reset)
  int32_t xerr;   // cooperative panel: an exchange wait expired
  int32_t xforce; // host-set test flag: cooperative launches report an expired wait at once
  int32_t csteps; // cooperative panel: pivot steps of this factorization
  int32_t cx3;    // ... of which took the second exchange (the candidate column)
};

// Look-ahead of the cooperative factorization: while the trailing update of
// panel b runs on part of the device, panel b + 1 factors its columns, which
// a near update (the 64-column strip at the trailing matrix's start) has
// already brought up to date.  Entries it reads outside that strip (the
// candidate column of a failed first Bunch-Kaufman test) it computes itself
// from panel b's input and multipliers: entry (i, c), i >= c, of its input is
// X[src(i), src(c)] - sum_t W[c, t] L[i, t] (lower triangle of X).
constexpr int kNearCols = 64;  // columns of the near update past its start
struct PanelPrev {
  const double *X;      // panel b's input, physical indices (FP64 storage), or
  const float *Xf;      // ... in FP32 storage (null both: no look-ahead)
  const int32_t *src;   // panel b's map: its output's row -> physical row of X
  const double *W;      // panel b's W = L D: W[c + t N]
  const double *L;      // panel b's multipliers: staged, L[i + t N], or in
  int labs;             // place (labs = 1), L[i + (k0_b + t) N]
  int amask;            // the strip starts at (k0 & amask): ~15 (FP64 tiles), -1 (FP32)
};

// One slot of a factorization's launch sequence (one panel launch and its
// trailing update): tail_nb 0 for the handle's panel kernel, else the tile
// width of the register tail; rows bounds the rows left at the slot's start
// and rows_after those left for its trailing update (the device's progress
// is not known to the host; every panel factors at least its tile width - 1
// columns unless the matrix ends).
struct SlotPlan {
  int tail_nb;
  long rows, rows_after;
};

// Pointers into the caller's workspace.
struct Work {
  double *M;          // N x N, full symmetric, column-major; L after factoring
  double *M2;         // second N x N buffer (register panel: ping-pong + L of even panels)
  float *X32[2];      // mixed precision: FP32 ping-pong buffers of the trailing matrix
  double *eq;         // mixed precision: equilibration S (N)
  int32_t *src;       // N: logical -> physical index map of the last panel
  double *W;          // N x (nb + 2) panel workspace (updated columns)
  // look-ahead: the second map and W (panels alternate), and two staging
  // buffers of a panel's multipliers (N x (nb + 2) each)
  int32_t *src2;
  double *W2;
  double *lst[2];
  double *dd, *ds;    // D diagonal / sub-diagonal (N)
  int32_t *ipiv;      // LAPACK-style pivots (N)
  int32_t *blk;       // 1: 1x1 pivot, 2: first of a 2x2, 3: second of a 2x2
  int32_t *panel_k0;  // panel start indices (max_panels + 1)
  FacState *fst;
  double *inv_d;      // D_s^{-1} (n_s)
  int32_t *csc_ptr;   // n_s + 1
  int32_t *csc_row;   // nnz
  double *csc_val;    // nnz
  int32_t *csc_fill;  // n_s scratch
  int32_t *flags;     // validation flags (16)
  double *red;        // reduction partials (kRedBlocks * 8)
  double *scal;       // device scalars (64)
  double *z;          // N: condensed rhs / solution
  double *z2;         // N: permuted solve vector
  int32_t *hmap;      // max_panels x N: row map of each panel's frame to the final order
  int32_t *perm;      // N: final row permutation of the factorization
  int32_t *colpanel;  // N: panel of each column
  int32_t *trsv;      // solve epoch, error word, pad, per-block flags (2 x blocks)
  uint64_t *xch;      // cooperative panel exchange words
  // Newton / IPM vectors
  // (vectors of length nx = n + m_I hold the variables, then the slacks of
  // the inequality rows)
  double *sig, *rx, *ry, *dsb;       // nx, nx, m, n_s
  double *dx, *dy, *dzl, *dzu, *xt;  // nx, m, nx, nx, nx
  double *xl_e, *xu_e;               // nx: bounds of the variables, then of the slacks
  double *dcv;                       // m: the IPM's (4,4) diagonal 1 / (Sigma_h + dw) (0 on equality rows)
  double *ry2;                       // m: rhs of the y rows with the slack step eliminated
  double *res, *cor, *prev, *kx;     // n + m each (refinement)
  double *tn, *tm, *tn2;             // scratch nx, m, nx
  double *kn_h, *kn_jd, *kn_y, *kn_js;  // ||K||_inf row-sum scratch: n_d, n_d, m, n_s
  // GMRES refinement (mixed precision): basis V (nK x (restart+1)), Z = P^{-1} V
  // (nK x restart), rhs, iterate, residual / work vector, dot partials, coefficients
  double *gV, *gZ, *grhs, *gx, *gw, *gpart, *gcoef;
};

}  // namespace mds

struct mds_handle {
  int device = 0;
  hipStream_t stream = nullptr;
  mds_dims dims{};
  int N = 0, n = 0, nb = 16, max_panels = 0;
  int mI = 0, mE = 0, nx = 0;  // inequality rows, equality rows, n + mI
  bool panel_reg = false;  // register-resident panel kernel (ping-pong layout)
  bool panel_coop = false; // ... spread over several workgroups
  bool panel_tail = false; // ... with the register panel once its rows fit one workgroup
  bool panel_lds = false;  // whole M in one workgroup's LDS, unblocked
  const double *dcv_user = nullptr;  // caller's per-row diagonal subtracted from M22 (m)
  // general-NLP mode (mds_set_nlp): the model, the quadratic problem it
  // replaced, workspace copies of the model objects and scratch of the
  // second-order correction and the restoration
  bool nlp_room = false, nlp_on = false, model_err = false;
  int nlp_force_resto = 0;  // debug: the next step enters the restoration
  mds_nlp_model nlp{};
  mds_problem Pq{};
  double *nlp_H = nullptr, *nlp_Jd = nullptr, *nlp_v = nullptr, *nlp_w = nullptr;
  double *nlp_zero = nullptr, *nlp_cx0 = nullptr, *nlp_csoc = nullptr, *nlp_yr = nullptr;
  double *nlp_xs = nullptr, *nlp_dxs = nullptr, *nlp_dys = nullptr, *nlp_xr = nullptr;
  double *nlp_dr = nullptr;
  int32_t *nlp_cmap = nullptr;  // CSC entry -> CSR entry of J_s
  mds_nlp_stats nlp_stats{};
  int sblk_max = 0;        // largest coupling block the workspace was sized for
  mds::SBlk sb{};          // coupling blocks of the sparse Hessian (sb.nblk = 0: none)
  const double *dcv_cur = nullptr;   // diagonal of the current M: dcv_user or w.dcv
  const double *sig_h = nullptr;     // IPM: slack barrier diagonal (mI) behind w.dcv
  // factorization mode and the kind of the current factor
  bool force64 = false;     // factor in FP64 in a mixed-precision handle
  bool coop_off = false;    // cooperative panel not co-resident: memory panel always
  bool fac_lowprec = false; // current factor is of the equilibrated FP32 matrix
  bool fac_pingpong = false;// current factor's L is spread over M and M2
  int64_t n_coop_abort = 0, n_fp64_refactor = 0;
  // look-ahead of the cooperative factorization: compute units reserved for
  // the panel and the near update (0: off), the far update's persistent
  // grid, the two CU-masked streams and the events between them
  int la_cus = 0, la_grid = 0;
  hipStream_t la_a = nullptr, la_b = nullptr;
  hipEvent_t la_ev[4] = {};
  // captured launch sequence of one factorization (replayed without timing)
  hipGraphExec_t fac_exec = nullptr;
  hipStream_t cap_stream = nullptr;
  bool fac_graph_off = false;
  int panel_threads = 512; // its workgroup size
  int precision = MDS_FP64;
  int adv = 16;            // least number of columns a panel factors
  std::vector<mds::SlotPlan> plan;  // slots of a factorization (register and memory panels)
  mds::Work w{};
  size_t ws_bytes = 0;
  mds_problem P{};
  bool have_problem = false, have_M = false, have_factor = false;
  bool std_ready = false;  // factor converted to standard form (in M)
  const double *sigma_d = nullptr, *dsbase = nullptr;  // last condense inputs
  double dw = 0.0, dc = 0.0;                           // shifts of current M / factor
  double alpha_bk = 0.0;                               // (1 + sqrt(17)) / 8
  // IPM state
  mds_ipm_opts ipm{};
  double theta_max = 0.0, theta_min = 0.0, dw_last = 0.0;
  std::vector<std::pair<double, double>> filter;
  bool ipm_ready = false;
  // per-launch timing (hipEvent pairs, resolved in mds_get_timings)
  bool timing = false;
  int64_t nsolves = 0;  // LDL' solves performed (statistics)
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used = 0;  // events of the pool taken since the last resolution
  std::vector<std::pair<int, std::pair<int, int>>> ev_marks;  // class, (start, stop)
  double t_ms[MDS_T_CLASSES] = {};
  int64_t t_n[MDS_T_CLASSES] = {};
  char err[512] = {0};
};

// ---- kernel launch wrappers (defined in the .hip files) --------------------
namespace mds {

// nlp.hip: helpers of the IPM's general-NLP mode: dst[q] = src[map[q]];
// out = a u + v; the restoration's x_R, D_R = min(1, 1/|x_R|), proximal
// Hessian, centred Newton system (Sigma, r_x, z) and centred multipliers
void nlp_gather(hipStream_t s, int64_t n, const int32_t *map, const double *src, double *dst);
void nlp_axpby(hipStream_t s, int n, double a, const double *u, const double *v, double *out);
void nlp_resto_init(hipStream_t s, int n, const double *x, double *xr, double *dr);
void nlp_resto_hess(hipStream_t s, int nd, int ns, double zeta, const double *dr, double *H,
                    double *w);
void nlp_resto_rhs(hipStream_t s, int n, double zeta, double mu, const double *x, const double *xr,
                   const double *dr, const double *jty, const double *xl, const double *xu,
                   double *sig, double *rx, double *zl, double *zu);
void nlp_check_nonneg(hipStream_t s, int n, const double *w, int32_t *flag);
void nlp_center_z(hipStream_t s, int n, double mu, const double *x, const double *xl,
                  const double *xu, double *zl, double *zu);

// sblock.hip: the blocks' L Delta L' (inv_d = 1/Delta), the values of Jh
// and its CSC copy, block solves (mode 0: u = L^{-1} u; mode 1: u = L^{-T}
// (inv_d .* L^{-1} u)), out (+)= blockdiag(Wb) u, and the (2,2) row pieces of
// ||K||_inf (off-diagonal |Wb| row sums added to jscol; dsb_eff = Wb_kk + dsb)
void sblk_factor(hipStream_t s, const SBlk &B, const double *dsb, double dw, double *inv_d);
void sblk_transform(hipStream_t s, const SBlk &B, int m, const double *jsv);
void sblk_solve(hipStream_t s, const SBlk &B, const double *inv_d, int mode, double *u);
void sblk_matvec(hipStream_t s, const SBlk &B, int ns, const double *u, bool accumulate,
                 double *out);
void sblk_absrow(hipStream_t s, const SBlk &B, int ns, const double *dsb, double *jscol,
                 double *dsb_eff);

// condense.hip
void launch_inv_d(hipStream_t s, int ns, const double *dsbase, double dw, double *inv_d);
void launch_condense_dense(hipStream_t s, int nd, int m, const double *H, const double *Jd,
                           const double *sigma_d, double dw, double *M);
void launch_condense_schur(hipStream_t s, int nd, int m, int N, const int32_t *rp,
                           const int32_t *ci, const double *v, const int32_t *cptr,
                           const int32_t *crow, const double *cval, const double *inv_d,
                           double dc, const double *dcv, double *M);
void launch_rhs_condense(hipStream_t s, int m, const int32_t *rp, const int32_t *ci,
                         const double *v, const double *inv_d, const double *r_s,
                         const double *r_y, double *out);
void launch_backsub(hipStream_t s, int ns, const int32_t *cptr, const int32_t *crow,
                    const double *cval, const double *inv_d, const double *r_s,
                    const double *dy, double *dx_s);
void launch_csc_build(hipStream_t s, int m, int ns, int64_t nnz, const int32_t *rp,
                      const int32_t *ci, const double *v, int32_t *cptr, int32_t *crow,
                      double *cval, int32_t *fill);
void launch_validate(hipStream_t s, const mds_dims &d, const mds_problem &p, int32_t *flags);

// bk.hip
void launch_fac_reset(hipStream_t s, FacState *st, int32_t *panel_k0);
void launch_bk_panel(hipStream_t s, int N, int nb, double alpha, double *M, double *W,
                     double *dd, double *ds, int32_t *ipiv, int32_t *blk, FacState *st,
                     int32_t *panel_k0);
// rem: an upper bound of the rows of the trailing matrix after the panel of
// slot `slot` (sizes the grid; 0 or less: nothing to update)
void launch_bk_trailing(hipStream_t s, int N, int nb, long rem, int slot, const double *W,
                        const double *X, double *Y, const double *Lsrc, const int32_t *src,
                        const FacState *st, const int32_t *panel_k0);
// look-ahead parts of the trailing update of slot `slot` (nb + 1 <= 36):
// part 1 the near strip (the first 64-column tile column), part 2 the rest;
// both persistent over at most `grid` workgroups; Lsrc holds the
// panel's multipliers staged (row i, column t at Lsrc[i + t N])
void launch_bk_trailing_part(hipStream_t s, int N, int nb, long rem, int slot, int part, int grid,
                             const double *W, const double *X, double *Y, const double *Lsrc,
                             const int32_t *src, const FacState *st, const int32_t *panel_k0);
// staged multipliers of slot `slot` into their place in Lout (columns
// k0 .. kend - 1, rows below the diagonal)
void launch_lstage_copy(hipStream_t s, int N, long rows, int slot, const double *Lst, double *Lout,
                        const FacState *st, const int32_t *panel_k0);

// bk_reg.hip: register-resident panel for N <= 4096 (X in FP64 or FP32),
// workgroup of `threads` = 512 or 1024
int bk_reg_rows(int N, int threads);
int bk_reg_nb(int N, int threads);
// register panel over the last rows of a cooperative factorization (rows >=
// N - k0, rows <= bk_reg_tail_rows(), nb <= 32); it factors at least
// bk_reg_tail_nb(rows) - 1 columns per launch (unless the matrix ends)
int bk_reg_tail_rows();
int bk_reg_tail_nb(int rows);
void launch_bk_panel_reg_tail(hipStream_t s, int rows, int N, int nb, double alpha,
                              const double *X, double *Lout, int32_t *src_out, double *W,
                              double *dd, double *ds, int32_t *ipiv, int32_t *blk, FacState *st,
                              int32_t *panel_k0);
void launch_bk_panel_reg_tail(hipStream_t s, int rows, int N, int nb, double alpha,
                              const float *X, double *Lout, int32_t *src_out, double *W,
                              double *dd, double *ds, int32_t *ipiv, int32_t *blk, FacState *st,
                              int32_t *panel_k0);
void launch_bk_panel_reg(hipStream_t s, int threads, int N, int nb, double alpha, const double *X,
                         double *Lout, int32_t *src_out, double *W, double *dd, double *ds,
                         int32_t *ipiv, int32_t *blk, FacState *st, int32_t *panel_k0);
void launch_bk_panel_reg(hipStream_t s, int threads, int N, int nb, double alpha, const float *X,
                         double *Lout, int32_t *src_out, double *W, double *dd, double *ds,
                         int32_t *ipiv, int32_t *blk, FacState *st, int32_t *panel_k0);

// bk_coop.hip: cooperative register panel over several workgroups (any N up
// to the solver limit; X in FP64 or FP32); xch: 2 * kCoopMaxP * kCoopSlotWords
// exchange words, zeroed once
int bk_coop_rows_per_wg();
// whether the device can hold every workgroup of the panel for order N at once
bool bk_coop_resident(int N);
int bk_coop_nb();
int bk_coop_wgs(int N);
// rows: at least the rows left at the panel's start (sizes the grid)
// Exchange round-trip probe of the cooperative panel (P <= kCoopMaxP workgroups,
// words <= kCoopSlotWords per workgroup, P * words <= 2048); -1: bad sizes.
int bk_xch_probe(hipStream_t s, int P, int rounds, int words, uint64_t *xch, int32_t *err,
                 uint64_t *out);
void launch_bk_panel_coop(hipStream_t s, int rows, int N, int nb, double alpha, const double *X,
                          double *Lout, int32_t *src_out, double *W, double *dd, double *ds,
                          int32_t *ipiv, int32_t *blk, FacState *st, int32_t *panel_k0,
                          uint64_t *xch);
// look-ahead form (FP64): X is valid in the near strip only, pv names the
// previous panel's pending update, and the multipliers go to the staging
// buffer Lst (row i, column t at Lst[i + t N])
void launch_bk_panel_coop_la(hipStream_t s, int rows, int N, int nb, double alpha, const double *X,
                             const PanelPrev &pv, double *Lst, int32_t *src_out, double *W,
                             double *dd, double *ds, int32_t *ipiv, int32_t *blk, FacState *st,
                             int32_t *panel_k0, uint64_t *xch);
// ... FP32 storage: the multipliers go to their place in Lout (FP64)
void launch_bk_panel_coop_la(hipStream_t s, int rows, int N, int nb, double alpha, const float *X,
                             const PanelPrev &pv, double *Lout, int32_t *src_out, double *W,
                             double *dd, double *ds, int32_t *ipiv, int32_t *blk, FacState *st,
                             int32_t *panel_k0, uint64_t *xch);
// the CU count the look-ahead keeps free of the far trailing update for a
// cooperative panel of order N (its workgroups, rounded up to a multiple of
// the XCD count); 0 when the panel would not fit beside it
int bk_coop_la_reserve(int N, int cus);
void launch_bk_panel_coop(hipStream_t s, int rows, int N, int nb, double alpha, const float *X,
                          double *Lout, int32_t *src_out, double *W, double *dd, double *ds,
                          int32_t *ipiv, int32_t *blk, FacState *st, int32_t *panel_k0,
                          uint64_t *xch);

// bk_lds.hip: unblocked factorization of an M held whole in one
// workgroup's LDS (N <= bk_lds_max_n(), threads 256 or 512); writes the
// standard-form L into M's strictly lower part, dd, ds, ipiv, blk, perm and
// the final FacState
size_t bk_lds_bytes(int N);
int bk_lds_max_n();
hipError_t bk_lds_prepare();
void launch_bk_lds(hipStream_t s, int threads, int N, double alpha, double *M, double *dd,
                   double *ds, int32_t *ipiv, int32_t *blk, int32_t *perm, FacState *st);

// bk_lp.hip: FP32-storage trailing update (mode MDS_FP32 or MDS_BF16 products)
void launch_trailing_lp(hipStream_t s, int mode, int N, int nb, long rem, int slot,
                        const double *W, const float *X, float *Y, const double *Lsrc,
                        const int32_t *src, const FacState *st, const int32_t *panel_k0);
// look-ahead parts (as launch_bk_trailing_part; Lsrc in place, not staged)
void launch_trailing_lp_part(hipStream_t s, int mode, int N, int nb, long rem, int slot, int part,
                             int grid, const double *W, const float *X, float *Y,
                             const double *Lsrc, const int32_t *src, const FacState *st,
                             const int32_t *panel_k0);
// scale = 1/sqrt(row max |M|), b = FP32(S M S); v = scale .* v
void launch_equilibrate_f32(hipStream_t s, int N, const double *M, double *scale, float *b);
void launch_vscale(hipStream_t s, int n, const double *scale, double *v);

// gmres.hip: Krylov products (partial[c * kDotBlocks + b]) and updates
void launch_dots(hipStream_t s, int64_t n, int ncol, const double *V, int64_t ldv,
                 const double *w, double *partial);
void launch_sub_cols(hipStream_t s, int64_t n, int ncol, const double *V, int64_t ldv,
                     const double *coef, double *w);
void launch_add_cols(hipStream_t s, int64_t n, int ncol, const double *Z, int64_t ldz,
                     const double *coef, double *x);
void launch_scale(hipStream_t s, int64_t n, double alpha, const double *w, double *out);

// solve_std.hip: standard form of the factor (L of panel b lives in M1 when
// pingpong and b is even, else in M0; the result may be M0 itself) and the
// multi-workgroup solve
int std_max_n();
int std_solve_blocks(int N);
size_t std_trsv_bytes(int N);  // the solve's control words (trsv below)
hipError_t std_prepare();
void launch_std_form(hipStream_t s, int N, const double *M0, const double *M1, int pingpong,
                     const int32_t *ipiv, const int32_t *blk, const int32_t *panel_k0,
                     const FacState *st, int32_t *hmap, int32_t *perm, int32_t *colpanel,
                     double *Lstd);
// out = M^{-1} v through P, L, D; z is scratch (N); trsv (std_trsv_bytes(N),
// 8-byte aligned, zeroed once when the handle is made): epoch, error word,
// pad, then the tagged solution words of the triangular solves
void launch_std_solve(hipStream_t s, int N, const double *Lstd, const double *dd,
                      const double *ds, const int32_t *blk, const int32_t *perm, const double *v,
                      double *z, double *out, int32_t *trsv);

// vec.hip
void launch_gemv_n(hipStream_t s, int rows, int cols, const double *A, int lda,
                   const double *x, double beta, double *y);
void launch_gemv_t(hipStream_t s, int rows, int cols, const double *A, int lda,
                   const double *x, double beta, double *y);
void launch_spmv_csr(hipStream_t s, int rows, const int32_t *rp, const int32_t *ci,
                     const double *v, const double *x, double beta, double *y);
void launch_spmv_csc(hipStream_t s, int cols, const int32_t *cptr, const int32_t *crow,
                     const double *cval, const double *x, double beta, double *y);

}  // namespace mds
