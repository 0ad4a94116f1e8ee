// C-ABI of the mdsipm library: handle and workspace management, validation,
// the inertia-correction loop, refinement and the host control of the filter
// line-search IPM.  Every numerical step on vectors and matrices runs in the
// HIP kernels; the host only sequences launches and takes scalar decisions.
#include <algorithm>
#include <cfloat>
#include <cmath>
#include <cstdarg>
#include <cstddef>
#include <cstring>
#include <new>
#include <vector>

#include "internal.hpp"
#include "ipm.hpp"

using namespace mds;

namespace {

int set_err(mds_handle *h, int code, const char *fmt, ...) {
  if (h) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(h->err, sizeof(h->err), fmt, ap);
    va_end(ap);
  }
  return code;
}

#define HIPCHK(expr)                                                                       \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess) return set_err(h, MDS_EHIP, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

#define TRY(expr)             \
  do {                        \
    int r_ = (expr);          \
    if (r_ < 0) return r_;    \
  } while (0)

// ---- per-launch timing ---------------------------------------------------
// Next free pair of the event pool (timers may nest: a pair is taken when
// a timer starts, its mark added when it stops).
int ev_take(mds_handle *h) {
  const size_t used = h->ev_used;
  while (h->ev_pool.size() < used + 2) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return -1;
    h->ev_pool.push_back(e);
  }
  h->ev_used += 2;
  return (int)used;
}

struct TimedLaunch {
  mds_handle *h;
  int cls, idx;
  hipStream_t s;
  TimedLaunch(mds_handle *h_, int c, hipStream_t s_ = nullptr)
      : h(h_), cls(c), idx(-1), s(s_ ? s_ : h_->stream) {
    if (!h->timing) return;
    idx = ev_take(h);
    if (idx >= 0) (void)hipEventRecord(h->ev_pool[idx], s);
  }
  ~TimedLaunch() {
    if (idx < 0) return;
    (void)hipEventRecord(h->ev_pool[idx + 1], s);
    h->ev_marks.push_back({cls, {idx, idx + 1}});
  }
};

int resolve_timings(mds_handle *h) {
  if (h->ev_marks.empty()) return MDS_OK;
  if (hipStreamSynchronize(h->stream) != hipSuccess) return MDS_EHIP;
  for (auto &mk : h->ev_marks) {
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, h->ev_pool[mk.second.first], h->ev_pool[mk.second.second]) ==
        hipSuccess) {
      h->t_ms[mk.first] += ms;
      h->t_n[mk.first] += 1;
    }
  }
  h->ev_marks.clear();
  h->ev_used = 0;
  return MDS_OK;
}

// Workspace slots, in carving order.
enum Slot {
  S_M, S_M2, S_SRC, S_W, S_DD, S_DS, S_IPIV, S_BLK, S_PK0, S_FST, S_INVD, S_CPTR, S_CROW, S_CVAL, S_CFILL,
  S_FLAGS, S_RED, S_SCAL, S_Z, S_Z2, S_HMAP, S_PERM, S_COLP, S_TRSV, S_SIG, S_RX, S_RY, S_DSB, S_DX, S_DY, S_DZL, S_DZU, S_XT, S_RES,
  S_COR, S_PREV, S_KX, S_TN, S_TM, S_TN2, S_KNH, S_KNJD, S_KNY, S_KNJS, S_EQ, S_GV,
  S_GZ, S_GRHS, S_GX, S_GW, S_GPART, S_GCOEF, S_XCH, S_XLE, S_XUE, S_DCV, S_RY2,
  S_BBP, S_BOFF, S_BKB, S_BL, S_HRP, S_HCI, S_HSRC, S_HVAL, S_HCPTR, S_HCROW, S_HCMAP, S_HCVAL,
  S_BT1, S_BT2, S_NH, S_NJD, S_NV, S_NW, S_NZERO, S_NCX0, S_NCSOC, S_NYR, S_NXS, S_NDXS, S_NDYS,
  S_NXR, S_NDR, S_NCMAP, S_SRC2, S_W2, S_LST, S_COUNT
};

struct Layout {
  size_t off[S_COUNT];
  size_t total;
};

int default_nb(int N) { return (N >= 64) ? 16 : 8; }

// entries of the transformed Jacobian J_s L^{-T} at most: every entry of J_s
// brings at most its block's other columns
size_t sblk_nnz_max(const mds_dims &d, int sblk_max) {
  if (sblk_max <= 0) return 0;
  const size_t a = (size_t)d.nnz_s * (size_t)sblk_max, b = (size_t)d.m * (size_t)d.n_s;
  return std::min(a, b);
}

Layout make_layout(const mds_dims &d, int nb, bool pingpong, int precision, int sblk_max,
                   bool nlp) {
  const size_t nd = d.n_d, ns = d.n_s, m = d.m, N = nd + m, n = nd + ns;
  const size_t nx = n + (size_t)d.m_I;
  const size_t nnz = (size_t)d.nnz_s;
  // panels: at least nb - 1 columns each, the register tail's 16-column
  // tile over the last 2048 rows adds at most 40 (see make_plan)
  const size_t maxp = N / (size_t)std::max(nb - 1, 1) + 42;
  size_t bytes[S_COUNT] = {};
  bytes[S_M] = 8 * N * N;
  const bool mixed = precision != MDS_FP64;
  // ping-pong partner of M; in a mixed-precision handle the same bytes hold
  // the two FP32 buffers of the trailing matrix (and serve as M2 again when
  // a Newton system is refactored in FP64)
  bytes[S_M2] = (pingpong || mixed) ? 8 * N * N : 0;
  bytes[S_EQ] = mixed ? 8 * N : 0;
  bytes[S_XLE] = bytes[S_XUE] = 8 * nx;
  bytes[S_DCV] = bytes[S_RY2] = 8 * m;
  const size_t nK = n + m, R = (size_t)kGmresRestart;
  bytes[S_GV] = mixed ? 8 * nK * (R + 1) : 0;
  bytes[S_GZ] = mixed ? 8 * nK * R : 0;
  bytes[S_GRHS] = bytes[S_GX] = bytes[S_GW] = mixed ? 8 * nK : 0;
  bytes[S_GPART] = 8 * (size_t)kDotBlocks * (R + 2);
  bytes[S_GCOEF] = 8 * (R + 2);
  bytes[S_XCH] = 8 * 2 * (size_t)kCoopMaxP * kCoopSlotWords;
  bytes[S_SRC] = 4 * N;
  bytes[S_W] = 8 * N * (size_t)(nb + 2);
  // look-ahead (ping-pong layout): second map and W, two staging buffers
  bytes[S_SRC2] = pingpong ? 4 * N : 0;
  bytes[S_W2] = pingpong ? 8 * N * (size_t)(nb + 2) : 0;
  bytes[S_LST] = pingpong ? 2 * 8 * N * (size_t)(nb + 2) : 0;
  bytes[S_DD] = bytes[S_DS] = 8 * N;
  bytes[S_IPIV] = bytes[S_BLK] = 4 * N;
  bytes[S_PK0] = 4 * (maxp + 2);
  bytes[S_FST] = sizeof(FacState);
  bytes[S_INVD] = 8 * ns;
  bytes[S_CPTR] = 4 * (ns + 1);
  bytes[S_CROW] = 4 * nnz;
  bytes[S_CVAL] = 8 * nnz;
  bytes[S_CFILL] = 4 * ns;
  bytes[S_FLAGS] = 4 * 16;
  bytes[S_RED] = 8 * (size_t)kRedBlocks * 8;
  bytes[S_SCAL] = 8 * 64;
  bytes[S_Z] = bytes[S_Z2] = 8 * N;
  bytes[S_HMAP] = 4 * maxp * N;
  bytes[S_PERM] = bytes[S_COLP] = 4 * N;
  bytes[S_TRSV] = std_trsv_bytes((int)N);
  bytes[S_SIG] = bytes[S_RX] = 8 * nx;
  bytes[S_RY] = 8 * m;
  bytes[S_DSB] = 8 * ns;
  bytes[S_DX] = bytes[S_DZL] = bytes[S_DZU] = bytes[S_XT] = 8 * nx;
  bytes[S_DY] = 8 * m;
  bytes[S_RES] = bytes[S_COR] = bytes[S_PREV] = bytes[S_KX] = 8 * (n + m);
  bytes[S_TN] = bytes[S_TN2] = 8 * nx;
  bytes[S_TM] = 8 * m;
  bytes[S_KNH] = bytes[S_KNJD] = 8 * nd;
  bytes[S_KNY] = 8 * m;
  bytes[S_KNJS] = 8 * ns;
  if (sblk_max > 0) {
    const size_t hn = sblk_nnz_max(d, sblk_max);
    bytes[S_BBP] = 4 * (ns + 1);
    bytes[S_BOFF] = bytes[S_BKB] = 4 * ns;
    bytes[S_BL] = 8 * ns * (size_t)sblk_max;
    bytes[S_HRP] = 4 * (m + 1);
    bytes[S_HCI] = bytes[S_HSRC] = bytes[S_HCROW] = bytes[S_HCMAP] = 4 * hn;
    bytes[S_HVAL] = bytes[S_HCVAL] = 8 * hn;
    bytes[S_HCPTR] = 4 * (ns + 1);
    bytes[S_BT1] = bytes[S_BT2] = 8 * ns;
  }
  if (nlp) {
    bytes[S_NH] = 8 * nd * nd;
    bytes[S_NJD] = 8 * m * nd;
    bytes[S_NV] = 8 * nnz;
    bytes[S_NW] = 8 * ns;
    bytes[S_NZERO] = bytes[S_NCX0] = bytes[S_NCSOC] = bytes[S_NYR] = bytes[S_NDYS] = 8 * m;
    bytes[S_NXS] = bytes[S_NDXS] = bytes[S_NXR] = bytes[S_NDR] = 8 * nx;
    bytes[S_NCMAP] = 4 * nnz;
  }
  Layout L{};
  size_t o = 0;
  for (int s = 0; s < S_COUNT; ++s) {
    L.off[s] = o;
    o += (bytes[s] + 255) & ~(size_t)255;
    if (bytes[s] == 0) o += 256;  // distinct valid addresses for empty arrays
  }
  L.total = o;
  return L;
}

bool dims_ok(const mds_dims *d) {
  return d && d->n_d >= 0 && d->n_s >= 0 && d->m >= 0 && d->nnz_s >= 0 && d->m_I >= 0 &&
         d->m_I <= d->m &&
         (int64_t)d->n_d + d->m <= std_max_n() && (int64_t)d->n_d + d->n_s < ((int64_t)1 << 30) &&
         d->nnz_s < ((int64_t)1 << 30);
}

struct PanelChoice {
  bool reg;   // panel output in the ping-pong layout (register or cooperative panel)
  bool coop;  // cooperative panel over several workgroups
  int nb, adv, threads;
  bool lds;   // unblocked factorization of the whole M in one workgroup's LDS
  bool tail = false;  // cooperative: the register panel once the rows left fit one workgroup
};

// workgroup size of the single-workgroup register panel: the option
// (64, 128, 256, 512 or 1024), else by order: 128 threads up to N = 128,
// 256 up to N = 256 (one row per thread: a pivot step waits on fewer waves,
// ~9% faster than 512 threads at N = 192), else 512
int panel_threads_of(const mds_options *o, int N) {
  const int t = o ? o->panel_threads : 0;
  if (t == 64 || t == 128 || t == 256 || t == 512 || t == 1024) return t;
  return (N <= 128) ? 128 : (N <= 256) ? 256 : 512;
}

// Panel choice.  panel option 1: memory panel; 2: register panel (N <= 4096);
// 3: cooperative register panel over several workgroups (any N); 4: the
// whole M in one workgroup's LDS (FP64, N <= bk_lds_max_n());
// 0 (automatic): the register panel while its tile keeps nb >= 16
// (N <= 2048 with 512 threads), else the cooperative panel (nb = 32, about
// 6 us per pivot at N = 4096 against 7-8 us for the memory panel, and half
// the trailing-update traffic), which hands over to the register panel once
// at most bk_reg_tail_rows() rows remain (option 3 keeps the cooperative
// panel to the end).  The mixed-precision modes need a register-resident
// panel (2 or 3).
PanelChoice panel_of(const mds_dims &d, const mds_options *o) {
  const int N = d.n_d + d.m;
  const int popt = o ? o->panel : 0;
  const int thr = panel_threads_of(o, N);
  const int rnb = bk_reg_nb(N, thr);
  PanelChoice c{};
  const int prec = o ? o->precision : MDS_FP64;
  if (prec != MDS_FP64 && prec != MDS_FP32 && prec != MDS_BF16 && prec != MDS_BF16X3)
    return c;  // nb = 0: invalid
  if (popt < 0 || popt > 4) return c;
  if (prec != MDS_FP64 && (popt == 1 || popt == 4)) return c;
  if (popt == 4) {
    if (N > bk_lds_max_n()) return c;
    const int t = o->panel_threads;
    const int nb = default_nb(N);
    return PanelChoice{false, false, nb, nb, (t == 256) ? 256 : 512, true};
  }
  if (popt == 2 && rnb == 0) return c;
  const bool use_reg = rnb > 0 && (popt == 2 || (popt == 0 && rnb >= 16));
  const bool use_coop = !use_reg && (popt == 3 || popt == 0);
  if (use_reg) {
    int nb = (o && o->nb > 0) ? o->nb : rnb;
    nb = std::min(std::max(nb, 2), rnb);
    c = {true, false, nb, std::max(nb - 1, 1), thr, false};
  } else if (use_coop) {
    int nb = (o && o->nb > 0) ? o->nb : bk_coop_nb();
    nb = std::min(std::max(nb, 2), bk_coop_nb());
    c = {true, true, nb, std::max(nb - 1, 1), 512, false};
    c.tail = (popt == 0);
  } else {
    int nb = (o && o->nb > 0) ? o->nb : default_nb(N);
    nb = std::min(std::max(nb, 2), kMaxNb);
    c = {false, false, nb, nb, 0, false};
  }
  return c;
}

int nb_of(const mds_dims &d, const mds_options *o) { return panel_of(d, o).nb; }

inline hipStream_t S(mds_handle *h) { return h->stream; }
inline int ND(mds_handle *h) { return h->dims.n_d; }
inline int NS(mds_handle *h) { return h->dims.n_s; }
inline int MM(mds_handle *h) { return h->dims.m; }

// ---- internal building blocks -------------------------------------------------

int condense_impl(mds_handle *h, double dw, double dc) {
  // (4,4) block of the inequality rows: the IPM's 1 / (Sigma_h + dw), which
  // follows the shift, or the caller's fixed diagonal
  h->dcv_cur = h->dcv_user;
  if (h->sig_h && h->mI > 0) {
    ipm_ineq_dcv(S(h), MM(h), h->mE, h->sig_h, dw, h->w.dcv);
    h->dcv_cur = h->w.dcv;
  }
  {
    TimedLaunch t(h, MDS_T_CONDENSE);
    const SBlk &B = h->sb;
    if (B.nblk > 0) {
      // blocks of Q_{x_s}: L Delta L', inv_d = 1/Delta, Jh = J_s L^{-T}
      sblk_factor(S(h), B, h->dsbase, dw, h->w.inv_d);
      sblk_transform(S(h), B, MM(h), h->P.Js_val);
    } else {
      launch_inv_d(S(h), NS(h), h->dsbase, dw, h->w.inv_d);
    }
    launch_condense_dense(S(h), ND(h), MM(h), h->P.H, h->P.J_d, h->sigma_d, dw, h->w.M);
    if (B.nblk > 0)
      launch_condense_schur(S(h), ND(h), MM(h), h->N, B.hrp, B.hci, B.hval, B.hcptr, B.hcrow,
                            B.hcval, h->w.inv_d, dc, h->dcv_cur, h->w.M);
    else
      launch_condense_schur(S(h), ND(h), MM(h), h->N, h->P.Js_rowptr, h->P.Js_col, h->P.Js_val,
                            h->w.csc_ptr, h->w.csc_row, h->w.csc_val, h->w.inv_d, dc,
                            h->dcv_cur, h->w.M);
  }
  HIPCHK(hipGetLastError());
  h->dw = dw;
  h->dc = dc;
  h->have_M = true;
  h->have_factor = false;
  return MDS_OK;
}

// Slot plan of a factorization (fixed per handle): the handle's panel until
// at most bk_reg_tail_rows() rows can remain (cooperative panel with the
// automatic tail), then the register tail, whose tile is 16 columns wide
// above 1024 rows and 32 below.
void make_plan(mds_handle *h) {
  h->plan.clear();
  long rows = h->N;
  while (rows > 0) {
    SlotPlan sp{0, rows, 0};
    if (h->panel_coop && h->panel_tail && rows <= bk_reg_tail_rows())
      sp.tail_nb = std::min(bk_reg_tail_nb((int)rows), h->nb);
    sp.rows_after = rows - (sp.tail_nb ? std::max(sp.tail_nb - 1, 1) : h->adv);
    h->plan.push_back(sp);
    rows = sp.rows_after;
  }
}

bool is_tail_slot(const mds_handle *h, int b) { return h->plan[b].tail_nb != 0; }

// Panel of slot b on the ping-pong layout: the cooperative panel, the
// register tail over its last rows, or the one-workgroup register panel.
template <typename TX>
void launch_reg_panel(mds_handle *h, hipStream_t s, int b, const TX *X, double *Y) {
  const int N = h->N;
  const SlotPlan &sp = h->plan[b];
  if (h->panel_coop && !sp.tail_nb)
    launch_bk_panel_coop(s, (int)sp.rows, N, h->nb, h->alpha_bk, X, Y, h->w.src, h->w.W, h->w.dd,
                         h->w.ds, h->w.ipiv, h->w.blk, h->w.fst, h->w.panel_k0, h->w.xch);
  else if (h->panel_coop)
    launch_bk_panel_reg_tail(s, (int)sp.rows, N, h->nb, h->alpha_bk, X, Y, h->w.src, h->w.W,
                             h->w.dd, h->w.ds, h->w.ipiv, h->w.blk, h->w.fst, h->w.panel_k0);
  else
    launch_bk_panel_reg(s, h->panel_threads, N, h->nb, h->alpha_bk, X, Y, h->w.src, h->w.W,
                        h->w.dd, h->w.ds, h->w.ipiv, h->w.blk, h->w.fst, h->w.panel_k0);
}

void factor_launches_la(mds_handle *h, hipStream_t s);

// Blocked Bunch-Kaufman of the current M; reads back the inertia.
// The launches of one factorization, on stream s.  Their number depends only
// on N and the panel's least width, so the sequence is fixed per handle.
void factor_launches(mds_handle *h, hipStream_t s) {
  const int N = h->N;
  if (h->la_cus > 0) {
    factor_launches_la(h, s);
    return;
  }
  launch_fac_reset(s, h->w.fst, h->w.panel_k0);
  const int slots = (int)h->plan.size();
  if (h->panel_lds) {
    TimedLaunch t(h, MDS_T_PANEL);
    launch_bk_lds(s, h->panel_threads, N, h->alpha_bk, h->w.M, h->w.dd, h->w.ds, h->w.ipiv,
                  h->w.blk, h->w.perm, h->w.fst);
  } else if (h->precision != MDS_FP64 && !h->force64) {
    // mixed precision: the trailing matrix lives in the FP32 ping-pong
    // buffers; L (FP64) goes to M, which then holds the whole factor
    {
      TimedLaunch t(h, MDS_T_CONDENSE);
      launch_equilibrate_f32(s, N, h->w.M, h->w.eq, h->w.X32[0]);
    }
    for (int b = 0; b < slots; ++b) {
      const float *X = h->w.X32[b & 1];
      float *Y = h->w.X32[(b + 1) & 1];
      {
        TimedLaunch t(h, is_tail_slot(h, b) ? MDS_T_PANEL_TAIL : MDS_T_PANEL);
        launch_reg_panel(h, s, b, X, h->w.M);
      }
      if (h->plan[b].rows_after > 0) {
        TimedLaunch t(h, MDS_T_TRAILING);
        launch_trailing_lp(s, h->precision, N, h->nb, h->plan[b].rows_after, b, h->w.W, X, Y,
                           h->w.M, h->w.src, h->w.fst, h->w.panel_k0);
      }
    }
  }
  const bool fp64 = h->precision == MDS_FP64 || h->force64;
  for (int b = 0; b < (fp64 && !h->panel_lds ? slots : 0); ++b) {
    // register panel: slot b reads buffer b%2 and writes its L and the
    // updated trailing matrix into the other buffer
    double *X = h->w.M, *Y = h->w.M;
    if (h->panel_reg && (b & 1)) X = h->w.M2;
    if (h->panel_reg && !(b & 1)) Y = h->w.M2;
    {
      TimedLaunch t(h, is_tail_slot(h, b) ? MDS_T_PANEL_TAIL : MDS_T_PANEL);
      if (h->panel_reg)
        launch_reg_panel(h, s, b, (const double *)X, Y);
      else
        launch_bk_panel(s, N, h->nb, h->alpha_bk, h->w.M, h->w.W, h->w.dd, h->w.ds,
                        h->w.ipiv, h->w.blk, h->w.fst, h->w.panel_k0);
    }
    if (h->plan[b].rows_after > 0) {
      TimedLaunch t(h, MDS_T_TRAILING);
      launch_bk_trailing(s, N, h->nb, h->plan[b].rows_after, b, h->w.W, X, Y, Y,
                         h->panel_reg ? h->w.src : nullptr, h->w.fst, h->w.panel_k0);
    }
  }
}

// Look-ahead form of the cooperative factorization.  Stream A (the
// reserved compute units) runs every panel and the near update of its
// trailing matrix (the 64-column strip the next panel reads); stream B (the
// other units) runs the rest of the update, while A goes on with the next
// panel.  Before the near update of slot b, A waits for B's update of slot
// b - 1: that update writes the strip and reads the buffer the near update
// writes.  Buffers of slot b: input buf[b % 2], output buf[(b + 1) % 2], map
// and W of parity b % 2 (the next panel still reads slot b's while it
// writes its own).  FP64 storage: the panel's multipliers go to a staging
// buffer of parity b % 2, which B copies into place before the rest of the
// update (the next panel's output buffer is the one that update reads).
// FP32 storage: they go straight to M, which no trailing update writes.
// Register-panel tail slots run in order on A.
void factor_launches_la(mds_handle *h, hipStream_t s) {
  const int N = h->N, nb = h->nb;
  const bool lowp = h->precision != MDS_FP64 && !h->force64;
  hipStream_t A = h->la_a, B = h->la_b;
  hipEvent_t ev_fork = h->la_ev[0], ev_near = h->la_ev[1], ev_far = h->la_ev[2],
             ev_join = h->la_ev[3];
  Work &w = h->w;
  double *buf[2] = {w.M, w.M2};
  float *buf32[2] = {w.X32[0], w.X32[1]};
  int32_t *src[2] = {w.src, w.src2};
  double *Wb[2] = {w.W, w.W2};
  if (lowp) {
    // on the handle's stream, which has every compute unit
    TimedLaunch t(h, MDS_T_CONDENSE, s);
    launch_equilibrate_f32(s, N, w.M, w.eq, buf32[0]);
  }
  (void)hipEventRecord(ev_fork, s);
  (void)hipStreamWaitEvent(A, ev_fork, 0);
  (void)hipStreamWaitEvent(B, ev_fork, 0);
  launch_fac_reset(A, w.fst, w.panel_k0);
  const int slots = (int)h->plan.size();
  bool far_pending = false;  // B holds an update A has not waited for
  auto wait_far = [&]() {
    if (far_pending) (void)hipStreamWaitEvent(A, ev_far, 0);
    far_pending = false;
  };
  for (int b = 0; b < slots; ++b) {
    const int p = b & 1, q = (b + 1) & 1;
    double *X = buf[p], *Y = buf[q];
    float *X32 = buf32[p], *Y32 = buf32[q];
    const long left = h->plan[b].rows, rem = h->plan[b].rows_after;
    const bool more = rem > 0;
    if (!is_tail_slot(h, b)) {
      {
        TimedLaunch t(h, MDS_T_PANEL, A);
        if (lowp) {
          PanelPrev pv{};
          if (b > 0) pv = PanelPrev{nullptr, buf32[q], src[q], Wb[q], w.M, 1, -1};
          launch_bk_panel_coop_la(A, (int)left, N, nb, h->alpha_bk, (const float *)X32, pv, w.M,
                                  src[p], Wb[p], w.dd, w.ds, w.ipiv, w.blk, w.fst, w.panel_k0,
                                  w.xch);
        } else {
          PanelPrev pv{};
          if (b > 0) pv = PanelPrev{buf[q], nullptr, src[q], Wb[q], w.lst[q], 0, ~15};
          launch_bk_panel_coop_la(A, (int)left, N, nb, h->alpha_bk, (const double *)X, pv,
                                  w.lst[p], src[p], Wb[p], w.dd, w.ds, w.ipiv, w.blk, w.fst,
                                  w.panel_k0, w.xch);
        }
      }
      wait_far();
      if (more) {
        {
          TimedLaunch t(h, MDS_T_NEAR, A);
          if (lowp)
            launch_trailing_lp_part(A, h->precision, N, nb, rem, b, 1, 2 * h->la_cus, Wb[p], X32,
                                    Y32, w.M, src[p], w.fst, w.panel_k0);
          else
            launch_bk_trailing_part(A, N, nb, rem, b, 1, 2 * h->la_cus, Wb[p], X, Y, w.lst[p],
                                    src[p], w.fst, w.panel_k0);
        }
        (void)hipEventRecord(ev_near, A);
        (void)hipStreamWaitEvent(B, ev_near, 0);
        if (!lowp) launch_lstage_copy(B, N, left, b, w.lst[p], Y, w.fst, w.panel_k0);
        {
          TimedLaunch t(h, MDS_T_TRAILING, B);
          if (lowp)
            launch_trailing_lp_part(B, h->precision, N, nb, rem, b, 2, h->la_grid, Wb[p], X32,
                                    Y32, w.M, src[p], w.fst, w.panel_k0);
          else
            launch_bk_trailing_part(B, N, nb, rem, b, 2, h->la_grid, Wb[p], X, Y, w.lst[p],
                                    src[p], w.fst, w.panel_k0);
        }
        (void)hipEventRecord(ev_far, B);
        far_pending = true;
      } else if (!lowp) {
        launch_lstage_copy(A, N, left, b, w.lst[p], Y, w.fst, w.panel_k0);
      }
    } else {
      wait_far();
      {
        TimedLaunch t(h, MDS_T_PANEL_TAIL, A);
        if (lowp)
          launch_bk_panel_reg_tail(A, (int)left, N, nb, h->alpha_bk, (const float *)X32, w.M,
                                   w.src, w.W, w.dd, w.ds, w.ipiv, w.blk, w.fst, w.panel_k0);
        else
          launch_bk_panel_reg_tail(A, (int)left, N, nb, h->alpha_bk, (const double *)X, Y, w.src,
                                   w.W, w.dd, w.ds, w.ipiv, w.blk, w.fst, w.panel_k0);
      }
      if (more) {
        TimedLaunch t(h, MDS_T_TRAILING, A);
        if (lowp)
          launch_trailing_lp(A, h->precision, N, nb, rem, b, w.W, X32, Y32, w.M, w.src, w.fst,
                             w.panel_k0);
        else
          launch_bk_trailing(A, N, nb, rem, b, w.W, X, Y, Y, w.src, w.fst, w.panel_k0);
      }
    }
  }
  wait_far();
  (void)hipEventRecord(ev_join, A);
  (void)hipStreamWaitEvent(s, ev_join, 0);
}

// CU-masked streams of the look-ahead: A on `reserve` compute units (the same
// count on every XCD: unit x + 8 j of XCD x, which is also XCD x when the
// mask's bits are dealt to the XCDs in turn), B on the others.  Leaves the
// look-ahead off when the device does not have 8 equal XCDs or a stream
// cannot be made.
void setup_lookahead(mds_handle *h) {
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, h->device) != hipSuccess) {
    (void)hipGetLastError();
    return;
  }
  if (cus < 64 || cus % 8 != 0) return;
  const int r = bk_coop_la_reserve(h->N, cus);
  const int per = cus / 8, m = r / 8;
  if (r == 0 || r % 8 != 0 || 7 + 8 * (m - 1) >= per) return;
  std::vector<uint32_t> ma((cus + 31) / 32, 0u), mb((cus + 31) / 32, 0u);
  for (int x = 0; x < 8; ++x)
    for (int j = 0; j < m; ++j) {
      const int bit = per * x + x + 8 * j;
      ma[bit / 32] |= 1u << (bit % 32);
    }
  for (int bit = 0; bit < cus; ++bit)
    if (!(ma[bit / 32] >> (bit % 32) & 1u)) mb[bit / 32] |= 1u << (bit % 32);
  bool ok = hipExtStreamCreateWithCUMask(&h->la_a, (uint32_t)ma.size(), ma.data()) == hipSuccess &&
            hipExtStreamCreateWithCUMask(&h->la_b, (uint32_t)mb.size(), mb.data()) == hipSuccess;
  for (int i = 0; ok && i < 4; ++i)
    ok = hipEventCreateWithFlags(&h->la_ev[i], hipEventDisableTiming) == hipSuccess;
  if (!ok) {
    (void)hipGetLastError();
    if (h->la_a) (void)hipStreamDestroy(h->la_a);
    if (h->la_b) (void)hipStreamDestroy(h->la_b);
    for (hipEvent_t &e : h->la_ev)
      if (e) (void)hipEventDestroy(e);
    h->la_a = h->la_b = nullptr;
    for (hipEvent_t &e : h->la_ev) e = nullptr;
    (void)hipGetLastError();
    return;
  }
  h->la_cus = r;
  h->la_grid = 2 * (cus - r);  // two trailing workgroups per compute unit
}

// Without per-launch timing, the factorization's launches are captured once
// into a hipGraph (on a private stream) and replayed on the handle's stream:
// ~266 dependent launches at N = 4096 leave smaller gaps that way.  Any
// failure to capture falls back to plain launches for the handle's life.
void capture_factor(mds_handle *h) {
  h->fac_graph_off = true;
  if (!h->cap_stream && hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking) != hipSuccess) {
    h->cap_stream = nullptr;
    (void)hipGetLastError();
    return;
  }
  if (hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    (void)hipGetLastError();
    return;
  }
  factor_launches(h, h->cap_stream);
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(h->cap_stream, &g);
  if (e == hipSuccess && g && hipGraphInstantiate(&h->fac_exec, g, nullptr, nullptr, 0) == hipSuccess)
    h->fac_graph_off = false;
  else
    h->fac_exec = nullptr;
  if (g) (void)hipGraphDestroy(g);
  (void)hipGetLastError();
}

// FP64 factorization of M in place by the memory panel (no exchanges between
// workgroups): the fallback of the cooperative panel.  Every panel advances
// at least nb columns.
void factor_launches_mem(mds_handle *h, hipStream_t s) {
  const int N = h->N, nb = h->nb;
  launch_fac_reset(s, h->w.fst, h->w.panel_k0);
  const int slots = (N + nb - 1) / nb;
  for (int b = 0; b < slots; ++b) {
    {
      TimedLaunch t(h, MDS_T_PANEL);
      launch_bk_panel(s, N, nb, h->alpha_bk, h->w.M, h->w.W, h->w.dd, h->w.ds, h->w.ipiv,
                      h->w.blk, h->w.fst, h->w.panel_k0);
    }
    if ((long)N - (long)(b + 1) * nb > 0) {
      TimedLaunch t(h, MDS_T_TRAILING);
      launch_bk_trailing(s, N, nb, (long)N - (long)(b + 1) * nb, b, h->w.W, h->w.M, h->w.M,
                         h->w.M, nullptr, h->w.fst, h->w.panel_k0);
    }
  }
}

int read_fac_state(mds_handle *h, FacState *st) {
  HIPCHK(hipGetLastError());
  HIPCHK(hipMemcpyAsync(st, h->w.fst, sizeof(*st), hipMemcpyDeviceToHost, S(h)));
  HIPCHK(hipStreamSynchronize(S(h)));
  return MDS_OK;
}

int factor_impl(mds_handle *h, mds_inertia *out) {
  const int N = h->N;
  FacState st{};
  bool mem = h->coop_off;
  if (!mem) {
    // the look-ahead's CU masks belong to its streams, which a graph would
    // not keep: its launches go out one by one
    const bool graph = !h->timing && !h->panel_lds && !h->fac_graph_off && !h->force64 &&
                       h->la_cus == 0;
    if (graph && !h->fac_exec) capture_factor(h);
    if (graph && h->fac_exec) {
      HIPCHK(hipGraphLaunch(h->fac_exec, S(h)));
    } else {
      TimedLaunch t(h, MDS_T_FACTOR);
      factor_launches(h, S(h));
    }
    TRY(read_fac_state(h, &st));
    if (st.xerr && h->panel_coop) {
      // an exchange wait of the cooperative panel expired (its workgroups
      // were not all resident): condense again (the ping-pong buffers hold a
      // partial factor) and factor in place with the memory panel
      h->n_coop_abort++;
      mem = true;
      TRY(condense_impl(h, h->dw, h->dc));
    } else if (st.xerr) {
      return set_err(h, MDS_EHIP, "panel aborted: rows beyond the register tile");
    }
  }
  if (mem) {
    factor_launches_mem(h, S(h));
    TRY(read_fac_state(h, &st));
  }
  if (st.k != N) return set_err(h, MDS_EHIP, "factorization stopped at %d of %d", st.k, N);
  h->fac_lowprec = !mem && !h->panel_lds && h->precision != MDS_FP64 && !h->force64;
  h->fac_pingpong = !mem && h->panel_reg && !h->fac_lowprec;
  out->npos = st.npos;
  out->nzero = st.nzero;
  out->nneg = st.nneg;
  out->n2x2 = st.n2x2;
  out->info = st.info;
  h->have_factor = true;
  h->have_M = false;
  h->std_ready = h->panel_lds;  // that kernel writes the standard form itself
  return MDS_OK;
}

// Standard form of the current factor, in place in M (once per factorization).
void ensure_std(mds_handle *h) {
  if (h->std_ready) return;
  TimedLaunch t(h, MDS_T_PERMUTE);
  const int pingpong = h->fac_pingpong ? 1 : 0;
  launch_std_form(S(h), h->N, h->w.M, h->w.M2, pingpong, h->w.ipiv, h->w.blk,
                  h->w.panel_k0, h->w.fst, h->w.hmap, h->w.perm, h->w.colpanel, h->w.M);
  h->std_ready = true;
}

// Error word of the triangular solves (a bounded wait that expired).
int solve_status(mds_handle *h) {
  int32_t e = 0;
  HIPCHK(hipMemcpyAsync(&e, h->w.trsv + 1, 4, hipMemcpyDeviceToHost, S(h)));
  HIPCHK(hipStreamSynchronize(S(h)));
  if (e) return set_err(h, MDS_EHIP, "triangular solve: dependency wait timed out");
  return MDS_OK;
}

bool inertia_ok(mds_handle *h, const mds_inertia &in) {
  return in.npos == ND(h) && in.nzero == 0 && in.nneg == MM(h);
}

// Inertia correction (Waechter & Biegler, Algorithm IC).
int correct_impl(mds_handle *h, mds_reg *reg, double mu, mds_inertia *out) {
  const double dw_min = 1e-20, dw0 = 1e-4, kw_minus = 1.0 / 3.0, kw_plus = 8.0,
               kw_plus_bar = 100.0, dc_bar = 1e-8, kappa_c = 0.25;
  const double dw_max = (reg->delta_w_max > 0.0) ? reg->delta_w_max : 1e20;
  const double dw_last = reg->delta_w_last;
  reg->trials = 1;
  TRY(condense_impl(h, 0.0, 0.0));
  TRY(factor_impl(h, out));
  if (inertia_ok(h, *out)) {
    reg->delta_w = 0.0;
    reg->delta_c = 0.0;
    return MDS_OK;
  }
  const double dc = (out->nzero > 0) ? dc_bar * std::pow(mu, kappa_c) : 0.0;
  double dw = (dw_last == 0.0) ? dw0 : std::max(dw_min, kw_minus * dw_last);
  for (;;) {
    reg->trials++;
    TRY(condense_impl(h, dw, dc));
    TRY(factor_impl(h, out));
    if (inertia_ok(h, *out)) {
      reg->delta_w_last = dw;
      reg->delta_w = dw;
      reg->delta_c = dc;
      return MDS_OK;
    }
    dw = (dw_last == 0.0) ? kw_plus_bar * dw : kw_plus * dw;
    if (dw > dw_max) {
      reg->delta_w = h->dw;
      reg->delta_c = h->dc;
      return MDS_INERTIA_FAIL;
    }
  }
}

int solve_impl(mds_handle *h, const double *r_d, const double *r_s, const double *r_y,
               double *dx_d, double *dx_s, double *dy) {
  const int nd = ND(h), ns = NS(h), m = MM(h), N = h->N;
  if (nd > 0) HIPCHK(hipMemcpyAsync(h->w.z, r_d, 8 * (size_t)nd, hipMemcpyDeviceToDevice, S(h)));
  const SBlk &B = h->sb;
  if (B.nblk > 0) {
    // r_y - Jh Delta^{-1} (L^{-1} r_s)
    vec_copy(S(h), ns, r_s, B.tmp);
    sblk_solve(S(h), B, h->w.inv_d, 0, B.tmp);
    launch_rhs_condense(S(h), m, B.hrp, B.hci, B.hval, h->w.inv_d, B.tmp, r_y, h->w.z + nd);
  } else {
    launch_rhs_condense(S(h), m, h->P.Js_rowptr, h->P.Js_col, h->P.Js_val, h->w.inv_d, r_s, r_y,
                        h->w.z + nd);
  }
  ensure_std(h);
  {
    TimedLaunch t(h, MDS_T_SOLVE);
    // mixed precision factors S M S: M^{-1} = S (S M S)^{-1} S
    if (h->fac_lowprec) launch_vscale(S(h), N, h->w.eq, h->w.z);
    launch_std_solve(S(h), N, h->w.M, h->w.dd, h->w.ds, h->w.blk, h->w.perm, h->w.z, h->w.z2,
                     h->w.z, h->w.trsv);
    if (h->fac_lowprec) launch_vscale(S(h), N, h->w.eq, h->w.z);
  }
  h->nsolves++;
  if (nd > 0) HIPCHK(hipMemcpyAsync(dx_d, h->w.z, 8 * (size_t)nd, hipMemcpyDeviceToDevice, S(h)));
  if (m > 0) HIPCHK(hipMemcpyAsync(dy, h->w.z + nd, 8 * (size_t)m, hipMemcpyDeviceToDevice, S(h)));
  if (B.nblk > 0) {
    // L^{-T} Delta^{-1} L^{-1} (r_s - J_s' dy): the unscaled back-substitution
    // (inverse diagonal of ones), then the block solves
    launch_backsub(S(h), ns, h->w.csc_ptr, h->w.csc_row, h->w.csc_val, nullptr, r_s, dy, dx_s);
    sblk_solve(S(h), B, h->w.inv_d, 1, dx_s);
  } else {
    launch_backsub(S(h), ns, h->w.csc_ptr, h->w.csc_row, h->w.csc_val, h->w.inv_d, r_s, dy,
                   dx_s);
  }
  HIPCHK(hipGetLastError());
  return MDS_OK;
}

// [od; os; oy] = K [dxd; dxs; dy] for the regularised full Newton system
void kkt_matvec(mds_handle *h, const double *dxd, const double *dxs, const double *dy,
                double *od, double *os, double *oy) {
  const int nd = ND(h), ns = NS(h), m = MM(h);
  const mds_problem &P = h->P;
  if (nd > 0) {
    launch_gemv_n(S(h), nd, nd, P.H, nd, dxd, 0.0, od);
    if (m > 0) launch_gemv_t(S(h), m, nd, P.J_d, m, dy, 1.0, od);
  }
  launch_spmv_csc(S(h), ns, h->w.csc_ptr, h->w.csc_row, h->w.csc_val, dy, 0.0, os);
  if (m > 0) {
    if (nd > 0) {
      launch_gemv_n(S(h), m, nd, P.J_d, m, dxd, 0.0, oy);
      launch_spmv_csr(S(h), m, P.Js_rowptr, P.Js_col, P.Js_val, dxs, 1.0, oy);
    } else {
      launch_spmv_csr(S(h), m, P.Js_rowptr, P.Js_col, P.Js_val, dxs, 0.0, oy);
    }
  }
  kkt_finish(S(h), nd, ns, m, h->sigma_d, h->dsbase, h->dw, h->dc, h->dcv_cur, dxd, dxs, dy, od,
             os, oy);
  if (h->sb.nblk > 0) sblk_matvec(S(h), h->sb, ns, dxs, true, os);
}

int read_scal(mds_handle *h, double *dst, int count) {
  HIPCHK(hipMemcpyAsync(dst, h->w.scal, 8 * (size_t)count, hipMemcpyDeviceToHost, S(h)));
  HIPCHK(hipStreamSynchronize(S(h)));
  return MDS_OK;
}

int amax3(mds_handle *h, int64_t na, const double *a, int64_t nb, const double *b, int64_t nc,
          const double *c, double out[3]) {
  ipm_red_amax3(S(h), na, a, nb, b, nc, c, h->w.red, h->w.scal);
  HIPCHK(hipGetLastError());
  double s[8];
  TRY(read_scal(h, s, 8));
  out[0] = s[0];
  out[1] = s[1];
  out[2] = s[2];
  return MDS_OK;
}

// ---- GMRES-based refinement (mixed precision) ---------------------------------
// Deterministic products of the columns V[:, 0..ncol) with w: the host adds
// the per-block partials in block order.
int krylov_dots(mds_handle *h, int64_t n, int ncol, const double *V, int64_t ldv,
                const double *w, double *out) {
  launch_dots(S(h), n, ncol, V, ldv, w, h->w.gpart);
  HIPCHK(hipGetLastError());
  double part[kDotBlocks * (kGmresRestart + 2)];
  HIPCHK(hipMemcpyAsync(part, h->w.gpart, 8 * (size_t)ncol * kDotBlocks, hipMemcpyDeviceToHost,
                        S(h)));
  HIPCHK(hipStreamSynchronize(S(h)));
  for (int c = 0; c < ncol; ++c) {
    double t = 0.0;
    for (int b = 0; b < kDotBlocks; ++b) t += part[c * kDotBlocks + b];
    out[c] = t;
  }
  return MDS_OK;
}

int set_coef(mds_handle *h, const double *c, int n) {
  HIPCHK(hipMemcpyAsync(h->w.gcoef, c, 8 * (size_t)n, hipMemcpyHostToDevice, S(h)));
  HIPCHK(hipStreamSynchronize(S(h)));
  return MDS_OK;
}

// Restarted GMRES(kGmresRestart) in FP64 on the full Newton system K x = r,
// right-preconditioned by the (low-precision) condensed LDL' solve P^{-1}:
// x = x0 + Z y with Z = P^{-1} V, classical Gram-Schmidt applied twice, Givens
// rotations on the host.  x0 = P^{-1} r.  Stops when the normwise backward
// error eta <= eta_tol or after max_iters GMRES iterations.
int gmres_refine(mds_handle *h, const double *r_d, const double *r_s, const double *r_y,
                 double *dx_d, double *dx_s, double *dy, int max_iters, double eta_tol,
                 mds_refine_info *info) {
  const int nd = ND(h), ns = NS(h), m = MM(h);
  const int64_t nK = (int64_t)nd + ns + m;
  const int R = kGmresRestart;
  double *r = h->w.grhs, *x = h->w.gx, *w = h->w.gw, *V = h->w.gV, *Z = h->w.gZ;
  vec_copy(S(h), nd, r_d, r);
  vec_copy(S(h), ns, r_s, r + nd);
  vec_copy(S(h), m, r_y, r + nd + ns);
  TRY(solve_impl(h, r, r + nd, r + nd + ns, x, x + nd, x + nd + ns));
  kkt_norm_parts(S(h), nd, ns, m, h->P.H, h->sigma_d, h->dw, h->P.J_d, h->P.Js_rowptr,
                 h->P.Js_val, h->w.csc_ptr, h->w.csc_val, h->dsbase, h->dc, h->dcv_cur, h->w.kn_h,
                 h->w.kn_jd, h->w.kn_y, h->w.kn_js, h->w.red, h->w.scal, &h->sb);
  HIPCHK(hipGetLastError());
  double s8[8];
  TRY(read_scal(h, s8, 8));
  const double nKn = std::max(s8[0], std::max(s8[1], s8[2]));
  double a3[3];
  TRY(amax3(h, nd, r, ns, r + nd, m, r + nd + ns, a3));
  const double nr = std::max(a3[0], std::max(a3[1], a3[2]));
  double eta = 0.0, nres = 0.0, den = 0.0;
  // w = r - K x and the backward error of x
  auto evaluate = [&]() -> int {
    kkt_matvec(h, x, x + nd, x + nd + ns, w, w + nd, w + nd + ns);
    vec_sub(S(h), nK, r, w, w);
    double rr[3], xx[3];
    TRY(amax3(h, nd, w, ns, w + nd, m, w + nd + ns, rr));
    TRY(amax3(h, nd, x, ns, x + nd, m, x + nd + ns, xx));
    nres = std::max(rr[0], std::max(rr[1], rr[2]));
    const double nx = std::max(xx[0], std::max(xx[1], xx[2]));
    den = nKn * nx + nr;
    eta = (den > 0.0) ? nres / den : 0.0;
    return MDS_OK;
  };
  TRY(evaluate());
  int iters = 0;
  std::vector<double> H((size_t)(R + 1) * R), cs(R), sn(R), g(R + 1), y(R);
  double h1[kGmresRestart + 2], h2[kGmresRestart + 2];
  while (eta > eta_tol && iters < max_iters) {
    double beta2 = 0.0;
    TRY(krylov_dots(h, nK, 1, w, nK, w, &beta2));
    const double beta = std::sqrt(beta2);
    if (!(beta > 0.0)) break;
    launch_scale(S(h), nK, 1.0 / beta, w, V);
    std::fill(g.begin(), g.end(), 0.0);
    g[0] = beta;
    int jdone = 0;
    for (int j = 0; j < R && iters < max_iters; ++j) {
      double *vj = V + (int64_t)j * nK, *zj = Z + (int64_t)j * nK;
      TRY(solve_impl(h, vj, vj + nd, vj + nd + ns, zj, zj + nd, zj + nd + ns));
      kkt_matvec(h, zj, zj + nd, zj + nd + ns, w, w + nd, w + nd + ns);
      TRY(krylov_dots(h, nK, j + 1, V, nK, w, h1));
      TRY(set_coef(h, h1, j + 1));
      launch_sub_cols(S(h), nK, j + 1, V, nK, h->w.gcoef, w);
      TRY(krylov_dots(h, nK, j + 1, V, nK, w, h2));
      TRY(set_coef(h, h2, j + 1));
      launch_sub_cols(S(h), nK, j + 1, V, nK, h->w.gcoef, w);
      double hn2 = 0.0;
      TRY(krylov_dots(h, nK, 1, w, nK, w, &hn2));
      const double hn = std::sqrt(hn2);
      double *Hj = &H[(size_t)j * (R + 1)];  // column j
      for (int i = 0; i <= j; ++i) Hj[i] = h1[i] + h2[i];
      Hj[j + 1] = hn;
      if (hn > 0.0) launch_scale(S(h), nK, 1.0 / hn, w, V + (int64_t)(j + 1) * nK);
      for (int i = 0; i < j; ++i) {
        const double t0 = cs[i] * Hj[i] + sn[i] * Hj[i + 1];
        Hj[i + 1] = -sn[i] * Hj[i] + cs[i] * Hj[i + 1];
        Hj[i] = t0;
      }
      const double rho = std::hypot(Hj[j], Hj[j + 1]);
      cs[j] = (rho > 0.0) ? Hj[j] / rho : 1.0;
      sn[j] = (rho > 0.0) ? Hj[j + 1] / rho : 0.0;
      Hj[j] = rho;
      Hj[j + 1] = 0.0;
      g[j + 1] = -sn[j] * g[j];
      g[j] = cs[j] * g[j];
      ++iters;
      jdone = j + 1;
      if (!(hn > 0.0) || std::fabs(g[j + 1]) <= eta_tol * den) break;
    }
    if (jdone == 0) break;
    for (int i = jdone - 1; i >= 0; --i) {
      double t = g[i];
      for (int c = i + 1; c < jdone; ++c) t -= H[(size_t)c * (R + 1) + i] * y[c];
      y[i] = t / H[(size_t)i * (R + 1) + i];
    }
    TRY(set_coef(h, y.data(), jdone));
    launch_add_cols(S(h), nK, jdone, Z, nK, h->w.gcoef, x);
    TRY(evaluate());
  }
  vec_copy(S(h), nd, x, dx_d);
  vec_copy(S(h), ns, x + nd, dx_s);
  vec_copy(S(h), m, x + nd + ns, dy);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(S(h)));
  TRY(solve_status(h));
  if (info) {
    info->eta = eta;
    info->rel_residual = (nr > 0.0) ? nres / nr : 0.0;
    info->steps = iters;
  }
  return (eta <= eta_tol) ? MDS_OK : MDS_REFINE_NOCONV;
}

int refine_impl(mds_handle *h, const double *r_d, const double *r_s, const double *r_y,
                double *dx_d, double *dx_s, double *dy, int max_steps, double eta_tol,
                mds_refine_info *info) {
  if (h->fac_lowprec)
    return gmres_refine(h, r_d, r_s, r_y, dx_d, dx_s, dy, max_steps, eta_tol, info);
  const int nd = ND(h), ns = NS(h), m = MM(h);
  const size_t nt = (size_t)nd + ns + m;
  double *res = h->w.res, *cor = h->w.cor, *prev = h->w.prev, *kx = h->w.kx;
  TRY(solve_impl(h, r_d, r_s, r_y, dx_d, dx_s, dy));
  // ||K||_inf parts and ||r||_inf: two reductions, one read-back
  kkt_norm_parts(S(h), nd, ns, m, h->P.H, h->sigma_d, h->dw, h->P.J_d, h->P.Js_rowptr,
                 h->P.Js_val, h->w.csc_ptr, h->w.csc_val, h->dsbase, h->dc, h->dcv_cur, h->w.kn_h,
                 h->w.kn_jd, h->w.kn_y, h->w.kn_js, h->w.red, h->w.scal, &h->sb);
  ipm_red_amax3(S(h), nd, r_d, ns, r_s, m, r_y, h->w.red, h->w.scal + 8);
  HIPCHK(hipGetLastError());
  double s16[16];
  TRY(read_scal(h, s16, 16));
  const double nK = std::max(s16[0], std::max(s16[1], s16[2]));
  const double nr = std::max(s16[8], std::max(s16[9], s16[10]));
  double eta_prev = INFINITY, eta = 0.0, rres = 0.0;
  int steps = 0;
  for (;;) {
    kkt_matvec(h, dx_d, dx_s, dy, kx, kx + nd, kx + nd + ns);
    vec_sub(S(h), nd, r_d, kx, res);
    vec_sub(S(h), ns, r_s, kx + nd, res + nd);
    vec_sub(S(h), m, r_y, kx + nd + ns, res + nd + ns);
    // ||res||_inf and ||x||_inf: one read-back
    ipm_red_amax3(S(h), nd, res, ns, res + nd, m, res + nd + ns, h->w.red, h->w.scal);
    ipm_red_amax3(S(h), nd, dx_d, ns, dx_s, m, dy, h->w.red, h->w.scal + 8);
    HIPCHK(hipGetLastError());
    TRY(read_scal(h, s16, 16));
    const double nres = std::max(s16[0], std::max(s16[1], s16[2]));
    const double nx = std::max(s16[8], std::max(s16[9], s16[10]));
    const double den = nK * nx + nr;
    eta = (den > 0.0) ? nres / den : 0.0;
    rres = (nr > 0.0) ? nres / nr : 0.0;
    if (steps > 0 && !(eta < eta_prev)) {
      // no decrease: keep the previous iterate
      vec_copy(S(h), nd, prev, dx_d);
      vec_copy(S(h), ns, prev + nd, dx_s);
      vec_copy(S(h), m, prev + nd + ns, dy);
      eta = eta_prev;
      break;
    }
    if (eta <= eta_tol || steps >= max_steps) break;
    vec_copy(S(h), nd, dx_d, prev);
    vec_copy(S(h), ns, dx_s, prev + nd);
    vec_copy(S(h), m, dy, prev + nd + ns);
    eta_prev = eta;
    TRY(solve_impl(h, res, res + nd, res + nd + ns, cor, cor + nd, cor + nd + ns));
    vec_add_inplace(S(h), nd, cor, dx_d);
    vec_add_inplace(S(h), ns, cor + nd, dx_s);
    vec_add_inplace(S(h), m, cor + nd + ns, dy);
    steps++;
  }
  HIPCHK(hipGetLastError());
  TRY(solve_status(h));  // synchronizes
  (void)nt;
  if (info) {
    info->eta = eta;
    info->rel_residual = rres;
    info->steps = steps;
  }
  return (eta <= eta_tol) ? MDS_OK : MDS_REFINE_NOCONV;
}

// Over the IPM's primal vector x = [variables; slacks] (nx entries):
// gf = grad f -> tn (0 on the slacks); jty = J'y -> tn2 (-y_h on the
// slacks); cx = c(x) = J x - [b; d] -> tm (and r_y = -c if ry).
void eval_grad_constr(mds_handle *h, const double *x, const double *y, double *ry) {
  const int nd = ND(h), ns = NS(h), m = MM(h), n = h->n;
  const mds_problem &P = h->P;
  double *gf = h->w.tn, *jty = h->w.tn2, *cx = h->w.tm;
  if (h->nlp_on) {
    // the model's gradient and rows; J' y from its last Jacobian
    if (h->nlp.gradient(h->nlp.ctx, x, gf) != 0) h->model_err = true;
  } else {
    launch_gemv_n(S(h), nd, nd, P.H, nd, x, 0.0, gf);
    ipm_grad_finish(S(h), nd, ns, P.c, P.w, P.g, x, gf);
    if (h->sb.nblk > 0) sblk_matvec(S(h), h->sb, ns, x + nd, true, gf + nd);
  }
  if (y) {
    if (nd > 0) {
      if (m > 0) launch_gemv_t(S(h), m, nd, P.J_d, m, y, 0.0, jty);
      else hipMemsetAsync(jty, 0, 8 * (size_t)nd, S(h));
    }
    launch_spmv_csc(S(h), ns, h->w.csc_ptr, h->w.csc_row, h->w.csc_val, y, 0.0, jty + nd);
  }
  ipm_slack_grad(S(h), h->mI, h->mE, y, gf + n, jty + n);
  if (m > 0) {
    if (h->nlp_on) {
      if (h->nlp.constraints(h->nlp.ctx, x, cx) != 0) h->model_err = true;
      ipm_constr_finish(S(h), m, h->mE, h->nlp_zero, x + n, cx, ry);
      return;
    }
    if (nd > 0) {
      launch_gemv_n(S(h), m, nd, P.J_d, m, x, 0.0, cx);
      launch_spmv_csr(S(h), m, P.Js_rowptr, P.Js_col, P.Js_val, x + nd, 1.0, cx);
    } else {
      launch_spmv_csr(S(h), m, P.Js_rowptr, P.Js_col, P.Js_val, x + nd, 0.0, cx);
    }
    ipm_constr_finish(S(h), m, h->mE, P.b, x + n, cx, ry);
  }
}

int opt_error_impl(mds_handle *h, const double *x, const double *y, const double *zl,
                   const double *zu, double mu, double *E, double *parts) {
  const int n = h->nx, m = MM(h);
  const double s_max = 100.0;
  eval_grad_constr(h, x, y, nullptr);
  ipm_red_opt(S(h), n, m, x, y, zl, zu, h->w.xl_e, h->w.xu_e, h->w.tn, h->w.tn2, h->w.tm, mu,
              h->w.red, h->w.scal);
  HIPCHK(hipGetLastError());
  double s[8];
  TRY(read_scal(h, s, 8));
  const double dual = s[0], prim = s[1], cl = s[2], cu = s[3], y1 = s[4], z1 = s[5];
  const double nz = s[6];
  const double sd = (m + nz > 0) ? std::max(s_max, (y1 + z1) / ((double)m + nz)) / s_max : 1.0;
  const double sc = (nz > 0) ? std::max(s_max, z1 / nz) / s_max : 1.0;
  *E = std::max(std::max(dual / sd, prim), std::max(cl, cu) / sc);
  if (parts) {
    parts[0] = dual;
    parts[1] = prim;
    parts[2] = cl;
    parts[3] = cu;
    parts[4] = sd;
    parts[5] = sc;
  }
  return MDS_OK;
}

// E_0 and E_mu at one mu from one reduction pass and one read-back.
int opt_error_pair(mds_handle *h, const double *x, const double *y, const double *zl,
                   const double *zu, double mu, double *E0, double *Emu) {
  const int n = h->nx, m = MM(h);
  const double s_max = 100.0;
  eval_grad_constr(h, x, y, nullptr);
  ipm_red_opt_pair(S(h), n, m, x, y, zl, zu, h->w.xl_e, h->w.xu_e, h->w.tn, h->w.tn2, h->w.tm,
                   mu, h->w.red, h->w.scal);
  HIPCHK(hipGetLastError());
  double s[8];
  TRY(read_scal(h, s, 8));
  const double dual = s[0], prim = s[1], cmu = s[2], c0 = s[3], y1 = s[4], z1 = s[5];
  const double nz = s[6];
  const double sd = (m + nz > 0) ? std::max(s_max, (y1 + z1) / ((double)m + nz)) / s_max : 1.0;
  const double sc = (nz > 0) ? std::max(s_max, z1 / nz) / s_max : 1.0;
  *Emu = std::max(std::max(dual / sd, prim), cmu / sc);
  *E0 = std::max(std::max(dual / sd, prim), c0 / sc);
  return MDS_OK;
}

// Launches the merit reductions at x = [variables; slacks] into out[0..7]
// (slot 4: f, 5: sum of log-slacks of the variables and the slacks, 6:
// theta, 7: the rounding scale of phi_mu, sum of the magnitudes of its
// terms); h->w.tn and h->w.tm are overwritten.
void merit_launch(mds_handle *h, const double *x, double mu, double *out) {
  const int nd = ND(h), ns = NS(h), m = MM(h);
  const mds_problem &P = h->P;
  double *hx = h->w.tn, *cx = h->w.tm;
  launch_gemv_n(S(h), nd, nd, P.H, nd, x, 0.0, hx);
  if (m > 0) {
    if (nd > 0) {
      launch_gemv_n(S(h), m, nd, P.J_d, m, x, 0.0, cx);
      launch_spmv_csr(S(h), m, P.Js_rowptr, P.Js_col, P.Js_val, x + nd, 1.0, cx);
    } else {
      launch_spmv_csr(S(h), m, P.Js_rowptr, P.Js_col, P.Js_val, x + nd, 0.0, cx);
    }
    ipm_constr_finish(S(h), m, h->mE, P.b, x + h->n, cx, nullptr);
  }
  const double *wbx = nullptr;
  if (h->sb.nblk > 0) {
    sblk_matvec(S(h), h->sb, ns, x + nd, false, h->sb.tmp2);
    wbx = h->sb.tmp2;
  }
  ipm_red_merit(S(h), nd, ns, h->nx, m, mu, x, hx, P.c, P.w, P.g, wbx, h->w.xl_e, h->w.xu_e,
                cx, h->w.red, out);
}

// NLP mode: the rows' residual at x (c(x) on the equality rows, h(x) - d on
// the inequality rows) into w.tm
int nlp_rows(mds_handle *h, const double *x) {
  const int m = MM(h);
  if (m == 0) return MDS_OK;
  if (h->nlp.constraints(h->nlp.ctx, x, h->w.tm) != 0)
    return set_err(h, MDS_EMODEL, "model constraints failed");
  ipm_constr_finish(S(h), m, h->mE, h->nlp_zero, x + h->n, h->w.tm, nullptr);
  return MDS_OK;
}

// NLP mode: theta, the log-slack sum (slot 5) and mu times its magnitude sum
// (slot 7) of x from the residual in w.tm, into out[0..7]
void nlp_merit_launch(mds_handle *h, const double *x, double mu, double *out) {
  ipm_red_merit(S(h), 0, 0, h->nx, MM(h), mu, x, nullptr, nullptr, nullptr, nullptr, nullptr,
                h->w.xl_e, h->w.xu_e, h->w.tm, h->w.red, out);
}

// NLP mode: theta at x (the residual stays in w.tm) and, when phi or scale
// is asked for, f from the model; scale = |f| + mu sum |log|, the rounding
// scale of phi for a model objective
int merit_nlp(mds_handle *h, const double *x, double mu, double *f, double *phi, double *theta,
              double *scale) {
  TRY(nlp_rows(h, x));
  nlp_merit_launch(h, x, mu, h->w.scal);
  HIPCHK(hipGetLastError());
  double fv = 0.0;
  if (f || phi || scale) {
    if (h->nlp.objective(h->nlp.ctx, x, &fv) != 0)
      return set_err(h, MDS_EMODEL, "model objective failed");
  }
  double s[8];
  TRY(read_scal(h, s, 8));
  if (f) *f = fv;
  if (phi) *phi = fv - mu * s[5];
  if (theta) *theta = s[6];
  if (scale) *scale = std::fabs(fv) + s[7];
  return MDS_OK;
}

int nlp_model_ok(mds_handle *h) {
  if (!h->model_err) return MDS_OK;
  h->model_err = false;
  return set_err(h, MDS_EMODEL, "a model callback failed");
}

// NLP mode: the model's Jacobian at x, and the column-compressed copy of
// its J_s values
int nlp_jacobian(mds_handle *h, const double *x) {
  if (h->nlp.jacobian(h->nlp.ctx, x, h->nlp_Jd, h->nlp_v) != 0)
    return set_err(h, MDS_EMODEL, "model Jacobian failed");
  nlp_gather(S(h), h->dims.nnz_s, h->nlp_cmap, h->nlp_v, h->w.csc_val);
  HIPCHK(hipGetLastError());
  return MDS_OK;
}

int merit_impl(mds_handle *h, const double *x, double mu, double *f, double *phi, double *theta) {
  if (h->nlp_on) return merit_nlp(h, x, mu, f, phi, theta, nullptr);
  merit_launch(h, x, mu, h->w.scal);
  HIPCHK(hipGetLastError());
  double s[8];
  TRY(read_scal(h, s, 8));
  if (f) *f = s[4];
  if (phi) *phi = s[4] - mu * s[5];
  if (theta) *theta = s[6];
  return MDS_OK;
}

int check_ready(mds_handle *h) {
  if (!h) return MDS_ENULL;
  if (!h->have_problem) return set_err(h, MDS_ESTATE, "no problem attached");
  return MDS_OK;
}

}  // namespace

// =============================================================================
// exported functions
// =============================================================================

extern "C" {

size_t mds_workspace_bytes(const mds_dims *dims, const mds_options *opts) {
  if (!dims_ok(dims)) return 0;
  const PanelChoice pc = panel_of(*dims, opts);
  if (pc.nb == 0) return 0;
  const int sbm = opts ? opts->sblk_max : 0;
  if (sbm < 0 || sbm > kSBlkMax) return 0;
  return make_layout(*dims, pc.nb, pc.reg, opts ? opts->precision : MDS_FP64, sbm,
                     opts && opts->nlp != 0).total;
}

int mds_create(mds_handle **out, const mds_dims *dims, const mds_options *opts, void *stream,
               void *workspace, size_t workspace_bytes) {
  if (!out || !dims) return MDS_ENULL;
  *out = nullptr;
  if (!dims_ok(dims)) return MDS_EDIMS;
  const int nb = nb_of(*dims, opts);
  if (nb == 0) return MDS_EINVAL;
  const int prec = opts ? opts->precision : MDS_FP64;
  const int sbm = opts ? opts->sblk_max : 0;
  if (sbm < 0 || sbm > kSBlkMax) return MDS_EINVAL;
  const bool nlp = opts && opts->nlp != 0;
  const int la_opt = opts ? opts->lookahead : 0;
  if (la_opt < 0 || la_opt > 2) return MDS_EINVAL;
  const Layout L = make_layout(*dims, nb, panel_of(*dims, opts).reg, prec, sbm, nlp);
  const PanelChoice pc = panel_of(*dims, opts);
  // every workgroup of the cooperative panel must be resident at once; if
  // the device cannot guarantee it, the memory panel (FP64) factors instead
  bool coop_off = false;
  if (pc.coop && !bk_coop_resident(dims->n_d + dims->m)) {
    if (prec != MDS_FP64) return MDS_EINVAL;
    coop_off = true;
  }
  if (!workspace) return MDS_ENULL;
  if (workspace_bytes < L.total || ((uintptr_t)workspace & 255) != 0) return MDS_EWORKSPACE;
  mds_handle *h = new (std::nothrow) mds_handle();
  if (!h) return MDS_EINVAL;
  h->stream = (hipStream_t)stream;
  if (hipGetDevice(&h->device) != hipSuccess) {
    delete h;
    return MDS_EHIP;
  }
  h->dims = *dims;
  h->N = dims->n_d + dims->m;
  h->n = dims->n_d + dims->n_s;
  h->mI = dims->m_I;
  h->mE = dims->m - dims->m_I;
  h->nx = h->n + h->mI;
  h->coop_off = coop_off;
  h->nb = nb;
  h->panel_reg = pc.reg;
  h->panel_coop = pc.coop;
  h->panel_tail = pc.tail;
  h->panel_lds = pc.lds;
  h->panel_threads = pc.threads;
  h->precision = prec;
  h->adv = pc.adv;
  h->max_panels = h->N / pc.adv + 2;
  make_plan(h);
  h->ws_bytes = workspace_bytes;
  h->alpha_bk = (1.0 + std::sqrt(17.0)) / 8.0;
  char *base = (char *)workspace;
  auto D = [&](int s) { return (double *)(base + L.off[s]); };
  auto I = [&](int s) { return (int32_t *)(base + L.off[s]); };
  Work &w = h->w;
  w.M = D(S_M);
  w.M2 = D(S_M2);
  w.X32[0] = (float *)(base + L.off[S_M2]);
  w.X32[1] = w.X32[0] + (size_t)h->N * (size_t)h->N;
  w.xl_e = D(S_XLE);
  w.xu_e = D(S_XUE);
  w.dcv = D(S_DCV);
  w.ry2 = D(S_RY2);
  w.eq = D(S_EQ);
  w.gV = D(S_GV);
  w.gZ = D(S_GZ);
  w.grhs = D(S_GRHS);
  w.gx = D(S_GX);
  w.gw = D(S_GW);
  w.gpart = D(S_GPART);
  w.gcoef = D(S_GCOEF);
  w.src = I(S_SRC);
  w.W = D(S_W);
  w.src2 = I(S_SRC2);
  w.W2 = D(S_W2);
  w.lst[0] = D(S_LST);
  w.lst[1] = w.lst[0] + (size_t)h->N * (size_t)(h->nb + 2);
  w.dd = D(S_DD);
  w.ds = D(S_DS);
  w.ipiv = I(S_IPIV);
  w.blk = I(S_BLK);
  w.panel_k0 = I(S_PK0);
  w.fst = (FacState *)(base + L.off[S_FST]);
  w.inv_d = D(S_INVD);
  w.csc_ptr = I(S_CPTR);
  w.csc_row = I(S_CROW);
  w.csc_val = D(S_CVAL);
  w.csc_fill = I(S_CFILL);
  w.flags = I(S_FLAGS);
  w.red = D(S_RED);
  w.scal = D(S_SCAL);
  w.z = D(S_Z);
  w.z2 = D(S_Z2);
  w.hmap = I(S_HMAP);
  w.perm = I(S_PERM);
  w.colpanel = I(S_COLP);
  w.trsv = I(S_TRSV);
  w.xch = (uint64_t *)(base + L.off[S_XCH]);
  w.sig = D(S_SIG);
  w.rx = D(S_RX);
  w.ry = D(S_RY);
  w.dsb = D(S_DSB);
  w.dx = D(S_DX);
  w.dy = D(S_DY);
  w.dzl = D(S_DZL);
  w.dzu = D(S_DZU);
  w.xt = D(S_XT);
  w.res = D(S_RES);
  w.cor = D(S_COR);
  w.prev = D(S_PREV);
  w.kx = D(S_KX);
  w.tn = D(S_TN);
  w.tm = D(S_TM);
  w.tn2 = D(S_TN2);
  w.kn_h = D(S_KNH);
  w.kn_jd = D(S_KNJD);
  w.kn_y = D(S_KNY);
  w.kn_js = D(S_KNJS);
  h->sblk_max = sbm;
  h->nlp_room = nlp;
  if (nlp) {
    h->nlp_H = D(S_NH);
    h->nlp_Jd = D(S_NJD);
    h->nlp_v = D(S_NV);
    h->nlp_w = D(S_NW);
    h->nlp_zero = D(S_NZERO);
    h->nlp_cx0 = D(S_NCX0);
    h->nlp_csoc = D(S_NCSOC);
    h->nlp_yr = D(S_NYR);
    h->nlp_xs = D(S_NXS);
    h->nlp_dxs = D(S_NDXS);
    h->nlp_dys = D(S_NDYS);
    h->nlp_xr = D(S_NXR);
    h->nlp_dr = D(S_NDR);
    h->nlp_cmap = I(S_NCMAP);
  }
  if (sbm > 0) {
    SBlk &B = h->sb;
    B.bp = I(S_BBP);
    B.boff = I(S_BOFF);
    B.kblk = I(S_BKB);
    B.lblk = D(S_BL);
    B.hrp = I(S_HRP);
    B.hci = I(S_HCI);
    B.hsrc = I(S_HSRC);
    B.hval = D(S_HVAL);
    B.hcptr = I(S_HCPTR);
    B.hcrow = I(S_HCROW);
    B.hcmap = I(S_HCMAP);
    B.hcval = D(S_HCVAL);
    B.tmp = D(S_BT1);
    B.tmp2 = D(S_BT2);
  }
  if (std_prepare() != hipSuccess || bk_lds_prepare() != hipSuccess ||
      hipMemsetAsync(w.trsv, 0, std_trsv_bytes(h->N), h->stream) !=
          hipSuccess ||
      hipMemsetAsync(w.xch, 0, 8 * 2 * (size_t)kCoopMaxP * kCoopSlotWords, h->stream) !=
          hipSuccess ||
      hipMemsetAsync(w.fst, 0, sizeof(FacState), h->stream) != hipSuccess ||
      hipStreamSynchronize(h->stream) != hipSuccess) {
    delete h;
    return MDS_EHIP;
  }
  // look-ahead: automatic from N = 8192 (below, the candidate columns it
  // computes on the fly cost about what the overlap saves)
  if (pc.coop && !coop_off && la_opt != 2 && (la_opt == 1 || h->N >= 8192)) setup_lookahead(h);
  *out = h;
  return MDS_OK;
}

void mds_destroy(mds_handle *h) {
  if (!h) return;
  for (hipEvent_t e : h->ev_pool) (void)hipEventDestroy(e);
  if (h->fac_exec) (void)hipGraphExecDestroy(h->fac_exec);
  if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
  if (h->la_a) (void)hipStreamDestroy(h->la_a);
  if (h->la_b) (void)hipStreamDestroy(h->la_b);
  for (hipEvent_t e : h->la_ev)
    if (e) (void)hipEventDestroy(e);
  delete h;
}

int mds_set_problem(mds_handle *h, const mds_problem *p) {
  if (!h || !p) return MDS_ENULL;
  const mds_dims &d = h->dims;
  const int64_t nd = d.n_d, ns = d.n_s, m = d.m;
  const int64_t mI = d.m_I, mE = m - mI;
  if ((nd > 0 && (!p->H || !p->c)) || (ns > 0 && (!p->w || !p->g)) ||
      (m > 0 && nd > 0 && !p->J_d) || (mE > 0 && !p->b) || !p->Js_rowptr ||
      (d.nnz_s > 0 && (!p->Js_col || !p->Js_val)) || (nd + ns > 0 && (!p->xl || !p->xu)) ||
      (mI > 0 && (!p->hl || !p->hu)))
    return set_err(h, MDS_ENULL, "problem array missing");
  h->have_problem = false;
  h->have_M = h->have_factor = false;
  h->ipm_ready = false;
  h->dcv_user = h->dcv_cur = nullptr;
  h->sig_h = nullptr;
  h->sb.nblk = 0;
  h->nlp_on = false;
  h->nlp_force_resto = 0;
  HIPCHK(hipMemsetAsync(h->w.flags, 0, 64, S(h)));
  launch_validate(S(h), d, *p, h->w.flags);
  check_ineq_bounds(S(h), (int)mI, p->hl, p->hu, h->w.flags + 5);
  HIPCHK(hipGetLastError());
  int32_t f[16];
  HIPCHK(hipMemcpyAsync(f, h->w.flags, 64, hipMemcpyDeviceToHost, S(h)));
  HIPCHK(hipStreamSynchronize(S(h)));
  if (f[3]) return set_err(h, MDS_EPATTERN, "J_s CSR pattern invalid (row pointers, range or order)");
  if (f[0]) return set_err(h, MDS_ENONFINITE_INPUT, "non-finite value in problem data");
  if (f[1]) return set_err(h, MDS_EDS_NONPOS, "w has a negative entry");
  if (f[2]) return set_err(h, MDS_EDS_NONPOS, "bounds violate xl < xu");
  if (f[4]) return set_err(h, MDS_EINVAL, "H is not exactly symmetric");
  if (f[5])
    return set_err(h, MDS_EDS_NONPOS,
                   "inequality bounds violate hl < hu or are both infinite");
  h->P = *p;
  // bounds of the IPM's primal vector: the variables', then the slacks'
  vec_copy(S(h), nd + ns, p->xl, h->w.xl_e);
  vec_copy(S(h), nd + ns, p->xu, h->w.xu_e);
  vec_copy(S(h), mI, p->hl, h->w.xl_e + nd + ns);
  vec_copy(S(h), mI, p->hu, h->w.xu_e + nd + ns);
  launch_csc_build(S(h), (int)m, (int)ns, d.nnz_s, p->Js_rowptr, p->Js_col, p->Js_val,
                   h->w.csc_ptr, h->w.csc_row, h->w.csc_val, h->w.csc_fill);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(S(h)));
  h->have_problem = true;
  return MDS_OK;
}

int mds_condense(mds_handle *h, const double *sigma_d, const double *dsbase, double delta_w,
                 double delta_c) {
  TRY(check_ready(h));
  if ((ND(h) > 0 && !sigma_d) || (NS(h) > 0 && !dsbase))
    return set_err(h, MDS_ENULL, "sigma_d / dsbase missing");
  if (!std::isfinite(delta_w) || !std::isfinite(delta_c) || delta_w < 0.0 || delta_c < 0.0)
    return set_err(h, MDS_EINVAL, "shifts must be finite and nonnegative");
  h->sigma_d = sigma_d;
  h->dsbase = dsbase;
  return condense_impl(h, delta_w, delta_c);
}

int mds_set_sparse_blocks(mds_handle *h, int32_t nblk, const int32_t *bp_host,
                          const double *Wb) {
  TRY(check_ready(h));
  SBlk &B = h->sb;
  if (nblk == 0) {
    B.nblk = 0;
    h->have_M = h->have_factor = false;
    return MDS_OK;
  }
  if (h->sblk_max <= 0)
    return set_err(h, MDS_ESTATE, "the workspace has no room for blocks (options.sblk_max = 0)");
  if (h->nlp_on) return set_err(h, MDS_ESTATE, "coupling blocks are not available in NLP mode");
  const int ns = NS(h), m = MM(h);
  if (nblk < 0 || nblk > ns) return set_err(h, MDS_EDIMS, "nblk must be in [0, n_s]");
  if (!bp_host || !Wb) return set_err(h, MDS_ENULL, "bp_host / Wb missing");
  if (bp_host[0] != 0 || bp_host[nblk] != ns)
    return set_err(h, MDS_EINVAL, "blocks must cover 0 .. n_s");
  std::vector<int32_t> boff(nblk), kblk(ns);
  int64_t words = 0;
  for (int b = 0; b < nblk; ++b) {
    const int sz = bp_host[b + 1] - bp_host[b];
    if (sz < 1 || sz > h->sblk_max)
      return set_err(h, MDS_EINVAL, "block %d has size %d (1 .. %d allowed)", b, sz, h->sblk_max);
    boff[b] = (int32_t)words;
    for (int k = bp_host[b]; k < bp_host[b + 1]; ++k) kblk[k] = b;
    words += (int64_t)sz * sz;
  }
  // the blocks: finite, exactly symmetric, positive semidefinite (their
  // L Delta L' after a shift of 1e-12 of the largest diagonal has Delta > 0)
  std::vector<double> wb((size_t)words);
  HIPCHK(hipMemcpyAsync(wb.data(), Wb, 8 * (size_t)words, hipMemcpyDeviceToHost, S(h)));
  HIPCHK(hipStreamSynchronize(S(h)));
  for (int b = 0; b < nblk; ++b) {
    const int sz = bp_host[b + 1] - bp_host[b];
    const double *Q = wb.data() + boff[b];
    double dmax = 0.0;
    for (int i = 0; i < sz; ++i) {
      for (int j = 0; j < sz; ++j) {
        if (!std::isfinite(Q[i + j * sz]))
          return set_err(h, MDS_ENONFINITE_INPUT, "non-finite entry in block %d", b);
        if (Q[i + j * sz] != Q[j + i * sz])
          return set_err(h, MDS_EINVAL, "block %d is not exactly symmetric", b);
      }
      dmax = std::max(dmax, Q[i + i * sz]);
    }
    double L[kSBlkMax * kSBlkMax], dl[kSBlkMax];
    const double shift = 1e-12 * dmax + 1e-300;
    for (int j = 0; j < sz; ++j) {
      double d = Q[j + j * sz] + shift;
      for (int t = 0; t < j; ++t) d -= L[j + t * sz] * L[j + t * sz] * dl[t];
      if (!(d > 0.0))
        return set_err(h, MDS_EDS_NONPOS, "block %d is not positive semidefinite", b);
      dl[j] = d;
      for (int i = j + 1; i < sz; ++i) {
        double e = Q[i + j * sz];
        for (int t = 0; t < j; ++t) e -= L[i + t * sz] * L[j + t * sz] * dl[t];
        L[i + j * sz] = e / d;
      }
    }
  }
  // pattern of J_s (host), then that of Jh = J_s L^{-T}: every column of
  // every block a row touches, blocks ascending
  const int64_t nnz = h->dims.nnz_s;
  std::vector<int32_t> rp(m + 1), ci((size_t)std::max<int64_t>(nnz, 1));
  HIPCHK(hipMemcpyAsync(rp.data(), h->P.Js_rowptr, 4 * (size_t)(m + 1), hipMemcpyDeviceToHost,
                        S(h)));
  if (nnz > 0)
    HIPCHK(hipMemcpyAsync(ci.data(), h->P.Js_col, 4 * (size_t)nnz, hipMemcpyDeviceToHost, S(h)));
  HIPCHK(hipStreamSynchronize(S(h)));
  std::vector<int32_t> hrp(m + 1, 0), hci, hsrc;
  for (int i = 0; i < m; ++i) {
    int a = rp[i];
    while (a < rp[i + 1]) {
      const int b = kblk[ci[a]], k0 = bp_host[b], sz = bp_host[b + 1] - k0;
      for (int p = 0; p < sz; ++p) {
        int src = -1;
        if (a < rp[i + 1] && ci[a] == k0 + p) src = a++;
        hci.push_back(k0 + p);
        hsrc.push_back(src);
      }
    }
    hrp[i + 1] = (int32_t)hci.size();
  }
  const int64_t hn = (int64_t)hci.size();
  if ((size_t)hn > sblk_nnz_max(h->dims, h->sblk_max))
    return set_err(h, MDS_EWORKSPACE, "transformed Jacobian exceeds the workspace");
  // its CSC copy: rows ascending in every column, with the CSR entry of each
  std::vector<int32_t> hcptr(ns + 1, 0), hcrow((size_t)std::max<int64_t>(hn, 1)),
      hcmap((size_t)std::max<int64_t>(hn, 1));
  for (int64_t e = 0; e < hn; ++e) hcptr[hci[e] + 1]++;
  for (int k = 0; k < ns; ++k) hcptr[k + 1] += hcptr[k];
  {
    std::vector<int32_t> fill(hcptr.begin(), hcptr.end() - 1);
    for (int i = 0; i < m; ++i)
      for (int e = hrp[i]; e < hrp[i + 1]; ++e) {
        const int q = fill[hci[e]]++;
        hcrow[q] = i;
        hcmap[q] = e;
      }
  }
  auto up = [&](void *dst, const void *src, size_t bytes) -> int {
    if (bytes == 0) return MDS_OK;
    HIPCHK(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, S(h)));
    return MDS_OK;
  };
  TRY(up((void *)B.bp, bp_host, 4 * (size_t)(nblk + 1)));
  TRY(up((void *)B.boff, boff.data(), 4 * (size_t)nblk));
  TRY(up((void *)B.kblk, kblk.data(), 4 * (size_t)ns));
  TRY(up(B.hrp, hrp.data(), 4 * (size_t)(m + 1)));
  TRY(up(B.hci, hci.data(), 4 * (size_t)hn));
  TRY(up(B.hsrc, hsrc.data(), 4 * (size_t)hn));
  TRY(up(B.hcptr, hcptr.data(), 4 * (size_t)(ns + 1)));
  TRY(up(B.hcrow, hcrow.data(), 4 * (size_t)hn));
  TRY(up(B.hcmap, hcmap.data(), 4 * (size_t)hn));
  HIPCHK(hipStreamSynchronize(S(h)));
  B.nblk = nblk;
  B.nnz = hn;
  B.Wb = Wb;
  h->have_M = h->have_factor = false;
  return MDS_OK;
}

int mds_set_nlp(mds_handle *h, const mds_nlp_model *model) {
  TRY(check_ready(h));
  const mds_dims &d = h->dims;
  const int nd = d.n_d, ns = d.n_s, m = d.m;
  const int64_t nnz = d.nnz_s;
  if (!model) {
    if (h->nlp_on) {
      // back to the quadratic problem: its values and J_s's column copy
      h->P = h->Pq;
      launch_csc_build(S(h), m, ns, nnz, h->P.Js_rowptr, h->P.Js_col, h->P.Js_val, h->w.csc_ptr,
                       h->w.csc_row, h->w.csc_val, h->w.csc_fill);
      HIPCHK(hipGetLastError());
      HIPCHK(hipStreamSynchronize(S(h)));
    }
    h->nlp_on = false;
    h->ipm_ready = h->have_M = h->have_factor = false;
    return MDS_OK;
  }
  if (!h->nlp_room) return set_err(h, MDS_ESTATE, "the workspace was created without options.nlp");
  if (!model->objective || !model->gradient || !model->constraints || !model->jacobian ||
      !model->hessian)
    return set_err(h, MDS_ENULL, "model callback missing");
  if (h->sb.nblk > 0) return set_err(h, MDS_ESTATE, "coupling blocks are set");
  if (!h->nlp_on) h->Pq = h->P;
  const mds_problem &Q = h->Pq;
  // the model's values start as the quadratic problem's
  vec_copy(S(h), (int64_t)nd * nd, Q.H, h->nlp_H);
  vec_copy(S(h), (int64_t)m * nd, Q.J_d, h->nlp_Jd);
  vec_copy(S(h), nnz, Q.Js_val, h->nlp_v);
  vec_copy(S(h), ns, Q.w, h->nlp_w);
  if (m > 0) HIPCHK(hipMemsetAsync(h->nlp_zero, 0, 8 * (size_t)m, S(h)));
  HIPCHK(hipGetLastError());
  // J_s's column copy takes the model's values through a map from each
  // column entry to its row-compressed entry
  if (nnz > 0) {
    std::vector<int32_t> cptr(ns + 1), crow(nnz), rp(m + 1), ci(nnz), map(nnz);
    HIPCHK(hipMemcpyAsync(cptr.data(), h->w.csc_ptr, 4 * (size_t)(ns + 1), hipMemcpyDeviceToHost,
                          S(h)));
    HIPCHK(hipMemcpyAsync(crow.data(), h->w.csc_row, 4 * (size_t)nnz, hipMemcpyDeviceToHost, S(h)));
    HIPCHK(hipMemcpyAsync(rp.data(), Q.Js_rowptr, 4 * (size_t)(m + 1), hipMemcpyDeviceToHost, S(h)));
    HIPCHK(hipMemcpyAsync(ci.data(), Q.Js_col, 4 * (size_t)nnz, hipMemcpyDeviceToHost, S(h)));
    HIPCHK(hipStreamSynchronize(S(h)));
    for (int j = 0; j < ns; ++j) {
      for (int32_t q = cptr[j]; q < cptr[j + 1]; ++q) {
        const int r = crow[q];
        const int32_t *b = ci.data() + rp[r], *e = ci.data() + rp[r + 1];
        const int32_t *f = std::lower_bound(b, e, j);
        if (f == e || *f != j) return set_err(h, MDS_EPATTERN, "J_s column copy out of step");
        map[q] = (int32_t)(f - ci.data());
      }
    }
    HIPCHK(hipMemcpyAsync(h->nlp_cmap, map.data(), 4 * (size_t)nnz, hipMemcpyHostToDevice, S(h)));
  }
  h->P.H = h->nlp_H;
  h->P.J_d = h->nlp_Jd;
  h->P.Js_val = h->nlp_v;
  h->P.w = h->nlp_w;
  h->P.b = h->nlp_zero;
  nlp_gather(S(h), nnz, h->nlp_cmap, h->nlp_v, h->w.csc_val);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(S(h)));
  h->nlp = *model;
  h->nlp_on = true;
  h->model_err = false;
  h->nlp_stats = mds_nlp_stats{};
  h->ipm_ready = h->have_M = h->have_factor = false;
  return MDS_OK;
}

int mds_get_nlp_stats(const mds_handle *h, mds_nlp_stats *out) {
  if (!h || !out) return MDS_ENULL;
  *out = h->nlp_stats;
  return MDS_OK;
}

int mds_set_m22_diag(mds_handle *h, const double *dcv) {
  TRY(check_ready(h));
  if (dcv && MM(h) > 0) {
    int32_t bad = 0;
    HIPCHK(hipMemsetAsync(h->w.flags, 0, 4, S(h)));
    check_nonneg(S(h), MM(h), dcv, h->w.flags);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(&bad, h->w.flags, 4, hipMemcpyDeviceToHost, S(h)));
    HIPCHK(hipStreamSynchronize(S(h)));
    if (bad) return set_err(h, MDS_EINVAL, "M22 diagonal: entries must be finite and nonnegative");
  }
  h->dcv_user = (MM(h) > 0) ? dcv : nullptr;
  h->have_M = false;
  h->have_factor = false;
  return MDS_OK;
}

int mds_factor_inertia(mds_handle *h, mds_reg *reg, double mu, mds_inertia *out_host) {
  TRY(check_ready(h));
  if (!out_host) return set_err(h, MDS_ENULL, "out_host is NULL");
  if (!reg) {
    if (!h->have_M) return set_err(h, MDS_ESTATE, "mds_condense must precede factorization");
    TRY(factor_impl(h, out_host));
    return out_host->info ? MDS_ZERO_PIVOT : MDS_OK;
  }
  if (!h->sigma_d && ND(h) > 0) return set_err(h, MDS_ESTATE, "mds_condense must precede factorization");
  if (!(mu >= 0.0)) return set_err(h, MDS_EINVAL, "mu must be nonnegative");
  return correct_impl(h, reg, mu, out_host);
}

int mds_solve(mds_handle *h, const double *r_d, const double *r_s, const double *r_y,
              double *dx_d, double *dx_s, double *dy) {
  TRY(check_ready(h));
  if (!h->have_factor) return set_err(h, MDS_ESTATE, "no factorization");
  if ((ND(h) > 0 && (!r_d || !dx_d)) || (NS(h) > 0 && (!r_s || !dx_s)) ||
      (MM(h) > 0 && (!r_y || !dy)))
    return set_err(h, MDS_ENULL, "vector missing");
  return solve_impl(h, r_d, r_s, r_y, dx_d, dx_s, dy);
}

int mds_refine(mds_handle *h, const double *r_d, const double *r_s, const double *r_y,
               double *dx_d, double *dx_s, double *dy, int32_t max_steps, double eta_tol,
               mds_refine_info *info_host) {
  TRY(check_ready(h));
  if (!h->have_factor) return set_err(h, MDS_ESTATE, "no factorization");
  if ((ND(h) > 0 && (!r_d || !dx_d)) || (NS(h) > 0 && (!r_s || !dx_s)) ||
      (MM(h) > 0 && (!r_y || !dy)))
    return set_err(h, MDS_ENULL, "vector missing");
  if (max_steps < 0) return set_err(h, MDS_EINVAL, "max_steps < 0");
  return refine_impl(h, r_d, r_s, r_y, dx_d, dx_s, dy, max_steps, eta_tol, info_host);
}

int mds_sigma_rhs(mds_handle *h, const double *x, const double *y, const double *zl,
                  const double *zu, double mu, double *sigma, double *r_x, double *r_y) {
  TRY(check_ready(h));
  if ((h->nx > 0 && (!x || !zl || !zu || !sigma || !r_x)) || (MM(h) > 0 && (!y || !r_y)))
    return set_err(h, MDS_ENULL, "vector missing");
  eval_grad_constr(h, x, y, r_y);
  ipm_sigma_rhs(S(h), h->nx, x, zl, zu, h->w.xl_e, h->w.xu_e, h->w.tn, h->w.tn2, mu, sigma, r_x);
  HIPCHK(hipGetLastError());
  return MDS_OK;
}

int mds_ftb(mds_handle *h, int64_t n, const double *v, const double *dv, double tau,
            double *alpha_host) {
  if (!h || !alpha_host) return MDS_ENULL;
  if (n < 0) return set_err(h, MDS_EDIMS, "n < 0");
  if (n > 0 && (!v || !dv)) return set_err(h, MDS_ENULL, "vector missing");
  if (n == 0) {
    *alpha_host = 1.0;
    return MDS_OK;
  }
  ipm_red_ftb1(S(h), n, v, dv, tau, h->w.red, h->w.scal);
  HIPCHK(hipGetLastError());
  double s[8];
  TRY(read_scal(h, s, 8));
  *alpha_host = -s[0];
  return MDS_OK;
}

int mds_opt_error(mds_handle *h, const double *x, const double *y, const double *zl,
                  const double *zu, double mu, double *E_host, double *parts_host) {
  TRY(check_ready(h));
  if (!E_host) return set_err(h, MDS_ENULL, "E_host is NULL");
  return opt_error_impl(h, x, y, zl, zu, mu, E_host, parts_host);
}

int mds_merit(mds_handle *h, const double *x, double mu, double *f_host, double *phi_host,
              double *theta_host) {
  TRY(check_ready(h));
  return merit_impl(h, x, mu, f_host, phi_host, theta_host);
}

}  // extern "C"

namespace {

// Slacks of the inequality rows at the start: the row values of J_h x pushed
// into [hl, hu] (x holds the start's variables).
void init_slacks(mds_handle *h, double *x) {
  if (h->mI <= 0) return;
  const int nd = ND(h), m = MM(h), n = h->n;
  const mds_problem &P = h->P;
  double *cx = h->w.tm;
  if (h->nlp_on) {
    // the model's row values at x
    if (h->nlp.constraints(h->nlp.ctx, x, cx) != 0) h->model_err = true;
    ipm_slack_project(S(h), h->mI, cx + h->mE, P.hl, P.hu, x + n);
    return;
  }
  if (nd > 0) {
    launch_gemv_n(S(h), m, nd, P.J_d, m, x, 0.0, cx);
    launch_spmv_csr(S(h), m, P.Js_rowptr, P.Js_col, P.Js_val, x + nd, 1.0, cx);
  } else {
    launch_spmv_csr(S(h), m, P.Js_rowptr, P.Js_col, P.Js_val, x + nd, 0.0, cx);
  }
  ipm_slack_project(S(h), h->mI, cx + h->mE, P.hl, P.hu, x + n);
}

// NLP mode, feasibility restoration (a reading of the phase Waechter and
// Biegler describe): from x_R = x, barrier steps of the problem
//   min zeta/2 ||D_R (x - x_R)||^2 - mu sum log(slacks)  s.t.  c(x) = 0,
// zeta = sqrt(mu), D_R = diag(min(1, 1 / |x_R|)), with the rows' curvature
// left out (a Gauss-Newton model) and the bound multipliers centred at
// mu / slack.  Each step is cut to the boundary fraction and halved until
// theta drops by 1e-4 alpha theta; the phase ends once theta <= 0.9
// theta(x_R) and the point is acceptable to the filter (at most 30 steps).
// *k receives the steps taken, or -1 when the phase failed.  y is kept; the
// phase's own multipliers live in nlp_yr.
int nlp_restore(mds_handle *h, double mu, double tau, int rsteps, double *x, double *zl,
                double *zu, int *k_out) {
  const int nd = ND(h), ns = NS(h), m = MM(h), n = h->nx;
  const double *xl = h->w.xl_e, *xu = h->w.xu_e;
  double *sig = h->w.sig, *rx = h->w.rx, *ry = h->w.ry, *ry2 = h->w.ry2, *dsb = h->w.dsb;
  double *dx = h->w.dx, *dy = h->w.dy, *dzl = h->w.dzl, *dzu = h->w.dzu, *xt = h->w.xt;
  double *xr = h->nlp_xr, *dr = h->nlp_dr, *yr = h->nlp_yr;
  const double zeta = std::sqrt(mu);
  *k_out = -1;
  nlp_resto_init(S(h), n, x, xr, dr);
  if (m > 0) HIPCHK(hipMemsetAsync(yr, 0, 8 * (size_t)m, S(h)));
  double thR = 0.0;
  TRY(merit_nlp(h, x, mu, nullptr, nullptr, &thR, nullptr));
  double dw_last = 0.0;
  // the condensation follows this phase's barrier diagonal
  h->sigma_d = sig;
  h->dsbase = dsb;
  h->sig_h = (h->mI > 0) ? sig + h->n : nullptr;
  struct SigReset {
    mds_handle *h;
    ~SigReset() { h->sig_h = nullptr; }
  } reset{h};
  for (int k = 0; k < 30; ++k) {
    double th = 0.0;
    TRY(merit_nlp(h, x, mu, nullptr, nullptr, &th, nullptr));
    if (k > 0 && th <= 0.9 * thR) {
      double ph = 0.0;
      TRY(merit_nlp(h, x, mu, nullptr, &ph, &th, nullptr));
      bool infilt = !(std::isfinite(th) && std::isfinite(ph)) || th >= h->theta_max;
      for (size_t f = 0; f < h->filter.size() && !infilt; ++f)
        if (th >= h->filter[f].first && ph >= h->filter[f].second) infilt = true;
      if (!infilt) {
        nlp_center_z(S(h), n, mu, x, xl, xu, zl, zu);
        HIPCHK(hipGetLastError());
        *k_out = k;
        return MDS_OK;
      }
    }
    TRY(nlp_jacobian(h, x));
    // proximal Hessian zeta D_R^2, no row curvature
    nlp_resto_hess(S(h), nd, ns, zeta, dr, h->nlp_H, h->nlp_w);
    // J' y_R into w.tn2 and -c(x) into ry
    eval_grad_constr(h, x, yr, ry);
    TRY(nlp_model_ok(h));
    nlp_resto_rhs(S(h), n, zeta, mu, x, xr, dr, h->w.tn2, xl, xu, sig, rx, zl, zu);
    ipm_dsbase(S(h), nd, ns, h->nlp_w, sig, dsb);
    HIPCHK(hipGetLastError());
    mds_reg reg{};
    reg.delta_w_last = dw_last;
    reg.delta_w_max = 1e20;
    mds_inertia in{};
    const int fst = correct_impl(h, &reg, mu, &in);
    if (fst < 0) return fst;
    if (fst == MDS_INERTIA_FAIL) return MDS_OK;
    dw_last = reg.delta_w_last;
    vec_copy(S(h), m, ry, ry2);
    ipm_ineq_rhs(S(h), h->mI, h->mE, h->w.dcv, rx + h->n, ry2);
    mds_refine_info ri{};
    const int rst = refine_impl(h, rx, rx + nd, ry2, dx, dx + nd, dy, rsteps, 1e-14, &ri);
    if (rst < 0) return rst;
    ipm_ineq_step(S(h), h->mI, h->mE, h->w.dcv, rx + h->n, dy, dx + h->n);
    ipm_red_ftb(S(h), n, x, xl, xu, dx, zl, zu, dzl, dzu, tau, h->w.red, h->w.scal);
    HIPCHK(hipGetLastError());
    double sf[8];
    TRY(read_scal(h, sf, 8));
    double a = -sf[0];
    for (;;) {
      ipm_axpy_to(S(h), n, x, dx, a, xt);
      double tht = 0.0;
      TRY(merit_nlp(h, xt, mu, nullptr, nullptr, &tht, nullptr));
      if (std::isfinite(tht) && tht <= (1.0 - 1e-4 * a) * th) break;
      a = 0.5 * a;
      if (a < 1e-12) return MDS_OK;
    }
    vec_copy(S(h), n, xt, x);
    nlp_axpby(S(h), m, a, dy, yr, yr);
    HIPCHK(hipGetLastError());
  }
  return MDS_OK;
}

int ipm_opts_check(mds_handle *h, mds_iterate *it) {
  if (!it || (h->nx > 0 && (!it->x || !it->zl || !it->zu)) || (MM(h) > 0 && !it->y))
    return set_err(h, MDS_ENULL, "iterate missing");
  if (h->dcv_user)
    return set_err(h, MDS_ESTATE,
                   "a caller's M22 diagonal is set: the IPM forms that block from its slacks");
  return MDS_OK;
}

}  // namespace

extern "C" {

int mds_ipm_init(mds_handle *h, mds_iterate *it, const mds_ipm_opts *opts) {
  TRY(check_ready(h));
  TRY(ipm_opts_check(h, it));
  h->model_err = false;
  h->nlp_stats = mds_nlp_stats{};
  mds_ipm_opts o{1e-8, 0.1, 200, 2, 1e20, 0, 0};
  if (opts) o = *opts;
  h->ipm = o;
  ipm_init_point(S(h), h->nx, MM(h), h->w.xl_e, h->w.xu_e, it->x, it->y, it->zl, it->zu);
  init_slacks(h, it->x);
  HIPCHK(hipGetLastError());
  TRY(nlp_model_ok(h));
  it->mu = o.mu0;
  it->tau = std::max(0.99, 1.0 - it->mu);
  it->iter = 0;
  h->dw_last = 0.0;
  h->filter.clear();
  double th0 = 0.0;
  TRY(merit_impl(h, it->x, it->mu, nullptr, nullptr, &th0));
  h->theta_max = 1e4 * std::max(1.0, th0);
  h->theta_min = 1e-4 * std::max(1.0, th0);
  h->ipm_ready = true;
  return MDS_OK;
}

int mds_ipm_init_warm(mds_handle *h, mds_iterate *it, const mds_ipm_opts *opts,
                      const double *x_d0, const double *y0, double mu0) {
  TRY(check_ready(h));
  TRY(ipm_opts_check(h, it));
  if ((ND(h) > 0 && !x_d0) || (MM(h) > 0 && !y0)) return set_err(h, MDS_ENULL, "start point missing");
  if (!(mu0 > 0.0) || !std::isfinite(mu0)) return set_err(h, MDS_EINVAL, "mu0 must be positive");
  if (h->sb.nblk > 0)
    return set_err(h, MDS_ESTATE, "the warm start completes x_s for a diagonal sparse Hessian "
                                  "(coupling blocks are set)");
  if (h->nlp_on) return set_err(h, MDS_ESTATE, "the warm start is for the quadratic problem");
  mds_ipm_opts o{1e-8, 0.1, 200, 2, 1e20, 0, 0};
  if (opts) o = *opts;
  h->ipm = o;
  // the slacks' entries first take the cold start's values (multipliers
  // mu0 / slack below), then the variables' warm values and the slacks
  ipm_init_point(S(h), h->nx, 0, h->w.xl_e, h->w.xu_e, it->x, it->y, it->zl, it->zu);
  ipm_init_warm(S(h), ND(h), NS(h), MM(h), h->P.xl, h->P.xu, h->P.w, h->P.g, h->w.csc_ptr,
                h->w.csc_row, h->w.csc_val, x_d0, y0, mu0, it->x, it->y, it->zl, it->zu);
  init_slacks(h, it->x);
  ipm_slack_duals(S(h), h->mI, h->w.xl_e + h->n, h->w.xu_e + h->n, it->x + h->n, mu0,
                  it->zl + h->n, it->zu + h->n);
  eval_grad_constr(h, it->x, MM(h) > 0 ? it->y : nullptr, nullptr);
  if (MM(h) == 0 && h->n > 0) HIPCHK(hipMemsetAsync(h->w.tn2, 0, 8 * (size_t)h->n, S(h)));
  ipm_warm_duals(S(h), h->nx, h->w.xl_e, h->w.xu_e, h->w.tn, h->w.tn2, it->zl, it->zu);
  HIPCHK(hipGetLastError());
  it->mu = mu0;
  it->tau = std::max(0.99, 1.0 - it->mu);
  it->iter = 0;
  h->dw_last = 0.0;
  h->filter.clear();
  double th0 = 0.0;
  TRY(merit_impl(h, it->x, it->mu, nullptr, nullptr, &th0));
  h->theta_max = 1e4 * std::max(1.0, th0);
  h->theta_min = 1e-4 * std::max(1.0, th0);
  h->ipm_ready = true;
  return MDS_OK;
}

// sync_end: wait for the iterate update before returning (mds_ipm_step);
// mds_ipm_solve leaves it stream-ordered between its own steps.
static int ipm_step_impl(mds_handle *h, mds_iterate *it, mds_step_info *info, bool sync_end) {
  TRY(check_ready(h));
  if (!h->ipm_ready) return set_err(h, MDS_ESTATE, "mds_ipm_init must precede mds_ipm_step");
  if (!it) return set_err(h, MDS_ENULL, "iterate missing");
  // Waechter & Biegler (2006) defaults
  const double tau_min = 0.99, kappa_eps = 10.0, kappa_mu = 0.2, theta_mu = 1.5;
  const double gamma_theta = 1e-5, gamma_phi = 1e-8, delta = 1.0, s_theta = 1.1, s_phi = 2.3;
  const double eta_phi = 1e-8, gamma_alpha = 0.05;
  const int nd = ND(h), ns = NS(h), m = MM(h), n = h->nx;  // n: variables + slacks
  const mds_problem &P = h->P;
  const double *xl = h->w.xl_e, *xu = h->w.xu_e;
  mds_step_info loc{};
  mds_step_info &I = info ? *info : loc;
  memset(&I, 0, sizeof(I));
  double *x = it->x, *y = it->y, *zl = it->zl, *zu = it->zu;
  double mu = it->mu, tau = it->tau;

  I.mu = mu;
  if (it->iter >= h->ipm.max_iter) return I.status = MDS_IPM_MAXITER;
  const bool nlp = h->nlp_on;
  if (nlp) TRY(nlp_jacobian(h, x));
  double E0 = 0.0, Emu0 = 0.0;  // E_0 and E_mu at the incoming mu, one pass
  TRY(opt_error_pair(h, x, y, zl, zu, mu, &E0, &Emu0));
  if (nlp) TRY(nlp_model_ok(h));
  I.E0 = E0;
  if (!std::isfinite(E0)) return I.status = MDS_IPM_NONFINITE;
  if (E0 <= h->ipm.tol) return I.status = MDS_IPM_CONVERGED;
  // barrier update while the barrier subproblem is solved to kappa_eps * mu
  for (bool first = true;; first = false) {
    double Emu = Emu0;
    if (!first) TRY(opt_error_impl(h, x, y, zl, zu, mu, &Emu, nullptr));
    if (!(Emu <= kappa_eps * mu)) break;
    const double mnew = std::max(h->ipm.tol / 10.0, std::min(kappa_mu * mu, std::pow(mu, theta_mu)));
    if (!(mnew < mu)) break;
    mu = mnew;
    tau = std::max(tau_min, 1.0 - mu);
    h->filter.clear();
  }
  I.mu = mu;
  if (nlp) {
    // the Lagrangian's Hessian at (x, y); its sparse block must stay >= 0
    if (h->nlp.hessian(h->nlp.ctx, x, y, h->nlp_H, h->nlp_w) != 0)
      return set_err(h, MDS_EMODEL, "model Hessian failed");
    HIPCHK(hipMemsetAsync(h->w.flags, 0, 4, S(h)));
    nlp_check_nonneg(S(h), ns, h->nlp_w, h->w.flags);
    HIPCHK(hipGetLastError());
    int32_t bad = 0;
    HIPCHK(hipMemcpyAsync(&bad, h->w.flags, 4, hipMemcpyDeviceToHost, S(h)));
    HIPCHK(hipStreamSynchronize(S(h)));
    if (bad) {
      it->mu = mu;
      it->tau = tau;
      I.status = MDS_EDS_NONPOS;
      return set_err(h, MDS_EDS_NONPOS, "the model's sparse Hessian w has a negative entry");
    }
  }
  // Newton system with inertia correction and refinement.  With inequality
  // rows the slack step is eliminated: their (4,4) diagonal is
  // 1 / (Sigma_h + dw) (formed by every condensation of the correction loop)
  // and their rhs gains dcv .* r_d.
  double *sig = h->w.sig, *rx = h->w.rx, *ry = h->w.ry, *ry2 = h->w.ry2, *dsb = h->w.dsb;
  double *dx = h->w.dx, *dy = h->w.dy, *dzl = h->w.dzl, *dzu = h->w.dzu, *xt = h->w.xt;
  TRY(mds_sigma_rhs(h, x, y, zl, zu, mu, sig, rx, ry));
  if (nlp) TRY(nlp_model_ok(h));
  ipm_dsbase(S(h), nd, ns, P.w, sig, dsb);
  h->sigma_d = sig;
  h->dsbase = dsb;
  h->sig_h = (h->mI > 0) ? sig + h->n : nullptr;
  const int64_t coop_aborts0 = h->n_coop_abort;
  const double dw_last0 = h->dw_last;
  mds_inertia in{};
  // correction loop, then the condensed solve refined on the full system
  auto newton = [&](int rsteps, mds_refine_info *ri) -> int {
    mds_reg reg{};
    reg.delta_w_last = dw_last0;
    reg.delta_w_max = h->ipm.dw_max;
    const int fst = correct_impl(h, &reg, mu, &in);
    if (fst < 0) return fst;
    h->dw_last = reg.delta_w_last;
    I.delta_w = reg.delta_w;
    I.delta_c = reg.delta_c;
    I.inertia[0] = in.npos;
    I.inertia[1] = in.nzero;
    I.inertia[2] = in.nneg;
    I.trials += reg.trials;
    if (fst == MDS_INERTIA_FAIL) return fst;
    vec_copy(S(h), m, ry, ry2);
    ipm_ineq_rhs(S(h), h->mI, h->mE, h->w.dcv, rx + h->n, ry2);
    const int rst = refine_impl(h, rx, rx + nd, ry2, dx, dx + nd, dy, rsteps, 1e-14, ri);
    if (rst < 0) return rst;
    I.solves += 1 + ri->steps;
    return rst;
  };
  mds_refine_info ri{};
  // mixed precision: the refinement budget counts GMRES iterations
  const int rsteps = (h->precision == MDS_FP64) ? h->ipm.refine_steps
                     : (h->ipm.gmres_max > 0) ? h->ipm.gmres_max : 60;
  int rst = newton(rsteps, &ri);
  if (rst == MDS_REFINE_NOCONV && h->fac_lowprec) {
    // the low-precision factor did not precondition GMRES down to the
    // tolerance: redo this Newton system from an FP64 factorization
    h->force64 = true;
    rst = newton(h->ipm.refine_steps, &ri);
    h->force64 = false;
    h->n_fp64_refactor++;
    I.fallback |= 1;
  }
  h->sig_h = nullptr;
  if (h->n_coop_abort != coop_aborts0) I.fallback |= 2;
  if (rst < 0) return rst;
  if (rst == MDS_INERTIA_FAIL) return I.status = MDS_INERTIA_FAIL;
  I.eta = ri.eta;
  // slack step from the multiplier step: dd = dcv .* (r_d + dy_h)
  ipm_ineq_step(S(h), h->mI, h->mE, h->w.dcv, rx + h->n, dy, dx + h->n);
  // fraction to the boundary, grad(phi_mu)' dx and the merit values at x:
  // three reductions into separate records, read back together
  ipm_dz(S(h), n, x, zl, zu, xl, xu, dx, mu, dzl, dzu);
  ipm_red_ftb(S(h), n, x, xl, xu, dx, zl, zu, dzl, dzu, tau, h->w.red, h->w.scal);
  // grad f at x (the refinement used the scratch), read by the gphi reduction
  // before the merit products overwrite it
  eval_grad_constr(h, x, nullptr, nullptr);
  ipm_red_gphi(S(h), n, h->w.tn, x, xl, xu, dx, mu, h->w.red, h->w.scal + 8);
  if (nlp) {
    // the gradient pass left the rows' residual at x in w.tm: keep it for
    // the second-order correction
    vec_copy(S(h), m, h->w.tm, h->nlp_cx0);
    nlp_merit_launch(h, x, mu, h->w.scal + 16);
  } else {
    merit_launch(h, x, mu, h->w.scal + 16);
  }
  HIPCHK(hipGetLastError());
  double s24[24];
  TRY(read_scal(h, s24, 24));
  double fx = s24[16 + 4], fscale = 0.0;
  if (nlp) {
    TRY(nlp_model_ok(h));
    if (h->nlp.objective(h->nlp.ctx, x, &fx) != 0)
      return set_err(h, MDS_EMODEL, "model objective failed");
    fscale = std::fabs(fx);
  }
  const double a_pr = -s24[0], a_du = -s24[1];
  const double gphi = s24[8 + 4];
  const double ph = fx - mu * s24[16 + 5], th = s24[16 + 6];
  // tests that compare barrier values allow ten machine epsilons of phi's
  // rounding scale at x: near a solution the decrease they ask for falls
  // below the rounding error of phi itself
  const double ph_tol = 10.0 * DBL_EPSILON * (fscale + s24[16 + 7]);
  double amin;
  if (gphi < 0.0) {
    amin = std::min(gamma_theta, gamma_phi * th / (-gphi));
    if (th <= h->theta_min) amin = std::min(amin, delta * std::pow(th, s_theta) / std::pow(-gphi, s_phi));
    amin = gamma_alpha * amin;
  } else {
    amin = gamma_alpha * gamma_theta;
  }
  // the acceptance tests of a trial point (tht, pht) reached with step al
  auto acceptable = [&](double al, double tht, double pht, bool *aug) -> bool {
    const bool ok = std::isfinite(tht) && std::isfinite(pht);
    bool infilt = !ok || tht >= h->theta_max;
    for (size_t f = 0; f < h->filter.size() && !infilt; ++f)
      if (tht >= h->filter[f].first && pht >= h->filter[f].second) infilt = true;
    if (infilt) return false;
    const bool sw = gphi < 0.0 && al * std::pow(-gphi, s_phi) > delta * std::pow(th, s_theta);
    const bool armijo = (pht - ph) - eta_phi * al * gphi <= ph_tol;
    bool acc = false;
    if (th <= h->theta_min && sw) {
      if (armijo) acc = true;
    } else if (tht <= (1.0 - gamma_theta) * th || (pht - ph) - (-gamma_phi * th) <= ph_tol) {
      acc = true;
    }
    if (acc) *aug = !(sw && armijo);
    return acc;
  };
  double alpha = a_pr;
  bool accepted = false, augment = true, soc = false;
  int nbt = 0;
  const double *xacc = xt;
  for (;;) {
    ipm_axpy_to(S(h), n, x, dx, alpha, xt);
    double tht = 0.0, pht = 0.0;
    TRY(merit_impl(h, xt, mu, nullptr, &pht, &tht));
    if (acceptable(alpha, tht, pht, &augment)) {
      accepted = true;
      break;
    }
    if (nlp && nbt == 0 && tht >= th) {
      // second-order correction of the first trial: re-solve the factored
      // system for the rows' right-hand side -c_soc, c_soc = alpha c(x) +
      // c(x_t) (the residual of the trial is in w.tm), then accumulate
      // c_soc = alpha_soc c_soc + c(x_soc) while theta keeps dropping
      const double kappa_soc = 0.99;
      double *dxs = h->nlp_dxs, *dys = h->nlp_dys, *xs = h->nlp_xs, *cs = h->nlp_csoc;
      nlp_axpby(S(h), m, alpha, h->nlp_cx0, h->w.tm, cs);
      double th_old = tht;
      for (int p = 0; p < 4; ++p) {
        h->nlp_stats.soc_trials++;
        nlp_axpby(S(h), m, -1.0, cs, h->nlp_zero, ry2);
        ipm_ineq_rhs(S(h), h->mI, h->mE, h->w.dcv, rx + h->n, ry2);
        mds_refine_info rs{};
        const int sst = refine_impl(h, rx, rx + nd, ry2, dxs, dxs + nd, dys, rsteps, 1e-14, &rs);
        if (sst < 0) return sst;
        I.solves += 1 + rs.steps;
        ipm_ineq_step(S(h), h->mI, h->mE, h->w.dcv, rx + h->n, dys, dxs + h->n);
        // primal fraction to the boundary along dxs (slot 0)
        ipm_red_ftb(S(h), n, x, xl, xu, dxs, zl, zu, dzl, dzu, tau, h->w.red, h->w.scal);
        HIPCHK(hipGetLastError());
        double sf[8];
        TRY(read_scal(h, sf, 8));
        const double a_soc = -sf[0];
        ipm_axpy_to(S(h), n, x, dxs, a_soc, xs);
        double ths = 0.0, phs = 0.0;
        TRY(merit_nlp(h, xs, mu, nullptr, &phs, &ths, nullptr));
        if (acceptable(alpha, ths, phs, &augment)) {
          accepted = soc = true;
          xacc = xs;
          h->nlp_stats.soc_accepted++;
          break;
        }
        if (!(ths <= kappa_soc * th_old)) break;
        th_old = ths;
        nlp_axpby(S(h), m, a_soc, cs, h->w.tm, cs);
      }
      if (accepted) break;
    }
    alpha = 0.5 * alpha;
    nbt++;
    if (alpha < amin || (nlp && nbt >= 200)) break;
  }
  I.theta = th;
  I.phi = ph;
  I.alpha_pr = soc ? a_pr : alpha;
  I.alpha_du = a_du;
  I.backtracks = nbt;
  I.nlp_event = soc ? 1 : 0;
  const bool force = nlp && h->nlp_force_resto;
  if (nlp && (!accepted || force)) {
    // feasibility restoration; the iterate that enters it joins the filter
    h->nlp_force_resto = 0;
    h->filter.emplace_back((1.0 - gamma_theta) * th, ph - gamma_phi * th);
    int k = -1;
    TRY(nlp_restore(h, mu, tau, rsteps, x, zl, zu, &k));
    h->nlp_stats.resto_calls++;
    I.nlp_event = 2;
    it->mu = mu;
    it->tau = tau;
    if (k < 0) return I.status = MDS_IPM_LS_FAIL;
    h->nlp_stats.resto_iters += k;
    if (sync_end) HIPCHK(hipStreamSynchronize(S(h)));
    it->iter++;
    I.status = MDS_OK;
    return MDS_OK;
  }
  if (!accepted) {
    it->mu = mu;
    it->tau = tau;
    return I.status = MDS_IPM_LS_FAIL;
  }
  if (augment) h->filter.emplace_back((1.0 - gamma_theta) * th, ph - gamma_phi * th);
  ipm_accept(S(h), n, m, xacc, x, y, dy, zl, zu, dzl, dzu, xl, xu, soc ? a_pr : alpha, a_du, mu);
  HIPCHK(hipGetLastError());
  if (sync_end) HIPCHK(hipStreamSynchronize(S(h)));
  it->mu = mu;
  it->tau = tau;
  it->iter++;
  I.status = MDS_OK;
  return MDS_OK;
}

int mds_ipm_step(mds_handle *h, mds_iterate *it, mds_step_info *info) {
  return ipm_step_impl(h, it, info, true);
}

int mds_ipm_solve(mds_handle *h, mds_iterate *it, const mds_ipm_opts *opts,
                  mds_step_info *trace_host, int32_t trace_cap, int32_t *iters_host) {
  TRY(mds_ipm_init(h, it, opts));
  int st = MDS_OK;
  int rows = 0;
  for (;;) {
    mds_step_info info{};
    // the next step's first read-back orders it after this step's update
    st = ipm_step_impl(h, it, &info, false);
    if (trace_host && rows < trace_cap) trace_host[rows] = info;
    rows++;
    if (st != MDS_OK) break;
  }
  if (hipStreamSynchronize(S(h)) != hipSuccess) return set_err(h, MDS_EHIP, "stream sync failed");
  if (iters_host) *iters_host = it->iter;
  return st;
}

int mds_get_matrix(mds_handle *h, double *M_host) {
  if (!h || !M_host) return MDS_ENULL;
  const size_t N = h->N;
  HIPCHK(hipMemcpyAsync(M_host, h->w.M, 8 * N * N, hipMemcpyDeviceToHost, S(h)));
  HIPCHK(hipStreamSynchronize(S(h)));
  return MDS_OK;
}

int mds_get_factor(mds_handle *h, double *L_host, double *dd_host, double *ds_host,
                   int32_t *ipiv_host) {
  if (!h) return MDS_ENULL;
  if (!h->have_factor) return set_err(h, MDS_ESTATE, "no factorization");
  const int N = h->N;
  ensure_std(h);
  if (ipiv_host) HIPCHK(hipMemcpyAsync(ipiv_host, h->w.ipiv, 4 * (size_t)N, hipMemcpyDeviceToHost, S(h)));
  if (dd_host) HIPCHK(hipMemcpyAsync(dd_host, h->w.dd, 8 * (size_t)N, hipMemcpyDeviceToHost, S(h)));
  if (ds_host) HIPCHK(hipMemcpyAsync(ds_host, h->w.ds, 8 * (size_t)N, hipMemcpyDeviceToHost, S(h)));
  if (L_host)
    HIPCHK(hipMemcpyAsync(L_host, h->w.M, 8 * (size_t)N * N, hipMemcpyDeviceToHost, S(h)));
  HIPCHK(hipStreamSynchronize(S(h)));
  if (L_host)  // keep the strictly lower part only
    for (int c = 0; c < N; ++c)
      for (int i = 0; i <= c; ++i) L_host[(size_t)i + (size_t)c * N] = 0.0;
  return MDS_OK;
}

int mds_get_pivots(mds_handle *h, int32_t *ipiv_host) {
  if (!h || !ipiv_host) return MDS_ENULL;
  if (!h->have_factor) return set_err(h, MDS_ESTATE, "no factorization");
  HIPCHK(hipMemcpyAsync(ipiv_host, h->w.ipiv, 4 * (size_t)h->N, hipMemcpyDeviceToHost, S(h)));
  HIPCHK(hipStreamSynchronize(S(h)));
  return MDS_OK;
}

int mds_get_inv_ds(mds_handle *h, double *inv_d_host) {
  if (!h || !inv_d_host) return MDS_ENULL;
  HIPCHK(hipMemcpyAsync(inv_d_host, h->w.inv_d, 8 * (size_t)NS(h), hipMemcpyDeviceToHost, S(h)));
  HIPCHK(hipStreamSynchronize(S(h)));
  return MDS_OK;
}

int mds_get_info(const mds_handle *h, mds_info *out) {
  if (!h || !out) return MDS_ENULL;
  out->nb = h->nb;
  // fewest columns a panel factors, the last panel aside (the register
  // tail's 16-column tile factors 15)
  int mw = h->adv;
  for (size_t b = 0; b + 1 < h->plan.size(); ++b)
    mw = (int)std::min<long>(mw, h->plan[b].rows - h->plan[b].rows_after);
  out->min_width = mw;
  out->panel = h->panel_lds ? 3 : h->panel_coop ? 2 : h->panel_reg ? 0 : 1;
  out->precision = h->precision;
  out->panel_threads = (h->panel_reg || h->panel_lds) ? h->panel_threads : 1024;
  out->lookahead_cus = h->la_cus;
  out->workspace_bytes = (int64_t)h->ws_bytes;
  return MDS_OK;
}

int mds_get_panel_stats(mds_handle *h, mds_panel_stats *out) {
  if (!h || !out) return MDS_ENULL;
  FacState st{};
  HIPCHK(hipMemcpyAsync(&st, h->w.fst, sizeof(st), hipMemcpyDeviceToHost, S(h)));
  HIPCHK(hipStreamSynchronize(S(h)));
  out->panels = st.npanel;
  out->coop_steps = st.csteps;
  out->coop_second = st.cx3;
  out->n2x2 = st.n2x2;
  return MDS_OK;
}

int mds_probe_exchange(mds_handle *h, int32_t P, int32_t rounds, int32_t words,
                       double *us_per_round_host) {
  if (!h || !us_per_round_host) return MDS_ENULL;
  if (rounds < 1 || rounds > (1 << 20)) return set_err(h, MDS_EINVAL, "rounds must be in [1, 2^20]");
  int32_t *err = h->w.flags + 15;
  uint64_t *out = reinterpret_cast<uint64_t *>(h->w.scal);
  HIPCHK(hipMemsetAsync(err, 0, 4, S(h)));
  if (bk_xch_probe(S(h), P, rounds, words, h->w.xch, err, out) != 0)
    return set_err(h, MDS_EINVAL, "P in [1, 32], words in [1, 512], P * words <= 2048");
  HIPCHK(hipGetLastError());
  int32_t e = 0;
  uint64_t ticks = 0;
  HIPCHK(hipMemcpyAsync(&e, err, 4, hipMemcpyDeviceToHost, S(h)));
  HIPCHK(hipMemcpyAsync(&ticks, out, 8, hipMemcpyDeviceToHost, S(h)));
  HIPCHK(hipStreamSynchronize(S(h)));
  if (e) return set_err(h, MDS_EHIP, "an exchange wait expired (workgroups not co-resident)");
  *us_per_round_host = (double)ticks / 100.0 / (double)rounds;  // 100 MHz wall clock
  return MDS_OK;
}

int mds_get_fallbacks(const mds_handle *h, mds_fallbacks *out) {
  if (!h || !out) return MDS_ENULL;
  out->coop_aborts = h->n_coop_abort;
  out->fp64_refactors = h->n_fp64_refactor;
  return MDS_OK;
}

int mds_set_debug(mds_handle *h, int32_t flags) {
  if (!h) return MDS_ENULL;
  if (flags & ~(int32_t)(MDS_DEBUG_COOP_ABORT | MDS_DEBUG_FORCE_RESTO))
    return set_err(h, MDS_EINVAL, "unknown debug flag");
  h->nlp_force_resto = (flags & MDS_DEBUG_FORCE_RESTO) ? 1 : 0;
  const int32_t force = (flags & MDS_DEBUG_COOP_ABORT) ? 1 : 0;
  // FacState::xforce, read by every cooperative panel launch
  HIPCHK(hipMemcpyAsync((char *)h->w.fst + offsetof(FacState, xforce), &force, sizeof(force),
                        hipMemcpyHostToDevice, S(h)));
  HIPCHK(hipStreamSynchronize(S(h)));
  return MDS_OK;
}

int mds_set_timing(mds_handle *h, int enable) {
  if (!h) return MDS_ENULL;
  if (resolve_timings(h) != MDS_OK) return set_err(h, MDS_EHIP, "event synchronization failed");
  h->timing = enable != 0;
  for (int c = 0; c < MDS_T_CLASSES; ++c) {
    h->t_ms[c] = 0.0;
    h->t_n[c] = 0;
  }
  return MDS_OK;
}

int mds_get_timings(mds_handle *h, mds_timings *out) {
  if (!h || !out) return MDS_ENULL;
  if (resolve_timings(h) != MDS_OK) return set_err(h, MDS_EHIP, "event synchronization failed");
  for (int c = 0; c < MDS_T_CLASSES; ++c) {
    out->ms[c] = h->t_ms[c];
    out->launches[c] = h->t_n[c];
  }
  return MDS_OK;
}

const char *mds_status_string(int s) {
  switch (s) {
    case MDS_OK: return "ok";
    case MDS_EINVAL: return "invalid argument";
    case MDS_ENULL: return "null pointer";
    case MDS_EDIMS: return "invalid dimensions";
    case MDS_EWORKSPACE: return "workspace too small or misaligned";
    case MDS_ESTATE: return "call order violated";
    case MDS_EHIP: return "HIP runtime error";
    case MDS_ENONFINITE_INPUT: return "non-finite input";
    case MDS_EDS_NONPOS: return "nonpositive diagonal or invalid bounds";
    case MDS_EPATTERN: return "invalid sparsity pattern";
    case MDS_ZERO_PIVOT: return "zero pivot";
    case MDS_INERTIA_FAIL: return "inertia correction failed";
    case MDS_REFINE_NOCONV: return "refinement did not reach its tolerance";
    case MDS_IPM_CONVERGED: return "converged";
    case MDS_IPM_LS_FAIL: return "line search failed";
    case MDS_IPM_MAXITER: return "iteration limit";
    case MDS_IPM_NONFINITE: return "non-finite iterate";
    default: return "unknown status";
  }
}

const char *mds_last_error(const mds_handle *h) { return h ? h->err : "null handle"; }

}  // extern "C"
