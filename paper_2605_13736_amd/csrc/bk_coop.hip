// Cooperative register-resident Bunch-Kaufman panel (Sec. 2.3) for orders
// too large for one workgroup's registers: P workgroups (one per CU) each
// keep the multipliers of their own block of rows in registers and take the
// same pivot decisions from data exchanged once or twice per pivot.
//
// Workgroup g of T threads owns the physical rows
//   rho = k0 + g (T R) + t + T r,   t < T, r < R,
// of the buffer X (the trailing matrix in logical order at the panel start).
// Interchanges move logical positions, never data: pos[r] is the logical
// position of an owned row, and s_map (replicated in every workgroup) maps a
// logical position to its physical row, which addresses the un-updated
// columns of X.  Each pivot step is the one of the single-workgroup register
// panel, with its two workgroup-wide reductions widened to the grid:
//
//   X1 (every step): each workgroup publishes its largest off-diagonal
//      candidate of the updated column k (magnitude, position, signed value,
//      L row) and, when it owns them, the rows at positions k, k+1, k+2
//      (updated column-k value and L row).  Every workgroup reads all of it in
//      one round trip and derives colmax, imax, a_kk, the W row of imax and,
//      later, the L row of the next pivot.
//   X3 (when the first test fails): per-wave partial maxima of the updated
//      column imax, a_ii from its owner, and the column-imax values at
//      positions k, k+1, k+2.
//
// Exchange words are 64 bits: 32 data bits under a 32-bit tag that names the
// panel launch and the exchange, written and read with relaxed agent-scope
// atomics.  A reader accepts a word when its tag is the expected one, so no
// fence or flag orders the payload.  Two buffers (by exchange parity)
// suffice: a workgroup writes exchange e only after reading every
// workgroup's exchange e-1, which each of them published after reading e-2.
// Every wait is bounded by the wall clock; an expired wait sets FacState::xerr
// and the workgroups leave (later panels of the same factorization return at
// once), so the grid always drains.
#include <algorithm>
#include <climits>

#include "panel_reg.hpp"

namespace mds {
namespace {

using panel::amax_combine;
using panel::keep_branch;
using panel::lds_wave_sync;
using panel::sym_at;
using panel::w_lane;

constexpr int kCoopMaxN = 20480;  // LDS map of logical positions
constexpr unsigned long long kCoopWaitTicks = 1ull << 26;  // ~0.67 s of the 100 MHz clock

__device__ inline void put_u32(uint64_t *p, uint32_t v, uint32_t tag) {
  __hip_atomic_store(p, ((uint64_t)tag << 32) | (uint64_t)v, __ATOMIC_RELAXED,
                     __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void put_f64(uint64_t *p, double v, uint32_t tag) {
  const uint64_t b = (uint64_t)__double_as_longlong(v);
  put_u32(p, (uint32_t)(b >> 32), tag);
  put_u32(p + 1, (uint32_t)b, tag);
}
__device__ inline uint64_t get_w(const uint64_t *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline bool tag_ok(uint64_t w, uint32_t tag) { return (uint32_t)(w >> 32) == tag; }
__device__ inline double as_f64(uint64_t hi, uint64_t lo) {
  return __longlong_as_double((long long)(((hi & 0xffffffffull) << 32) | (lo & 0xffffffffull)));
}

// Look-ahead: entry (hi, lo) of the panel's input, hi and lo the larger and
// smaller of (rho, c), where the near update has not written it:
// X_prev[src(hi), src(lo)] - sum_t W(lo, t) L(hi, t), X_prev in the storage
// type TX (in FP32 the result is rounded to FP32, as the trailing update
// stores it).  The row's own L row (rho > c) or W row (rho <= c) meets the
// candidate c's W or L row, which the caller put in LDS (pw, pl: zero past
// jw, 40 entries).  Two rows per call (rows with on = false give 0), their
// loads in flight together.  Not inlined: its loads then take registers only
// while it runs, not in the pivot loop.
template <typename TX>
__device__ __attribute__((noinline)) double2 pending_entries(const TX *pX, const int32_t *psrc,
                                                             const double *pW, const double *pL,
                                                             int rho0, int rho1, bool on0, bool on1,
                                                             int c, int jw, int ld,
                                                             const double *pw, const double *pl) {
  const int rho[2] = {rho0, rho1};
  const bool on[2] = {on0, on1};
  double x[2], acc[2];
  const double *row[2], *bc[2];
#pragma unroll
  for (int r = 0; r < 2; ++r) {
    const int hi = max(rho[r], c), lo = min(rho[r], c);
    const int a = on[r] ? psrc[hi] : 0, b = on[r] ? psrc[lo] : 0;
    const int q = (a >= b) ? a + b * ld : b + a * ld;
    x[r] = on[r] ? (double)pX[q] : 0.0;
    row[r] = (rho[r] > c) ? pL : pW;
    bc[r] = (rho[r] > c) ? pw : pl;
    acc[r] = 0.0;
  }
  for (int t0 = 0; t0 < jw; t0 += 8) {
    double v[2][8];
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
      for (int u = 0; u < 8; ++u) v[r][u] = (on[r] && t0 + u < jw) ? row[r][rho[r] + (t0 + u) * ld] : 0.0;
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
      for (int u = 0; u < 8; ++u) acc[r] = fma(v[r][u], bc[r][t0 + u], acc[r]);
  }
  return double2{(double)(TX)(x[0] - acc[0]), (double)(TX)(x[1] - acc[1])};
}

template <int T, int R, int NB, int PMAX, typename TX, bool LA>
__global__ __launch_bounds__(T) void k_bk_panel_coop(int N, int nb, double alpha, int Pmax,
                                                     const TX *__restrict__ X,
                                                     const PanelPrev pv,
                                                     double *__restrict__ Lout,
                                                     int32_t *__restrict__ src_out,
                                                     double *__restrict__ W,
                                                     double *__restrict__ dd,
                                                     double *__restrict__ ds,
                                                     int32_t *__restrict__ ipiv,
                                                     int32_t *__restrict__ blk, FacState *st,
                                                     int32_t *__restrict__ panel_k0,
                                                     uint64_t *__restrict__ xch, int lstage) {
  constexpr int NWV = T / 64;
  constexpr int RW = T * R;
  constexpr int NR = NB + 1;          // row record: value + L row
  constexpr int PREC = 2 * NR;        // words of a row record
  constexpr int X1_CAND = 3;          // [0] position, [1,2] magnitude, then the row record
  constexpr int X1_POS = X1_CAND + PREC;
  constexpr int X3_AII = 2 * NWV;     // after the per-wave partial maxima
  constexpr int X3_POS = X3_AII + 2;
  // waves that read the first exchange: all of them on the wide grids
  constexpr int XW = (PMAX >= 12) ? NWV : 1;
  constexpr int U1 = ((PMAX + 3) * NR + 64 * XW - 1) / (64 * XW);  // row-record pairs per lane
  constexpr int U3 = (PMAX * NWV + 63) / 64;       // partial maxima per lane
  static_assert(NB % 8 == 0 && NR <= 64 && NWV <= 64, "tile");
  static_assert(X1_POS + 3 * PREC <= kCoopSlotWords && X3_POS + 6 <= kCoopSlotWords, "slot");

  __shared__ double s_wk[NB], s_wi[NB], s_cA[NB], s_cB[NB], s_cC[NB], s_nrow[NB];
  __shared__ double s_acur[R * T], s_wkc[R * T], s_wic[R * T];
  __shared__ int s_map[kCoopMaxN];
  __shared__ double s_cv[NWV];
  __shared__ int s_ci[NWV];
  __shared__ double s_crow[NWV][NR];  // wave candidates: signed value + L row
  __shared__ double s_prow[3][NR];    // owned rows at positions k, k+1, k+2
  __shared__ double s_xb[PMAX + 3][NR];  // X1: candidate rows, then position rows
  __shared__ double s_xwic[3];
  __shared__ double s_colmax, s_rowmax, s_aii;
  __shared__ int s_imax, s_gw, s_k0, s_abort, s_force;
  __shared__ int s_xok[2][NWV];  // X1 poll: bit 0 all tags seen, bit 1 wait expired
  __shared__ uint32_t s_tag0;
  __shared__ double s_pdd[NB], s_pds[NB];  // the panel's D and pivot records (written at its end)
  __shared__ int s_pip[NB], s_pbk[NB];
  __shared__ double s_pw[40], s_pl[40];  // look-ahead: W and L rows of the candidate
  __shared__ int s_jwp, s_kprev;         // ... and the previous panel's width and start

  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int g = blockIdx.x;
  if (tid == 0) {
    s_k0 = st->k;
    s_tag0 = st->xtag;
    s_abort = st->xerr;
    s_force = st->xforce;
    const int np = st->npanel;
    const bool pvon = pv.X != nullptr || pv.Xf != nullptr;
    s_kprev = (pvon && np > 0) ? panel_k0[np - 1] : 0;
    s_jwp = (pvon && np > 0) ? min(s_k0 - s_kprev, NB + 1) : 0;
  }
  if (tid < NB) {
    s_wk[tid] = 0.0;
    s_wi[tid] = 0.0;
    s_cA[tid] = 0.0;
    s_cB[tid] = 0.0;
    s_cC[tid] = 0.0;
  }
  __syncthreads();
  const int k0 = s_k0;
  if (k0 >= N || s_abort) return;
  if (s_force) {
    // host-set test flag: report an expired exchange wait without waiting
    if (tid == 0) __hip_atomic_store(&st->xerr, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return;
  }
  const int P = min(Pmax, (N - k0 + RW - 1) / RW);
  if (g >= P) return;
  const int ld = N;  // N <= 20480: every offset fits in 32 bits
  const int gbase = k0 + g * RW;
  // look-ahead: columns below kstrip are up to date in X; the previous
  // panel factored jwp columns
  const int kstrip = (k0 & pv.amask) + kNearCols, jwp = s_jwp;
  const bool la = LA && (pv.X != nullptr || pv.Xf != nullptr) && jwp > 0;
  const uint32_t tagb = ((s_tag0 % 0xffffffu) + 1u) << 8;
  auto slot = [&](int par, int wg) { return xch + (size_t)(par * kCoopMaxP + wg) * kCoopSlotWords; };
  auto owner = [&](int phys) { return (phys - k0) / RW; };

  double Lr[R][NB];
  // prefetched un-updated column values, kept in the storage type and
  // widened where used: a widening next to a conditional load would make the
  // compiler wait for the load there
  TX pre1[R], pre2[R];
  int pos[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
#pragma unroll
    for (int t = 0; t < NB; ++t) Lr[r][t] = 0.0;
    const int rho = gbase + tid + T * r;
    pos[r] = (rho < N) ? rho : -1;
    s_acur[r * T + tid] = (rho < N) ? (double)X[rho + k0 * ld] : 0.0;
    pre1[r] = pre2[r] = (TX)0;
  }
  for (int i = tid; i < N - k0; i += T) s_map[i] = k0 + i;
  __syncthreads();

  int k = k0, j = 0, c = 0;
  int c_pos = 0, c_zero = 0, c_neg = 0, c_2x2 = 0, first_zero = 0, nsteps = 0;
  int pj = -1;
  bool p2 = false;
  double pA0 = 0.0, pB0 = 0.0, pA1 = 0.0;

  while (j < nb - 1 && k < N) {
    ++nsteps;
    if (tid == 0 && pj >= 0) {
      s_cA[pj] = pA0;
      s_cB[pj] = pB0;
      if (p2) {
        s_cA[pj + 1] = pA1;
        s_cC[pj + 1] = pB0;
      }
    }
    // ---- updated column k, this workgroup's candidates ----------------------
    double a[R];
#pragma unroll
    for (int r = 0; r < R; ++r) a[r] = s_acur[r * T + tid];
#pragma unroll
    for (int t0 = 0; t0 < NB; t0 += 8) {
      if (t0 < j) {
        keep_branch();
        // columns t >= j: L = 0 and the W entries are zeros too (a W row
        // comes from an L row, which ends before column j), so their
        // products add an exact zero (no per-column branch or select)
        double wv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) wv[u] = s_wk[t0 + u];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
#pragma unroll
          for (int r = 0; r < R; ++r) a[r] = fma(-Lr[r][t0 + u], wv[u], a[r]);
        }
      }
    }
    // ---- prefetch the un-updated column k+1 (needed at the end of the step;
    //      issued after the column update's LDS reads so that no wait for
    //      older memory operations ahead of them includes it) ----------------
    {
      const int sc1 = (k + 1 < N) ? s_map[k + 1 - k0] : 0;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int rho = gbase + tid + T * r;
        if (pos[r] >= k && k + 1 < N) pre1[r] = sym_at(X, rho, sc1, ld);
      }
    }
    double bv = -1.0;
    int bi = INT_MAX, br = -1;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      if (pos[r] >= k) {
        s_wkc[r * T + tid] = a[r];
        if (pos[r] != k) {
          const double v = fabs(a[r]);
          if (v > bv || (v == bv && pos[r] < bi)) {
            bv = v;
            bi = pos[r];
            br = r;
          }
        }
        const int po = pos[r] - k;
        if (po <= 2) {
          keep_branch();
          s_prow[po][0] = a[r];
#pragma unroll
          for (int t = 0; t < NB; ++t) s_prow[po][1 + t] = Lr[r][t];
        }
      }
    }
    const int mybi = bi;
    wave::amax(bv, bi);
    if (lane == 0) {
      s_cv[wid] = bv;
      s_ci[wid] = bi;
    }
    if (mybi != INT_MAX && mybi == bi) {
      keep_branch();
#pragma unroll
      for (int r = 0; r < R; ++r) {
        if (br == r) {
          keep_branch();
          s_crow[wid][0] = a[r];
#pragma unroll
          for (int t = 0; t < NB; ++t) s_crow[wid][1 + t] = Lr[r][t];
        }
      }
    }
    __syncthreads();

    // ---- X1: publish (wave 0), then every wave reads its share ----------------
    const int par = c & 1;
    const uint32_t tag = tagb + (uint32_t)c;
    // owners of the rows at positions k, k+1, k+2 (-1: past N)
    const int o0 = owner(s_map[k - k0]);
    const int o1 = (k + 1 < N) ? owner(s_map[k + 1 - k0]) : -1;
    const int o2 = (k + 2 < N) ? owner(s_map[k + 2 - k0]) : -1;
    if (wid == 0) {
      double cv = -1.0;
      int ci = INT_MAX, cw = 0;
      if (lane < NWV) {
        cv = s_cv[lane];
        ci = s_ci[lane];
        cw = lane;
      }
      wave::amax(cv, ci, cw);  // every lane: lanes <= NB publish the winner's row
      uint64_t *mine = slot(par, g);
      if (lane == 0) {
        put_u32(mine, (uint32_t)ci, tag);
        put_f64(mine + 1, cv, tag);
      }
      if (lane < NR) put_f64(mine + X1_CAND + 2 * lane, s_crow[cw][lane], tag);
      if (lane < NR) {
        if (o0 == g) put_f64(mine + X1_POS + 2 * lane, s_prow[0][lane], tag);
        if (o1 == g) put_f64(mine + X1_POS + PREC + 2 * lane, s_prow[1][lane], tag);
        if (o2 == g) put_f64(mine + X1_POS + 2 * PREC + 2 * lane, s_prow[2][lane], tag);
      }
    }
    // One round trip reads all: the headers in wave 0's lanes < P, the row
    // records spread over the XW reading waves (pair p = lane + 64 (wid + XW
    // u): record p / NR, word p % NR).  Every lane issues every load (a lane
    // with nothing to read loads its own slot's first word and ignores it),
    // so the loads leave back to back and one wait covers them.  With one
    // reading wave its ballot decides; with all waves reading (the wide
    // grids, where one wave's U1 pairs next to its register tile would spill
    // to scratch) the waves agree through LDS after each poll
    // (double-buffered by poll parity): done when every wave saw all its
    // tags, time-out when any wave's wait expired.
    if (wid < XW) {
      const uint64_t *hp = slot(par, (wid == 0 && lane < P) ? lane : g);
      const uint64_t *ap[U1];
      bool need[U1];
#pragma unroll
      for (int u = 0; u < U1; ++u) {
        const int p = lane + 64 * (wid + XW * u), rec = p / NR, w = p % NR;
        const int ip = rec - P, op = (ip == 0) ? o0 : (ip == 1) ? o1 : o2;
        need[u] = rec < P || (ip < 3 && op >= 0);
        ap[u] = (rec < P) ? slot(par, rec) + X1_CAND + 2 * w
                : (ip < 3 && op >= 0) ? slot(par, op) + X1_POS + ip * PREC + 2 * w
                : slot(par, g);
      }
      const bool hneed = (wid == 0) && (lane < P);
      uint64_t h0, h1, h2, whi[U1], wlo[U1];
      const uint64_t t0 = wall_clock64();
      bool done = false;
      for (int it = 0;; ++it) {
        h0 = get_w(hp);
        h1 = get_w(hp + 1);
        h2 = get_w(hp + 2);
#pragma unroll
        for (int u = 0; u < U1; ++u) {
          whi[u] = get_w(ap[u]);
          wlo[u] = get_w(ap[u] + 1);
        }
        // branch-free checks: every load is consumed on every path, so no
        // later wait mistakes one of them for an outstanding one
        bool ok = (!hneed) | (tag_ok(h0, tag) & tag_ok(h1, tag) & tag_ok(h2, tag));
#pragma unroll
        for (int u = 0; u < U1; ++u) ok = ok & ((!need[u]) | (tag_ok(whi[u], tag) & tag_ok(wlo[u], tag)));
        const bool wok = __ballot(!ok) == 0;
        const bool expired = wall_clock64() - t0 > kCoopWaitTicks;
        if constexpr (XW == 1) {
          if (wok) {
            done = true;
            break;
          }
          if (expired) break;
        } else {
          if (lane == 0) s_xok[it & 1][wid] = (wok ? 1 : 0) | (expired ? 2 : 0);
          __syncthreads();
          int all = 1, any_exp = 0;
#pragma unroll
          for (int q = 0; q < XW; ++q) {
            const int v = s_xok[it & 1][q];
            all &= v;
            any_exp |= v >> 1;
          }
          if (all & 1) {
            done = true;
            break;
          }
          if (any_exp) break;
        }
      }
      if (!done) {
        if (tid == 0) {
          __hip_atomic_store(&st->xerr, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          s_abort = 1;
        }
      } else {
#pragma unroll
        for (int u = 0; u < U1; ++u) {
          const int p = lane + 64 * (wid + XW * u), rec = p / NR, w = p % NR;
          if (rec < P + 3) s_xb[rec][w] = need[u] ? as_f64(whi[u], wlo[u]) : 0.0;
        }
      }
      if constexpr (XW == 1) {
        lds_wave_sync();
      } else {
        __syncthreads();
      }
      if (!s_abort && wid == 0) {
        double gv = -1.0;
        int gi = INT_MAX, gw = 0;
        if (lane < P) {
          gv = as_f64(h1, h2);
          gi = (int)(uint32_t)h0;
          gw = lane;
        }
        wave::amax(gv, gi, gw);
        if (gv < 0.0) {
          gv = 0.0;
          gi = k;
        }
        // W row of imax from its L row (used when the first test fails)
        if (lane < NB)
          s_wi[lane] = w_lane<NB>(&s_xb[gw][1], s_cA, s_cB, s_cC, lane, 0, false, false, 0.0,
                                  0.0, 0.0);
        if (lane == 0) {
          s_colmax = gv;
          s_imax = gi;
          s_gw = gw;
        }
      }
    }
    __syncthreads();
    if (s_abort) return;
    ++c;
    const double colmax = s_colmax;
    const int imax = s_imax;
    const double akk = s_xb[P][0], absakk = fabs(akk);

    // ---- Bunch-Kaufman decision ----------------------------------------------
    int kind;  // 0 zero, 1 1x1, 2 1x1 (second test), 3 1x1 swap, 4 2x2
    int kstep = 1, q = k;
    double aii = 0.0, wki = 0.0;
    if (fmax(absakk, colmax) == 0.0 || isnan(absakk)) {
      kind = 0;
    } else if (absakk >= alpha * colmax) {
      kind = 1;
    } else {
      const int src_i = s_map[imax - k0];
      const int src_k2 = (k + 2 < N) ? s_map[k + 2 - k0] : 0;
      // look-ahead with the candidate past the strip: its entries in rows
      // past the strip still lack the previous panel's update (the column of
      // position k + 2 lies in the strip: every position up to k0 + nb holds
      // a physical row of the strip)
      const bool fly = la && src_i >= kstrip;
      // the previous panel's multipliers from column 0 (computed here, not
      // kept live through the pivot loop)
      const double *pL = pv.L + (pv.labs ? (size_t)s_kprev * (size_t)N : 0);
      if constexpr (LA) if (fly) {
        if (tid < 40) s_pw[tid] = (tid < jwp) ? pv.W[src_i + tid * ld] : 0.0;
        else if (tid >= 64 && tid < 104)
          s_pl[tid - 64] = (tid - 64 < jwp) ? pL[src_i + (tid - 64) * ld] : 0.0;
        __syncthreads();
      }
      double wic[R];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int rho = gbase + tid + T * r;
        wic[r] = 0.0;
        if (pos[r] >= k) {
          if (!fly || rho < kstrip) wic[r] = (double)sym_at(X, rho, src_i, ld);
          if (k + 2 < N) pre2[r] = sym_at(X, rho, src_k2, ld);
        }
      }
      if constexpr (LA) if (fly) {
        keep_branch();
        static_assert(R == 2, "two rows per call");
        const int rho0 = gbase + tid, rho1 = gbase + tid + T;
        const bool on0 = pos[0] >= k && rho0 >= kstrip, on1 = pos[1] >= k && rho1 >= kstrip;
        const TX *pX;
        if constexpr (sizeof(TX) == 8) pX = pv.X;
        else pX = pv.Xf;
        const double2 e = pending_entries<TX>(pX, pv.src, pv.W, pL, rho0, rho1, on0, on1, src_i,
                                              jwp, ld, s_pw, s_pl);
        if (on0) wic[0] = e.x;
        if (on1) wic[1] = e.y;
      }
#pragma unroll
      for (int t0 = 0; t0 < NB; t0 += 8) {
        if (t0 < j) {
          keep_branch();
          // columns t >= j: L = 0 and the W entries are zeros too, so
          // their products add an exact zero (no per-column select)
          double wv[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) wv[u] = s_wi[t0 + u];
#pragma unroll
          for (int u = 0; u < 8; ++u) {
#pragma unroll
            for (int r = 0; r < R; ++r) wic[r] = fma(-Lr[r][t0 + u], wv[u], wic[r]);
          }
        }
      }
      // ---- X3: partial maxima of the updated column imax -----------------------
      const int par = c & 1;
      const uint32_t tag = tagb + (uint32_t)c;
      uint64_t *mine = slot(par, g);
      double rv = 0.0;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        if (pos[r] >= k) {
          s_wic[r * T + tid] = wic[r];
          if (pos[r] == imax) put_f64(mine + X3_AII, wic[r], tag);
          else rv = fmax(rv, fabs(wic[r]));
          const int po = pos[r] - k;
          if (po <= 2) put_f64(mine + X3_POS + 2 * po, wic[r], tag);
        }
      }
      rv = wave::max(rv);
      if (lane == 0) put_f64(mine + 2 * wid, rv, tag);
      if (wid == 0) {
        const int oi = owner(src_i);
        // lane 1 + i < 4 reads the column-imax value at position k + i
        const int ol = (lane >= 1 && lane <= 3 && k + lane - 1 < N)
                           ? owner(s_map[k + lane - 1 - k0]) : -1;
        // unconditional loads (see X1): partial maxima, then lane 0: a_ii,
        // lanes 1..3: the column-imax values at positions k..k+2
        const uint64_t *pp[U3];
#pragma unroll
        for (int u = 0; u < U3; ++u) {
          const int p = lane + 64 * u;
          pp[u] = (p < P * NWV) ? slot(par, p / NWV) + 2 * (p % NWV) : slot(par, g);
        }
        const bool needa = (lane == 0) || (lane <= 3 && ol >= 0);
        const uint64_t *aq = (lane == 0) ? slot(par, oi) + X3_AII
                             : (lane <= 3 && ol >= 0) ? slot(par, ol) + X3_POS + 2 * (lane - 1)
                             : slot(par, g);
        uint64_t phi[U3], plo[U3], ahi, alo;
        const uint64_t t0 = wall_clock64();
        bool done = false;
        for (;;) {
#pragma unroll
          for (int u = 0; u < U3; ++u) {
            phi[u] = get_w(pp[u]);
            plo[u] = get_w(pp[u] + 1);
          }
          ahi = get_w(aq);
          alo = get_w(aq + 1);
          bool ok = (!needa) | (tag_ok(ahi, tag) & tag_ok(alo, tag));
#pragma unroll
          for (int u = 0; u < U3; ++u)
            ok = ok & ((lane + 64 * u >= P * NWV) | (tag_ok(phi[u], tag) & tag_ok(plo[u], tag)));
          if (__ballot(!ok) == 0) {
            done = true;
            break;
          }
          if (wall_clock64() - t0 > kCoopWaitTicks) break;
        }
        if (!done) {
          if (lane == 0) {
            __hip_atomic_store(&st->xerr, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            s_abort = 1;
          }
        } else {
          double m = 0.0;
#pragma unroll
          for (int u = 0; u < U3; ++u)
            if (lane + 64 * u < P * NWV) m = fmax(m, as_f64(phi[u], plo[u]));
          m = wave::max(m);
          if (lane == 0) {
            s_rowmax = m;
            s_aii = as_f64(ahi, alo);
          } else if (lane <= 3) {
            s_xwic[lane - 1] = needa ? as_f64(ahi, alo) : 0.0;
          }
        }
      }
      __syncthreads();
      if (s_abort) return;
      ++c;
      const double rowmax = s_rowmax;
      aii = s_aii;
      wki = s_xb[s_gw][0];
      if (absakk >= alpha * colmax * (colmax / rowmax)) {
        kind = 2;
      } else if (fabs(aii) >= alpha * rowmax) {
        kind = 3;
        q = imax;
      } else {
        kind = 4;
        q = imax;
        kstep = 2;
      }
    }
    const int p = k + kstep - 1;
    const bool sw = (q != p);
    const int kn = k + kstep;
    double Da = akk, Dc = 0.0, Db = 0.0, det = 1.0;
    if (kind == 3) Da = aii;
    const double Dw = (kind == 0) ? 0.0 : Da;
    if (kind == 4) {
      Db = wki;
      Dc = aii;
      det = Da * Dc - Db * Db;
    }
    const double rD = (kind == 4) ? 1.0 / det : (kind == 3) ? 1.0 / aii : 1.0 / akk;

    // ---- multipliers, new positions, next column ------------------------------
    double l0[R], l1[R];
    bool act[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int pr = pos[r];
      l1[r] = 0.0;
      if (kind == 4) {
        act[r] = pr >= k + 1 && pr != q;
        const double x0 = s_wkc[r * T + tid], y0 = s_wic[r * T + tid];
        l0[r] = (x0 * Dc - y0 * Db) * rD;
        l1[r] = (y0 * Da - x0 * Db) * rD;
      } else if (kind == 3) {
        act[r] = pr >= k && pr != q;
        l0[r] = s_wic[r * T + tid] * rD;
      } else {
        act[r] = pr > k;
        l0[r] = (kind == 0) ? 0.0 : s_wkc[r * T + tid] * rD;
      }
      int np = pr;
      if (sw) {
        if (pr == p) np = q;
        else if (pr == q) np = p;
      }
      pos[r] = np;
      double an = (double)pre1[r];
      if (kind == 3 && q == k + 1) an = s_acur[r * T + tid];
      if (kind == 4 && q != k + 2) an = (double)pre2[r];
      s_acur[r * T + tid] = an;
    }
    // the step's column(s) of the register tile (j is uniform: one scalar
    // compare per column, which every wave runs on the compute unit's shared
    // scalar unit; the 2x2 pivot's second column only on 2x2 steps)
#pragma unroll
    for (int t = 0; t < NB; ++t) {
      if (t == j) {
        keep_branch();
#pragma unroll
        for (int r = 0; r < R; ++r) Lr[r][t] = act[r] ? l0[r] : Lr[r][t];
      }
    }
    if (kind == 4) {
      keep_branch();
#pragma unroll
      for (int t = 1; t < NB; ++t) {
        if (t == j + 1) {
          keep_branch();
#pragma unroll
          for (int r = 0; r < R; ++r) Lr[r][t] = act[r] ? l1[r] : Lr[r][t];
        }
      }
    }

    // ---- W row of the next pivot, from the exchanged rows (wave 0) -------------
    if (wid == 0 && kn < N) {
      // the row at position kn came from position k + inx before the interchange
      const int inx = (kind == 4) ? ((q == k + 2) ? 1 : 2) : (kind == 3 && q == k + 1) ? 0 : 1;
      const double x0 = s_xb[P + inx][0], y0 = s_xwic[inx];
      double n0, n1 = 0.0;
      if (kind == 4) {
        n0 = (x0 * Dc - y0 * Db) * rD;
        n1 = (y0 * Da - x0 * Db) * rD;
      } else if (kind == 3) {
        n0 = y0 * rD;
      } else {
        n0 = (kind == 0) ? 0.0 : x0 * rD;
      }
      if (lane < NB) {
        double v = s_xb[P + inx][1 + lane];
        if (lane == j) v = n0;
        if (kind == 4 && lane == j + 1) v = n1;
        s_nrow[lane] = v;
      }
      lds_wave_sync();
      if (lane < NB)
        s_wk[lane] = w_lane<NB>(s_nrow, s_cA, s_cB, s_cC, lane, j, true, kind == 4,
                                (kind == 4) ? Da : Dw, Dc, Db);
    }

    // ---- pivot records and map -------------------------------------------------
    if (tid == 0) {
      if (sw) {
        const int t0 = s_map[p - k0];
        s_map[p - k0] = s_map[q - k0];
        s_map[q - k0] = t0;
      }
      // the pivot records go to global memory at the end of the panel: a
      // store here would make this wave wait for its prefetch of the next
      // column at the next write of the store's source registers
      if (kind == 4) {
        s_pdd[j] = Da;
        s_pdd[j + 1] = Dc;
        s_pds[j] = Db;
        s_pds[j + 1] = 0.0;
        s_pip[j] = -(q + 1);
        s_pip[j + 1] = -(q + 1);
        s_pbk[j] = 2;
        s_pbk[j + 1] = 3;
        c_pos++;
        c_neg++;
        c_2x2++;
      } else {
        s_pdd[j] = Da;
        s_pds[j] = 0.0;
        s_pip[j] = q + 1;
        s_pbk[j] = 1;
        if (Da > 0.0) c_pos++;
        else if (Da < 0.0) c_neg++;
        else {
          c_zero++;
          if (first_zero == 0) first_zero = k + 1;
        }
      }
    }
    pj = j;
    p2 = (kind == 4);
    pA0 = (kind == 4) ? Da : Dw;
    pB0 = Db;
    pA1 = Dc;
    j += kstep;
    k = kn;
    __syncthreads();
  }

  // ---- write the panel's multipliers and W = L D for the trailing rows ---------
  const int kend = k, jend = j;
  const int lcol = lstage ? 0 : k0;  // staged multipliers: column t at t N
  if (tid == 0 && pj >= 0) {
    s_cA[pj] = pA0;
    s_cB[pj] = pB0;
    if (p2) {
      s_cA[pj + 1] = pA1;
      s_cC[pj + 1] = pB0;
    }
  }
  __syncthreads();
  if (g == 0) {
    for (int t = tid; t < jend; t += T) {
      dd[k0 + t] = s_pdd[t];
      ds[k0 + t] = s_pds[t];
      ipiv[k0 + t] = s_pip[t];
      blk[k0 + t] = s_pbk[t];
    }
  }
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int pr = pos[r];
    if (pr < 0) continue;
    const int rho = gbase + tid + T * r;
#pragma unroll
    for (int t = 0; t < NB; ++t)
      if (t < jend && pr > k0 + t) Lout[pr + (lcol + t) * ld] = Lr[r][t];
    if (pr >= kend) {
#pragma unroll
      for (int t = 0; t < NB; ++t) {
        if (t < jend) {
          double v = Lr[r][t] * s_cA[t];
          if (t + 1 < NB) v = v + Lr[r][t + 1 < NB ? t + 1 : t] * s_cB[t];
          if (t >= 1) v = v + Lr[r][t >= 1 ? t - 1 : 0] * s_cC[t];
          W[pr + t * ld] = v;
        }
      }
      src_out[pr] = rho;
    }
  }
  if (g == 0 && tid == 0) {
    const int b = st->npanel;
    panel_k0[b + 1] = kend;
    st->npanel = b + 1;
    st->k = kend;
    st->npos += c_pos;
    st->nzero += c_zero;
    st->nneg += c_neg;
    st->n2x2 += c_2x2;
    if (st->info == 0 && first_zero != 0) st->info = first_zero;
    st->xtag = s_tag0 + 1u;
    // every step takes the first exchange; c counts both
    st->csteps += nsteps;
    st->cx3 += c - nsteps;
  }
}

// Exchange probe: P workgroups of T threads run `rounds` exchanges of the
// cooperative panel's kind with no other work.  In each round every
// workgroup's wave 0 publishes `words` tagged words; then all waves read every
// workgroup's words in one round trip (word q = thread + T u of the P *
// words), polling until every tag matches, and agree through LDS as the
// panel's first exchange does.  Tags are 1..255 in the low bits with zero
// launch bits, which no panel launch uses, so stale probe words are never
// taken for panel data.  out[0] = wall-clock ticks (100 MHz) of workgroup 0
// over all rounds; *err = 1 when a wait expired (every workgroup then
// leaves).
template <int T, int U>
__global__ __launch_bounds__(T) void k_xch_probe(int P, int rounds, int words,
                                                 uint64_t *__restrict__ xch,
                                                 int32_t *__restrict__ err,
                                                 uint64_t *__restrict__ out) {
  constexpr int NWV = T / 64;
  __shared__ int s_ok[2][NWV];
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6, g = blockIdx.x;
  auto slot = [&](int par, int wg) { return xch + (size_t)(par * kCoopMaxP + wg) * kCoopSlotWords; };
  const uint64_t t_start = wall_clock64();
  int it = 0;
  for (int e = 0; e < rounds; ++e) {
    const int par = e & 1;
    const uint32_t tag = (uint32_t)(e % 255) + 1u;
    uint64_t *mine = slot(par, g);
    if (wid == 0)
      for (int w = lane; w < words; w += 64) put_u32(mine + w, (uint32_t)(w + e), tag);
    const uint64_t *ap[U];
    bool need[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int q = tid + T * u, rec = q / words, w = q % words;
      need[u] = rec < P;
      ap[u] = need[u] ? slot(par, rec) + w : mine;
    }
    uint64_t v[U];
    const uint64_t t0 = wall_clock64();
    bool done = false;
    for (;; ++it) {
#pragma unroll
      for (int u = 0; u < U; ++u) v[u] = get_w(ap[u]);
      bool ok = true;
#pragma unroll
      for (int u = 0; u < U; ++u) ok = ok & ((!need[u]) | tag_ok(v[u], tag));
      const bool wok = __ballot(!ok) == 0;
      const bool expired = wall_clock64() - t0 > kCoopWaitTicks;
      if (lane == 0) s_ok[it & 1][wid] = (wok ? 1 : 0) | (expired ? 2 : 0);
      __syncthreads();
      int all = 1, any_exp = 0;
#pragma unroll
      for (int q = 0; q < NWV; ++q) {
        const int x = s_ok[it & 1][q];
        all &= x;
        any_exp |= x >> 1;
      }
      if (all & 1) {
        done = true;
        ++it;
        break;
      }
      if (any_exp) {
        ++it;
        break;
      }
    }
    if (!done) {
      if (tid == 0) __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return;
    }
  }
  if (g == 0 && tid == 0) out[0] = wall_clock64() - t_start;
}

// Variants: (threads, rows per thread, register tile, most workgroups)
constexpr int kCoopT = 512, kCoopR = 2, kCoopNB = 32;
constexpr int kCoopP = (kCoopMaxN + kCoopT * kCoopR - 1) / (kCoopT * kCoopR);

}  // namespace

int bk_coop_rows_per_wg() { return kCoopT * kCoopR; }

// Occupancy of the instantiation used at order N times the compute units must
// cover its workgroups: they spin on each other's exchange words.
bool bk_coop_resident(int N) {
  const int P = (N + kCoopT * kCoopR - 1) / (kCoopT * kCoopR);
  int dev = 0, cus = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  hipError_t e;
  if (P <= 4)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &per, k_bk_panel_coop<kCoopT, kCoopR, kCoopNB, 4, double, false>, kCoopT, 0);
  else if (P <= 8)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &per, k_bk_panel_coop<kCoopT, kCoopR, kCoopNB, 8, double, false>, kCoopT, 0);
  else if (P <= 12)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &per, k_bk_panel_coop<kCoopT, kCoopR, kCoopNB, 12, double, false>, kCoopT, 0);
  else
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &per, k_bk_panel_coop<kCoopT, kCoopR, kCoopNB, kCoopP, double, false>, kCoopT, 0);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return (long)per * cus >= P;
}
int bk_coop_nb() { return kCoopNB; }
int bk_coop_wgs(int N) { return (N + kCoopT * kCoopR - 1) / (kCoopT * kCoopR); }

// The exchange reads of X1 hold (PMAX + 3) (NB + 1) / 64 word pairs per lane
// in registers (every lane issues all of them on every poll), so the grid
// picks the smallest instantiation that covers the panel: `rows` bounds the
// rows left at the panel's start (every earlier panel factored at least
// nb - 1 columns), and with them its workgroups.
template <typename TX, bool LA>
static void panel_coop(hipStream_t s, int rows, int N, int nb, double alpha, const TX *X,
                       const PanelPrev &pv, double *Lout, int lstage, int32_t *src_out, double *W,
                       double *dd, double *ds, int32_t *ipiv, int32_t *blk, FacState *st,
                       int32_t *panel_k0, uint64_t *xch) {
  const int P = std::max(1, std::min(bk_coop_wgs(N), bk_coop_wgs(rows)));
#define MDS_COOP(PM_)                                                                  \
  k_bk_panel_coop<kCoopT, kCoopR, kCoopNB, PM_, TX, LA><<<P, kCoopT, 0, s>>>(          \
      N, nb, alpha, P, X, pv, Lout, src_out, W, dd, ds, ipiv, blk, st, panel_k0, xch, lstage)
  if (P <= 4) MDS_COOP(4);
  else if (P <= 8) MDS_COOP(8);
  else if (P <= 12) MDS_COOP(12);
  else MDS_COOP(kCoopP);
#undef MDS_COOP
}

int bk_xch_probe(hipStream_t s, int P, int rounds, int words, uint64_t *xch, int32_t *err,
                 uint64_t *out) {
  constexpr int U = 4;  // words read per thread: P * words <= 4 * 512
  if (P < 1 || P > kCoopMaxP || words < 1 || words > kCoopSlotWords || P * words > U * kCoopT ||
      rounds < 1)
    return -1;
  k_xch_probe<kCoopT, U><<<P, kCoopT, 0, s>>>(P, rounds, words, xch, err, out);
  return 0;
}

void launch_bk_panel_coop(hipStream_t s, int rows, int N, int nb, double alpha, const double *X,
                          double *Lout, int32_t *src_out, double *W, double *dd, double *ds,
                          int32_t *ipiv, int32_t *blk, FacState *st, int32_t *panel_k0,
                          uint64_t *xch) {
  panel_coop<double, false>(s, rows, N, nb, alpha, X, PanelPrev{}, Lout, 0, src_out, W, dd, ds,
                            ipiv, blk, st, panel_k0, xch);
}

void launch_bk_panel_coop(hipStream_t s, int rows, int N, int nb, double alpha, const float *X,
                          double *Lout, int32_t *src_out, double *W, double *dd, double *ds,
                          int32_t *ipiv, int32_t *blk, FacState *st, int32_t *panel_k0,
                          uint64_t *xch) {
  panel_coop<float, false>(s, rows, N, nb, alpha, X, PanelPrev{}, Lout, 0, src_out, W, dd, ds,
                           ipiv, blk, st, panel_k0, xch);
}

void launch_bk_panel_coop_la(hipStream_t s, int rows, int N, int nb, double alpha, const double *X,
                             const PanelPrev &pv, double *Lst, int32_t *src_out, double *W,
                             double *dd, double *ds, int32_t *ipiv, int32_t *blk, FacState *st,
                             int32_t *panel_k0, uint64_t *xch) {
  panel_coop<double, true>(s, rows, N, nb, alpha, X, pv, Lst, 1, src_out, W, dd, ds, ipiv, blk, st,
                           panel_k0, xch);
}

void launch_bk_panel_coop_la(hipStream_t s, int rows, int N, int nb, double alpha, const float *X,
                             const PanelPrev &pv, double *Lout, int32_t *src_out, double *W,
                             double *dd, double *ds, int32_t *ipiv, int32_t *blk, FacState *st,
                             int32_t *panel_k0, uint64_t *xch) {
  panel_coop<float, true>(s, rows, N, nb, alpha, X, pv, Lout, 0, src_out, W, dd, ds, ipiv, blk, st,
                          panel_k0, xch);
}

// One panel workgroup per compute unit (each takes the whole register file),
// so the reserved units must number at least the first panel's workgroups;
// at least 32 (4 per XCD), since the near update runs on them too, and a
// multiple of the XCD count so that every XCD keeps the same share.
int bk_coop_la_reserve(int N, int cus) {
  const int P = bk_coop_wgs(N);
  const int r = std::max(32, (P + 7) / 8 * 8);
  return (r <= cus / 4) ? r : 0;
}

}  // namespace mds
