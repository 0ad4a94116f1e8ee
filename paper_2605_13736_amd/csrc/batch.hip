// Batched condensed-KKT Newton solves (scenario problems of uneven size, the
// motivation of Sec. 1): one persistent kernel in which every workgroup takes
// problems from an atomic queue (largest first) and runs the whole Newton
// system for each inside the workgroup:
//   condense (same IEEE sequence as condense.hip, so M is bit-identical),
//   blocked Bunch-Kaufman (panel::panel_reg_dev + per-wave trailing tiles on
//   FP64 MFMA, ping-pong buffers), inertia correction (Algorithm IC),
//   LDL' solve in the panels' own row frames, back-substitution of dx_s.
// Each workgroup owns one slot of scratch buffers sized for the largest
// problem.  The host captures the queue reset and the kernel in a hipGraph and
// chooses the panel width and the grid by timing candidates (autotune).
//
// Mixed precision: M is equilibrated (S M S, S = diag(1/sqrt(max_j |M_ij|)))
// and stored in FP32, the trailing tiles run on FP32 MFMA with the panel's W
// and L rounded to FP32, every panel decision and L, D stay FP64; the solution
// is then refined in FP64 on the full (uncondensed) Newton system,
// x += K^-1 (r - K x) through the low-precision factor.
#include <algorithm>
#include <cfloat>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "panel_reg.hpp"

namespace mds {
namespace {

constexpr int BT = 512;   // threads per workgroup (the register panel's)
constexpr int BR = 4;     // register rows per thread: N <= 2048
constexpr int BNB = 16;   // register panel tile
constexpr int BMAX_N = BT * BR;
constexpr int TW = 32;    // per-wave trailing tile
constexpr int NWAVE = BT / 64;

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

struct ProbDev {
  int32_t nd, ns, m, nnz;
  const double *H, *Jd;
  const int32_t *rp, *ci;
  const double *v;
  const int32_t *cptr, *crow;
  const double *cval;
  const double *sigma_d, *dsbase, *r_d, *r_s, *r_y;
  double *dx_d, *dx_s, *dy;
};

struct SlotDev {
  double *buf[2], *W, *dd, *ds, *inv_d;
  int32_t *src, *ipiv, *blk, *pk0;
  FacState *st;
  float *x32[2];  // mixed precision: FP32 ping-pong halves of buf[1]
  double *eq;     // mixed precision: equilibration S (N)
  double *res;    // residual of the full system (n_d + n_s + m)
  const double *zero;  // 64 zeros (written at creation, never after)
  // whole-IPM vectors (null without IPM memory): n = n_d + n_s entries
  // (sig, rx, dx, dzl, dzu, xt, gf, jty), m (ry, dy, cx), n_s (dsb), n_d
  // (hx), n + m (prev); filter pairs (theta, phi)
  double *sig, *rx, *ry, *dsb, *dx, *dy, *dzl, *dzu, *xt, *gf, *jty, *cx, *hx, *prev, *filt;
};

// whole-IPM data of one problem (caller's device arrays)
struct IpmDev {
  const double *c, *w, *g, *b, *xl, *xu;
  double *x, *y, *zl, *zu;
};

struct IpmResDev {
  int32_t status, iters;
  double mu, E0;
  int64_t t_start, t_done;
  int32_t slot, facs;
};

struct IpmIterDev {
  double mu, alpha_pr, delta_w;
  int32_t inertia[3], trials, backtracks, pad;
};

struct IpmParams {
  double tol, mu0, dw_max;
  int32_t max_iter, refine_steps, trace_rows, pad;
};

struct ResultDev {
  int32_t npos, nzero, nneg, trials;
  double delta_w, delta_c;
  int64_t t_start, t_done;
  int32_t status, pad;
  int32_t refine_steps, pad2;
  double residual;  // max |r - K x| / max |r| before the last correction
};

// ---- condensation (bit-identical to k_condense_dense / k_condense_schur) ----
__device__ __attribute__((noinline)) void condense_wg(const ProbDev &P, double *inv_d, double dw, double dc, double *M) {
  const int tid = threadIdx.x, nd = P.nd, m = P.m, N = nd + m;
  for (int k = tid; k < P.ns; k += BT) inv_d[k] = 1.0 / (P.dsbase[k] + dw);
  for (int j = 0; j < N; ++j)
  for (int i = tid; i < N; i += BT) {
    double v;
    if (i < nd && j < nd) {
      v = P.H[(size_t)i + (size_t)j * nd];
      if (i == j) v = (v + P.sigma_d[i]) + dw;
    } else if (j < nd) {
      v = P.Jd[(size_t)(i - nd) + (size_t)j * m];
    } else if (i < nd) {
      v = P.Jd[(size_t)(j - nd) + (size_t)i * m];
    } else {
      v = 0.0;
    }
    M[(size_t)i + (size_t)j * N] = v;
  }
  __syncthreads();
  for (int r = tid; r < m; r += BT) {
    const size_t col = (size_t)(nd + r) * N;
    for (int a = P.rp[r]; a < P.rp[r + 1]; ++a) {
      const int k = P.ci[a];
      const double jrk = P.v[a], dk = inv_d[k];
      for (int e = P.cptr[k]; e < P.cptr[k + 1]; ++e) {
        const int i = P.crow[e];
        if (i < r) continue;
        const size_t pos = (size_t)(nd + i) + col;
        double acc = M[pos];
        acc = acc - (P.cval[e] * dk) * jrk;
        M[pos] = acc;
        if (i != r) M[(size_t)(nd + r) + (size_t)(nd + i) * N] = acc;
      }
    }
    const size_t dpos = (size_t)(nd + r) + col;
    M[dpos] = M[dpos] - dc;
  }
  __syncthreads();
}

// ---- trailing update: every wave takes 32 x 32 lower tiles on its own --------
// D[c][i] = sum_t W[c, t] L[i, t]; Y(i, c) = X(src i, src c) - D[c][i] for the
// lower tile only (every reader takes entries above the diagonal from the
// lower triangle).
typedef __attribute__((address_space(1))) const double gdouble;
typedef __attribute__((address_space(1))) const float gfloat;
typedef __attribute__((address_space(1))) const int32_t gint;
typedef __attribute__((address_space(1))) double gdouble_out;
typedef __attribute__((address_space(1))) float gfloat_out;

// a pointer that is the same in every lane, as a global-memory base in SGPRs
__device__ inline unsigned long long ubase(const void *p) {
  const unsigned long long a = (unsigned long long)p;
  const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)a);
  const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(a >> 32));
  return ((unsigned long long)hi << 32) | lo;
}
__device__ __attribute__((noinline)) void trailing_wg(int N, int k0, int kend, const double *W, const double *X, double *Y,
                            const int32_t *src, const double *zero, double (*s_t)[TW + 1]) {
  // The FP64 tiles keep guarded loads: with the zero-block loads of the FP32
  // tiles below, the FP64 batch measured 7% slower (its traffic is twice the
  // FP32 tiles' and the extra loads in flight did not pay).
  (void)zero;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int l16 = lane & 15, l4 = lane >> 4;
  const int jw = kend - k0, n = N - kend;
  const int nt = (n + TW - 1) / TW;
  const int ntiles = nt * (nt + 1) / 2;
  const size_t ld = (size_t)N;
  (void)s_t;
  for (int x = wv; x < ntiles; x += NWAVE) {
    int ti = (int)((sqrt(8.0 * (double)x + 1.0) - 1.0) * 0.5);
    while ((ti + 1) * (ti + 2) / 2 <= x) ++ti;
    while (ti * (ti + 1) / 2 > x) --ti;
    const int tj = x - ti * (ti + 1) / 2;
    const int i0 = kend + ti * TW, c0 = kend + tj * TW;
    // Every load of the tile is issued before the first use: the panel's map
    // for the tile's rows (lanes 0-31) and columns (lanes 32-63), the W and L
    // operands of every k-step, then the un-updated entries.
    const int li = (lane < 32) ? i0 + lane : c0 + (lane - 32);
    const int sidx = (li < N) ? src[li] : 0;
    constexpr int KS = (BNB + 1 + 3) / 4;  // a panel has at most nb + 1 columns
    double av[KS][2], bv[KS][2];
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const int tt = 4 * ks + l4;
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        const int c = c0 + a * 16 + l16;
        av[ks][a] = (tt < jw && c < N) ? W[(size_t)c + (size_t)tt * ld] : 0.0;
      }
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        const int i = i0 + b * 16 + l16;
        bv[ks][b] = (tt < jw && i < N) ? Y[(size_t)i + (size_t)(k0 + tt) * ld] : 0.0;
      }
    }
    const bool diag = (ti == tj);
    double xv[2][2][4];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int cl = a * 16 + l4 + 4 * r, il = b * 16 + l16;
          const int si = __shfl(sidx, il), sc = __shfl(sidx, 32 + cl);
          const int c = c0 + cl, i = i0 + il;
          const bool ok = c < N && i < N && (!diag || i >= c);
          // lower triangle only: entry (max, min) of the physical indices
          xv[a][b][r] = ok ? X[(si >= sc) ? (size_t)si + (size_t)sc * ld : (size_t)sc + (size_t)si * ld] : 0.0;
        }
    d4 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) acc[a][b] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      if (4 * ks < jw) {
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
          for (int b = 0; b < 2; ++b)
            acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[ks][a], bv[ks][b], acc[a][b], 0, 0, 0);
      }
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          // FP64 16 x 16 MFMA result: lane l, register r holds row l/16 + 4 r
          const int c = c0 + a * 16 + l4 + 4 * r;
          const int i = i0 + b * 16 + l16;
          if (c < N && i < N && (!diag || i >= c)) Y[(size_t)i + (size_t)c * ld] = xv[a][b][r] - acc[a][b][r];
        }
  }
}

// Mixed precision: the same tiles with FP32 storage of the trailing matrix.
// Every load of a tile is issued before the first use: an operand outside
// the tile (past N, or a panel column past the panel's width) is read from
// the slot's zero block instead, each load is unconditional from a
// workgroup-uniform global base plus a selected 32-bit element offset, and
// the conversion to FP32 comes after all loads are issued; with the operands
// loaded as (float)(guard ? W[..] : 0) every load waited on its own.  19%
// more problems per second than the guarded form.  The products run on FP32
// MFMA with W and L (FP64, L in Lsrc) rounded after loading.
// v_mfma_f32_16x16x4f32: result register r of lane l holds row 4 (l/16) + r.
__device__ __attribute__((noinline)) void trailing_wg_lp(int N, int k0, int kend, const double *W,
                                                         const double *Lsrc, const float *X,
                                                         float *Y, const int32_t *src,
                                                         const double *zero,
                                                         double (*s_t)[TW + 1]) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  gdouble *gW = (gdouble *)ubase(W), *gL = (gdouble *)ubase(Lsrc), *gZ = (gdouble *)ubase(zero);
  gfloat *gX = (gfloat *)ubase(X), *gZf = (gfloat *)ubase(zero);
  gint *gsrc = (gint *)ubase(src);
  gfloat_out *oY = (gfloat_out *)ubase(Y);
  const int zW = (int)(gZ - gW), zL = (int)(gZ - gL), zX = (int)(gZf - gX);
  const int l16 = lane & 15, l4 = lane >> 4;
  const int jw = kend - k0, n = N - kend;
  const int nt = (n + TW - 1) / TW;
  (void)s_t;
  constexpr int KS = (BNB + 1 + 3) / 4;
  // Each wave walks whole tile columns, top to bottom: the W operands and
  // the columns' map stay in registers for all the column's tiles (5% more
  // FP32 batch problems per second than one lower tile per wave iteration;
  // the same walk in trailing_wg doubled its spills and gained nothing)
  for (int tj = wv; tj < nt; tj += NWAVE) {
    const int c0 = kend + tj * TW;
    const int scol = gsrc[(unsigned)min(c0 + (lane & 31), N - 1)];
    float av[KS][2];
    {
      double aw[KS][2];
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) {
        const int tt = 4 * ks + l4;
#pragma unroll
        for (int a = 0; a < 2; ++a) {
          const int c = c0 + a * 16 + l16;
          aw[ks][a] = gW[(unsigned)((tt < jw && c < N) ? c + tt * N : zW)];
        }
      }
#pragma unroll
      for (int ks = 0; ks < KS; ++ks)
#pragma unroll
        for (int a = 0; a < 2; ++a) av[ks][a] = (float)aw[ks][a];
    }
    for (int ti = tj; ti < nt; ++ti) {
      const int i0 = kend + ti * TW;
      const int srow = gsrc[(unsigned)min(i0 + (lane & 31), N - 1)];
      const int sidx = (lane < 32) ? srow : scol;
      double bw[KS][2];  // converted to FP32 after all loads are issued
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) {
        const int tt = 4 * ks + l4;
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          const int i = i0 + b * 16 + l16;
          bw[ks][b] = gL[(unsigned)((tt < jw && i < N) ? i + (k0 + tt) * N : zL)];
        }
      }
      const bool diag = (ti == tj);
      float xv[2][2][4];
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int cl = a * 16 + 4 * l4 + r, il = b * 16 + l16;
            const int si = __shfl(sidx, il), sc = __shfl(sidx, 32 + cl);
            const int c = c0 + cl, i = i0 + il;
            const bool ok = c < N && i < N && (!diag || i >= c);
            xv[a][b][r] = gX[(unsigned)(ok ? ((si >= sc) ? si + sc * N : sc + si * N) : zX)];
          }
      float bv[KS][2];
#pragma unroll
      for (int ks = 0; ks < KS; ++ks)
#pragma unroll
        for (int b = 0; b < 2; ++b) bv[ks][b] = (float)bw[ks][b];
      f4 acc[2][2];
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) {
        if (4 * ks < jw) {
#pragma unroll
          for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b)
              acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[ks][a], bv[ks][b], acc[a][b], 0, 0, 0);
        }
      }
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int c = c0 + a * 16 + 4 * l4 + r;
            const int i = i0 + b * 16 + l16;
            if (c < N && i < N && (!diag || i >= c)) oY[(unsigned)(i + c * N)] = xv[a][b][r] - acc[a][b][r];
          }
    }
  }
}

// Mixed precision: S = diag(1/sqrt(max_j |M_ij|)) (1 on a zero row) and
// X = FP32(S M S), the same scaling as the single-problem path.
__device__ __attribute__((noinline)) void equilibrate_wg(int N, const double *M, double *eq,
                                                         float *X) {
  const int tid = threadIdx.x;
  const size_t ld = (size_t)N;
  for (int i = tid; i < N; i += BT) {
    double mx = 0.0;
    for (int j = 0; j < N; ++j) mx = fmax(mx, fabs(M[(size_t)i + (size_t)j * ld]));
    eq[i] = (mx > 0.0) ? 1.0 / sqrt(mx) : 1.0;
  }
  __syncthreads();
  for (int j = 0; j < N; ++j) {
    const double sj = eq[j];
    for (int i = tid; i < N; i += BT)
      X[(size_t)i + (size_t)j * ld] = (float)((eq[i] * M[(size_t)i + (size_t)j * ld]) * sj);
  }
  __syncthreads();
}

// The phases are kept out of line so that each gets its own register
// allocation (the panel needs most of the register file for L).
__device__ __attribute__((noinline)) void panel_call(int N, int nb, double alpha, const double *X,
                                                     double *Y, const SlotDev &S) {
  panel::panel_reg_dev<BT, BR, BNB, double>(N, nb, alpha, X, Y, S.src, S.W, S.dd, S.ds, S.ipiv,
                                            S.blk, S.st, S.pk0);
}

__device__ __attribute__((noinline)) void panel_call_lp(int N, int nb, double alpha,
                                                        const float *X, const SlotDev &S) {
  panel::panel_reg_dev<BT, BR, BNB, float>(N, nb, alpha, X, S.buf[0], S.src, S.W, S.dd, S.ds,
                                           S.ipiv, S.blk, S.st, S.pk0);
}

// Mixed precision: blocked factorization of X32[0] = FP32(S M S); L (FP64)
// of every panel lands in buf[0].
__device__ void factor_wg_lp(int N, int nb, double alpha, const SlotDev &S,
                             double (*s_t)[TW + 1]) {
  const int tid = threadIdx.x;
  if (tid == 0) {
    FacState z{};
    *S.st = z;
    S.pk0[0] = 0;
  }
  __syncthreads();
  for (int b = 0;; ++b) {
    const int k0 = S.st->k;
    if (k0 >= N) break;
    const float *X = S.x32[b & 1];
    float *Y = S.x32[(b + 1) & 1];
    panel_call_lp(N, nb, alpha, X, S);
    __syncthreads();
    const int kend = S.st->k;
    if (kend < N) trailing_wg_lp(N, k0, kend, S.W, S.buf[0], X, Y, S.src, S.zero, s_t);
    __syncthreads();
  }
}

// ---- blocked factorization of the slot's buf[0] --------------------------------
__device__ void factor_wg(int N, int nb, double alpha, const SlotDev &S,
                          double (*s_t)[TW + 1]) {
  const int tid = threadIdx.x;
  if (tid == 0) {
    FacState z{};
    *S.st = z;
    S.pk0[0] = 0;
  }
  __syncthreads();
  for (int b = 0;; ++b) {
    const int k0 = S.st->k;
    if (k0 >= N) break;
    const double *X = S.buf[b & 1];
    double *Y = S.buf[(b + 1) & 1];
    panel_call(N, nb, alpha, X, Y, S);
    __syncthreads();
    const int kend = S.st->k;
    if (kend < N) trailing_wg(N, k0, kend, S.W, X, Y, S.src, S.zero, s_t);
    __syncthreads();
  }
}

// ---- LDL' solve in the panels' row frames (z in LDS) ----------------------------
// L of panel b: buf[(b + 1) % 2] (FP64 ping-pong) or buf[0] (mixed precision).
// Per panel, the pivot records are read in parallel into s_pq (one entry
// per thread: (k, q) for a 1x1 pivot, (k + 1, q) for the first row of a 2x2
// one, p = -1 for its second row) and the panel's diagonal block of L into
// s_db (w x w, one load per entry, all in flight at once); the sequential
// steps then touch only LDS and broadcast a lane's value with readlane.
constexpr int BDB = BNB + 1;  // widest panel (a final 2x2 pivot)

__device__ inline void panel_records(const SlotDev &S, int k0, int w, int *s_pq) {
  const int tid = threadIdx.x;
  if (tid < w) {
    const int k = k0 + tid, bk = S.blk[k], iv = S.ipiv[k];
    s_pq[2 * tid] = (bk == 1) ? k : (bk == 2) ? k + 1 : -1;
    s_pq[2 * tid + 1] = (bk == 1) ? iv - 1 : -iv - 1;
  }
}

__device__ inline void diag_block(const double *Lb, size_t ld, int k0, int w, double *s_db) {
  const int tid = threadIdx.x;
  if (tid < BDB * BDB) {
    const int r = tid % BDB, c = tid / BDB;
    if (r < w && c < w) s_db[r * BDB + c] = Lb[(size_t)(k0 + r) + (size_t)(k0 + c) * ld];
  }
}

__device__ __attribute__((noinline)) void solve_wg(int N, const SlotDev &S, double *z, double *s_part,
                                                   bool mixed, double *s_db, int *s_pq) {
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int np = S.st->npanel;
  const size_t ld = (size_t)N;
  // forward: P_b, then L_b
  for (int b = 0; b < np; ++b) {
    const int k0 = S.pk0[b], k1 = S.pk0[b + 1];
    const int w = k1 - k0;
    const double *Lb = mixed ? S.buf[0] : S.buf[(b + 1) & 1];
    panel_records(S, k0, w, s_pq);
    diag_block(Lb, ld, k0, w, s_db);
    __syncthreads();
    if (tid == 0) {
      for (int e = 0; e < w; ++e) {
        const int p = s_pq[2 * e], q = s_pq[2 * e + 1];
        if (p >= 0 && p != q) {
          const double t = z[p];
          z[p] = z[q];
          z[q] = t;
        }
      }
    }
    __syncthreads();
    if (wv == 0) {
      double v = (lane < w) ? z[k0 + lane] : 0.0;
      for (int c = 0; c + 1 < w; ++c) {
        const double zc = wave::lane_read(v, c);
        if (lane > c && lane < w) v = fma(-s_db[lane * BDB + c], zc, v);
      }
      if (lane < w) z[k0 + lane] = v;
    }
    __syncthreads();
    for (int x = k1 + tid; x < N; x += BT) {
      double v = z[x];
      for (int c = k0; c < k1; ++c) v = fma(-Lb[(size_t)x + (size_t)c * ld], z[c], v);
      z[x] = v;
    }
    __syncthreads();
  }
  // D
  for (int k = tid; k < N; k += BT) {
    const int bk = S.blk[k];
    if (bk == 1) {
      z[k] = z[k] / S.dd[k];
    } else if (bk == 2) {
      const double a = S.dd[k], c = S.dd[k + 1], s = S.ds[k];
      const double det = a * c - s * s;
      const double y0 = z[k], y1 = z[k + 1];
      z[k] = (c * y0 - s * y1) / det;
      z[k + 1] = (a * y1 - s * y0) / det;
    }
  }
  __syncthreads();
  // backward: L_b', then P_b'
  for (int b = np - 1; b >= 0; --b) {
    const int k0 = S.pk0[b], k1 = S.pk0[b + 1], w = k1 - k0;
    const double *Lb = mixed ? S.buf[0] : S.buf[(b + 1) & 1];
    panel_records(S, k0, w, s_pq);
    diag_block(Lb, ld, k0, w, s_db);
    double acc[BNB + 1];
#pragma unroll
    for (int c = 0; c <= BNB; ++c) acc[c] = 0.0;
    for (int x = k1 + tid; x < N; x += BT) {
      const double zx = z[x];
#pragma unroll
      for (int c = 0; c <= BNB; ++c)
        if (c < w) acc[c] = fma(Lb[(size_t)x + (size_t)(k0 + c) * ld], zx, acc[c]);
    }
#pragma unroll
    for (int c = 0; c <= BNB; ++c) {
      const double v = wave::sum(acc[c]);
      if (lane == 0) s_part[wv * (BNB + 1) + c] = v;
    }
    __syncthreads();
    if (wv == 0) {
      double v = 0.0;
      if (lane < w) {
        double s = 0.0;
        for (int q = 0; q < NWAVE; ++q) s += s_part[q * (BNB + 1) + lane];
        v = z[k0 + lane] - s;
      }
      for (int c = w - 1; c > 0; --c) {
        const double xc = wave::lane_read(v, c);
        if (lane < c) v = fma(-s_db[c * BDB + lane], xc, v);
      }
      if (lane < w) z[k0 + lane] = v;
    }
    __syncthreads();
    if (tid == 0) {
      for (int e = w - 1; e >= 0; --e) {
        const int p = s_pq[2 * e], q = s_pq[2 * e + 1];
        if (p >= 0 && p != q) {
          const double t = z[p];
          z[p] = z[q];
          z[q] = t;
        }
      }
    }
    __syncthreads();
  }
}

// Maximum of v over the workgroup (every thread; s_part holds NWAVE doubles).
__device__ inline double block_max(double v, double *s_part) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  v = wave::max(v);
  __syncthreads();
  if (lane == 0) s_part[wv] = v;
  __syncthreads();
  double m = 0.0;
  for (int q = 0; q < NWAVE; ++q) m = fmax(m, s_part[q]);
  __syncthreads();
  return m;
}

// Condensed solve of the full Newton system for the right-hand side
// (rd, rs, ry): z = [rd; ry - J_s (inv_d .* rs)], [x_d; x_y] = M^-1 z through
// the factor (S-scaled on both sides in mixed precision), then
// x_s = inv_d .* (rs - J_s' x_y).  Writes x, or adds it to x when accumulate;
// returns max |increment| and max |x| (after) over the workgroup.
__device__ __attribute__((noinline)) void kkt_solve_wg(const ProbDev &P, const SlotDev &S, bool mixed,
                                                      const double *rd, const double *rs,
                                                      const double *ry, bool accumulate,
                                                      double *s_z, double *s_part, double *s_db,
                                                      int *s_pq, double *cmax, double *xmax) {
  const int tid = threadIdx.x, nd = P.nd, N = P.nd + P.m;
  for (int i = tid; i < N; i += BT) {
    double t;
    if (i < nd) {
      t = rd[i];
    } else {
      const int r = i - nd;
      t = ry[r];
      for (int a = P.rp[r]; a < P.rp[r + 1]; ++a) {
        const int k = P.ci[a];
        t = t - P.v[a] * (S.inv_d[k] * rs[k]);
      }
    }
    s_z[i] = mixed ? S.eq[i] * t : t;
  }
  __syncthreads();
  solve_wg(N, S, s_z, s_part, mixed, s_db, s_pq);
  if (mixed) {
    for (int i = tid; i < N; i += BT) s_z[i] = S.eq[i] * s_z[i];
    __syncthreads();
  }
  double cm = 0.0, xm = 0.0;
  for (int i = tid; i < N; i += BT) {
    double *dst = (i < nd) ? &P.dx_d[i] : &P.dy[i - nd];
    const double c = s_z[i];
    const double v = accumulate ? *dst + c : c;
    *dst = v;
    cm = fmax(cm, fabs(c));
    xm = fmax(xm, fabs(v));
  }
  for (int k = tid; k < P.ns; k += BT) {
    double t = rs[k];
    for (int e = P.cptr[k]; e < P.cptr[k + 1]; ++e) t = t - P.cval[e] * s_z[nd + P.crow[e]];
    const double c = S.inv_d[k] * t;
    const double v = accumulate ? P.dx_s[k] + c : c;
    P.dx_s[k] = v;
    cm = fmax(cm, fabs(c));
    xm = fmax(xm, fabs(v));
  }
  __syncthreads();
  *cmax = block_max(cm, s_part);
  *xmax = block_max(xm, s_part);
}

// res = r - K x on the full Newton system
//   K = [[H + diag(Sigma_d) + dw I, 0, J_d'], [0, diag(dsbase) + dw I, J_s'],
//        [J_d, J_s, -dc I]]
// in FP64 (res: n_d, n_s, m consecutive); returns max |res| / max |r|.
__device__ __attribute__((noinline)) double residual_wg(const ProbDev &P, const SlotDev &S, double dw,
                                                        double dc, double *s_part) {
  const int tid = threadIdx.x, nd = P.nd, ns = P.ns, m = P.m;
  double *res = S.res;
  double rm = 0.0, bm = 0.0;
  for (int i = tid; i < nd; i += BT) {
    double t = P.r_d[i];
    bm = fmax(bm, fabs(t));
    for (int j = 0; j < nd; ++j) t = t - P.H[(size_t)i + (size_t)j * nd] * P.dx_d[j];
    t = t - (P.sigma_d[i] + dw) * P.dx_d[i];
    for (int r = 0; r < m; ++r) t = t - P.Jd[(size_t)r + (size_t)i * m] * P.dy[r];
    res[i] = t;
    rm = fmax(rm, fabs(t));
  }
  for (int k = tid; k < ns; k += BT) {
    double t = P.r_s[k];
    bm = fmax(bm, fabs(t));
    t = t - (P.dsbase[k] + dw) * P.dx_s[k];
    for (int e = P.cptr[k]; e < P.cptr[k + 1]; ++e) t = t - P.cval[e] * P.dy[P.crow[e]];
    res[nd + k] = t;
    rm = fmax(rm, fabs(t));
  }
  for (int r = tid; r < m; r += BT) {
    double t = P.r_y[r];
    bm = fmax(bm, fabs(t));
    for (int i = 0; i < nd; ++i) t = t - P.Jd[(size_t)r + (size_t)i * m] * P.dx_d[i];
    for (int a = P.rp[r]; a < P.rp[r + 1]; ++a) t = t - P.v[a] * P.dx_s[P.ci[a]];
    t = t + dc * P.dy[r];
    res[nd + ns + r] = t;
    rm = fmax(rm, fabs(t));
  }
  __syncthreads();
  rm = block_max(rm, s_part);
  bm = block_max(bm, s_part);
  return (bm > 0.0) ? rm / bm : rm;
}

__global__ void k_batch_reset(int32_t *queue, unsigned long long *t0) {
  if (threadIdx.x == 0) {
    queue[0] = 0;
    t0[0] = ~0ull;
  }
}

// The persistent kernel.  dc_sing = 1e-8 mu^(1/4), computed on the host.
// MIXED: FP32 trailing storage and products, then up to refine_max FP64
// refinement steps (stop when the correction is below 1e-15 of the solution).
// One instantiation per mode: each holds one register panel and its LDS.
template <bool MIXED>
__global__ __launch_bounds__(BT) void k_batch(int count, const int32_t *__restrict__ order,
                                              const ProbDev *__restrict__ probs,
                                              const SlotDev *__restrict__ slots, int nb,
                                              double alpha, const double *dc_sing_p,
                                              int32_t *queue, unsigned long long *t0,
                                              ResultDev *results, int refine_max) {
  constexpr bool mixed = MIXED;
  const double dc_sing = *dc_sing_p;
  __shared__ double s_t[NWAVE * TW][TW + 1];
  __shared__ double s_z[BMAX_N];
  __shared__ double s_part[NWAVE * (BNB + 1)];
  // the solves' diagonal block and pivot records live in the trailing
  // update's transpose tiles, which no solve uses
  double *s_db = &s_t[0][0];
  int *s_pq = (int *)(s_db + BDB * BDB);
  static_assert(BDB * BDB * 8 + 2 * BDB * 4 <= NWAVE * TW * (TW + 1) * 8, "solve staging");
  __shared__ int s_p;
  const int tid = threadIdx.x;
  const SlotDev S = slots[blockIdx.x];
  if (tid == 0) atomicMin(t0, (unsigned long long)wall_clock64());
  for (;;) {
    if (tid == 0) s_p = atomicAdd(queue, 1);
    __syncthreads();
    const int p = s_p;
    __syncthreads();
    if (p >= count) break;
    const int pid = order[p];
    const ProbDev P = probs[pid];
    const int N = P.nd + P.m;
    const unsigned long long ts = wall_clock64();
    // inertia correction (Waechter & Biegler, Algorithm IC) from delta_w_last = 0
    const double dw0 = 1e-4, kw_plus_bar = 100.0, dw_max = 1e20;
    int trials = 1, status = 0;
    double dw = 0.0, dc = 0.0;
    condense_wg(P, S.inv_d, 0.0, 0.0, S.buf[0]);
    if constexpr (MIXED) {
      equilibrate_wg(N, S.buf[0], S.eq, S.x32[0]);
      factor_wg_lp(N, nb, alpha, S, s_t);
    } else {
      factor_wg(N, nb, alpha, S, s_t);
    }
    bool ok = S.st->npos == P.nd && S.st->nzero == 0 && S.st->nneg == P.m;
    if (!ok) {
      dc = (S.st->nzero > 0) ? dc_sing : 0.0;
      dw = dw0;
      for (;;) {
        trials++;
        condense_wg(P, S.inv_d, dw, dc, S.buf[0]);
        if constexpr (MIXED) {
          equilibrate_wg(N, S.buf[0], S.eq, S.x32[0]);
          factor_wg_lp(N, nb, alpha, S, s_t);
        } else {
          factor_wg(N, nb, alpha, S, s_t);
        }
        ok = S.st->npos == P.nd && S.st->nzero == 0 && S.st->nneg == P.m;
        if (ok) break;
        dw = kw_plus_bar * dw;
        if (dw > dw_max) {
          status = MDS_INERTIA_FAIL;
          break;
        }
      }
    }
    // condensed right-hand side, solve, back-substitution; in mixed
    // precision FP64 refinement on the full system
    double cmax, xmax, rel = 0.0;
    kkt_solve_wg(P, S, mixed, P.r_d, P.r_s, P.r_y, false, s_z, s_part, s_db, s_pq, &cmax, &xmax);
    int steps = 0;
    if constexpr (MIXED) {
      const double *res = S.res;
      while (steps < refine_max) {
        rel = residual_wg(P, S, dw, dc, s_part);
        kkt_solve_wg(P, S, true, res, res + P.nd, res + P.nd + P.ns, true, s_z, s_part, s_db, s_pq, &cmax,
                     &xmax);
        ++steps;
        if (cmax <= 1e-15 * xmax) break;
      }
    }
    if (tid == 0) {
      ResultDev r;
      r.npos = S.st->npos;
      r.nzero = S.st->nzero;
      r.nneg = S.st->nneg;
      r.trials = trials;
      r.delta_w = dw;
      r.delta_c = dc;
      r.t_start = (int64_t)ts;
      r.t_done = (int64_t)wall_clock64();
      r.status = status;
      r.pad = (int32_t)blockIdx.x;
      r.refine_steps = steps;
      r.pad2 = 0;
      r.residual = rel;
      results[pid] = r;
    }
  }
}


// ============================ whole IPM per problem ==============================
// The filter line-search IPM of Sec. 2.1 (mds_ipm_step's iteration, with the
// same constants, start point and tests) run by one workgroup per problem of
// the scenario batch: every reduction is workgroup-local, so problems never
// wait for one another and the queue keeps the device busy.  The Newton
// systems go through the batch's own condense / factor / correction / solve
// above, with FP64 iterative refinement on the full system as in
// or_newton_refine (stop at backward error 1e-14, no decrease, or the step
// limit).

// deterministic workgroup sum (wave sums, then the waves in order)
__device__ inline double block_sum(double v, double *s_part) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  v = wave::sum(v);
  __syncthreads();
  if (lane == 0) s_part[wv] = v;
  __syncthreads();
  double t = 0.0;
  for (int q = 0; q < NWAVE; ++q) t = t + s_part[q];
  __syncthreads();
  return t;
}

// workgroup maximum starting from lo (fmax: NaN operands are ignored)
__device__ inline double block_max_from(double v, double lo, double *s_part) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  v = wave::max(v);
  __syncthreads();
  if (lane == 0) s_part[wv] = v;
  __syncthreads();
  double t = lo;
  for (int q = 0; q < NWAVE; ++q) t = fmax(t, s_part[q]);
  __syncthreads();
  return t;
}

// workgroup OR of a flag
__device__ inline bool block_any(bool f, int *s_flag) {
  __syncthreads();
  if (threadIdx.x == 0) *s_flag = 0;
  __syncthreads();
  if (f) *s_flag = 1;
  __syncthreads();
  const bool r = *s_flag != 0;
  __syncthreads();
  return r;
}

// gf = grad f(x) = [H x_d + c; w .* x_s + g] (hx = H x_d), jty = J' y (when
// y is given), cx = J x - b; each entry summed in ascending index
__device__ __attribute__((noinline)) void ipm_eval_wg(const ProbDev &P, const IpmDev &Q, const SlotDev &S, const double *x,
                            const double *y, double *gf, double *jty, double *cx) {
  const int tid = threadIdx.x, nd = P.nd, ns = P.ns, m = P.m;
  for (int i = tid; i < nd; i += BT) {
    double t = 0.0;
    for (int j = 0; j < nd; ++j) t = t + P.H[(size_t)i + (size_t)j * nd] * x[j];
    S.hx[i] = t;
    gf[i] = t + Q.c[i];
  }
  for (int k = tid; k < ns; k += BT) gf[nd + k] = Q.w[k] * x[nd + k] + Q.g[k];
  if (y) {
    for (int j = tid; j < nd; j += BT) {
      double t = 0.0;
      for (int r = 0; r < m; ++r) t = t + P.Jd[(size_t)r + (size_t)j * m] * y[r];
      jty[j] = t;
    }
    for (int k = tid; k < ns; k += BT) {
      double t = 0.0;
      for (int e = P.cptr[k]; e < P.cptr[k + 1]; ++e) t = t + P.cval[e] * y[P.crow[e]];
      jty[nd + k] = t;
    }
  }
  for (int r = tid; r < m; r += BT) {
    double t = 0.0;
    for (int j = 0; j < nd; ++j) t = t + P.Jd[(size_t)r + (size_t)j * m] * x[j];
    for (int a = P.rp[r]; a < P.rp[r + 1]; ++a) t = t + P.v[a] * x[nd + P.ci[a]];
    cx[r] = t - Q.b[r];
  }
  __syncthreads();
}

// scaled optimality error parts at (x, y, zl, zu) from gf, jty, cx:
// out[0] dual inf, [1] primal inf, [2] sum |y| + |z| (s_d numerator),
// [3] number of finite bounds, [4] sum |z|; the complementarity maxima
// depend on mu and come from ipm_compl_wg
__device__ __attribute__((noinline)) void ipm_parts_wg(const ProbDev &P, const IpmDev &Q, const SlotDev &S,
                             const double *x, const double *y, const double *zl,
                             const double *zu, double *s_part, double *out) {
  const int tid = threadIdx.x, n = P.nd + P.ns, m = P.m;
  double dual = 0.0, z1 = 0.0, nz = 0.0, y1 = 0.0, prim = 0.0;
  bool bad = false;
  for (int i = tid; i < n; i += BT) {
    double r = S.gf[i] + S.jty[i];
    if (isfinite(Q.xl[i])) {
      r = r - zl[i];
      z1 += fabs(zl[i]);
      nz += 1.0;
    }
    if (isfinite(Q.xu[i])) {
      r = r + zu[i];
      z1 += fabs(zu[i]);
      nz += 1.0;
    }
    bad = bad || !isfinite(r);
    dual = fmax(dual, fabs(r));
  }
  for (int r = tid; r < m; r += BT) {
    bad = bad || !isfinite(S.cx[r]) || !isfinite(y[r]);
    prim = fmax(prim, fabs(S.cx[r]));
    y1 += fabs(y[r]);
  }
  out[0] = block_max_from(dual, 0.0, s_part);
  out[1] = block_max_from(prim, 0.0, s_part);
  const double zs = block_sum(z1, s_part);
  out[2] = block_sum(y1, s_part) + zs;
  out[3] = block_sum(nz, s_part);
  out[4] = zs;
  int *flag = reinterpret_cast<int *>(s_part + NWAVE);
  if (block_any(bad, flag)) out[0] = NAN;
}

// max |(x - l) zl - mu| and max |(u - x) zu - mu| over the finite bounds
__device__ __attribute__((noinline)) double ipm_compl_wg(const ProbDev &P, const IpmDev &Q, const double *x,
                               const double *zl, const double *zu, double mu, double *s_part) {
  const int tid = threadIdx.x, n = P.nd + P.ns;
  double c = 0.0;
  for (int i = tid; i < n; i += BT) {
    if (isfinite(Q.xl[i])) c = fmax(c, fabs((x[i] - Q.xl[i]) * zl[i] - mu));
    if (isfinite(Q.xu[i])) c = fmax(c, fabs((Q.xu[i] - x[i]) * zu[i] - mu));
  }
  return block_max_from(c, 0.0, s_part);
}

__device__ inline double ipm_error(const double *pt, double compl_, int m) {
  const double s_max = 100.0;
  if (!isfinite(pt[0])) return pt[0];  // a non-finite residual entry
  const double nz = pt[3];
  const double sd = ((double)m + nz > 0.0) ? fmax(s_max, pt[2] / ((double)m + nz)) / s_max : 1.0;
  const double sc = (nz > 0.0) ? fmax(s_max, pt[4] / nz) / s_max : 1.0;
  return fmax(fmax(pt[0] / sd, pt[1]), compl_ / sc);
}

// f, sum of log-slacks, theta = ||J x - b||_1 and phi's rounding scale at
// x: out[0..3]; S.hx must hold H x_d and S.cx = J x - b
__device__ __attribute__((noinline)) void ipm_merit_wg(const ProbDev &P, const IpmDev &Q, const SlotDev &S, const double *x,
                             double mu, double *s_part, double *out) {
  const int tid = threadIdx.x, nd = P.nd, n = P.nd + P.ns, m = P.m;
  double f = 0.0, lg = 0.0, th = 0.0, sc = 0.0;
  bool bad = false;
  for (int i = tid; i < n; i += BT) {
    double t;
    if (i < nd) {
      t = x[i] * (0.5 * S.hx[i] + Q.c[i]);
    } else {
      const double xs = x[i];
      t = xs * (0.5 * Q.w[i - nd] * xs + Q.g[i - nd]);
    }
    f += t;
    sc += fabs(t);
    if (isfinite(Q.xl[i])) {
      const double l = log(x[i] - Q.xl[i]);
      lg += l;
      sc += mu * fabs(l);
    }
    if (isfinite(Q.xu[i])) {
      const double l = log(Q.xu[i] - x[i]);
      lg += l;
      sc += mu * fabs(l);
    }
  }
  for (int r = tid; r < m; r += BT) th += fabs(S.cx[r]);
  bad = !isfinite(f) || !isfinite(lg) || !isfinite(th);
  out[0] = block_sum(f, s_part);
  out[1] = block_sum(lg, s_part);
  out[2] = block_sum(th, s_part);
  out[3] = block_sum(sc, s_part);
  int *flag = reinterpret_cast<int *>(s_part + NWAVE);
  if (block_any(bad, flag)) out[0] = NAN;
}

// J x - b and H x_d at x only (the trial points of the line search)
__device__ __attribute__((noinline)) void ipm_constr_wg(const ProbDev &P, const IpmDev &Q, const SlotDev &S, const double *x) {
  const int tid = threadIdx.x, nd = P.nd, m = P.m;
  for (int i = tid; i < nd; i += BT) {
    double t = 0.0;
    for (int j = 0; j < nd; ++j) t = t + P.H[(size_t)i + (size_t)j * nd] * x[j];
    S.hx[i] = t;
  }
  for (int r = tid; r < m; r += BT) {
    double t = 0.0;
    for (int j = 0; j < nd; ++j) t = t + P.Jd[(size_t)r + (size_t)j * m] * x[j];
    for (int a = P.rp[r]; a < P.rp[r + 1]; ++a) t = t + P.v[a] * x[nd + P.ci[a]];
    S.cx[r] = t - Q.b[r];
  }
  __syncthreads();
}

// ||K||_inf of the regularised Newton matrix (row sums of |K|)
__device__ __attribute__((noinline)) double ipm_knorm_wg(const ProbDev &P, double dw, double dc, double *s_part) {
  const int tid = threadIdx.x, nd = P.nd, ns = P.ns, m = P.m;
  double best = 0.0;
  for (int i = tid; i < nd; i += BT) {
    double t = 0.0;
    for (int j = 0; j < nd; ++j) {
      double h = P.H[(size_t)i + (size_t)j * nd];
      if (i == j) h = h + P.sigma_d[i] + dw;
      t += fabs(h);
    }
    for (int r = 0; r < m; ++r) t += fabs(P.Jd[(size_t)r + (size_t)i * m]);
    best = fmax(best, t);
  }
  for (int k = tid; k < ns; k += BT) {
    double t = fabs(P.dsbase[k] + dw);
    for (int e = P.cptr[k]; e < P.cptr[k + 1]; ++e) t += fabs(P.cval[e]);
    best = fmax(best, t);
  }
  for (int r = tid; r < m; r += BT) {
    double t = fabs(dc);
    for (int j = 0; j < nd; ++j) t += fabs(P.Jd[(size_t)r + (size_t)j * m]);
    for (int a = P.rp[r]; a < P.rp[r + 1]; ++a) t += fabs(P.v[a]);
    best = fmax(best, t);
  }
  return block_max_from(best, 0.0, s_part);
}

// max |v| over the Newton solution or right-hand side stored as three pieces
__device__ __attribute__((noinline)) double amax3_wg(const double *a, int na, const double *b, int nb_, const double *c,
                           int nc, double *s_part) {
  const int tid = threadIdx.x;
  double t = 0.0;
  for (int i = tid; i < na; i += BT) t = fmax(t, fabs(a[i]));
  for (int i = tid; i < nb_; i += BT) t = fmax(t, fabs(b[i]));
  for (int i = tid; i < nc; i += BT) t = fmax(t, fabs(c[i]));
  return block_max_from(t, 0.0, s_part);
}

// FP64 refinement of the Newton solve (P.dx_*, P.dy) on the full system with
// right-hand side (P.r_d, P.r_s, P.r_y), as or_newton_refine
__device__ __attribute__((noinline)) void ipm_refine_wg(const ProbDev &P, const SlotDev &S, double dw, double dc,
                              int max_steps, double *s_z, double *s_part, double *s_db,
                              int *s_pq) {
  const int tid = threadIdx.x, nd = P.nd, ns = P.ns, m = P.m;
  const int nt = nd + ns + m;
  double cmax, xmax;
  kkt_solve_wg(P, S, false, P.r_d, P.r_s, P.r_y, false, s_z, s_part, s_db, s_pq, &cmax, &xmax);
  const double nK = ipm_knorm_wg(P, dw, dc, s_part);
  const double nr = amax3_wg(P.r_d, nd, P.r_s, ns, P.r_y, m, s_part);
  double eta_prev = INFINITY;
  int steps = 0;
  for (;;) {
    residual_wg(P, S, dw, dc, s_part);  // S.res = r - K x
    const double nres = amax3_wg(S.res, nt, nullptr, 0, nullptr, 0, s_part);
    const double nx = amax3_wg(P.dx_d, nd, P.dx_s, ns, P.dy, m, s_part);
    const double den = nK * nx + nr;
    const double eta = (den > 0.0) ? nres / den : 0.0;
    if (steps > 0 && !(eta < eta_prev)) {
      // no decrease: keep the previous iterate
      for (int i = tid; i < nd; i += BT) P.dx_d[i] = S.prev[i];
      for (int i = tid; i < ns; i += BT) P.dx_s[i] = S.prev[nd + i];
      for (int i = tid; i < m; i += BT) P.dy[i] = S.prev[nd + ns + i];
      __syncthreads();
      break;
    }
    if (eta <= 1e-14 || steps >= max_steps) break;
    for (int i = tid; i < nd; i += BT) S.prev[i] = P.dx_d[i];
    for (int i = tid; i < ns; i += BT) S.prev[nd + i] = P.dx_s[i];
    for (int i = tid; i < m; i += BT) S.prev[nd + ns + i] = P.dy[i];
    __syncthreads();
    eta_prev = eta;
    kkt_solve_wg(P, S, false, S.res, S.res + nd, S.res + nd + ns, true, s_z, s_part, s_db, s_pq,
                 &cmax, &xmax);
    ++steps;
  }
}

// Condense + factor with the shifts, and whether In(M) = (n_d, 0, m)
__device__ inline bool ipm_factor_wg(const ProbDev &P, const SlotDev &S, int nb, double alpha,
                                     double dw, double dc, double (*s_t)[TW + 1]) {
  condense_wg(P, S.inv_d, dw, dc, S.buf[0]);
  factor_wg(P.nd + P.m, nb, alpha, S, s_t);
  return S.st->npos == P.nd && S.st->nzero == 0 && S.st->nneg == P.m;
}

__global__ __launch_bounds__(BT) void k_batch_ipm(int count, const int32_t *__restrict__ order,
                                                  const ProbDev *__restrict__ probs,
                                                  const IpmDev *__restrict__ ipms,
                                                  const SlotDev *__restrict__ slots, int nb,
                                                  double alpha, IpmParams prm, int32_t *queue,
                                                  unsigned long long *t0, IpmResDev *results,
                                                  IpmIterDev *trace) {
  __shared__ double s_t[NWAVE * TW][TW + 1];
  __shared__ double s_z[BMAX_N];
  __shared__ double s_part[NWAVE * (BNB + 1)];
  double *s_db = &s_t[0][0];
  int *s_pq = (int *)(s_db + BDB * BDB);
  __shared__ int s_p;
  const int tid = threadIdx.x;
  const SlotDev S = slots[blockIdx.x];
  if (tid == 0) atomicMin(t0, (unsigned long long)wall_clock64());
  // Waechter & Biegler (2006) constants, as the single-problem step
  const double tau_min = 0.99, kappa_eps = 10.0, kappa_mu = 0.2, theta_mu = 1.5;
  const double kappa_sigma = 1e10, gamma_theta = 1e-5, gamma_phi = 1e-8, delta = 1.0;
  const double s_theta = 1.1, s_phi = 2.3, eta_phi = 1e-8, gamma_alpha = 0.05;
  const double dw_min = 1e-20, dw0 = 1e-4, kw_minus = 1.0 / 3.0, kw_plus = 8.0;
  const double kw_plus_bar = 100.0, dc_bar = 1e-8, kappa_c = 0.25;
  for (;;) {
    if (tid == 0) s_p = atomicAdd(queue, 1);
    __syncthreads();
    const int p = s_p;
    __syncthreads();
    if (p >= count) break;
    const int pid = order[p];
    const IpmDev Q = ipms[pid];
    ProbDev P = probs[pid];
    const int nd = P.nd, ns = P.ns, m = P.m, n = nd + ns;
    P.sigma_d = S.sig;
    P.dsbase = S.dsb;
    P.r_d = S.rx;
    P.r_s = S.rx + nd;
    P.r_y = S.ry;
    P.dx_d = S.dx;
    P.dx_s = S.dx + nd;
    P.dy = S.dy;
    const unsigned long long ts = wall_clock64();
    double *x = Q.x, *y = Q.y, *zl = Q.zl, *zu = Q.zu;
    // start point: x = 0 pushed inside its bounds (kappa_1 = kappa_2 = 1e-2),
    // y = 0, z = 1 on finite bounds
    for (int i = tid; i < n; i += BT) {
      const double l = Q.xl[i], u = Q.xu[i];
      const bool hl = isfinite(l), hu = isfinite(u);
      double xi = 0.0;
      if (hl && hu) {
        const double pl = fmin(1e-2 * fmax(1.0, fabs(l)), 1e-2 * (u - l));
        const double pu = fmin(1e-2 * fmax(1.0, fabs(u)), 1e-2 * (u - l));
        xi = fmin(fmax(xi, l + pl), u - pu);
      } else if (hl) {
        xi = fmax(xi, l + 1e-2 * fmax(1.0, fabs(l)));
      } else if (hu) {
        xi = fmin(xi, u - 1e-2 * fmax(1.0, fabs(u)));
      }
      x[i] = xi;
      zl[i] = hl ? 1.0 : 0.0;
      zu[i] = hu ? 1.0 : 0.0;
    }
    for (int r = tid; r < m; r += BT) y[r] = 0.0;
    __syncthreads();
    double mu = prm.mu0, tau = fmax(tau_min, 1.0 - mu), dw_last = 0.0;
    double mv[4], pt[5];
    ipm_constr_wg(P, Q, S, x);
    ipm_merit_wg(P, Q, S, x, mu, s_part, mv);
    const double theta_max = 1e4 * fmax(1.0, mv[2]), theta_min = 1e-4 * fmax(1.0, mv[2]);
    int nf = 0, status = MDS_IPM_MAXITER, it = 0, facs = 0;
    double E0 = 0.0;
    for (it = 0; it < prm.max_iter; ++it) {
      ipm_eval_wg(P, Q, S, x, y, S.gf, S.jty, S.cx);
      ipm_parts_wg(P, Q, S, x, y, zl, zu, s_part, pt);
      E0 = ipm_error(pt, ipm_compl_wg(P, Q, x, zl, zu, 0.0, s_part), m);
      if (!isfinite(E0)) {
        status = MDS_IPM_NONFINITE;
        break;
      }
      if (E0 <= prm.tol) {
        status = MDS_IPM_CONVERGED;
        break;
      }
      // barrier update while the barrier problem is solved to kappa_eps mu
      while (ipm_error(pt, ipm_compl_wg(P, Q, x, zl, zu, mu, s_part), m) <= kappa_eps * mu) {
        const double mnew = fmax(prm.tol / 10.0, fmin(kappa_mu * mu, pow(mu, theta_mu)));
        if (!(mnew < mu)) break;
        mu = mnew;
        tau = fmax(tau_min, 1.0 - mu);
        nf = 0;
      }
      // barrier diagonal and Newton right-hand side; D_s base w + Sigma_s
      for (int i = tid; i < n; i += BT) {
        double sg = 0.0, gb = S.gf[i] + S.jty[i];
        if (isfinite(Q.xl[i])) {
          const double sl = x[i] - Q.xl[i];
          sg = sg + zl[i] / sl;
          gb = gb - mu / sl;
        }
        if (isfinite(Q.xu[i])) {
          const double su = Q.xu[i] - x[i];
          sg = sg + zu[i] / su;
          gb = gb + mu / su;
        }
        S.sig[i] = sg;
        S.rx[i] = -gb;
        if (i >= nd) S.dsb[i - nd] = Q.w[i - nd] + sg;
      }
      for (int r = tid; r < m; r += BT) S.ry[r] = -S.cx[r];
      __syncthreads();
      // inertia correction (Algorithm IC)
      int trials = 1;
      double dw = 0.0, dc = 0.0;
      bool ok = ipm_factor_wg(P, S, nb, alpha, 0.0, 0.0, s_t);
      if (!ok) {
        dc = (S.st->nzero > 0) ? dc_bar * pow(mu, kappa_c) : 0.0;
        dw = (dw_last == 0.0) ? dw0 : fmax(dw_min, kw_minus * dw_last);
        for (;;) {
          trials++;
          ok = ipm_factor_wg(P, S, nb, alpha, dw, dc, s_t);
          if (ok) {
            dw_last = dw;
            break;
          }
          dw = (dw_last == 0.0) ? kw_plus_bar * dw : kw_plus * dw;
          if (dw > prm.dw_max) break;
        }
      }
      facs += trials;
      const int inn0 = S.st->npos, inn1 = S.st->nzero, inn2 = S.st->nneg;
      if (!ok) {
        status = MDS_INERTIA_FAIL;
        break;
      }
      ipm_refine_wg(P, S, dw, dc, prm.refine_steps, s_z, s_part, s_db, s_pq);
      // bound-multiplier steps and the fraction to the boundary
      double apr = -1.0, adu = -1.0;  // largest -(step limit)
      for (int i = tid; i < n; i += BT) {
        double a = 0.0, b = 0.0;
        const double d = S.dx[i];
        if (isfinite(Q.xl[i])) {
          const double sl = x[i] - Q.xl[i];
          a = mu / sl - zl[i] - (zl[i] / sl) * d;
          if (d < 0.0) apr = fmax(apr, -(-tau * sl / d));
          if (a < 0.0) adu = fmax(adu, -(-tau * zl[i] / a));
        }
        if (isfinite(Q.xu[i])) {
          const double su = Q.xu[i] - x[i];
          b = mu / su - zu[i] + (zu[i] / su) * d;
          if (-d < 0.0) apr = fmax(apr, -(-tau * su / (-d)));
          if (b < 0.0) adu = fmax(adu, -(-tau * zu[i] / b));
        }
        S.dzl[i] = a;
        S.dzu[i] = b;
      }
      const double a_pr = -block_max_from(apr, -1.0, s_part);
      const double a_du = -block_max_from(adu, -1.0, s_part);
      // merit at x and grad(phi)' dx
      ipm_constr_wg(P, Q, S, x);
      ipm_merit_wg(P, Q, S, x, mu, s_part, mv);
      const double th = mv[2], ph = mv[0] - mu * mv[1];
      const double ph_tol = 10.0 * DBL_EPSILON * mv[3];
      double gp = 0.0;
      for (int i = tid; i < n; i += BT) {
        double gi = S.gf[i];
        if (isfinite(Q.xl[i])) gi = gi - mu / (x[i] - Q.xl[i]);
        if (isfinite(Q.xu[i])) gi = gi + mu / (Q.xu[i] - x[i]);
        gp += gi * S.dx[i];
      }
      const double gphi = block_sum(gp, s_part);
      double amin;
      if (gphi < 0.0) {
        amin = fmin(gamma_theta, gamma_phi * th / (-gphi));
        if (th <= theta_min) amin = fmin(amin, delta * pow(th, s_theta) / pow(-gphi, s_phi));
        amin = gamma_alpha * amin;
      } else {
        amin = gamma_alpha * gamma_theta;
      }
      double alpha_s = a_pr;
      bool accepted = false, augment = true;
      int nbt = 0;
      for (;;) {
        for (int i = tid; i < n; i += BT) S.xt[i] = x[i] + alpha_s * S.dx[i];
        __syncthreads();
        ipm_constr_wg(P, Q, S, S.xt);
        ipm_merit_wg(P, Q, S, S.xt, mu, s_part, mv);
        const double tht = mv[2], pht = mv[0] - mu * mv[1];
        const bool okv = isfinite(tht) && isfinite(pht);
        bool infilt = !okv || tht >= theta_max;
        for (int f = 0; f < nf && !infilt; ++f)
          if (tht >= S.filt[2 * f] && pht >= S.filt[2 * f + 1]) infilt = true;
        if (!infilt) {
          const bool sw = gphi < 0.0 && alpha_s * pow(-gphi, s_phi) > delta * pow(th, s_theta);
          const bool armijo = (pht - ph) - eta_phi * alpha_s * gphi <= ph_tol;
          if (th <= theta_min && sw) {
            if (armijo) accepted = true;
          } else if (tht <= (1.0 - gamma_theta) * th || (pht - ph) - (-gamma_phi * th) <= ph_tol) {
            accepted = true;
          }
          if (accepted) augment = !(sw && armijo);
        }
        if (accepted) break;
        alpha_s = 0.5 * alpha_s;
        nbt++;
        // alpha_min can be 0 (theta = 0 and a descent direction); past 2^-200
        // the step is nil, and the workgroup must not spin on it
        if (alpha_s < amin || nbt >= 200) break;
      }
      if (tid == 0 && it < prm.trace_rows) {
        IpmIterDev r;
        r.mu = mu;
        r.alpha_pr = alpha_s;
        r.delta_w = dw;
        r.inertia[0] = inn0;
        r.inertia[1] = inn1;
        r.inertia[2] = inn2;
        r.trials = trials;
        r.backtracks = nbt;
        r.pad = 0;
        trace[(size_t)pid * prm.trace_rows + it] = r;
      }
      if (!accepted) {
        status = MDS_IPM_LS_FAIL;
        break;
      }
      if (augment) {
        if (tid == 0) {
          S.filt[2 * nf] = (1.0 - gamma_theta) * th;
          S.filt[2 * nf + 1] = ph - gamma_phi * th;
        }
        nf++;
      }
      // accept: x, y, and the bound multipliers with the kappa_Sigma safeguard
      for (int i = tid; i < n; i += BT) {
        const double xi = S.xt[i];
        x[i] = xi;
        if (isfinite(Q.xl[i])) {
          const double z = zl[i] + a_du * S.dzl[i], sl = xi - Q.xl[i];
          zl[i] = fmax(fmin(z, kappa_sigma * mu / sl), mu / (kappa_sigma * sl));
        }
        if (isfinite(Q.xu[i])) {
          const double z = zu[i] + a_du * S.dzu[i], su = Q.xu[i] - xi;
          zu[i] = fmax(fmin(z, kappa_sigma * mu / su), mu / (kappa_sigma * su));
        }
      }
      for (int r = tid; r < m; r += BT) y[r] = y[r] + alpha_s * S.dy[r];
      __syncthreads();
    }
    if (tid == 0) {
      IpmResDev r;
      r.status = status;
      r.iters = it;
      r.mu = mu;
      r.E0 = E0;
      r.t_start = (int64_t)ts;
      r.t_done = (int64_t)wall_clock64();
      r.slot = (int32_t)blockIdx.x;
      r.facs = facs;
      results[pid] = r;
    }
    __syncthreads();
  }
}


// ============================ host side ========================================

}  // namespace

struct mds_batch_impl {
  hipStream_t caller = nullptr;  // the caller's stream (inputs are ordered on it)
  hipStream_t stream = nullptr;  // the batch's own stream (capturable)
  int count = 0, Nmax = 0, nsmax = 0, nslots = 0;
  int nb = BNB, grid = 0;
  bool use_graph = true;
  int mixed = 0;       // 1: FP32 trailing storage and products + FP64 refinement
  int refine_max = 0;  // refinement steps at most (mixed precision)
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  int g_nb = -1, g_grid = -1;
  double alpha = 0.0;
  ProbDev *d_probs = nullptr;
  SlotDev *d_slots = nullptr;
  int32_t *d_order = nullptr, *d_queue = nullptr;
  unsigned long long *d_t0 = nullptr;
  double *d_dc = nullptr;
  ResultDev *d_results = nullptr;
  std::vector<ResultDev> h_results;
  // whole-IPM mode
  int ipm_rows = 0;          // trace rows per problem (0: no IPM memory)
  bool newton_io = true;     // every problem has Newton-system inputs and outputs
  IpmDev *d_ipms = nullptr;
  IpmResDev *d_ipm_res = nullptr;
  IpmIterDev *d_trace = nullptr;
  char err[256] = {0};
};

namespace {

size_t al256(size_t b) { return (b + 255) & ~(size_t)255; }
inline size_t al256_(size_t b) { return ((b + 255) & ~(size_t)255) + (b == 0 ? 256 : 0); }

struct BatchLayout {
  size_t probs, slots, order, ctl, results, csc_total, slot_bytes, total;
  size_t ipms = 0, ipm_res = 0, trace = 0, slot_ipm = 0;
  int Nmax, nsmax, nslots, ndmax = 0, mmax = 0, ipm_rows = 0;
  std::vector<size_t> csc_off;
};

// per-slot IPM vectors, in carving order: sig, rx, dx, dzl, dzu, xt, gf, jty
// (n each), ry, dy, cx (m), dsb (n_s), hx (n_d), prev (n + m), filt
size_t ipm_slot_bytes(size_t n, size_t m, size_t ns, size_t nd, int rows) {
  return 8 * al256_(8 * n) + 3 * al256_(8 * m) + al256_(8 * ns) + al256_(8 * nd) +
         al256_(8 * (n + m)) + al256_(16 * (size_t)(rows + 1));
}

bool batch_layout(const mds_batch_problem *ps, int count, const mds_batch_opts *o, BatchLayout &L) {
  if (!ps || count <= 0) return false;
  L.Nmax = 0;
  L.nsmax = 0;
  L.csc_off.resize(count);
  size_t csc = 0;
  for (int p = 0; p < count; ++p) {
    const mds_batch_problem &q = ps[p];
    if (q.n_d < 0 || q.n_s < 0 || q.m < 0 || q.nnz_s < 0) return false;
    const int N = q.n_d + q.m;
    if (N < 1 || N > BMAX_N || q.nnz_s >= (1LL << 30)) return false;
    L.Nmax = std::max(L.Nmax, N);
    L.nsmax = std::max(L.nsmax, q.n_s);
    L.csc_off[p] = csc;
    csc += al256(4 * ((size_t)q.n_s + 1)) + al256(4 * (size_t)q.nnz_s + 4) +
           al256(8 * (size_t)q.nnz_s + 8) + al256(4 * (size_t)q.n_s + 4);
  }
  L.ipm_rows = (o && o->ipm_max_iter > 0) ? o->ipm_max_iter + 1 : 0;
  size_t nmax = 0;
  for (int p = 0; p < count; ++p) {
    L.ndmax = std::max(L.ndmax, ps[p].n_d);
    L.mmax = std::max(L.mmax, ps[p].m);
    nmax = std::max(nmax, (size_t)ps[p].n_d + (size_t)ps[p].n_s);
  }
  const int want = (o && o->grid > 0) ? o->grid : 256;
  L.nslots = std::max(1, std::min(count, want));
  const size_t N = (size_t)L.Nmax;
  L.slot_bytes = 2 * al256(8 * N * N) + al256(8 * N * (kMaxNb + 2)) + al256(8 * 64) +
                 2 * al256(8 * N) +
                 al256(8 * (size_t)std::max(L.nsmax, 1)) + 3 * al256(4 * N) + al256(4 * (N + 4)) +
                 al256(sizeof(FacState)) + al256(8 * N) + al256(8 * (N + (size_t)L.nsmax));
  L.probs = al256(sizeof(ProbDev) * count);
  L.slots = al256(sizeof(SlotDev) * L.nslots);
  L.order = al256(4 * (size_t)count);
  L.ctl = 256;
  L.results = al256(sizeof(ResultDev) * count);
  L.csc_total = csc;
  if (L.ipm_rows > 0) {
    L.slot_ipm = ipm_slot_bytes(nmax, (size_t)L.mmax, (size_t)L.nsmax, (size_t)L.ndmax,
                                L.ipm_rows);
    L.ipms = al256(sizeof(IpmDev) * count);
    L.ipm_res = al256(sizeof(IpmResDev) * count);
    L.trace = al256(sizeof(IpmIterDev) * (size_t)count * (size_t)L.ipm_rows);
  }
  L.total = L.probs + L.slots + L.order + L.ctl + L.results + L.csc_total +
            (L.slot_bytes + L.slot_ipm) * L.nslots + L.ipms + L.ipm_res + L.trace;
  return true;
}

int fail(mds_batch_impl *b, int code, const char *what, hipError_t e) {
  snprintf(b->err, sizeof(b->err), "%s: %s", what, hipGetErrorString(e));
  return code;
}

int launch_batch(mds_batch_impl *b) {
  k_batch_reset<<<1, 64, 0, b->stream>>>(b->d_queue, b->d_t0);
  if (b->mixed)
    k_batch<true><<<(unsigned)b->grid, BT, 0, b->stream>>>(
        b->count, b->d_order, b->d_probs, b->d_slots, b->nb, b->alpha, b->d_dc, b->d_queue,
        b->d_t0, b->d_results, b->refine_max);
  else
    k_batch<false><<<(unsigned)b->grid, BT, 0, b->stream>>>(
        b->count, b->d_order, b->d_probs, b->d_slots, b->nb, b->alpha, b->d_dc, b->d_queue,
        b->d_t0, b->d_results, b->refine_max);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? MDS_OK : fail(b, MDS_EHIP, "batch launch", e);
}

int run_once(mds_batch_impl *b) {
  if (!b->use_graph) return launch_batch(b);
  if (!b->gexec || b->g_nb != b->nb || b->g_grid != b->grid) {
    if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->gexec = nullptr;
    b->graph = nullptr;
    hipError_t e = hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return fail(b, MDS_EHIP, "hipStreamBeginCapture", e);
    const int st = launch_batch(b);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(b->stream, &g);
    if (e != hipSuccess) return fail(b, MDS_EHIP, "hipStreamEndCapture", e);
    if (st != MDS_OK) return st;
    b->graph = g;
    e = hipGraphInstantiate(&b->gexec, g, nullptr, nullptr, 0);
    if (e != hipSuccess) return fail(b, MDS_EHIP, "hipGraphInstantiate", e);
    b->g_nb = b->nb;
    b->g_grid = b->grid;
  }
  const hipError_t e = hipGraphLaunch(b->gexec, b->stream);
  return e == hipSuccess ? MDS_OK : fail(b, MDS_EHIP, "hipGraphLaunch", e);
}

}  // namespace
}  // namespace mds

using namespace mds;

struct mds_batch : mds_batch_impl {};

extern "C" {

size_t mds_batch_workspace_bytes(const mds_batch_problem *probs_host, int32_t count,
                                 const mds_batch_opts *opts) {
  BatchLayout L;
  if (!batch_layout(probs_host, count, opts, L)) return 0;
  return L.total;
}

int mds_batch_create(mds_batch **out, const mds_batch_problem *probs_host, int32_t count,
                     const mds_batch_opts *opts, void *stream, void *workspace, size_t bytes) {
  if (!out || !probs_host || !workspace) return MDS_ENULL;
  *out = nullptr;
  BatchLayout L;
  if (!batch_layout(probs_host, count, opts, L)) return MDS_EDIMS;
  if (bytes < L.total || ((uintptr_t)workspace & 255) != 0) return MDS_EWORKSPACE;
  if (opts && (opts->nb < 0 || opts->nb == 1 || opts->nb > BNB)) return MDS_EINVAL;
  if (opts && opts->precision != MDS_FP64 && opts->precision != MDS_FP32) return MDS_EINVAL;
  if (opts && (opts->refine_steps < 0 || opts->refine_steps > 100)) return MDS_EINVAL;
  if (opts && (opts->ipm_max_iter < 0 || opts->ipm_max_iter > 1000)) return MDS_EINVAL;
  bool newton_io = true;
  for (int p = 0; p < count; ++p) {
    const mds_batch_problem &q = probs_host[p];
    if ((q.n_d > 0 && !q.H) || (q.m > 0 && q.n_d > 0 && !q.J_d) || !q.Js_rowptr ||
        (q.nnz_s > 0 && (!q.Js_col || !q.Js_val)))
      return MDS_ENULL;
    const bool io = !((q.n_d > 0 && (!q.sigma_d || !q.r_d || !q.dx_d)) ||
                      (q.n_s > 0 && (!q.dsbase || !q.r_s || !q.dx_s)) ||
                      (q.m > 0 && (!q.r_y || !q.dy)));
    // the Newton-system arrays are required unless the batch holds IPM memory
    if (!io && L.ipm_rows == 0) return MDS_ENULL;
    newton_io = newton_io && io;
  }
  mds_batch *b = new (std::nothrow) mds_batch();
  if (!b) return MDS_EINVAL;
  b->caller = (hipStream_t)stream;
  if (hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) != hipSuccess) {
    delete b;
    return MDS_EHIP;
  }
  b->count = count;
  b->Nmax = L.Nmax;
  b->nsmax = L.nsmax;
  b->nslots = L.nslots;
  b->grid = L.nslots;
  b->nb = (opts && opts->nb > 0) ? opts->nb : BNB;
  b->use_graph = !(opts && opts->use_graph == 0);
  b->mixed = (opts && opts->precision == MDS_FP32) ? 1 : 0;
  b->refine_max = (opts && opts->refine_steps > 0) ? opts->refine_steps : 10;
  b->alpha = (1.0 + std::sqrt(17.0)) / 8.0;
  b->ipm_rows = L.ipm_rows;
  b->newton_io = newton_io;
  char *base = (char *)workspace;
  size_t o = 0;
  b->d_probs = (ProbDev *)(base + o);
  o += L.probs;
  b->d_slots = (SlotDev *)(base + o);
  o += L.slots;
  b->d_order = (int32_t *)(base + o);
  o += L.order;
  b->d_queue = (int32_t *)(base + o);
  b->d_t0 = (unsigned long long *)(base + o + 64);
  b->d_dc = (double *)(base + o + 128);
  o += L.ctl;
  b->d_results = (ResultDev *)(base + o);
  o += L.results;
  char *csc_base = base + o;
  o += L.csc_total;
  if (L.ipm_rows > 0) {
    b->d_ipms = (IpmDev *)(base + o);
    o += L.ipms;
    b->d_ipm_res = (IpmResDev *)(base + o);
    o += L.ipm_res;
    b->d_trace = (IpmIterDev *)(base + o);
    o += L.trace;
  }
  std::vector<ProbDev> hp(count);
  hipStream_t s = b->caller;
  for (int p = 0; p < count; ++p) {
    const mds_batch_problem &q = probs_host[p];
    char *c = csc_base + L.csc_off[p];
    int32_t *cptr = (int32_t *)c;
    c += al256(4 * ((size_t)q.n_s + 1));
    int32_t *crow = (int32_t *)c;
    c += al256(4 * (size_t)q.nnz_s + 4);
    double *cval = (double *)c;
    c += al256(8 * (size_t)q.nnz_s + 8);
    int32_t *fill = (int32_t *)c;
    launch_csc_build(s, q.m, q.n_s, q.nnz_s, q.Js_rowptr, q.Js_col, q.Js_val, cptr, crow, cval,
                     fill);
    ProbDev d{};
    d.nd = q.n_d;
    d.ns = q.n_s;
    d.m = q.m;
    d.nnz = (int32_t)q.nnz_s;
    d.H = q.H;
    d.Jd = q.J_d;
    d.rp = q.Js_rowptr;
    d.ci = q.Js_col;
    d.v = q.Js_val;
    d.cptr = cptr;
    d.crow = crow;
    d.cval = cval;
    d.sigma_d = q.sigma_d;
    d.dsbase = q.dsbase;
    d.r_d = q.r_d;
    d.r_s = q.r_s;
    d.r_y = q.r_y;
    d.dx_d = q.dx_d;
    d.dx_s = q.dx_s;
    d.dy = q.dy;
    hp[p] = d;
  }
  std::vector<SlotDev> hs(L.nslots);
  const size_t N = (size_t)L.Nmax;
  const size_t nmax_ipm = [&]() {
    size_t t = 0;
    for (int p = 0; p < count; ++p)
      t = std::max(t, (size_t)probs_host[p].n_d + (size_t)probs_host[p].n_s);
    return t;
  }();
  for (int k = 0; k < L.nslots; ++k) {
    char *c = base + o + (size_t)k * (L.slot_bytes + L.slot_ipm);
    SlotDev &S = hs[k];
    if (L.ipm_rows > 0) {
      char *q = c + L.slot_bytes;
      double **vn[8] = {&S.sig, &S.rx, &S.dx, &S.dzl, &S.dzu, &S.xt, &S.gf, &S.jty};
      for (double **v : vn) {
        *v = (double *)q;
        q += al256_(8 * nmax_ipm);
      }
      double **vm[3] = {&S.ry, &S.dy, &S.cx};
      for (double **v : vm) {
        *v = (double *)q;
        q += al256_(8 * (size_t)L.mmax);
      }
      S.dsb = (double *)q;
      q += al256_(8 * (size_t)L.nsmax);
      S.hx = (double *)q;
      q += al256_(8 * (size_t)L.ndmax);
      S.prev = (double *)q;
      q += al256_(8 * (nmax_ipm + (size_t)L.mmax));
      S.filt = (double *)q;
    }
    S.buf[0] = (double *)c;
    c += al256(8 * N * N);
    S.buf[1] = (double *)c;
    c += al256(8 * N * N);
    S.W = (double *)c;
    c += al256(8 * N * (kMaxNb + 2));
    S.zero = (double *)c;  // after both matrix buffers and W: every offset to it is positive
    c += al256(8 * 64);
    S.dd = (double *)c;
    c += al256(8 * N);
    S.ds = (double *)c;
    c += al256(8 * N);
    S.inv_d = (double *)c;
    c += al256(8 * (size_t)std::max(L.nsmax, 1));
    S.src = (int32_t *)c;
    c += al256(4 * N);
    S.ipiv = (int32_t *)c;
    c += al256(4 * N);
    S.blk = (int32_t *)c;
    c += al256(4 * N);
    S.pk0 = (int32_t *)c;
    c += al256(4 * (N + 4));
    S.st = (FacState *)c;
    c += al256(sizeof(FacState));
    S.eq = (double *)c;
    c += al256(8 * N);
    S.res = (double *)c;
    // mixed precision: two FP32 N x N halves of buf[1]
    S.x32[0] = (float *)S.buf[1];
    S.x32[1] = (float *)S.buf[1] + N * N;
  }
  // largest problems first (LPT), ties by index
  std::vector<int32_t> order(count);
  for (int p = 0; p < count; ++p) order[p] = p;
  std::stable_sort(order.begin(), order.end(), [&](int a, int c) {
    return probs_host[a].n_d + probs_host[a].m > probs_host[c].n_d + probs_host[c].m;
  });
  bool ok = true;
  for (int k = 0; k < L.nslots && ok; ++k)
    ok = hipMemsetAsync((void *)hs[k].zero, 0, 8 * 64, s) == hipSuccess;
  ok = ok &&
       hipMemcpyAsync(b->d_probs, hp.data(), sizeof(ProbDev) * count, hipMemcpyHostToDevice,
                           s) == hipSuccess &&
            hipMemcpyAsync(b->d_slots, hs.data(), sizeof(SlotDev) * L.nslots,
                           hipMemcpyHostToDevice, s) == hipSuccess &&
            hipMemcpyAsync(b->d_order, order.data(), 4 * (size_t)count, hipMemcpyHostToDevice,
                           s) == hipSuccess &&
            hipGetLastError() == hipSuccess && hipStreamSynchronize(s) == hipSuccess;
  if (!ok) {
    (void)hipStreamDestroy(b->stream);
    delete b;
    return MDS_EHIP;
  }
  b->h_results.resize(count);
  *out = b;
  return MDS_OK;
}

int mds_batch_run(mds_batch *b, double mu, mds_batch_result *results_host) {
  if (!b) return MDS_ENULL;
  if (!(mu >= 0.0)) return MDS_EINVAL;
  if (!b->newton_io) {
    snprintf(b->err, sizeof(b->err), "the batch was created without Newton-system arrays");
    return MDS_ESTATE;
  }
  const double dc = 1e-8 * std::pow(mu, 0.25);
  // inputs and outputs are ordered on the caller's stream
  hipError_t e = hipStreamSynchronize(b->caller);
  if (e != hipSuccess) return fail(b, MDS_EHIP, "caller stream", e);
  e = hipMemcpyAsync(b->d_dc, &dc, 8, hipMemcpyHostToDevice, b->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
  if (e != hipSuccess) return fail(b, MDS_EHIP, "batch parameters", e);
  int st = run_once(b);
  if (st != MDS_OK) return st;
  unsigned long long t0 = 0;
  if (hipMemcpyAsync(b->h_results.data(), b->d_results, sizeof(ResultDev) * b->count,
                     hipMemcpyDeviceToHost, b->stream) != hipSuccess ||
      hipMemcpyAsync(&t0, b->d_t0, 8, hipMemcpyDeviceToHost, b->stream) != hipSuccess ||
      hipStreamSynchronize(b->stream) != hipSuccess)
    return MDS_EHIP;
  if (results_host) {
    for (int p = 0; p < b->count; ++p) {
      const ResultDev &r = b->h_results[p];
      mds_batch_result &o = results_host[p];
      o.npos = r.npos;
      o.nzero = r.nzero;
      o.nneg = r.nneg;
      o.trials = r.trials;
      o.delta_w = r.delta_w;
      o.delta_c = r.delta_c;
      o.t_start = r.t_start - (int64_t)t0;
      o.t_done = r.t_done - (int64_t)t0;
      o.status = r.status;
      o.slot = r.pad;
      o.refine_steps = r.refine_steps;
      o.pad = 0;
      o.residual = r.residual;
    }
  }
  return MDS_OK;
}

int mds_batch_ipm(mds_batch *b, const mds_batch_ipm_problem *ipm_host,
                  const mds_ipm_opts *opts, mds_batch_ipm_result *results_host,
                  mds_batch_ipm_iter *trace_host) {
  if (!b || !ipm_host) return MDS_ENULL;
  if (b->ipm_rows <= 0) {
    snprintf(b->err, sizeof(b->err), "the batch was created without IPM memory");
    return MDS_ESTATE;
  }
  if (b->mixed) {
    snprintf(b->err, sizeof(b->err), "the whole-IPM batch runs in FP64");
    return MDS_ESTATE;
  }
  mds_ipm_opts o{1e-8, 0.1, 200, 2, 1e20, 0, 0};
  if (opts) o = *opts;
  if (!(o.tol > 0.0) || !(o.mu0 > 0.0) || o.max_iter < 1 || o.max_iter + 1 > b->ipm_rows ||
      o.refine_steps < 0 || !(o.dw_max > 0.0))
    return MDS_EINVAL;
  std::vector<IpmDev> hq(b->count);
  for (int p = 0; p < b->count; ++p) {
    const mds_batch_ipm_problem &q = ipm_host[p];
    IpmDev d{};
    d.c = q.c;
    d.w = q.w;
    d.g = q.g;
    d.b = q.b;
    d.xl = q.xl;
    d.xu = q.xu;
    d.x = q.x;
    d.y = q.y;
    d.zl = q.zl;
    d.zu = q.zu;
    hq[p] = d;
  }
  std::vector<ProbDev> hp(b->count);
  hipError_t e = hipMemcpyAsync(hp.data(), b->d_probs, sizeof(ProbDev) * b->count,
                                hipMemcpyDeviceToHost, b->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
  if (e != hipSuccess) return fail(b, MDS_EHIP, "batch problems", e);
  for (int p = 0; p < b->count; ++p) {
    const mds_batch_ipm_problem &q = ipm_host[p];
    const int nd = hp[p].nd, ns = hp[p].ns, m = hp[p].m;
    if ((nd > 0 && !q.c) || (ns > 0 && (!q.w || !q.g)) || (m > 0 && (!q.b || !q.y)) ||
        (nd + ns > 0 && (!q.xl || !q.xu || !q.x || !q.zl || !q.zu)))
      return MDS_ENULL;
  }
  e = hipStreamSynchronize(b->caller);
  if (e != hipSuccess) return fail(b, MDS_EHIP, "caller stream", e);
  e = hipMemcpyAsync(b->d_ipms, hq.data(), sizeof(IpmDev) * b->count, hipMemcpyHostToDevice,
                     b->stream);
  if (e != hipSuccess) return fail(b, MDS_EHIP, "ipm descriptors", e);
  IpmParams prm{o.tol, o.mu0, o.dw_max, o.max_iter, o.refine_steps, b->ipm_rows, 0};
  k_batch_reset<<<1, 64, 0, b->stream>>>(b->d_queue, b->d_t0);
  k_batch_ipm<<<(unsigned)b->grid, BT, 0, b->stream>>>(b->count, b->d_order, b->d_probs,
                                                       b->d_ipms, b->d_slots, b->nb, b->alpha,
                                                       prm, b->d_queue, b->d_t0, b->d_ipm_res,
                                                       b->d_trace);
  e = hipGetLastError();
  if (e != hipSuccess) return fail(b, MDS_EHIP, "batch ipm launch", e);
  std::vector<IpmResDev> hr(b->count);
  unsigned long long t0 = 0;
  e = hipMemcpyAsync(hr.data(), b->d_ipm_res, sizeof(IpmResDev) * b->count,
                     hipMemcpyDeviceToHost, b->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(&t0, b->d_t0, 8, hipMemcpyDeviceToHost, b->stream);
  std::vector<IpmIterDev> ht;
  if (e == hipSuccess && trace_host) {
    ht.resize((size_t)b->count * b->ipm_rows);
    e = hipMemcpyAsync(ht.data(), b->d_trace, sizeof(IpmIterDev) * ht.size(),
                       hipMemcpyDeviceToHost, b->stream);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
  if (e != hipSuccess) return fail(b, MDS_EHIP, "batch ipm results", e);
  if (results_host) {
    for (int p = 0; p < b->count; ++p) {
      const IpmResDev &r = hr[p];
      mds_batch_ipm_result &d = results_host[p];
      memset(&d, 0, sizeof(d));
      d.status = r.status;
      d.iters = r.iters;
      d.mu = r.mu;
      d.E0 = r.E0;
      d.t_start = r.t_start - (int64_t)t0;
      d.t_done = r.t_done - (int64_t)t0;
      d.slot = r.slot;
      d.factorizations = r.facs;
    }
  }
  if (trace_host) {
    for (size_t k = 0; k < ht.size(); ++k) {
      const IpmIterDev &r = ht[k];
      mds_batch_ipm_iter &d = trace_host[k];
      memset(&d, 0, sizeof(d));
      d.mu = r.mu;
      d.alpha_pr = r.alpha_pr;
      d.delta_w = r.delta_w;
      d.inertia[0] = r.inertia[0];
      d.inertia[1] = r.inertia[1];
      d.inertia[2] = r.inertia[2];
      d.trials = r.trials;
      d.backtracks = r.backtracks;
    }
  }
  return MDS_OK;
}

int mds_batch_autotune(mds_batch *b, double mu, mds_batch_opts *chosen_host) {
  if (!b) return MDS_ENULL;
  const int nbs[3] = {8, 12, BNB};
  int grids[3] = {std::min(b->nslots, 64), std::min(b->nslots, 128), b->nslots};
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return MDS_EHIP;
  float best = 1e30f;
  int bnb = b->nb, bgrid = b->grid;
  for (int gi = 0; gi < 3; ++gi) {
    if (gi > 0 && grids[gi] == grids[gi - 1]) continue;
    for (int ni = 0; ni < 3; ++ni) {
      b->nb = nbs[ni];
      b->grid = grids[gi];
      int st = mds_batch_run(b, mu, nullptr);  // warm (and builds the graph)
      if (st != MDS_OK) return st;
      (void)hipEventRecord(e0, b->stream);
      st = run_once(b);
      (void)hipEventRecord(e1, b->stream);
      if (st != MDS_OK || hipEventSynchronize(e1) != hipSuccess) return MDS_EHIP;
      float ms = 0.0f;
      (void)hipEventElapsedTime(&ms, e0, e1);
      if (ms < best) {
        best = ms;
        bnb = b->nb;
        bgrid = b->grid;
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  b->nb = bnb;
  b->grid = bgrid;
  if (chosen_host) {
    memset(chosen_host, 0, sizeof(*chosen_host));
    chosen_host->nb = bnb;
    chosen_host->grid = bgrid;
    chosen_host->use_graph = b->use_graph ? 1 : 0;
    chosen_host->precision = b->mixed ? MDS_FP32 : MDS_FP64;
    chosen_host->refine_steps = b->refine_max;
  }
  return MDS_OK;
}

int mds_batch_get_config(const mds_batch *b, mds_batch_opts *out_host) {
  if (!b || !out_host) return MDS_ENULL;
  memset(out_host, 0, sizeof(*out_host));
  out_host->nb = b->nb;
  out_host->grid = b->grid;
  out_host->use_graph = b->use_graph ? 1 : 0;
  out_host->precision = b->mixed ? MDS_FP32 : MDS_FP64;
  out_host->refine_steps = b->refine_max;
  return MDS_OK;
}

const char *mds_batch_last_error(const mds_batch *b) { return b ? b->err : "null batch"; }

void mds_batch_destroy(mds_batch *b) {
  if (!b) return;
  if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->stream) (void)hipStreamDestroy(b->stream);
  delete b;
}

}  // extern "C"
