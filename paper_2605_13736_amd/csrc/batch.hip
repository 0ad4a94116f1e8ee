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
// lower tile, mirrored through the wave's LDS tile.
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
  double(*t)[TW + 1] = s_t + wv * TW;
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
          xv[a][b][r] = ok ? X[(size_t)si + (size_t)sc * ld] : 0.0;
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
          if (c < N && i < N && (!diag || i >= c)) {
            const double v = xv[a][b][r] - acc[a][b][r];
            Y[(size_t)i + (size_t)c * ld] = v;
            t[c - c0][i - i0] = v;
          }
        }
    __builtin_amdgcn_wave_barrier();
    __asm__ __volatile__("s_waitcnt lgkmcnt(0)" ::: "memory");
    for (int e = lane; e < TW * TW; e += 64) {
      const int cl = e & (TW - 1), il = e / TW;
      const int c = c0 + cl, i = i0 + il;
      if (c < N && i < N && i > c && (!diag || il >= cl)) Y[(size_t)c + (size_t)i * ld] = t[cl][il];
    }
    __builtin_amdgcn_wave_barrier();
    __asm__ __volatile__("s_waitcnt lgkmcnt(0)" ::: "memory");
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
  const int ntiles = nt * (nt + 1) / 2;
  const size_t ld = (size_t)N;
  double(*t)[TW + 1] = s_t + wv * TW;
  for (int x = wv; x < ntiles; x += NWAVE) {
    int ti = (int)((sqrt(8.0 * (double)x + 1.0) - 1.0) * 0.5);
    while ((ti + 1) * (ti + 2) / 2 <= x) ++ti;
    while (ti * (ti + 1) / 2 > x) --ti;
    const int tj = x - ti * (ti + 1) / 2;
    const int i0 = kend + ti * TW, c0 = kend + tj * TW;
    const int li = (lane < 32) ? i0 + lane : c0 + (lane - 32);
    const int sidx = gsrc[(unsigned)min(li, N - 1)];
    constexpr int KS = (BNB + 1 + 3) / 4;
    double aw[KS][2], bw[KS][2];  // converted to FP32 after all loads are issued
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const int tt = 4 * ks + l4;
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        const int c = c0 + a * 16 + l16;
        aw[ks][a] = gW[(unsigned)((tt < jw && c < N) ? c + tt * N : zW)];
      }
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
          xv[a][b][r] = gX[(unsigned)(ok ? si + sc * N : zX)];
        }
    float av[KS][2], bv[KS][2];
#pragma unroll
    for (int ks = 0; ks < KS; ++ks)
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        av[ks][a] = (float)aw[ks][a];
        bv[ks][a] = (float)bw[ks][a];
      }
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
          if (c < N && i < N && (!diag || i >= c)) {
            const float v = xv[a][b][r] - acc[a][b][r];
            oY[(unsigned)(i + c * N)] = v;
            t[c - c0][i - i0] = (double)v;
          }
        }
    __builtin_amdgcn_wave_barrier();
    __asm__ __volatile__("s_waitcnt lgkmcnt(0)" ::: "memory");
    for (int e = lane; e < TW * TW; e += 64) {
      const int cl = e & (TW - 1), il = e / TW;
      const int c = c0 + cl, i = i0 + il;
      if (c < N && i < N && i > c && (!diag || il >= cl)) oY[(unsigned)(c + i * N)] = (float)t[cl][il];
    }
    __builtin_amdgcn_wave_barrier();
    __asm__ __volatile__("s_waitcnt lgkmcnt(0)" ::: "memory");
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
  char err[256] = {0};
};

namespace {

size_t al256(size_t b) { return (b + 255) & ~(size_t)255; }

struct BatchLayout {
  size_t probs, slots, order, ctl, results, csc_total, slot_bytes, total;
  int Nmax, nsmax, nslots;
  std::vector<size_t> csc_off;
};

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
  L.total = L.probs + L.slots + L.order + L.ctl + L.results + L.csc_total + L.slot_bytes * L.nslots;
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
  for (int p = 0; p < count; ++p) {
    const mds_batch_problem &q = probs_host[p];
    if ((q.n_d > 0 && (!q.H || !q.sigma_d || !q.r_d || !q.dx_d)) ||
        (q.m > 0 && q.n_d > 0 && !q.J_d) || !q.Js_rowptr ||
        (q.nnz_s > 0 && (!q.Js_col || !q.Js_val)) ||
        (q.n_s > 0 && (!q.dsbase || !q.r_s || !q.dx_s)) || (q.m > 0 && (!q.r_y || !q.dy)))
      return MDS_ENULL;
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
  for (int k = 0; k < L.nslots; ++k) {
    char *c = base + o + (size_t)k * L.slot_bytes;
    SlotDev &S = hs[k];
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
