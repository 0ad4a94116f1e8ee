#pragma once
// Register-resident Bunch-Kaufman panel (Sec. 2.3), as a workgroup-level
// device function shared by the panel kernel and the batched kernel: same decisions and the
// same output layout as the panel in bk.hip, for at most R * T rows left.
//
// One workgroup of 512 threads (two waves per SIMD).  Thread t owns the
// physical rows rho = k0 + t + 512 r (r < R) of the buffer X for the whole
// panel and keeps their multipliers L[rho, k0:k0+nb] in registers
// (R * nb <= 64 doubles).  An interchange p <-> q only changes which logical
// position a physical row holds (pos[r], and the logical -> physical map
// s_map used to address columns); multipliers stay with their physical row,
// which is exactly the row interchange of the panel's L.  The updated column
//   w = A0[:, c] - L_panel W_panel[c, :]'
// therefore costs no memory traffic for L, and the un-updated values of the
// next pivot column are the prefetched values of one of the columns k, k+1
// or k+2 (whichever the interchange puts at the next position).
//
// Every VALU instruction of a pivot step costs a wave several cycles, so the
// step is written for a small instruction count: register indices are
// static, groups of 8 columns not yet factored are skipped by wave-uniform
// branches (inside a group, a column not yet factored has L = 0 and its W
// entry is forced to 0, an exact no-op), and the W row (L D) of a pivot
// candidate is formed lane-parallel by the wave that owns the row.
//
// The panel stops once j >= nb - 1 (width nb - 1, or nb after a final 2x2),
// so that a 2x2 pivot always fits the register tile.
#include <climits>

#include "internal.hpp"
#include "wave.hpp"

namespace mds {
namespace panel {

// Entry (r, c) of the symmetric trailing matrix, of which only the lower
// triangle is kept current: (r, c) itself when r >= c, else its mirror (c, r).
// Offsets fit in 32 bits (N <= 20480).
template <typename TX>
__device__ inline TX sym_at(const TX *X, int r, int c, int ld) {
  return X[(r >= c) ? r + c * ld : c + r * ld];
}

__device__ inline void amax_combine(double &v, int &i, double v2, int i2) {
  if (v2 > v || (v2 == v && i2 < i)) {
    v = v2;
    i = i2;
  }
}

// Keeps a wave-uniform branch a branch: a block holding it cannot be
// if-converted into selects that would execute its instructions always.
__device__ inline void keep_branch() { __asm__ __volatile__(""); }

// Orders this wave's earlier LDS writes before its later LDS reads.
__device__ inline void lds_wave_sync() { __asm__ __volatile__("s_waitcnt lgkmcnt(0)" ::: "memory"); }

// Lane t < NB of the calling wave: W[t] of the L row in Lrow, from the stored
// coefficients (cA diagonal, cB / cC off-diagonal of a 2x2 for its first /
// second column; zero for columns not yet stored) plus, for the step that
// just factored columns jc (and jc + 1 if two), its D from registers.
template <int NB>
__device__ inline double w_lane(const double *Lrow, const double *cA, const double *cB,
                                const double *cC, int t, int jc, bool cur, bool two, double d0,
                                double d1, double db) {
  const double lt = Lrow[t];
  const double ln = (t + 1 < NB) ? Lrow[t + 1] : 0.0;
  const double lp = (t >= 1) ? Lrow[t - 1] : 0.0;
  double v = lt * cA[t];
  v = v + ln * cB[t];
  v = v + lp * cC[t];
  if (cur) {
    if (t == jc) v = v + (two ? (lt * d0 + ln * db) : lt * d0);
    if (two && t == jc + 1) v = v + (lt * d1 + lp * db);
  }
  return v;
}

// X holds the trailing matrix in FP64 or (mixed precision) FP32; every
// value is widened to FP64 on load and all panel arithmetic is FP64.
template <int T, int R, int NB, typename TX>
__device__ inline void panel_reg_dev(int N, int nb, double alpha,
                                                    const TX *__restrict__ X,
                                                    double *__restrict__ Lout,
                                                    int32_t *__restrict__ src_out,
                                                    double *__restrict__ W,
                                                    double *__restrict__ dd,
                                                    double *__restrict__ ds,
                                                    int32_t *__restrict__ ipiv,
                                                    int32_t *__restrict__ blk, FacState *st,
                                                    int32_t *__restrict__ panel_k0) {
  constexpr int NWV = T / 64;
  static_assert(NB <= 64 && NB % 8 == 0, "one lane per panel column, chunks of 8");
  __shared__ double s_wk[NB], s_wi[NB];            // W rows of the pivot k and of imax
  __shared__ double s_cA[NB], s_cB[NB], s_cC[NB];  // W = L D coefficients per panel column
  __shared__ double s_lrow[NB];                    // L row of imax / of the next pivot
  __shared__ double s_pdd[NB], s_pds[NB];          // D and pivot records (written at the end)
  __shared__ int s_pip[NB], s_pbk[NB];
  __shared__ double s_rv[NWV];
  __shared__ int s_ri[NWV];
  __shared__ double s_akk, s_aii, s_wki;
  __shared__ int s_k0, s_err;
  // per owned row: un-updated values of the current pivot column, its updated
  // values, the updated candidate column
  __shared__ double s_acur[R * T], s_wkc[R * T], s_wic[R * T];
  // logical -> physical row of the active part (X is addressed physically)
  __shared__ int s_map[R * T];

  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  if (tid == 0) {
    s_k0 = st->k;
    s_err = st->xerr;  // an earlier panel of this factorization aborted
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
  if (k0 >= N || s_err) return;
  // the tile must hold every remaining row (the host guarantees it); if not,
  // the factorization is flagged as failed rather than left incomplete
  if (N - k0 > R * T) {
    if (tid == 0) st->xerr = 1;
    return;
  }
  const int ld = N;  // N <= 20480 (a cooperative factorization's tail): offsets fit in 32 bits

  double Lr[R][NB];
  // prefetched un-updated column values, kept in the storage type and
  // widened where used: a widening next to a conditional load would make the
  // compiler wait for the load there
  TX pre1[R], pre2[R];
  int pos[R];  // logical position of the owned physical row (-1: past N)
#pragma unroll
  for (int r = 0; r < R; ++r) {
#pragma unroll
    for (int t = 0; t < NB; ++t) Lr[r][t] = 0.0;
    const int rho = k0 + tid + T * r;
    pos[r] = (rho < N) ? rho : -1;
    s_map[r * T + tid] = rho;
    s_acur[r * T + tid] = (rho < N) ? (double)X[rho + k0 * ld] : 0.0;
    pre1[r] = pre2[r] = (TX)0;
  }
  __syncthreads();

  int k = k0, j = 0;
  int c_pos = 0, c_zero = 0, c_neg = 0, c_2x2 = 0, first_zero = 0;
  // D of the previous step; thread 0 stores its coefficients at the start of
  // the next step (the W row of the next pivot takes them from registers)
  int pj = -1;
  bool p2 = false;
  double pA0 = 0.0, pB0 = 0.0, pA1 = 0.0;

  while (j < nb - 1 && k < N) {
    if (tid == 0 && pj >= 0) {
      s_cA[pj] = pA0;
      s_cB[pj] = pB0;
      if (p2) {
        s_cA[pj + 1] = pA1;
        s_cC[pj + 1] = pB0;
      }
    }
    // ---- prefetch the un-updated column k+1 --------------------------------
    {
      const int sc1 = (k + 1 < N) ? s_map[k + 1 - k0] : 0;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int rho = k0 + tid + T * r;
        if (pos[r] >= k && k + 1 < N) pre1[r] = sym_at(X, rho, sc1, ld);
      }
    }
    // ---- updated column k and its largest off-diagonal magnitude -----------
    double a[R];
#pragma unroll
    for (int r = 0; r < R; ++r) a[r] = s_acur[r * T + tid];
    // columns t < j in chunks of 8: one batch of LDS reads per chunk
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
    double bv = -1.0;
    int bi = INT_MAX;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      if (pos[r] >= k) {
        s_wkc[r * T + tid] = a[r];
        if (pos[r] == k) s_akk = a[r];
        else amax_combine(bv, bi, fabs(a[r]), pos[r]);
      }
    }
    wave::amax(bv, bi);
    if (lane == 0) {
      s_rv[wid] = bv;
      s_ri[wid] = bi;
    }
    __syncthreads();
    double colmax = -1.0;
    int imax = INT_MAX;
#pragma unroll
    for (int w = 0; w < NWV; ++w) amax_combine(colmax, imax, s_rv[w], s_ri[w]);
    if (colmax < 0.0) {
      colmax = 0.0;
      imax = k;
    }
    const double akk = s_akk, absakk = fabs(akk);

    // ---- Bunch-Kaufman decision ----------------------------------------------
    int kind;  // 0 zero, 1 1x1, 2 1x1 (second test), 3 1x1 swap, 4 2x2
    int kstep = 1, q = k;
    double aii = 0.0, wki = 0.0;
    if (fmax(absakk, colmax) == 0.0 || isnan(absakk)) {
      kind = 0;
    } else if (absakk >= alpha * colmax) {
      kind = 1;
    } else {
      // candidate column imax (and column k+2, which follows a 2x2 pivot):
      // un-updated values, and the W row of imax
      const int src_i = s_map[imax - k0];
      const int src_k2 = (k + 2 < N) ? s_map[k + 2 - k0] : 0;
      double wic[R];
      bool own = false;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int rho = k0 + tid + T * r;
        wic[r] = 0.0;
        if (pos[r] >= k) {
          wic[r] = (double)sym_at(X, rho, src_i, ld);
          if (k + 2 < N) pre2[r] = sym_at(X, rho, src_k2, ld);
        }
        if (pos[r] == imax) {
          own = true;
#pragma unroll
          for (int t = 0; t < NB; ++t) s_lrow[t] = Lr[r][t];
          s_wki = s_wkc[r * T + tid];
        }
      }
      if (__ballot(own) != 0) {
        lds_wave_sync();
        if (lane < NB)
          s_wi[lane] = w_lane<NB>(s_lrow, s_cA, s_cB, s_cC, lane, 0, false, false, 0.0, 0.0, 0.0);
      }
      __syncthreads();
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
      double rv = 0.0;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        if (pos[r] >= k) {
          s_wic[r * T + tid] = wic[r];
          if (pos[r] == imax) s_aii = wic[r];
          else rv = fmax(rv, fabs(wic[r]));
        }
      }
      rv = wave::max(rv);
      if (lane == 0) s_rv[wid] = rv;
      __syncthreads();
      double rowmax = 0.0;
#pragma unroll
      for (int w = 0; w < NWV; ++w) rowmax = fmax(rowmax, s_rv[w]);
      aii = s_aii;
      wki = s_wki;
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
    // D of this step (identical in every thread)
    double Da = akk, Dc = 0.0, Db = 0.0, det = 1.0;
    if (kind == 3) Da = aii;
    // a zero (or NaN) pivot eliminates nothing: its W column is zero
    const double Dw = (kind == 0) ? 0.0 : Da;
    if (kind == 4) {
      Db = wki;
      Dc = aii;
      det = Da * Dc - Db * Db;
    }
    // one reciprocal per step (wave-uniform), multipliers by multiplication
    const double rD = (kind == 4) ? 1.0 / det : (kind == 3) ? 1.0 / aii : 1.0 / akk;

    // ---- multipliers, new positions, next column ------------------------------
    double l0[R], l1[R];
    bool act[R];
    bool ownn = false;
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
#pragma unroll
    for (int r = 0; r < R; ++r) {
      if (pos[r] == kn) {
        ownn = true;
#pragma unroll
        for (int t = 0; t < NB; ++t) s_lrow[t] = Lr[r][t];
      }
    }

    // ---- pivot records, map, and the W row of the next pivot -----------------
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
    if (__ballot(ownn) != 0 && kn < N) {
      lds_wave_sync();
      if (lane < NB)
        s_wk[lane] = w_lane<NB>(s_lrow, s_cA, s_cB, s_cC, lane, j, true, kind == 4,
                                (kind == 4) ? Da : Dw, Dc, Db);
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
  if (tid == 0 && pj >= 0) {
    s_cA[pj] = pA0;
    s_cB[pj] = pB0;
    if (p2) {
      s_cA[pj + 1] = pA1;
      s_cC[pj + 1] = pB0;
    }
  }
  __syncthreads();
  for (int t = tid; t < jend; t += T) {
    dd[k0 + t] = s_pdd[t];
    ds[k0 + t] = s_pds[t];
    ipiv[k0 + t] = s_pip[t];
    blk[k0 + t] = s_pbk[t];
  }
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int pr = pos[r];
    if (pr < 0) continue;
    const int rho = k0 + tid + T * r;
#pragma unroll
    for (int t = 0; t < NB; ++t)
      if (t < jend && pr > k0 + t) Lout[pr + (k0 + t) * ld] = Lr[r][t];
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
  if (tid == 0) {
    const int b = st->npanel;
    panel_k0[b + 1] = kend;
    st->npanel = b + 1;
    st->k = kend;
    st->npos += c_pos;
    st->nzero += c_zero;
    st->nneg += c_neg;
    st->n2x2 += c_2x2;
    if (st->info == 0 && first_zero != 0) st->info = first_zero;
  }
}

}  // namespace panel
}  // namespace mds
