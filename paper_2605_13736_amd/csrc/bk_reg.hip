// Register-resident Bunch-Kaufman panel (Sec. 2.3): same decisions and the
// same output layout as the panel in bk.hip, for N <= 4096.
//
// One workgroup of 512 threads (two waves per SIMD); thread t owns the fixed
// rows k0 + t + 512 r (r < R) of the panel for its whole duration and keeps
// their multipliers L[i, k0:k0+nb] in registers (R * nb <= 64 doubles), so the updated column
//   w = A0[:, c] - L_panel W_panel[c, :]'
// costs no memory traffic for L.  W rows are formed on demand as L D.  The
// un-updated values of the next candidate column k+1 are prefetched at the
// start of every pivot step (column k+2 as soon as a 2x2 pivot is chosen) and
// patched for the interchange the step makes, so the only global-memory round trip on the critical path is the
// column of a pivot candidate imax.  When an interchange p <-> q moves row
// contents between threads, the rows involved (k, k+1, imax) are published
// in LDS before the reduction barriers that precede the decision.
//
// The panel stops once j >= nb - 1 (width nb - 1, or nb after a final 2x2),
// so that a 2x2 pivot always fits the register tile.
#include <climits>

#include "internal.hpp"

namespace mds {
namespace {

constexpr int TMAX = 512;

__device__ inline void amax_combine(double &v, int &i, double v2, int i2) {
  if (v2 > v || (v2 == v && i2 < i)) {
    v = v2;
    i = i2;
  }
}

// W[i, t] = sum_s L[i, s] D[s, t] over the pivot block holding column t.
// Columns t < jlim use the panel's D from LDS; column jlim (and jlim+1) use
// the current step's D passed in registers (kind_cur: 1 = 1x1 d0, 2 = 2x2).
// Compiler-level memory barrier: keeps the LDS reads of a rarely taken row
// move inside its branch (hoisting them would pin NB doubles in registers).
__device__ inline void row_barrier() { __asm__ __volatile__("" ::: "memory"); }

template <int NB>
__device__ inline void w_row(const double (&L)[NB], const double *sD0, const double *sD1,
                             const int *sB, int jlim, int kind_cur, double d0, double d1,
                             double dsub, double *out) {
#pragma unroll
  for (int t = 0; t < NB; ++t) {
    double v = 0.0;
    if (t < jlim) {
      const int b = sB[t];
      if (b == 1) {
        v = L[t] * sD0[t];
      } else if (b == 2) {
        if (t + 1 < NB) v = L[t] * sD0[t] + L[t + 1] * sD1[t];
      } else if (b == 3) {
        if (t >= 1) v = L[t - 1] * sD1[t - 1] + L[t] * sD0[t];
      }
    } else if (t == jlim) {
      if (kind_cur == 1) {
        v = L[t] * d0;
      } else if (kind_cur == 2) {
        if (t + 1 < NB) v = L[t] * d0 + L[t + 1] * dsub;
      }
    } else if (t == jlim + 1 && kind_cur == 2) {
      if (t >= 1) v = L[t - 1] * dsub + L[t] * d1;
    }
    out[t] = v;
  }
}

// W[i, t] for t < jend into global memory (stride ld)
template <int NB>
__device__ inline void w_row_global(const double (&L)[NB], const double *sD0, const double *sD1,
                                    const int *sB, int jend, double *out, int ld) {
#pragma unroll
  for (int t = 0; t < NB; ++t) {
    if (t >= jend) continue;
    const int b = sB[t];
    double v = 0.0;
    if (b == 1) v = L[t] * sD0[t];
    else if (b == 2) {
      if (t + 1 < NB) v = L[t] * sD0[t] + L[t + 1] * sD1[t];
    } else if (b == 3) {
      if (t >= 1) v = L[t - 1] * sD1[t - 1] + L[t] * sD0[t];
    }
    out[t * ld] = v;
  }
}

template <int T, int R, int NB>
__global__ __launch_bounds__(T) void k_bk_panel_reg(int N, int nb, double alpha,
                                                    const double *__restrict__ X,
                                                    double *__restrict__ Lout,
                                                    int32_t *__restrict__ src_out,
                                                    double *__restrict__ W,
                                                    double *__restrict__ dd,
                                                    double *__restrict__ ds,
                                                    int32_t *__restrict__ ipiv,
                                                    int32_t *__restrict__ blk, FacState *st,
                                                    int32_t *__restrict__ panel_k0) {
  constexpr int NWV = T / 64;
  __shared__ double s_wk[NB], s_wi[NB];            // W rows of pivot k and candidate imax
  __shared__ double s_Lk[NB], s_Lk1[NB], s_Li[NB];  // L rows of k, k+1, imax
  __shared__ double s_D0[NB], s_D1[NB];            // panel D: diagonal, sub-diagonal
  __shared__ int s_B[NB];                          // 1: 1x1, 2/3: first/second of 2x2
  __shared__ double s_rv[NWV];
  __shared__ int s_ri[NWV];
  __shared__ double s_akk, s_aii;
  // s_x: [0] w_k[k+1], [1] w_i[k], [2] w_i[k+1], [3] w_k[imax], [4] A0[k+1,k+1],
  //      [5] A0[k,k], [6] A0[k+1,k], [7] A0[k+2,k+1]
  __shared__ double s_x[8];
  __shared__ int s_k0;

  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  if (tid == 0) s_k0 = st->k;
  for (int t = tid; t < NB; t += T) {
    s_wk[t] = 0.0;
    s_wi[t] = 0.0;
    s_D0[t] = 0.0;
    s_D1[t] = 0.0;
    s_B[t] = 0;
  }
  __syncthreads();
  const int k0 = s_k0;
  if (k0 >= N) return;
  const int ld = N;  // N <= 4096: every offset fits in 32 bits

  // un-updated values of the current column for the owned rows live in LDS
  // (s_acur[r * T + tid]) to leave the registers to L
  __shared__ double s_acur[R * T];
  // updated candidate column w_imax for the owned rows (LDS, for the same reason)
  __shared__ double s_wic[R * T];
  // updated pivot column w_k for the owned rows (LDS)
  __shared__ double s_wkc[R * T];
  // logical -> physical index map of the active part: the logical entry (x, c)
  // of the matrix is X[src(x) + src(c) * N].  Interchanges only update the map.
  __shared__ int s_map[T * R];
  double Lr[R][NB];
  double pre1[R], pre2[R];
  int srcr[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
#pragma unroll
    for (int t = 0; t < NB; ++t) Lr[r][t] = 0.0;
    const int i = k0 + tid + T * r;
    srcr[r] = i;
    s_map[r * T + tid] = i;
    s_acur[r * T + tid] = (i < N) ? X[i + k0 * ld] : 0.0;
    pre1[r] = pre2[r] = 0.0;
  }
  __syncthreads();

  int k = k0, j = 0;
  int c_pos = 0, c_zero = 0, c_neg = 0, c_2x2 = 0, first_zero = 0;

  while (j < nb - 1 && k < N) {
    // ---- prefetch the un-updated candidate next column k+1 ------------------
    {
      const int sc1 = (k + 1 < N) ? s_map[k + 1 - k0] : 0;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int i = k0 + tid + T * r;
        pre1[r] = (i > k && i < N) ? X[srcr[r] + sc1 * ld] : 0.0;
      }
    }
    // ---- updated column k and its largest off-diagonal magnitude -----------
    double bv = -1.0;
    int bi = INT_MAX;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int i = k0 + tid + T * r;
      if (i >= k && i < N) {
        const double ac = s_acur[r * T + tid];
        double a = ac;
#pragma unroll
        for (int t = 0; t < NB; ++t) a = fma(-Lr[r][t], s_wk[t], a);
        s_wkc[r * T + tid] = a;
        if (i == k) {
          s_akk = a;
          s_x[5] = ac;
#pragma unroll
          for (int t = 0; t < NB; ++t) s_Lk[t] = Lr[r][t];
        } else {
          if (i == k + 1) {
            s_x[0] = a;
            s_x[6] = ac;
#pragma unroll
            for (int t = 0; t < NB; ++t) s_Lk1[t] = Lr[r][t];
          }
          const double v = fabs(a);
          if (v > bv) {
            bv = v;
            bi = i;
          }
        }
      }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      const double v2 = __shfl_xor(bv, off);
      const int i2 = __shfl_xor(bi, off);
      amax_combine(bv, bi, v2, i2);
    }
    if (lane == 0) {
      s_rv[wid] = bv;
      s_ri[wid] = bi;
    }
    __syncthreads();
    double colmax = -1.0;
    int imax = INT_MAX;
#pragma unroll
    for (int q = 0; q < NWV; ++q) amax_combine(colmax, imax, s_rv[q], s_ri[q]);
    if (colmax < 0.0) {
      colmax = 0.0;
      imax = k;
    }
    const double akk = s_akk, absakk = fabs(akk);
    // physical indices of the rows that may move this step (read before any
    // thread updates the map)
    const int src_k = s_map[k - k0];
    const int src_k1 = (k + 1 < N) ? s_map[k + 1 - k0] : 0;
    const int src_k2 = (k + 2 < N) ? s_map[k + 2 - k0] : 0;
    const int src_i = s_map[imax - k0];

    // ---- Bunch-Kaufman decision ----------------------------------------------
    int kind;  // 0 zero, 1 1x1, 2 1x1 (second test), 3 1x1 swap, 4 2x2
    int kstep = 1, q = k;
    double aii = 0.0;
    if (fmax(absakk, colmax) == 0.0 || isnan(absakk)) {
      kind = 0;
    } else if (absakk >= alpha * colmax) {
      kind = 1;
    } else {
      // candidate column imax: publish its row (W, L, w_k) and load A0[:, imax]
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int i = k0 + tid + T * r;
        if (i == imax) {
          w_row<NB>(Lr[r], s_D0, s_D1, s_B, j, 0, 0.0, 0.0, 0.0, s_wi);
#pragma unroll
          for (int t = 0; t < NB; ++t) s_Li[t] = Lr[r][t];
          s_x[3] = s_wkc[r * T + tid];
        }
        if (i == k + 2) s_x[7] = pre1[r];
        s_wic[r * T + tid] = (i >= k && i < N) ? X[srcr[r] + src_i * ld] : 0.0;
      }
      __syncthreads();
      double rv = 0.0;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int i = k0 + tid + T * r;
        if (i >= k && i < N) {
          double a = s_wic[r * T + tid];
#pragma unroll
          for (int t = 0; t < NB; ++t) a = fma(-Lr[r][t], s_wi[t], a);
          s_wic[r * T + tid] = a;
          if (i == imax) s_aii = a;
          else rv = fmax(rv, fabs(a));
          if (i == k) s_x[1] = a;
          if (i == k + 1) {
            s_x[2] = a;
            s_x[4] = pre1[r];
          }
        }
      }
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) rv = fmax(rv, __shfl_xor(rv, off));
      if (lane == 0) s_rv[wid] = rv;
      __syncthreads();
      double rowmax = 0.0;
#pragma unroll
      for (int qq = 0; qq < NWV; ++qq) rowmax = fmax(rowmax, s_rv[qq]);
      aii = s_aii;
      if (absakk >= alpha * colmax * (colmax / rowmax)) {
        kind = 2;
      } else if (fabs(aii) >= alpha * rowmax) {
        kind = 3;
        q = imax;
      } else {
        kind = 4;
        q = imax;
        kstep = 2;
        // next column is k+2: load its un-updated values now (the patch below
        // replaces the entries this step's interchange changes)
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const int i = k0 + tid + T * r;
          pre2[r] = (i > k + 1 && i < N) ? X[srcr[r] + src_k2 * ld] : 0.0;
        }
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
      Db = s_x[3];
      Dc = aii;
      det = Da * Dc - Db * Db;
    }

    // ---- multipliers, row moves, copy of index p into index q, next column --
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int i = k0 + tid + T * r;
      if (i < k || i >= N) continue;
      if (kind <= 2) {
        if (i > k) {
          const double l = (kind == 0) ? 0.0 : s_wkc[r * T + tid] / akk;
#pragma unroll
          for (int t = 0; t < NB; ++t)
            if (t == j) Lr[r][t] = l;
        }
      } else if (kind == 3) {
        if (i == k) {
row_barrier();
#pragma unroll
          for (int t = 0; t < NB; ++t)
            if (t < j) Lr[r][t] = s_Li[t];
          srcr[r] = src_i;
          s_map[k - k0] = src_i;
        } else {
          const double c = (i == q) ? s_x[1] : s_wic[r * T + tid];
          if (i == q) {
row_barrier();
#pragma unroll
            for (int t = 0; t < NB; ++t)
              if (t < j) Lr[r][t] = s_Lk[t];
            srcr[r] = src_k;
            s_map[q - k0] = src_k;
          }
          const double l = c / aii;
#pragma unroll
          for (int t = 0; t < NB; ++t)
            if (t == j) Lr[r][t] = l;
        }
      } else {  // kind 4: 2x2 on (k, k+1) after k+1 <-> q
        if (i == k + 1) {
          if (sw) {
row_barrier();
#pragma unroll
            for (int t = 0; t < NB; ++t)
              if (t < j) Lr[r][t] = s_Li[t];
            srcr[r] = src_i;
            s_map[k + 1 - k0] = src_i;
          }
        } else if (i >= k + 2) {
          const bool isq = sw && (i == q);
          const double x0 = isq ? s_x[0] : s_wkc[r * T + tid];
          const double y0 = isq ? s_x[2] : s_wic[r * T + tid];
          if (isq) {
row_barrier();
#pragma unroll
            for (int t = 0; t < NB; ++t)
              if (t < j) Lr[r][t] = s_Lk1[t];
            srcr[r] = src_k1;
            s_map[q - k0] = src_k1;
          }
          const double l0 = (x0 * Dc - y0 * Db) / det;
          const double l1 = (y0 * Da - x0 * Db) / det;
#pragma unroll
          for (int t = 0; t < NB; ++t) {
            if (t == j) Lr[r][t] = l0;
            if (t == j + 1) Lr[r][t] = l1;
          }
        }
      }
      // un-updated values of the next column kn after this step's interchange
      double an = (kstep == 1) ? pre1[r] : pre2[r];
      if (sw) {
        if (q == kn) {
          if (i == q) an = (kind == 3) ? s_x[5] : s_x[4];
          else an = (kind == 3) ? s_acur[r * T + tid] : pre1[r];
        } else if (i == q) {
          an = (kind == 3) ? s_x[6] : s_x[7];
        }
      }
      s_acur[r * T + tid] = an;
    }

    // ---- pivot records and the W row of the next pivot -----------------------
    if (tid == 0) {
      if (kind == 4) {
        dd[k] = Da;
        dd[k + 1] = Dc;
        ds[k] = Db;
        ds[k + 1] = 0.0;
        ipiv[k] = -(q + 1);
        ipiv[k + 1] = -(q + 1);
        blk[k] = 2;
        blk[k + 1] = 3;
        s_D0[j] = Da;
        s_D0[j + 1] = Dc;
        s_D1[j] = Db;
        s_B[j] = 2;
        s_B[j + 1] = 3;
        c_pos++;
        c_neg++;
        c_2x2++;
      } else {
        dd[k] = Da;
        ds[k] = 0.0;
        ipiv[k] = q + 1;
        blk[k] = 1;
        s_D0[j] = Dw;
        s_B[j] = 1;
        if (Da > 0.0) c_pos++;
        else if (Da < 0.0) c_neg++;
        else {
          c_zero++;
          if (first_zero == 0) first_zero = k + 1;
        }
      }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int i = k0 + tid + T * r;
      if (i == kn && kn < N)
        w_row<NB>(Lr[r], s_D0, s_D1, s_B, j, (kind == 4) ? 2 : 1, Dw, Dc, Db, s_wk);
    }
    k = kn;
    j += kstep;
    __syncthreads();
  }

  // ---- write the panel's multipliers and W = L D for the trailing rows ---------
  const int kend = k, jend = j;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int i = k0 + tid + T * r;
    if (i >= N) continue;
#pragma unroll
    for (int t = 0; t < NB; ++t)
      if (t < jend && i > k0 + t) Lout[i + (k0 + t) * ld] = Lr[r][t];
    if (i >= kend) {
      w_row_global<NB>(Lr[r], s_D0, s_D1, s_B, jend, W + i, ld);
      src_out[i] = srcr[r];
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

}  // namespace

// Panel variant for a matrix of order N: 1024 threads and R rows per thread
// (R * 1024 >= N), with the register tile NB chosen so that R * NB = 32
// doubles of L per thread.
int bk_reg_rows(int N) {
  for (int r = 1; r <= 8; r *= 2)
    if (N <= r * TMAX) return r;
  return 0;
}

int bk_reg_nb(int N) {
  switch (bk_reg_rows(N)) {
    case 1: return 32;
    case 2: return 32;
    case 4: return 16;
    case 8: return 8;
    default: return 0;
  }
}

void launch_bk_panel_reg(hipStream_t s, int N, int nb, double alpha, const double *X,
                         double *Lout, int32_t *src_out, double *W, double *dd, double *ds,
                         int32_t *ipiv, int32_t *blk, FacState *st, int32_t *panel_k0) {
#define MDS_PANEL_REG(R_, NB_)                                                         \
  k_bk_panel_reg<TMAX, R_, NB_><<<1, TMAX, 0, s>>>(N, nb, alpha, X, Lout, src_out, W, dd, ds, \
                                                   ipiv, blk, st, panel_k0)
  switch (bk_reg_rows(N)) {
    case 1: MDS_PANEL_REG(1, 32); break;
    case 2: MDS_PANEL_REG(2, 32); break;
    case 4: MDS_PANEL_REG(4, 16); break;
    case 8: MDS_PANEL_REG(8, 8); break;
    default: break;
  }
#undef MDS_PANEL_REG
}

}  // namespace mds
