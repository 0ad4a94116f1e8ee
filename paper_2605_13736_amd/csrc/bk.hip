// Blocked Bunch-Kaufman LDL' of the condensed matrix (Sec. 2.3, kernel class
// K4), right-looking, lower, left to right.
//
// Data layout.  M (N x N, column-major, leading dimension N) holds the
// symmetric matrix; the condensation writes both triangles, but from then on
// only the LOWER triangle of the active submatrix is kept current (the upper
// one is stale after the first trailing update).  Columns not yet factored
// hold the current un-updated values of the active submatrix (the lazily
// updated form): the part of a column at or below the diagonal is one
// contiguous read, the part above it is the matching row of the lower
// triangle.  Factored columns receive the unit-lower multipliers L in place
// (strictly lower part).
//
// Panel step (one workgroup, up to nb pivots).  For a panel starting at k0,
// with W[:, t] the updated pivot column(s) of the t-th panel pivot (before
// division by D) and L[:, k0+t] the multipliers:
//   updated column c of the active matrix = M[:, c] - sum_t L[:, k0+t] W[c, t].
// At each pivot index k the kernel forms the updated column k, finds its
// largest off-diagonal magnitude (first index on ties), and when the diagonal
// is too small forms the updated column imax and its largest off-diagonal
// magnitude, then takes the Bunch-Kaufman decision with alpha = (1+sqrt 17)/8:
//   |a_kk| >= alpha colmax                          -> 1x1, no interchange
//   |a_kk| >= alpha colmax (colmax / rowmax)        -> 1x1, no interchange
//   |a_imax,imax| >= alpha rowmax                   -> 1x1, interchange k<->imax
//   otherwise                                       -> 2x2, interchange k+1<->imax
// A zero column gives a zero 1x1 pivot (recorded in info).  An interchange
// p<->q swaps rows p,q of the panel's L and W columns, and gives index q the
// un-updated values of index p in the lower triangle of the active part.  Rows of
// earlier panels' L are NOT permuted by later interchanges; the solve applies
// each panel's interchanges in turn.
//
// Trailing update: M22 -= L21 W21' over the lower tiles of the trailing
// matrix with FP64 MFMA (v_mfma_f64_16x16x4), lower triangle only (16 bytes
// of traffic per entry: read and write).  With the register-resident panel
// (bk_reg.hip) the update also applies the panel's interchanges: it reads
// the un-updated entry through the panel's index map (from the lower
// triangle: entry (max, min) of the two physical indices) from one buffer
// and writes the other.
#include <algorithm>
#include <climits>

#include "internal.hpp"
#include "tile_order.hpp"
#include "wave.hpp"

namespace mds {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int NT = kPanelThreads;
constexpr int NW = NT / 64;

__device__ inline void amax_combine(double &v, int &i, double v2, int i2) {
  if (v2 > v || (v2 == v && i2 < i)) {
    v = v2;
    i = i2;
  }
}

__device__ inline void wave_argmax(double &v, int &i) { wave::amax(v, i); }

__device__ inline double wave_max(double v) { return wave::max(v); }

__global__ void k_fac_reset(FacState *st, int32_t *panel_k0) {
  if (threadIdx.x == 0) {
    st->k = 0;
    st->npanel = 0;
    st->info = 0;
    st->npos = st->nzero = st->nneg = st->n2x2 = 0;
    st->xerr = 0;
    st->csteps = st->cx3 = 0;
    panel_k0[0] = 0;
  }
}

__global__ __launch_bounds__(NT) void k_bk_panel(int N, int nb, double alpha,
                                                 double *__restrict__ M,
                                                 double *__restrict__ W,
                                                 double *__restrict__ dd,
                                                 double *__restrict__ ds,
                                                 int32_t *__restrict__ ipiv,
                                                 int32_t *__restrict__ blk, FacState *st,
                                                 int32_t *__restrict__ panel_k0) {
  __shared__ double s_wk[kMaxNb + 2];
  __shared__ double s_wi[kMaxNb + 2];
  __shared__ double s_rv[NW];
  __shared__ int s_ri[NW];
  __shared__ double s_akk, s_aii;
  __shared__ double s_sw[4];  // W[p,j], W[q,j], W[p,j+1], W[q,j+1] before an interchange
  __shared__ int s_k0;

  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  if (tid == 0) s_k0 = st->k;
  __syncthreads();
  const int k0 = s_k0;
  if (k0 >= N) return;
  const size_t ld = (size_t)N;

  int k = k0, j = 0;
  int c_pos = 0, c_zero = 0, c_neg = 0, c_2x2 = 0, first_zero = 0;

  while (j < nb && k < N) {
    // ---- updated column k ----------------------------------------------
    if (tid < j) s_wk[tid] = W[(size_t)k + tid * ld];
    __syncthreads();
    double bv = -1.0;
    int bi = INT_MAX;
    for (int i = k + tid; i < N; i += NT) {
      double a = M[(size_t)i + (size_t)k * ld];
      for (int t = 0; t < j; ++t) a = fma(-M[(size_t)i + (size_t)(k0 + t) * ld], s_wk[t], a);
      W[(size_t)i + (size_t)j * ld] = a;
      if (i == k) {
        s_akk = a;
      } else {
        double v = fabs(a);
        if (v > bv) {
          bv = v;
          bi = i;
        }
      }
    }
    wave_argmax(bv, bi);
    if (lane == 0) {
      s_rv[wid] = bv;
      s_ri[wid] = bi;
    }
    __syncthreads();
    double colmax = -1.0;
    int imax = INT_MAX;
    for (int q = 0; q < NW; ++q) amax_combine(colmax, imax, s_rv[q], s_ri[q]);
    if (colmax < 0.0) {
      colmax = 0.0;
      imax = k;
    }
    const double akk = s_akk, absakk = fabs(akk);

    // ---- Bunch-Kaufman decision ------------------------------------------
    int kind;  // 0 zero, 1 1x1, 2 1x1 (second test), 3 1x1 swap, 4 2x2
    int kp = k, kstep = 1;
    double aii = 0.0;
    if (fmax(absakk, colmax) == 0.0 || isnan(absakk)) {
      kind = 0;
    } else if (absakk >= alpha * colmax) {
      kind = 1;
    } else {
      // updated column imax (rows >= k) into W[:, j+1]
      __syncthreads();  // everyone has read s_rv / s_ri
      if (tid < j) s_wi[tid] = W[(size_t)imax + tid * ld];
      __syncthreads();
      double rv = 0.0;
      for (int i = k + tid; i < N; i += NT) {
        // lower triangle only: rows above imax read row imax
        double a = (i >= imax) ? M[(size_t)i + (size_t)imax * ld] : M[(size_t)imax + (size_t)i * ld];
        for (int t = 0; t < j; ++t) a = fma(-M[(size_t)i + (size_t)(k0 + t) * ld], s_wi[t], a);
        W[(size_t)i + (size_t)(j + 1) * ld] = a;
        if (i == imax) s_aii = a;
        else rv = fmax(rv, fabs(a));
      }
      rv = wave_max(rv);
      if (lane == 0) s_rv[wid] = rv;
      __syncthreads();
      double rowmax = 0.0;
      for (int q = 0; q < NW; ++q) rowmax = fmax(rowmax, s_rv[q]);
      aii = s_aii;
      if (absakk >= alpha * colmax * (colmax / rowmax)) {
        kind = 2;
      } else if (fabs(aii) >= alpha * rowmax) {
        kind = 3;
        kp = imax;
      } else {
        kind = 4;
        kp = imax;
        kstep = 2;
      }
    }
    const int p = k + kstep - 1, q = kp;
    const bool swap = (q != p);

    // ---- snapshot the entries of rows p, q that change hands ---------------
    if (tid == 0 && swap) {
      s_sw[0] = W[(size_t)p + (size_t)j * ld];
      s_sw[1] = W[(size_t)q + (size_t)j * ld];
      s_sw[2] = W[(size_t)p + (size_t)(j + 1) * ld];
      s_sw[3] = W[(size_t)q + (size_t)(j + 1) * ld];
    }
    __syncthreads();

    // ---- interchange: rows p,q of the panel's L and W columns ---------------
    if (swap && tid < j) {
      double *a = &M[(size_t)p + (size_t)(k0 + tid) * ld];
      double *b = &M[(size_t)q + (size_t)(k0 + tid) * ld];
      double t0 = *a;
      *a = *b;
      *b = t0;
      double *c = &W[(size_t)p + (size_t)tid * ld];
      double *d = &W[(size_t)q + (size_t)tid * ld];
      double t1 = *c;
      *c = *d;
      *d = t1;
    }

    // ---- pivot column(s) after the interchange, multipliers, and the copy of
    //      index p's un-updated values into index q --------------------------
    if (kind == 4) {
      // 2x2 on (k, k+1) after k+1 <-> q; c0 = column k, c1 = column imax
      const double a = akk;
      const double b = swap ? s_sw[1] : W[(size_t)(k + 1) + (size_t)j * ld];
      const double c = aii;
      const double det = a * c - b * b;
      for (int i = k + 2 + tid; i < N; i += NT) {
        double x, y;
        if (swap && i == q) {
          x = s_sw[0];
          y = s_sw[2];
        } else {
          x = W[(size_t)i + (size_t)j * ld];
          y = W[(size_t)i + (size_t)(j + 1) * ld];
        }
        if (swap && i != q) {
          const double a0 = M[(size_t)i + (size_t)p * ld];
          if (i > q) M[(size_t)i + (size_t)q * ld] = a0;
          else M[(size_t)q + (size_t)i * ld] = a0;
        }
        M[(size_t)i + (size_t)k * ld] = (x * c - y * b) / det;
        M[(size_t)i + (size_t)(k + 1) * ld] = (y * a - x * b) / det;
        if (swap && i == q) {
          W[(size_t)i + (size_t)j * ld] = x;
          W[(size_t)i + (size_t)(j + 1) * ld] = y;
        }
      }
      if (tid == 0) {
        if (swap) {
          M[(size_t)q + (size_t)q * ld] = M[(size_t)p + (size_t)p * ld];
          W[(size_t)p + (size_t)j * ld] = s_sw[1];
          W[(size_t)p + (size_t)(j + 1) * ld] = s_sw[3];
        }
        M[(size_t)(k + 1) + (size_t)k * ld] = 0.0;
        dd[k] = a;
        dd[k + 1] = c;
        ds[k] = b;
        ds[k + 1] = 0.0;
        ipiv[k] = -(q + 1);
        ipiv[k + 1] = -(q + 1);
        blk[k] = 2;
        blk[k + 1] = 3;
        c_pos++;
        c_neg++;
        c_2x2++;
      }
    } else {
      // 1x1: pivot column is W[:, j] (kinds 0-2) or column imax moved to k (3)
      const double d = (kind == 3) ? aii : akk;
      for (int i = k + 1 + tid; i < N; i += NT) {
        double x;
        if (kind == 3) {
          if (i == q) x = s_sw[2];  // old W[k, j+1]
          else x = W[(size_t)i + (size_t)(j + 1) * ld];
          W[(size_t)i + (size_t)j * ld] = x;
          if (i != q) {
            const double a0 = M[(size_t)i + (size_t)p * ld];
            if (i > q) M[(size_t)i + (size_t)q * ld] = a0;
            else M[(size_t)q + (size_t)i * ld] = a0;
          }
        } else {
          x = W[(size_t)i + (size_t)j * ld];
        }
        M[(size_t)i + (size_t)k * ld] = (kind == 0) ? 0.0 : x / d;
        if (kind == 0) W[(size_t)i + (size_t)j * ld] = 0.0;  // eliminates nothing
      }
      if (tid == 0) {
        if (kind == 3) {
          M[(size_t)q + (size_t)q * ld] = M[(size_t)p + (size_t)p * ld];
          W[(size_t)k + (size_t)j * ld] = aii;
        }
        dd[k] = d;
        ds[k] = 0.0;
        ipiv[k] = q + 1;
        blk[k] = 1;
        if (d > 0.0) c_pos++;
        else if (d < 0.0) c_neg++;
        else {
          c_zero++;
          if (first_zero == 0) first_zero = k + 1;
        }
      }
    }
    k += kstep;
    j += kstep;
    __syncthreads();
  }
  if (tid == 0) {
    const int b = st->npanel;
    panel_k0[b + 1] = k;
    st->npanel = b + 1;
    st->k = k;
    st->npos += c_pos;
    st->nzero += c_zero;
    st->nneg += c_neg;
    st->n2x2 += c_2x2;
    if (st->info == 0 && first_zero != 0) st->info = first_zero;
  }
}

// ---- trailing update -------------------------------------------------------
// Workgroup = 4 waves = one 64 x 64 lower tile of the trailing matrix; each
// wave owns a 32 (columns c) x 32 (rows i) quarter as 2 x 2 MFMA blocks.
// MFMA computes D'[c][i] = sum_t W[c,t] L[i,t] so that each accumulator
// register holds 16 consecutive rows i of one column c (coalesced access).
// Register layout of v_mfma_f64_16x16x4 on gfx950 (measured): operand A lane
// l holds A[l%16][l/16], operand B lane l holds B[l/16][l%16], and result
// register r of lane l holds D[l/16 + 4r][l%16].
constexpr int TT = 64;
static_assert(TT == kNearCols, "the near strip is one tile column");
constexpr int TS = 36;        // panel columns staged in LDS per chunk (multiple of 4)
constexpr int TS1 = TS + 1;   // odd row stride of the staged panels
constexpr int TSTAGE = TT * TS / 256;  // staged entries per thread and panel
constexpr int kTrailingGrid = kTileGrid;  // persistent trailing update: 512 workgroups (2 per CU at 194 VGPRs)
static_assert(TT * TS % 256 == 0, "staging");

// X: matrix the panel read (entry (x, c) at X[src(x) + src(c) N]); Y: output
// buffer (may equal X when src is null); Lsrc: buffer holding the panel's L.
__global__ __launch_bounds__(256) void k_bk_trailing(int N, int nb, const double *__restrict__ W,
                                                     const double *X, double *Y,
                                                     const double *Lsrc,
                                                     const int32_t *__restrict__ src,
                                                     const FacState *__restrict__ st,
                                                     const int32_t *__restrict__ panel_k0,
                                                     int slot, int part) {
  // the staged panels: W rows c0.., L rows i0..
  __shared__ double s_buf[2 * TT * TS1];
  double *s_w = s_buf, *s_l = s_buf + TT * TS1;
  // only slots whose panel ran in this factorization have valid bounds
  if (slot >= st->npanel) return;
  const int k0 = panel_k0[slot], kend = panel_k0[slot + 1];
  if (kend >= N || kend <= k0 || kend - k0 > nb + 1) return;
  const int jw = kend - k0;
  // tiles start at the 16-row (128-byte) boundary at or below kend, so that a
  // tile's 64-row column segments cover 4 cache lines rather than 5 (when
  // N is a multiple of 16); rows and columns below kend are masked
  const int a0 = kend & ~15;
  const int nt = (N - a0 + TT - 1) / TT;
  // look-ahead's near strip (part 1): tile (blockIdx.x, 0), the multipliers
  // staged; otherwise triangular tile index -> (ti >= tj)
  const int lk0 = (part == 1) ? 0 : k0;
  const int x = blockIdx.x;
  int ti = (int)((sqrt(8.0 * (double)x + 1.0) - 1.0) * 0.5);
  while ((ti + 1) * (ti + 2) / 2 <= x) ++ti;
  while (ti * (ti + 1) / 2 > x) --ti;
  int tj = x - ti * (ti + 1) / 2;
  if (part == 1) {
    ti = x;
    tj = 0;
  }
  if (ti >= nt) return;
  const int i0 = a0 + ti * TT, c0 = a0 + tj * TT;
  const size_t ld = (size_t)N;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int wc = c0 + (wv & 1) * 32, wi = i0 + (wv >> 1) * 32;
  const int l16 = lane & 15, l4 = lane >> 4;

  const bool diag = (ti == tj);
  // the entries this lane updates, loaded before the product loop so that
  // their memory latency overlaps it
  int si[2], sc[2][4];
#pragma unroll
  for (int b = 0; b < 2; ++b) {
    const int i = wi + b * 16 + l16;
    si[b] = (i >= kend && i < N) ? (src ? src[i] : i) : 0;
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int c = wc + a * 16 + l4 + 4 * r;
      sc[a][r] = (c >= kend && c < N) ? (src ? src[c] : c) : 0;
    }
  double xv[2][2][4];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int c = wc + a * 16 + l4 + 4 * r;
        const int i = wi + b * 16 + l16;
        const int pi = si[b], pc = sc[a][r];  // physical row and column
        xv[a][b][r] = (c >= kend && c < N && i < N && (!diag || i >= c))
                          ? X[(pi >= pc) ? (size_t)pi + (size_t)pc * ld : (size_t)pc + (size_t)pi * ld]
                          : 0.0;
      }

  d4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = d4{0.0, 0.0, 0.0, 0.0};

  // panel columns in chunks of TS: every load of a chunk is issued before
  // the LDS stores, so one memory latency covers the chunk
  for (int tb = 0; tb < jw; tb += TS) {
    const int tw = min(TS, jw - tb);
    if (tb > 0) __syncthreads();  // the previous chunk has been read
    double vw[TSTAGE], vl[TSTAGE];
#pragma unroll
    for (int u = 0; u < TSTAGE; ++u) {
      const int e = tid + 256 * u, r = e & (TT - 1), t = e >> 6;
      const int c = c0 + r, i = i0 + r;
      vw[u] = (t < tw && c >= kend && c < N) ? W[(size_t)c + (size_t)(tb + t) * ld] : 0.0;
      vl[u] = (t < tw && i >= kend && i < N) ? Lsrc[(size_t)i + (size_t)(lk0 + tb + t) * ld] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < TSTAGE; ++u) {
      const int e = tid + 256 * u, r = e & (TT - 1), t = e >> 6;
      s_w[r * TS1 + t] = vw[u];
      s_l[r * TS1 + t] = vl[u];
    }
    __syncthreads();
    for (int t0 = 0; t0 < tw; t0 += 4) {
      const int t = t0 + l4;  // < TS; entries past tw are zero
      double av[2], bv[2];
#pragma unroll
      for (int a = 0; a < 2; ++a) av[a] = s_w[(wc - c0 + a * 16 + l16) * TS1 + t];
#pragma unroll
      for (int b = 0; b < 2; ++b) bv[b] = s_l[(wi - i0 + b * 16 + l16) * TS1 + t];
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
          acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[b], acc[a][b], 0, 0, 0);
    }
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int c = wc + a * 16 + l4 + 4 * r;
        const int i = wi + b * 16 + l16;
        if (c >= kend && c < N && i < N && (!diag || i >= c))
          Y[(size_t)i + (size_t)c * ld] = xv[a][b][r] - acc[a][b][r];
      }
}

// Persistent form of k_bk_trailing for panels of at most TS - 1 columns
// (one staging chunk): a grid of a few workgroups per compute unit walks the
// tiles in row-major triangular order, and while it computes one tile the
// loads of its next tile (the entries it updates and the panel rows it
// stages) are already in flight.  Per entry the arithmetic is the one of
// k_bk_trailing, in the same order.
__device__ inline void tr_load(int i0, int c0, bool diag, int N, int kend, int lk0, int jw,
                               const double *__restrict__ W, const double *X,
                               const double *Lsrc, const int32_t *__restrict__ src,
                               double (&xv)[2][2][4], double (&vw)[TSTAGE],
                               double (&vl)[TSTAGE]) {
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int l16 = lane & 15, l4 = lane >> 4;
  const size_t ld = (size_t)N;
  const int wc = c0 + (wv & 1) * 32, wi = i0 + (wv >> 1) * 32;
  int si[2], sc[2][4];
#pragma unroll
  for (int b = 0; b < 2; ++b) {
    const int i = wi + b * 16 + l16;
    si[b] = (i >= kend && i < N) ? (src ? src[i] : i) : 0;
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int c = wc + a * 16 + l4 + 4 * r;
      sc[a][r] = (c >= kend && c < N) ? (src ? src[c] : c) : 0;
    }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int c = wc + a * 16 + l4 + 4 * r;
        const int i = wi + b * 16 + l16;
        const int pi = si[b], pc = sc[a][r];  // physical row and column
        xv[a][b][r] = (c >= kend && c < N && i < N && (!diag || i >= c))
                          ? X[(pi >= pc) ? (size_t)pi + (size_t)pc * ld : (size_t)pc + (size_t)pi * ld]
                          : 0.0;
      }
#pragma unroll
  for (int u = 0; u < TSTAGE; ++u) {
    const int e = tid + 256 * u, r = e & (TT - 1), t = e >> 6;
    const int c = c0 + r, i = i0 + r;
    vw[u] = (t < jw && c >= kend && c < N) ? W[(size_t)c + (size_t)t * ld] : 0.0;
    vl[u] = (t < jw && i >= kend && i < N) ? Lsrc[(size_t)i + (size_t)(lk0 + t) * ld] : 0.0;
  }
}


__global__ __launch_bounds__(256) void k_bk_trailing_ps(int N, int nb,
                                                        const double *__restrict__ W,
                                                        const double *X, double *Y,
                                                        const double *Lsrc,
                                                        const int32_t *__restrict__ src,
                                                        const FacState *__restrict__ st,
                                                        const int32_t *__restrict__ panel_k0,
                                                        int slot, int part) {
  __shared__ double s_buf[2 * TT * TS1];
  double *s_w = s_buf, *s_l = s_buf + TT * TS1;
  if (slot >= st->npanel) return;
  const int k0 = panel_k0[slot], kend = panel_k0[slot + 1];
  if (kend >= N || kend <= k0 || kend - k0 > nb + 1 || kend - k0 > TS) return;
  const int jw = kend - k0;
  // the look-ahead parts read the panel's multipliers from its staging buffer
  const int lk0 = (part == 0) ? k0 : 0;
  const int a0 = kend & ~15;
  const int nt = (N - a0 + TT - 1) / TT;
  // plain row-major order: measured at N = 16384, the super-tile order of
  // tile_order.hpp cut this kernel's fetched bytes by 17% but made it 3.5%
  // slower (188.8 against 182.4 us per launch), and as the look-ahead's rest
  // of the update 4% slower (113.0 against 108.5 ms per factorization); the
  // FP32 update keeps it
  const bool xcd = false;
  const long nslots = part_slots(part, nt, xcd);
  const size_t ld = (size_t)N;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int l16 = lane & 15, l4 = lane >> 4;
  // first slot of this workgroup that holds a tile
  long x = blockIdx.x;
  int ti = 0, tj = 0;
  while (x < nslots && !part_tile(part, x, nt, xcd, ti, tj)) x += gridDim.x;
  if (x >= nslots) return;
  double xn[2][2][4], vwn[TSTAGE], vln[TSTAGE];
  tr_load(a0 + ti * TT, a0 + tj * TT, ti == tj, N, kend, lk0, jw, W, X, Lsrc, src, xn, vwn, vln);
  while (x < nslots) {
    const int i0 = a0 + ti * TT, c0 = a0 + tj * TT;
    const bool diag = (ti == tj);
    const int wc = c0 + (wv & 1) * 32, wi = i0 + (wv >> 1) * 32;
    double xv[2][2][4];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int r = 0; r < 4; ++r) xv[a][b][r] = xn[a][b][r];
    __syncthreads();  // the previous tile is done with the staging buffer
#pragma unroll
    for (int u = 0; u < TSTAGE; ++u) {
      const int e = tid + 256 * u, r = e & (TT - 1), t = e >> 6;
      s_w[r * TS1 + t] = vwn[u];
      s_l[r * TS1 + t] = vln[u];
    }
    __syncthreads();
    // the next slot that holds a tile, its loads in flight during this one
    long xnext = x + gridDim.x;
    int tin = 0, tjn = 0;
    while (xnext < nslots && !part_tile(part, xnext, nt, xcd, tin, tjn)) xnext += gridDim.x;
    if (xnext < nslots)
      tr_load(a0 + tin * TT, a0 + tjn * TT, tin == tjn, N, kend, lk0, jw, W, X, Lsrc, src, xn, vwn,
              vln);
    d4 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) acc[a][b] = d4{0.0, 0.0, 0.0, 0.0};
    for (int t0 = 0; t0 < jw; t0 += 4) {
      const int t = t0 + l4;  // < TS; entries past jw are zero
      double av[2], bv[2];
#pragma unroll
      for (int a = 0; a < 2; ++a) av[a] = s_w[(wc - c0 + a * 16 + l16) * TS1 + t];
#pragma unroll
      for (int b = 0; b < 2; ++b) bv[b] = s_l[(wi - i0 + b * 16 + l16) * TS1 + t];
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
          acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[b], acc[a][b], 0, 0, 0);
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int c = wc + a * 16 + l4 + 4 * r;
          const int i = wi + b * 16 + l16;
          if (c >= kend && c < N && i < N && (!diag || i >= c))
            Y[(size_t)i + (size_t)c * ld] = xv[a][b][r] - acc[a][b][r];
        }
    x = xnext;
    ti = tin;
    tj = tjn;
  }
}

// Staged multipliers of a look-ahead panel into their column of the factor:
// column t of Lst (rows below the diagonal) -> column k0 + t of Lout.
__global__ __launch_bounds__(256) void k_lstage_copy(int N, const double *__restrict__ Lst,
                                                     double *__restrict__ Lout,
                                                     const FacState *__restrict__ st,
                                                     const int32_t *__restrict__ panel_k0,
                                                     int slot) {
  if (slot >= st->npanel) return;
  const int k0 = panel_k0[slot], kend = panel_k0[slot + 1];
  const int t = blockIdx.y;
  if (t >= kend - k0) return;
  const size_t ld = (size_t)N;
  for (int i = k0 + t + 1 + blockIdx.x * 256 + threadIdx.x; i < N; i += gridDim.x * 256)
    Lout[(size_t)i + (size_t)(k0 + t) * ld] = Lst[(size_t)i + (size_t)t * ld];
}

}  // namespace

void launch_fac_reset(hipStream_t s, FacState *st, int32_t *panel_k0) {
  k_fac_reset<<<1, 64, 0, s>>>(st, panel_k0);
}

void launch_bk_panel(hipStream_t s, int N, int nb, double alpha, double *M, double *W,
                     double *dd, double *ds, int32_t *ipiv, int32_t *blk, FacState *st,
                     int32_t *panel_k0) {
  k_bk_panel<<<1, NT, 0, s>>>(N, nb, alpha, M, W, dd, ds, ipiv, blk, st, panel_k0);
}

void launch_bk_trailing(hipStream_t s, int N, int nb, long rem, int slot, const double *W,
                        const double *X, double *Y, const double *Lsrc, const int32_t *src,
                        const FacState *st, const int32_t *panel_k0) {
  // rem bounds the rows of the trailing matrix after slot `slot`; the
  // kernel's tiles start up to 15 rows earlier (at a 16-row boundary)
  if (rem <= 0) return;
  const long nt = (rem + 15 + TT - 1) / TT;
  const long tiles = nt * (nt + 1) / 2;
  if (nb + 1 <= TS) {
    // persistent: a few workgroups per compute unit walk the tiles
    const long grid = std::min(tiles, (long)kTrailingGrid);
    k_bk_trailing_ps<<<(unsigned)grid, 256, 0, s>>>(N, nb, W, X, Y, Lsrc, src, st, panel_k0,
                                                     slot, 0);
  } else {
    k_bk_trailing<<<(unsigned)tiles, 256, 0, s>>>(N, nb, W, X, Y, Lsrc, src, st, panel_k0, slot,
                                                  0);
  }
}

void launch_bk_trailing_part(hipStream_t s, int N, int nb, long rem, int slot, int part, int grid,
                             const double *W, const double *X, double *Y, const double *Lsrc,
                             const int32_t *src, const FacState *st, const int32_t *panel_k0) {
  if (rem <= 0 || nb + 1 > TS) return;
  const long nt = (rem + 15 + TT - 1) / TT;
  const long tiles = (part == 1) ? nt : (nt - 1) * nt / 2;
  if (tiles <= 0) return;
  if (part == 1) {
    // one tile per workgroup (104 VGPRs: more workgroups per compute unit
    // than the persistent form's two)
    k_bk_trailing<<<(unsigned)nt, 256, 0, s>>>(N, nb, W, X, Y, Lsrc, src, st, panel_k0, slot, 1);
    return;
  }
  const long g = std::min(tiles, (long)std::max(grid, 1));
  k_bk_trailing_ps<<<(unsigned)g, 256, 0, s>>>(N, nb, W, X, Y, Lsrc, src, st, panel_k0, slot,
                                                part);
}

void launch_lstage_copy(hipStream_t s, int N, long rows, int slot, const double *Lst, double *Lout,
                        const FacState *st, const int32_t *panel_k0) {
  // rows: the rows at the panel's start, at most
  if (rows <= 0) return;
  const unsigned gx = (unsigned)std::min<long>((rows + 1023) / 1024, 64);
  k_lstage_copy<<<dim3(gx, (unsigned)(TS + 1)), 256, 0, s>>>(N, Lst, Lout, st, panel_k0, slot);
}

}  // namespace mds
