// Unblocked Bunch-Kaufman factorization (Sec. 2.3) of a small M held whole
// in one workgroup's LDS.
//
// Up to N = 199 the lower triangle of M (N (N + 1) / 2 doubles, packed
// column by column) and two work columns fit in the 160 KB of one CU's LDS,
// so the factorization needs no panel / trailing-update split and touches
// global memory only to load M and to store the factor.  Each pivot step is
// the plain one, separated by three workgroup barriers:
//   search  wave 0 reads column k (and, when the first test fails, row and
//           column imax), takes the decision and leaves it in LDS;
//   swap    the symmetric interchange of p = k + s - 1 with q over whole
//           rows (the earlier columns of L included, so L ends in standard
//           form P M P' = L D L'); thread e owns the swapped pair indexed by
//           e and, for its row e >= k + s, forms the multipliers
//           l = w D^{-1} (Cramer's rule for a 2x2 pivot), writes them into
//           column k (and k + 1) and saves the unscaled w for the update;
//   update  A(i, j) -= l(i) w(j) (rank 1) or l0(i) w0(j) + l1(i) w1(j)
//           (rank 2) for k + s <= j <= i < N: waves take pairs of columns in
//           turn; a column and the multipliers beside it are contiguous, so
//           lane x reads rows j + x + 64 c at one base address plus
//           immediate offsets, both columns' loads are issued before any
//           store, and only the stores of a column's last 64-row chunk are
//           masked (loads past a column's end read the next column or the
//           slack after the triangle and are discarded).
// Products and sums are evaluated as written, without contraction into
// fused multiply-adds, and divisions are IEEE divisions: every operation
// rounds exactly as in the plain definition of the method.
#include <climits>

#include "internal.hpp"
#include "wave.hpp"

namespace mds {
namespace {

// start of packed column j: entry (i, j), i >= j, lives at poff(j) + i - j
__device__ inline int poff(int N, int j) { return j * N - (j * (j - 1)) / 2; }

constexpr int kLdsChunks = 4;  // 64-row chunks of a column: N <= 256
constexpr int kLdsSlack = 64;  // doubles after the triangle (over-reads)

__device__ inline int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }

template <int T>
__global__ __launch_bounds__(T) void k_bk_lds(int N, double alpha, double *M,
                                              double *__restrict__ dd, double *__restrict__ ds,
                                              int32_t *__restrict__ ipiv,
                                              int32_t *__restrict__ blk,
                                              int32_t *__restrict__ perm, FacState *st) {
#pragma clang fp contract(off)
  constexpr int NW = T / 64, U = kLdsChunks;
  extern __shared__ double s_dyn[];
  __shared__ double s_val[3];  // akk, aii, wki of the step
  __shared__ int s_dec[2];     // kind, imax of the step
  const int tid = threadIdx.x, lane = tid & 63;
  const int wid = uni(tid >> 6);
  const int PN = N * (N + 1) / 2;
  double *A = s_dyn;
  double *w0 = A + PN + kLdsSlack, *w1 = w0 + N;
  int *orig = (int *)(w1 + N);  // original index of the row at each position
  auto at = [&](int i, int j) -> double & { return A[poff(N, j) + (i - j)]; };

  for (int j = wid; j < N; j += NW) {
    const int o = poff(N, j) - j;
    double v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int i = j + lane + 64 * u;
      v[u] = (i < N) ? M[(size_t)i + (size_t)j * N] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int i = j + lane + 64 * u;
      if (i < N) A[o + i] = v[u];
    }
  }
  for (int x = tid; x < N; x += T) orig[x] = x;
  for (int x = tid; x < kLdsSlack; x += T) A[PN + x] = 0.0;
  __syncthreads();

  int c_pos = 0, c_zero = 0, c_neg = 0, c_2x2 = 0, info = 0;
  int k = 0;
  while (k < N) {
    const int ok = poff(N, k);
    // ---- search (wave 0) -----------------------------------------------------
    if (wid == 0) {
      const double akk = A[ok], absakk = fabs(akk);
      double cv[U];
#pragma unroll
      for (int u = 0; u < U; ++u) cv[u] = A[ok + (min(k + 1 + lane + 64 * u, N - 1) - k)];
      double bv = -1.0;
      int bi = INT_MAX;
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int i = k + 1 + lane + 64 * u;
        const double v = fabs(cv[u]);
        if (i < N && v > bv) {  // rows rise along a lane: the first maximum stays
          bv = v;
          bi = i;
        }
      }
      wave::amax(bv, bi);
      double colmax = bv;
      int imax = bi;
      if (bv < 0.0) {  // no row below, or only NaN
        colmax = 0.0;
        imax = k;
      }
      int kind;  // 0 zero, 1 / 2 / 3 1x1, 4 2x2
      double aii = 0.0, wki = 0.0;
      if (fmax(absakk, colmax) == 0.0 || isnan(absakk)) {
        kind = 0;
      } else if (absakk >= alpha * colmax) {
        kind = 1;
      } else {
        // row imax left of the diagonal (r < imax: A(imax, r)) and column
        // imax below it (r > imax: A(r, imax)), r = k + lane + 64 u
        const int oi = poff(N, imax);
        double rvv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int r = min(k + lane + 64 * u, N - 1);
          rvv[u] = A[(r < imax) ? poff(N, r) + (imax - r) : oi + (r - imax)];
        }
        double rv = 0.0;
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int r = k + lane + 64 * u;
          if (r < N && r != imax) rv = fmax(rv, fabs(rvv[u]));
        }
        const double rowmax = wave::max(rv);
        aii = A[oi];
        wki = A[ok + (imax - k)];
        if (absakk >= alpha * colmax * (colmax / rowmax)) kind = 2;
        else if (fabs(aii) >= alpha * rowmax) kind = 3;
        else kind = 4;
      }
      if (lane == 0) {
        s_dec[0] = kind;
        s_dec[1] = imax;
        s_val[0] = akk;
        s_val[1] = aii;
        s_val[2] = wki;
      }
    }
    __syncthreads();
    const int kind = uni(s_dec[0]);
    const int kstep = (kind == 4) ? 2 : 1;
    const int q = (kind >= 3) ? uni(s_dec[1]) : k;
    const double akk = s_val[0], aii = s_val[1], wki = s_val[2];

    // ---- interchange p <-> q and multipliers ---------------------------------
    const int p = k + kstep - 1, kn = k + kstep;
    const bool sw = q != p;
    // pivot block after the interchange: a = A(k,k), b = A(k+1,k) (old
    // A(q,k)), c = A(k+1,k+1) (old A(q,q)); a 1x1 pivot is A(k,k)
    const double d = (kind == 3) ? aii : akk;
    const double Da = akk, Db = wki, Dc = aii;
    const double det = (kind == 4) ? Da * Dc - Db * Db : 1.0;
    for (int e = tid; e < N; e += T) {
      // the pair this thread interchanges: rows p, q of column e (e < p),
      // the diagonal (e == p), (e, p) <-> (q, e) (p < e < q), (e, p) <-> (e, q)
      // (e > q); for a 2x2 pivot thread q takes rows p, q of column k
      int ua = 0, va = 0;
      bool two = false;
      if (sw) {
        if (e < p) {
          two = !(kstep == 2 && e == k);
          ua = poff(N, e) + (p - e);
          va = poff(N, e) + (q - e);
        } else if (e == p) {
          two = true;
          ua = poff(N, p);
          va = poff(N, q);
        } else if (e != q) {
          two = true;
          ua = poff(N, p) + (e - p);
          va = (e < q) ? poff(N, e) + (q - e) : poff(N, q) + (e - q);
        }
      }
      double nu = 0.0;  // new value at ua
      if (two) {
        const double u = A[ua], v = A[va];
        A[ua] = v;
        A[va] = u;
        nu = v;
      }
      if (sw && e == p) {
        const int o = orig[p];
        orig[p] = orig[q];
        orig[q] = o;
      }
      double xk = 0.0;  // old A(p, k) for thread q of a 2x2 pivot
      if (kind == 4 && ((sw && e == q) || (!sw && e == p))) {
        if (sw) xk = A[ok + (p - k)];
        A[ok + (p - k)] = 0.0;  // belongs to D
      }
      if (kind != 0 && e >= kn) {
        // column k (k + 1) at row e after the interchange
        const bool moved = sw && e != q;  // (e, p) came from the swap
        if (kstep == 1) {
          const double x0 = moved ? nu : A[ok + (e - k)];
          w0[e] = x0;
          A[ok + (e - k)] = x0 / d;
        } else {
          const int o1 = poff(N, k + 1) + (e - k - 1);
          const double x0 = (sw && e == q) ? xk : A[ok + (e - k)];
          const double y0 = moved ? nu : A[o1];
          w0[e] = x0;
          w1[e] = y0;
          A[ok + (e - k)] = (x0 * Dc - y0 * Db) / det;
          A[o1] = (y0 * Da - x0 * Db) / det;
        }
      }
    }
    __syncthreads();
    // pivot records (issued after the barrier, whose wait for outstanding
    // memory operations they would otherwise lengthen)
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
        c_pos++;
        c_neg++;
        c_2x2++;
      } else {
        dd[k] = d;
        ds[k] = 0.0;
        ipiv[k] = q + 1;
        blk[k] = 1;
        if (d > 0.0) c_pos++;
        else if (d < 0.0) c_neg++;
        else {
          c_zero++;
          if (info == 0) info = k + 1;
        }
      }
    }

    // ---- rank-1 / rank-2 update of the trailing triangle ----------------------
    if (kind != 0) {
      // l0(i) = A[lk0 + i], l1(i) = A[lk1 + i]
      const int lk0 = ok - k, lk1 = poff(N, k + 1) - (k + 1);
      for (int j = kn + wid; j < N; j += 2 * NW) {
        const int j2 = j + NW;
        const int n1 = N - j, n2 = N - j2;  // rows of each column (n2 <= 0: none)
        double *pa = A + poff(N, j) + lane;
        double *pb = (n2 > 0) ? A + poff(N, j2) + lane : pa;
        const double *la0 = A + lk0 + j + lane, *la1 = A + lk1 + j + lane;
        const double *lb0 = A + lk0 + j2 + lane, *lb1 = A + lk1 + j2 + lane;
        const double wa0 = w0[j], wa1 = w1[j];
        const double wb0 = (n2 > 0) ? w0[j2] : 0.0, wb1 = (n2 > 0) ? w1[j2] : 0.0;
        double ra[U], rb[U], xa0[U], xa1[U], xb0[U], xb1[U];
#pragma unroll
        for (int c = 0; c < U; ++c) {
          if (64 * c < n1) {
            ra[c] = pa[64 * c];
            xa0[c] = la0[64 * c];
            if (kstep == 2) xa1[c] = la1[64 * c];
          }
          if (64 * c < n2) {
            rb[c] = pb[64 * c];
            xb0[c] = lb0[64 * c];
            if (kstep == 2) xb1[c] = lb1[64 * c];
          }
        }
#pragma unroll
        for (int c = 0; c < U; ++c) {
          if (64 * c < n1) {
            const double v = (kstep == 1) ? ra[c] - xa0[c] * wa0
                                          : ra[c] - (xa0[c] * wa0 + xa1[c] * wa1);
            if (64 * (c + 1) <= n1 || lane + 64 * c < n1) pa[64 * c] = v;
          }
          if (64 * c < n2) {
            const double v = (kstep == 1) ? rb[c] - xb0[c] * wb0
                                          : rb[c] - (xb0[c] * wb0 + xb1[c] * wb1);
            if (64 * (c + 1) <= n2 || lane + 64 * c < n2) pb[64 * c] = v;
          }
        }
      }
    }
    __syncthreads();
    k = kn;
  }

  // ---- standard-form factor: strictly lower L into M, permutation ------------
  for (int j = wid; j < N; j += NW) {
    const int o = poff(N, j) - j;
    for (int i = j + 1 + lane; i < N; i += 64) M[(size_t)i + (size_t)j * N] = A[o + i];
  }
  for (int y = tid; y < N; y += T) perm[orig[y]] = y;
  if (tid == 0) {
    st->k = N;
    st->npanel = 1;
    st->info = info;
    st->npos = c_pos;
    st->nzero = c_zero;
    st->nneg = c_neg;
    st->n2x2 = c_2x2;
    st->xerr = 0;
  }
}

}  // namespace

size_t bk_lds_bytes(int N) {
  return 8 * ((size_t)N * (size_t)(N + 1) / 2 + kLdsSlack + 2 * (size_t)N) + 4 * (size_t)N;
}

int bk_lds_max_n() {
  int n = 0;  // 64 bytes of the 160 KB stay for the kernel's static LDS
  while (bk_lds_bytes(n + 1) + 64 <= 160 * 1024) ++n;
  return n;
}

hipError_t bk_lds_prepare() {
  constexpr int dyn = 160 * 1024 - 64;  // static LDS of the kernel: under 64 bytes
  hipError_t e = hipFuncSetAttribute((const void *)k_bk_lds<256>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, dyn);
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute((const void *)k_bk_lds<512>,
                             hipFuncAttributeMaxDynamicSharedMemorySize, dyn);
}

void launch_bk_lds(hipStream_t s, int threads, int N, double alpha, double *M, double *dd,
                   double *ds, int32_t *ipiv, int32_t *blk, int32_t *perm, FacState *st) {
  if (N <= 0 || N > bk_lds_max_n()) return;
  const size_t bytes = bk_lds_bytes(N);
  if (threads >= 512)
    k_bk_lds<512><<<1, 512, bytes, s>>>(N, alpha, M, dd, ds, ipiv, blk, perm, st);
  else
    k_bk_lds<256><<<1, 256, bytes, s>>>(N, alpha, M, dd, ds, ipiv, blk, perm, st);
}

}  // namespace mds
