// Condensation of the sparse block (Sec. 2.2, eq. (compressed); kernel class
// K3) and the sparse helpers around it: D_s^{-1}, the condensed right-hand
// side, back-substitution of dx_s, the column-compressed copy of J_s and the
// input validation.
//
// M is stored full (both triangles) and column-major with leading dimension N.
// Every entry is produced by a fixed sequence of IEEE operations so that the
// assembled matrix is bitwise reproducible:
//   M11 = H, diagonal (H_ii + Sigma_d,i) + dw;   M21 = J_d;   M12 = J_d';
//   M22(i,j) = 0 - sum_k (J_ik * Dinv_k) * J_jk  over the shared columns k of
//              rows i >= j in ascending k, then - dc on the diagonal and,
//              when a per-row diagonal is set, - dcv[r] after it.
#include "internal.hpp"

namespace mds {
namespace {

constexpr int kTile = 64;

__global__ void k_inv_d(int ns, const double *__restrict__ dsbase, double dw,
                        double *__restrict__ inv_d) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < ns) inv_d[i] = 1.0 / (dsbase[i] + dw);
}

// One 64 x 64 tile of M per workgroup (256 threads).  Everything but the
// (1,2) block J_d' is read along columns (coalesced); the J_d' block is
// transposed through LDS.
__global__ __launch_bounds__(256) void k_condense_dense(int nd, int m, int N,
                                                        const double *__restrict__ H,
                                                        const double *__restrict__ Jd,
                                                        const double *__restrict__ sig,
                                                        double dw, double *__restrict__ M) {
  __shared__ double t[kTile][kTile + 1];
  const int I0 = blockIdx.x * kTile, J0 = blockIdx.y * kTile;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  const bool has_t = (I0 < nd) && (J0 + kTile > nd);  // tile touches the J_d' block
  if (has_t) {
    // stage J_d'(i, j) = J_d(j - nd, i): read along j (contiguous rows of J_d)
    for (int ii = ty; ii < kTile; ii += 4) {
      int i = I0 + ii, j = J0 + tx;
      double v = 0.0;
      if (i < nd && j >= nd && j < N) v = Jd[(size_t)(j - nd) + (size_t)i * m];
      t[tx][ii] = v;
    }
    __syncthreads();
  }
  // every entry of this thread's column strip is loaded before the first
  // store, so that the loads of one thread overlap
  double vals[kTile / 4];
#pragma unroll
  for (int u = 0; u < kTile / 4; ++u) {
    const int jj = ty + 4 * u, i = I0 + tx, j = J0 + jj;
    double v = 0.0;
    if (i < N && j < N) {
      if (i < nd && j < nd) {
        v = H[(size_t)i + (size_t)j * nd];
        if (i == j) v = (v + sig[i]) + dw;
      } else if (j < nd) {
        v = Jd[(size_t)(i - nd) + (size_t)j * m];
      } else if (i < nd) {
        v = t[jj][tx];
      }
    }
    vals[u] = v;
  }
#pragma unroll
  for (int u = 0; u < kTile / 4; ++u) {
    const int i = I0 + tx, j = J0 + ty + 4 * u;
    if (i < N && j < N) M[(size_t)i + (size_t)j * N] = vals[u];
  }
}

// One thread per constraint r: accumulates column r of M22 (rows i >= r) in
// ascending shared column k and mirrors each entry into row r.  The dense
// kernel has zeroed M22 before this runs (stream order).
__global__ void k_condense_schur(int nd, int m, int N, const int32_t *__restrict__ rp,
                                 const int32_t *__restrict__ ci, const double *__restrict__ v,
                                 const int32_t *__restrict__ cptr,
                                 const int32_t *__restrict__ crow,
                                 const double *__restrict__ cval,
                                 const double *__restrict__ inv_d, double dc,
                                 const double *__restrict__ dcv, double *__restrict__ M) {
  int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= m) return;
  const size_t col = (size_t)(nd + r) * N;
  for (int a = rp[r]; a < rp[r + 1]; ++a) {
    const int k = ci[a];
    const double jrk = v[a], dk = inv_d[k];
    for (int e = cptr[k]; e < cptr[k + 1]; ++e) {
      const int i = crow[e];
      if (i < r) continue;
      const size_t pos = (size_t)(nd + i) + col;
      double acc = M[pos];
      acc = acc - (cval[e] * dk) * jrk;
      M[pos] = acc;
      if (i != r) M[(size_t)(nd + r) + (size_t)(nd + i) * N] = acc;
    }
  }
  const size_t dpos = (size_t)(nd + r) + col;
  M[dpos] = M[dpos] - dc;
  if (dcv) M[dpos] = M[dpos] - dcv[r];
}

__global__ void k_rhs_condense(int m, const int32_t *__restrict__ rp,
                               const int32_t *__restrict__ ci, const double *__restrict__ v,
                               const double *__restrict__ inv_d,
                               const double *__restrict__ r_s,
                               const double *__restrict__ r_y, double *__restrict__ out) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  double t = r_y[i];
  for (int a = rp[i]; a < rp[i + 1]; ++a) {
    const int k = ci[a];
    t = t - v[a] * (inv_d[k] * r_s[k]);
  }
  out[i] = t;
}

__global__ void k_backsub(int ns, const int32_t *__restrict__ cptr,
                          const int32_t *__restrict__ crow, const double *__restrict__ cval,
                          const double *__restrict__ inv_d, const double *__restrict__ r_s,
                          const double *__restrict__ dy, double *__restrict__ dx_s) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= ns) return;
  double t = r_s[k];
  for (int e = cptr[k]; e < cptr[k + 1]; ++e) t = t - cval[e] * dy[crow[e]];
  dx_s[k] = inv_d ? inv_d[k] * t : t;
}

// ---- column-compressed copy of J_s ----------------------------------------
__global__ void k_zero_i32(int64_t n, int32_t *p) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

__global__ void k_csc_count(int m, const int32_t *__restrict__ rp,
                            const int32_t *__restrict__ ci, int32_t *cnt) {
  int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= m) return;
  for (int a = rp[r]; a < rp[r + 1]; ++a) atomicAdd(&cnt[ci[a]], 1);
}

// Exclusive scan of cnt[0..n) into ptr[0..n], single workgroup of 1024.
__global__ __launch_bounds__(1024) void k_scan(int n, const int32_t *__restrict__ cnt,
                                               int32_t *__restrict__ ptr) {
  __shared__ int64_t part[1024];
  const int t = threadIdx.x;
  const int64_t chunk = ((int64_t)n + 1023) / 1024;
  const int64_t b = t * chunk, e = (b + chunk < n) ? b + chunk : n;
  int64_t s = 0;
  for (int64_t i = b; i < e; ++i) s += cnt[i];
  part[t] = s;
  __syncthreads();
  if (t == 0) {
    int64_t acc = 0;
    for (int i = 0; i < 1024; ++i) {
      int64_t x = part[i];
      part[i] = acc;
      acc += x;
    }
    ptr[n] = (int32_t)acc;
  }
  __syncthreads();
  int64_t acc = part[t];
  for (int64_t i = b; i < e; ++i) {
    ptr[i] = (int32_t)acc;
    acc += cnt[i];
  }
}

__global__ void k_csc_fill(int m, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                           const double *__restrict__ v, const int32_t *__restrict__ cptr,
                           int32_t *fill, int32_t *__restrict__ crow,
                           double *__restrict__ cval) {
  int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= m) return;
  for (int a = rp[r]; a < rp[r + 1]; ++a) {
    const int k = ci[a];
    const int pos = cptr[k] + atomicAdd(&fill[k], 1);
    crow[pos] = r;
    cval[pos] = v[a];
  }
}

// Insertion sort of each column by row: the atomic fill order is arbitrary,
// the sorted result is unique (rows within a column are distinct).
__global__ void k_csc_sort(int ns, const int32_t *__restrict__ cptr, int32_t *__restrict__ crow,
                           double *__restrict__ cval) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= ns) return;
  const int b = cptr[k], e = cptr[k + 1];
  for (int a = b + 1; a < e; ++a) {
    int r = crow[a];
    double x = cval[a];
    int q = a - 1;
    while (q >= b && crow[q] > r) {
      crow[q + 1] = crow[q];
      cval[q + 1] = cval[q];
      --q;
    }
    crow[q + 1] = r;
    cval[q + 1] = x;
  }
}

// ---- validation: flags[0] non-finite, [1] w < 0, [2] xl >= xu, [3] pattern,
// [4] H not exactly symmetric.
__global__ void k_check_finite(int64_t n, const double *__restrict__ a, int32_t *flags) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && !isfinite(a[i])) flags[0] = 1;
}

__global__ void k_check_w(int64_t n, const double *__restrict__ w, int32_t *flags) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && !(w[i] >= 0.0)) flags[1] = 1;
}

__global__ void k_check_bounds(int64_t n, const double *__restrict__ xl,
                               const double *__restrict__ xu, int32_t *flags) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double l = xl[i], u = xu[i];
  if (!(l < u) || isnan(l) || isnan(u) || l == INFINITY || u == -INFINITY) flags[2] = 1;
}

__global__ void k_check_pattern(int m, int ns, int64_t nnz, const int32_t *__restrict__ rp,
                                const int32_t *__restrict__ ci, int32_t *flags) {
  int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r > m) return;
  if (r == 0 && rp[0] != 0) flags[3] = 1;
  if (r == m) {
    if ((int64_t)rp[m] != nnz) flags[3] = 1;
    return;
  }
  const int b = rp[r], e = rp[r + 1];
  if (e < b || b < 0 || (int64_t)e > nnz) {
    flags[3] = 1;
    return;
  }
  for (int a = b; a < e; ++a) {
    const int k = ci[a];
    if (k < 0 || k >= ns || (a > b && k <= ci[a - 1])) flags[3] = 1;
  }
}

__global__ void k_check_sym(int nd, const double *__restrict__ H, int32_t *flags) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  int j = blockIdx.y;
  if (i >= nd || i <= j) return;
  const double a = H[(size_t)i + (size_t)j * nd], b = H[(size_t)j + (size_t)i * nd];
  if (!(a == b)) flags[4] = 1;
}

inline unsigned grid1(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

void launch_inv_d(hipStream_t s, int ns, const double *dsbase, double dw, double *inv_d) {
  if (ns <= 0) return;
  k_inv_d<<<grid1(ns, 256), 256, 0, s>>>(ns, dsbase, dw, inv_d);
}

void launch_condense_dense(hipStream_t s, int nd, int m, const double *H, const double *Jd,
                           const double *sigma_d, double dw, double *M) {
  const int N = nd + m;
  if (N <= 0) return;
  dim3 g(grid1(N, kTile), grid1(N, kTile));
  k_condense_dense<<<g, 256, 0, s>>>(nd, m, N, H, Jd, sigma_d, dw, M);
}

void launch_condense_schur(hipStream_t s, int nd, int m, int N, const int32_t *rp,
                           const int32_t *ci, const double *v, const int32_t *cptr,
                           const int32_t *crow, const double *cval, const double *inv_d,
                           double dc, const double *dcv, double *M) {
  if (m <= 0) return;
  k_condense_schur<<<grid1(m, 128), 128, 0, s>>>(nd, m, N, rp, ci, v, cptr, crow, cval, inv_d,
                                                 dc, dcv, M);
}

void launch_rhs_condense(hipStream_t s, int m, const int32_t *rp, const int32_t *ci,
                         const double *v, const double *inv_d, const double *r_s,
                         const double *r_y, double *out) {
  if (m <= 0) return;
  k_rhs_condense<<<grid1(m, 256), 256, 0, s>>>(m, rp, ci, v, inv_d, r_s, r_y, out);
}

void launch_backsub(hipStream_t s, int ns, const int32_t *cptr, const int32_t *crow,
                    const double *cval, const double *inv_d, const double *r_s,
                    const double *dy, double *dx_s) {
  if (ns <= 0) return;
  k_backsub<<<grid1(ns, 256), 256, 0, s>>>(ns, cptr, crow, cval, inv_d, r_s, dy, dx_s);
}

void launch_csc_build(hipStream_t s, int m, int ns, int64_t nnz, const int32_t *rp,
                      const int32_t *ci, const double *v, int32_t *cptr, int32_t *crow,
                      double *cval, int32_t *fill) {
  if (ns <= 0) return;
  k_zero_i32<<<grid1(ns, 256), 256, 0, s>>>(ns, fill);
  if (m > 0) k_csc_count<<<grid1(m, 256), 256, 0, s>>>(m, rp, ci, fill);
  k_scan<<<1, 1024, 0, s>>>(ns, fill, cptr);
  k_zero_i32<<<grid1(ns, 256), 256, 0, s>>>(ns, fill);
  if (m > 0 && nnz > 0) {
    k_csc_fill<<<grid1(m, 256), 256, 0, s>>>(m, rp, ci, v, cptr, fill, crow, cval);
    k_csc_sort<<<grid1(ns, 256), 256, 0, s>>>(ns, cptr, crow, cval);
  }
}

void launch_validate(hipStream_t s, const mds_dims &d, const mds_problem &p, int32_t *flags) {
  const int64_t nd = d.n_d, ns = d.n_s, m = d.m, n = nd + ns;
  auto fin = [&](int64_t len, const double *a) {
    if (len > 0) k_check_finite<<<grid1(len, 256), 256, 0, s>>>(len, a, flags);
  };
  fin(nd * nd, p.H);
  fin(nd, p.c);
  fin(ns, p.w);
  fin(ns, p.g);
  fin(m * nd, p.J_d);
  fin(d.nnz_s, p.Js_val);
  fin(m - d.m_I, p.b);  // the equality rows' right-hand side
  if (ns > 0) k_check_w<<<grid1(ns, 256), 256, 0, s>>>(ns, p.w, flags);
  if (n > 0) k_check_bounds<<<grid1(n, 256), 256, 0, s>>>(n, p.xl, p.xu, flags);
  k_check_pattern<<<grid1(m + 1, 256), 256, 0, s>>>((int)m, (int)ns, d.nnz_s, p.Js_rowptr,
                                                    p.Js_col, flags);
  if (nd > 1) {
    dim3 g(grid1(nd, 256), (unsigned)nd);
    k_check_sym<<<g, 256, 0, s>>>((int)nd, p.H, flags);
  }
}

}  // namespace mds
