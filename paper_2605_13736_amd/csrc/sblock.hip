// Coupling blocks of the sparse Hessian (assumption A2 of Sec. 2 in its
// general form: the sparse block of the Hessian has a pattern that makes
// solves with Q_{x_s} = W_s + D_{x_s} cheap).  Here W_s = diag(w) +
// blockdiag(Wb): consecutive blocks of at most kSBlkMax sparse variables.
//
// Every block of Q_{x_s} = blockdiag(Wb) + diag(dsbase) + dw I is factored
// L Delta L' (unit lower L, no pivoting; positive definite when Wb is
// positive semidefinite and dsbase + dw > 0).  Then
//   J_s Q_{x_s}^{-1} J_s' = (J_s L^{-T}) Delta^{-1} (J_s L^{-T})',
// so the condensation of eq. (compressed) runs unchanged on the transformed
// Jacobian Jh = J_s L^{-T} with the diagonal middle factor 1/Delta.  Row i of
// Jh holds every column of every block that row i of J_s touches.
//
// Evaluation order (bitwise the same as the CPU reference): per block,
// column j: Delta_j = ((Wb_jj + dsbase_j) + dw) - sum_{t<j} (L_jt Delta_t) L_jt
// and L_ij = (Wb_ij - sum_{t<j} (L_it Delta_t) L_jt) / Delta_j, sums in
// ascending t; Jh(i, k0+p) = u_p - sum_{t<p} L_pt Jh(i, k0+t), u_p the entry
// of J_s (0 where J_s has none), ascending t.
#include "internal.hpp"

namespace mds {
namespace {

inline unsigned grid1(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

__global__ void k_sblk_factor(int nblk, const int32_t *__restrict__ bp,
                              const int32_t *__restrict__ boff, const double *__restrict__ Wb,
                              const double *__restrict__ dsb, double dw,
                              double *__restrict__ lblk, double *__restrict__ inv_d) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nblk) return;
  const int k0 = bp[b], sz = bp[b + 1] - k0;
  const double *Q = Wb + boff[b];
  double *L = lblk + boff[b];
  double dl[kSBlkMax];
  for (int j = 0; j < sz; ++j) {
    double d = (Q[j + j * sz] + dsb[k0 + j]) + dw;
    for (int t = 0; t < j; ++t) d = d - (L[j + t * sz] * dl[t]) * L[j + t * sz];
    dl[j] = d;
    L[j + j * sz] = 1.0;
    for (int i = j + 1; i < sz; ++i) {
      double e = Q[i + j * sz];
      for (int t = 0; t < j; ++t) e = e - (L[i + t * sz] * dl[t]) * L[j + t * sz];
      L[i + j * sz] = e / d;
    }
  }
  for (int j = 0; j < sz; ++j) inv_d[k0 + j] = 1.0 / dl[j];
}

// one thread per row of Jh: its entries come block after block, each block
// complete and in ascending column order
__global__ void k_sblk_transform(int m, const int32_t *__restrict__ hrp,
                                 const int32_t *__restrict__ hci,
                                 const int32_t *__restrict__ hsrc,
                                 const double *__restrict__ jsv,
                                 const int32_t *__restrict__ kblk,
                                 const int32_t *__restrict__ bp,
                                 const int32_t *__restrict__ boff,
                                 const double *__restrict__ lblk, double *__restrict__ hv) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  int e = hrp[i];
  const int ee = hrp[i + 1];
  while (e < ee) {
    const int b = kblk[hci[e]], k0 = bp[b], sz = bp[b + 1] - k0;
    const double *L = lblk + boff[b];
    for (int p = 0; p < sz; ++p) {
      const int a = hsrc[e + p];
      double u = (a >= 0) ? jsv[a] : 0.0;
      for (int t = 0; t < p; ++t) u = u - L[p + t * sz] * hv[e + t];
      hv[e + p] = u;
    }
    e += sz;
  }
}

__global__ void k_gather(int64_t n, const int32_t *__restrict__ map,
                         const double *__restrict__ src, double *__restrict__ dst) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) dst[e] = src[map[e]];
}

// u <- L^{-1} u (mode 0), or u <- L^{-T} (inv_d .* (L^{-1} u)) (mode 1), per block
__global__ void k_sblk_solve(int nblk, const int32_t *__restrict__ bp,
                             const int32_t *__restrict__ boff, const double *__restrict__ lblk,
                             const double *__restrict__ inv_d, int mode,
                             double *__restrict__ u) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nblk) return;
  const int k0 = bp[b], sz = bp[b + 1] - k0;
  const double *L = lblk + boff[b];
  double v[kSBlkMax];
  for (int p = 0; p < sz; ++p) {
    double t = u[k0 + p];
    for (int q = 0; q < p; ++q) t = t - L[p + q * sz] * v[q];
    v[p] = t;
  }
  if (mode == 1) {
    for (int p = 0; p < sz; ++p) v[p] = inv_d[k0 + p] * v[p];
    for (int p = sz - 1; p >= 0; --p) {
      double t = v[p];
      for (int q = p + 1; q < sz; ++q) t = t - L[q + p * sz] * v[q];
      v[p] = t;
    }
  }
  for (int p = 0; p < sz; ++p) u[k0 + p] = v[p];
}

// out[k] (+)= sum_j Wb(k, j) u_j over k's block (full symmetric block read
// from its lower triangle), in ascending j; accumulate: add to out
__global__ void k_sblk_matvec(int ns, const int32_t *__restrict__ kblk,
                              const int32_t *__restrict__ bp, const int32_t *__restrict__ boff,
                              const double *__restrict__ Wb, const double *__restrict__ u,
                              int accumulate, double *__restrict__ out) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= ns) return;
  const int b = kblk[k], k0 = bp[b], sz = bp[b + 1] - k0, i = k - k0;
  const double *Q = Wb + boff[b];
  double t = accumulate ? out[k] : 0.0;
  for (int j = 0; j < sz; ++j) t = t + ((i >= j) ? Q[i + j * sz] : Q[j + i * sz]) * u[k0 + j];
  out[k] = t;
}

// norm pieces of the (2,2) block row: jscol[k] += sum_{j != i} |Wb(k, j)|,
// dsb_eff[k] = Wb(k, k) + dsb[k]
__global__ void k_sblk_absrow(int ns, const int32_t *__restrict__ kblk,
                              const int32_t *__restrict__ bp, const int32_t *__restrict__ boff,
                              const double *__restrict__ Wb, const double *__restrict__ dsb,
                              double *__restrict__ jscol, double *__restrict__ dsb_eff) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= ns) return;
  const int b = kblk[k], k0 = bp[b], sz = bp[b + 1] - k0, i = k - k0;
  const double *Q = Wb + boff[b];
  double t = 0.0;
  for (int j = 0; j < sz; ++j)
    if (j != i) t += fabs((i > j) ? Q[i + j * sz] : Q[j + i * sz]);
  jscol[k] += t;
  dsb_eff[k] = Q[i + i * sz] + dsb[k];
}

}  // namespace

void sblk_factor(hipStream_t s, const SBlk &B, const double *dsb, double dw, double *inv_d) {
  if (B.nblk > 0)
    k_sblk_factor<<<grid1(B.nblk, 64), 64, 0, s>>>(B.nblk, B.bp, B.boff, B.Wb, dsb, dw, B.lblk,
                                                    inv_d);
}

void sblk_transform(hipStream_t s, const SBlk &B, int m, const double *jsv) {
  if (m > 0)
    k_sblk_transform<<<grid1(m, 64), 64, 0, s>>>(m, B.hrp, B.hci, B.hsrc, jsv, B.kblk, B.bp,
                                                  B.boff, B.lblk, B.hval);
  if (B.nnz > 0)
    k_gather<<<grid1(B.nnz, 256), 256, 0, s>>>(B.nnz, B.hcmap, B.hval, B.hcval);
}

void sblk_solve(hipStream_t s, const SBlk &B, const double *inv_d, int mode, double *u) {
  if (B.nblk > 0)
    k_sblk_solve<<<grid1(B.nblk, 64), 64, 0, s>>>(B.nblk, B.bp, B.boff, B.lblk, inv_d, mode, u);
}

void sblk_matvec(hipStream_t s, const SBlk &B, int ns, const double *u, bool accumulate,
                 double *out) {
  if (ns > 0)
    k_sblk_matvec<<<grid1(ns, 256), 256, 0, s>>>(ns, B.kblk, B.bp, B.boff, B.Wb, u,
                                                  accumulate ? 1 : 0, out);
}

void sblk_absrow(hipStream_t s, const SBlk &B, int ns, const double *dsb, double *jscol,
                 double *dsb_eff) {
  if (ns > 0)
    k_sblk_absrow<<<grid1(ns, 256), 256, 0, s>>>(ns, B.kblk, B.bp, B.boff, B.Wb, dsb, jscol,
                                                  dsb_eff);
}

}  // namespace mds
