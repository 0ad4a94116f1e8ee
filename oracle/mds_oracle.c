/*
 * Plain FP64 CPU oracle for the mixed dense-sparse interior-point Newton step.
 * TEST INFRASTRUCTURE ONLY (see mds_oracle.h).  Build: gcc -O2 -ffp-contract=off.
 *
 * The paper (Peles et al., HiOp on accelerators) fixes the method:
 *  - Sec. 2, eqs. (obj)-(bounds): the MDS problem; assumptions A1/A2;
 *  - Sec. 2.1, eq. (linsys4x4): the Newton/KKT system, the inertia requirement
 *    (n,0,m) and its enforcement by diagonal shifts;
 *  - Sec. 2.2, eq. (compressed): Gauss elimination of the sparse block;
 *  - Sec. 2.3: kernel classes K1-K4, Bunch-Kaufman LDL' and Haynsworth
 *    inertia additivity.
 * Where the paper defers to Waechter & Biegler (the filter line-search IPM and
 * its inertia-correction algorithm) the constants are theirs.
 */
#include "mds_oracle.h"

#include <float.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Threads of the Bunch-Kaufman elimination (1 unless set).  Each entry of
 * the trailing triangle is updated by one thread with the same expression,
 * so every thread count gives bit-identical factors. */
static int g_threads = 1;

void or_set_threads(int32_t n) { g_threads = (n > 0) ? n : 1; }

#define IDX(i, j, ld) ((size_t)(j) * (size_t)(ld) + (size_t)(i))

/* ======================================================================== */
/* Condensation: Sec. 2.2, eq. (compressed).  dcv (optional, m entries) is
 * the per-row diagonal by which inequality rows enter the (2,2) block
 * (-D_h^{-1} of the compressed form); NULL when there is none.             */
/* ======================================================================== */

/* ---- blocks of Q_{x_s} (assumption A2, general form) --------------------- */

int64_t or_blk_words(const orq_problem *P) {
  int64_t t = 0;
  for (int b = 0; b < P->nblk; ++b) {
    const int64_t sz = P->bp[b + 1] - P->bp[b];
    t += sz * sz;
  }
  return t;
}

/* L Delta L' of every block of Q_{x_s} = blockdiag(Wb) + diag(dsbase) + dw I,
 * column by column (no pivoting: the blocks are positive definite when
 * dsbase + dw > 0 and Wb is positive semidefinite).  Diagonal entries are
 * (Wb_jj + dsbase_j) + dw.  For column j of a block:
 *   Delta_j = Q_jj - sum_{t<j} (L_jt Delta_t) L_jt,
 *   L_ij = (Q_ij - sum_{t<j} (L_it Delta_t) L_jt) / Delta_j   (i > j),
 * each sum in ascending t.  inv_d = 1/Delta. */
static void blk_factor(const orq_problem *P, const double *dsbase, double dw, double *lblk,
                       double *inv_d) {
  int smax = 1;
  for (int b = 0; b < P->nblk; ++b) smax = (P->bp[b + 1] - P->bp[b] > smax) ? P->bp[b + 1] - P->bp[b] : smax;
  double *dl = (double *)malloc(sizeof(double) * (size_t)smax);
  int64_t off = 0;
  for (int b = 0; b < P->nblk; ++b) {
    const int k0 = P->bp[b], sz = P->bp[b + 1] - k0;
    const double *Q = P->Wb + off;
    double *L = lblk + off;
    for (int j = 0; j < sz; ++j) {
      double d = (Q[IDX(j, j, sz)] + dsbase[k0 + j]) + dw;
      for (int t = 0; t < j; ++t) d = d - (L[IDX(j, t, sz)] * dl[t]) * L[IDX(j, t, sz)];
      dl[j] = d;
      L[IDX(j, j, sz)] = 1.0;
      for (int i = j + 1; i < sz; ++i) {
        double e = Q[IDX(i, j, sz)];
        for (int t = 0; t < j; ++t) e = e - (L[IDX(i, t, sz)] * dl[t]) * L[IDX(j, t, sz)];
        L[IDX(i, j, sz)] = e / d;
      }
    }
    for (int j = 0; j < sz; ++j) inv_d[k0 + j] = 1.0 / dl[j];
    off += (int64_t)sz * sz;
  }
  free(dl);
}

/* block index of every sparse variable and the offset of every block */
static void blk_maps(const orq_problem *P, int32_t *bid, int64_t *boff) {
  int64_t off = 0;
  for (int b = 0; b < P->nblk; ++b) {
    boff[b] = off;
    for (int k = P->bp[b]; k < P->bp[b + 1]; ++k) bid[k] = b;
    off += (int64_t)(P->bp[b + 1] - P->bp[b]) * (P->bp[b + 1] - P->bp[b]);
  }
}

/* Transformed Jacobian Jh = J_s L^{-T} in CSR: row i holds every column of
 * every block that row i of J_s touches (blocks in ascending order, columns
 * ascending inside a block).  Inside a block of size s starting at k0, with
 * u_p = J_s(i, k0 + p) (0 where J_s has no entry):
 *   Jh(i, k0 + p) = u_p - sum_{t<p} L_pt Jh(i, k0 + t)   (ascending t). */
typedef struct { int32_t *rp, *ci; double *v; } csr_t;

static csr_t blk_transform(const orq_problem *P, const double *lblk) {
  const int m = P->m, ns = P->n_s;
  int32_t *bid = (int32_t *)malloc(sizeof(int32_t) * (size_t)(ns > 0 ? ns : 1));
  int64_t *boff = (int64_t *)malloc(sizeof(int64_t) * (size_t)(P->nblk > 0 ? P->nblk : 1));
  blk_maps(P, bid, boff);
  csr_t J;
  J.rp = (int32_t *)malloc(sizeof(int32_t) * (size_t)(m + 1));
  J.rp[0] = 0;
  for (int i = 0; i < m; ++i) {
    int cnt = 0, last = -1;
    for (int a = P->rp[i]; a < P->rp[i + 1]; ++a) {
      const int b = bid[P->ci[a]];
      if (b != last) { cnt += P->bp[b + 1] - P->bp[b]; last = b; }
    }
    J.rp[i + 1] = J.rp[i] + cnt;
  }
  const int nnz = J.rp[m];
  J.ci = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nnz > 0 ? nnz : 1));
  J.v = (double *)malloc(sizeof(double) * (size_t)(nnz > 0 ? nnz : 1));
  for (int i = 0; i < m; ++i) {
    int e = J.rp[i], a = P->rp[i];
    const int ae = P->rp[i + 1];
    while (a < ae) {
      const int b = bid[P->ci[a]], k0 = P->bp[b], sz = P->bp[b + 1] - k0;
      const double *L = lblk + boff[b];
      for (int p = 0; p < sz; ++p) {
        double u = 0.0;
        if (a < ae && P->ci[a] == k0 + p) { u = P->v[a]; ++a; }
        for (int t = 0; t < p; ++t) u = u - L[IDX(p, t, sz)] * J.v[e + t];
        J.ci[e + p] = k0 + p;
        J.v[e + p] = u;
      }
      e += sz;
    }
  }
  free(bid); free(boff);
  return J;
}

/* u <- L^{-1} u (forward) or L^{-T} u (backward), block by block */
static void blk_lsolve(const orq_problem *P, const double *lblk, double *u, int transpose) {
  int64_t off = 0;
  for (int b = 0; b < P->nblk; ++b) {
    const int k0 = P->bp[b], sz = P->bp[b + 1] - k0;
    const double *L = lblk + off;
    if (!transpose) {
      for (int p = 0; p < sz; ++p) {
        double t = u[k0 + p];
        for (int q = 0; q < p; ++q) t = t - L[IDX(p, q, sz)] * u[k0 + q];
        u[k0 + p] = t;
      }
    } else {
      for (int p = sz - 1; p >= 0; --p) {
        double t = u[k0 + p];
        for (int q = p + 1; q < sz; ++q) t = t - L[IDX(q, p, sz)] * u[k0 + q];
        u[k0 + p] = t;
      }
    }
    off += (int64_t)sz * sz;
  }
}

void or_condense_dcv(const orq_problem *P, const double *sigma_d, const double *dsbase,
                     double dw, double dc, const double *dcv, double *M, double *inv_d,
                     double *lblk) {
  const int nd = P->n_d, ns = P->n_s, m = P->m, N = nd + m;
  /* D_s^{-1} (diagonal Q_{x_s}), or the blocks' factors and the transformed
   * Jacobian whose (2,2) Schur term has the diagonal middle factor 1/Delta */
  csr_t J = {(int32_t *)P->rp, (int32_t *)P->ci, (double *)P->v};
  if (P->nblk > 0) {
    blk_factor(P, dsbase, dw, lblk, inv_d);
    J = blk_transform(P, lblk);
  } else {
    for (int k = 0; k < ns; ++k) inv_d[k] = 1.0 / (dsbase[k] + dw);
  }
  /* (1,1) block: H + Sigma_d + dw I  (Q_{x_d} with its shift) */
  for (int j = 0; j < nd; ++j)
    for (int i = 0; i < nd; ++i) {
      double h = (i >= j) ? P->H[IDX(i, j, nd)] : P->H[IDX(j, i, nd)];
      if (i == j) h = (h + sigma_d[i]) + dw;
      M[IDX(i, j, N)] = h;
    }
  /* (2,1) and (1,2) blocks: the dense Jacobian J_d and its transpose */
  for (int j = 0; j < nd; ++j)
    for (int i = 0; i < m; ++i) {
      M[IDX(nd + i, j, N)] = P->Jd[IDX(i, j, m)];
      M[IDX(j, nd + i, N)] = P->Jd[IDX(i, j, m)];
    }
  /* (2,2) block: -J_s D_s^{-1} J_s' - dc I - diag(dcv).  Entry (i,j), i >= j,
   * sums over the shared columns k of rows i and j in ascending k. */
  for (int j = 0; j < m; ++j)
    for (int i = j; i < m; ++i) {
      double acc = 0.0;
      int a = J.rp[i], ae = J.rp[i + 1], b = J.rp[j], be = J.rp[j + 1];
      while (a < ae && b < be) {
        int ka = J.ci[a], kb = J.ci[b];
        if (ka < kb) ++a;
        else if (kb < ka) ++b;
        else {
          acc = acc - (J.v[a] * inv_d[ka]) * J.v[b];
          ++a; ++b;
        }
      }
      if (i == j) {
        acc = acc - dc;
        if (dcv) acc = acc - dcv[i];
      }
      M[IDX(nd + i, nd + j, N)] = acc;
      M[IDX(nd + j, nd + i, N)] = acc;
    }
  if (P->nblk > 0) { free(J.rp); free(J.ci); free(J.v); }
}

void or_condense(const orq_problem *P, const double *sigma_d, const double *dsbase,
                 double dw, double dc, double *M, double *inv_d, double *lblk) {
  or_condense_dcv(P, sigma_d, dsbase, dw, dc, NULL, M, inv_d, lblk);
}

void or_rhs_condense(const orq_problem *P, const double *inv_d, const double *lblk,
                     const double *r_s, const double *r_y, double *rhat) {
  if (P->nblk > 0) {
    /* r_y - (J_s L^{-T}) Delta^{-1} (L^{-1} r_s) */
    double *u = (double *)malloc(sizeof(double) * (size_t)(P->n_s > 0 ? P->n_s : 1));
    for (int k = 0; k < P->n_s; ++k) u[k] = r_s[k];
    blk_lsolve(P, lblk, u, 0);
    csr_t J = blk_transform(P, lblk);
    for (int i = 0; i < P->m; ++i) {
      double t = r_y[i];
      for (int a = J.rp[i]; a < J.rp[i + 1]; ++a) {
        int k = J.ci[a];
        t = t - J.v[a] * (inv_d[k] * u[k]);
      }
      rhat[i] = t;
    }
    free(J.rp); free(J.ci); free(J.v); free(u);
    return;
  }
  for (int i = 0; i < P->m; ++i) {
    double t = r_y[i];
    for (int a = P->rp[i]; a < P->rp[i + 1]; ++a) {
      int k = P->ci[a];
      t = t - P->v[a] * (inv_d[k] * r_s[k]);
    }
    rhat[i] = t;
  }
}

void or_backsub(const orq_problem *P, const double *inv_d, const double *lblk,
                const double *r_s, const double *dy, double *dx_s) {
  /* t = r_s - J_s' dy, accumulated row by row in ascending row order */
  double *t = (double *)malloc(sizeof(double) * (size_t)(P->n_s > 0 ? P->n_s : 1));
  for (int k = 0; k < P->n_s; ++k) t[k] = r_s[k];
  for (int i = 0; i < P->m; ++i)
    for (int a = P->rp[i]; a < P->rp[i + 1]; ++a) t[P->ci[a]] = t[P->ci[a]] - P->v[a] * dy[i];
  if (P->nblk > 0) {
    /* L^{-T} Delta^{-1} L^{-1} t */
    blk_lsolve(P, lblk, t, 0);
    for (int k = 0; k < P->n_s; ++k) t[k] = inv_d[k] * t[k];
    blk_lsolve(P, lblk, t, 1);
    for (int k = 0; k < P->n_s; ++k) dx_s[k] = t[k];
  } else {
    for (int k = 0; k < P->n_s; ++k) dx_s[k] = inv_d[k] * t[k];
  }
  free(t);
}

/* ======================================================================== */
/* Bunch-Kaufman diagonal pivoting, lower triangle, left to right (Sec. 2.3). */
/* ======================================================================== */

static void swap_d(double *a, double *b) {
  double t = *a; *a = *b; *b = t;
}

static int bk_until(int32_t N, double *A, int32_t *ipiv, double *dd, double *ds, int32_t *kind,
                    int32_t kstop);

int or_bk(int32_t N, double *A, int32_t *ipiv, double *dd, double *ds, int32_t *kind) {
  return bk_until(N, A, ipiv, dd, ds, kind, N);
}

int or_bk_partial(int32_t N, double *A, int32_t *ipiv, double *dd, double *ds, int32_t kstop) {
  return bk_until(N, A, ipiv, dd, ds, NULL, kstop);
}

/* The elimination of or_bk, stopped once kstop pivot columns are done. */
static int bk_until(int32_t N, double *A, int32_t *ipiv, double *dd, double *ds, int32_t *kind,
                    int32_t kstop) {
  const double alpha = (1.0 + sqrt(17.0)) / 8.0;
  int info = 0;
  double *w0 = (double *)malloc(sizeof(double) * (size_t)(N > 0 ? N : 1));
  double *w1 = (double *)malloc(sizeof(double) * (size_t)(N > 0 ? N : 1));
  double *l0 = (double *)malloc(sizeof(double) * (size_t)(N > 0 ? N : 1));
  double *l1 = (double *)malloc(sizeof(double) * (size_t)(N > 0 ? N : 1));
  for (int i = 0; i < N; ++i) { dd[i] = 0.0; ds[i] = 0.0; }
  int k = 0;
  while (k < N && k < kstop) {
    double absakk = fabs(A[IDX(k, k, N)]);
    /* column maximum below the diagonal; the first index wins ties */
    int imax = k;
    double colmax = 0.0;
    for (int i = k + 1; i < N; ++i) {
      double t = fabs(A[IDX(i, k, N)]);
      if (t > colmax) { colmax = t; imax = i; }
    }
    if (fmax(absakk, colmax) == 0.0 || isnan(absakk)) {
      /* zero column: record a zero 1x1 pivot and move on without elimination */
      if (info == 0) info = k + 1;
      ipiv[k] = k + 1;
      dd[k] = A[IDX(k, k, N)];
      if (kind) kind[k] = 0;
      k += 1;
      continue;
    }
    int kp = k, kstep = 1, br = 1;
    if (absakk >= alpha * colmax) {
      kp = k; br = 1;
    } else {
      /* largest off-diagonal magnitude in row/column imax of the active part */
      double rowmax = 0.0;
      for (int j = k; j < imax; ++j) rowmax = fmax(rowmax, fabs(A[IDX(imax, j, N)]));
      for (int i = imax + 1; i < N; ++i) rowmax = fmax(rowmax, fabs(A[IDX(i, imax, N)]));
      if (absakk >= alpha * colmax * (colmax / rowmax)) {
        kp = k; br = 2;
      } else if (fabs(A[IDX(imax, imax, N)]) >= alpha * rowmax) {
        kp = imax; br = 3;
      } else {
        kp = imax; kstep = 2; br = 4;
      }
    }
    if (kind) { kind[k] = br; if (kstep == 2) kind[k + 1] = br; }
    /* symmetric interchange of indices p = k+kstep-1 and q = kp (lower storage) */
    int p = k + kstep - 1, q = kp;
    if (q != p) {
      for (int j = 0; j < p; ++j) swap_d(&A[IDX(p, j, N)], &A[IDX(q, j, N)]);
      for (int j = p + 1; j < q; ++j) swap_d(&A[IDX(j, p, N)], &A[IDX(q, j, N)]);
      swap_d(&A[IDX(p, p, N)], &A[IDX(q, q, N)]);
      for (int i = q + 1; i < N; ++i) swap_d(&A[IDX(i, p, N)], &A[IDX(i, q, N)]);
    }
    if (kstep == 1) {
      double d = A[IDX(k, k, N)];
      dd[k] = d;
      ipiv[k] = kp + 1;
      for (int i = k + 1; i < N; ++i) { w0[i] = A[IDX(i, k, N)]; l0[i] = w0[i] / d; }
      /* rank-1 update of the trailing lower triangle: A -= l w' (columns
       * split over the threads; each entry's expression is unchanged) */
#pragma omp parallel for schedule(dynamic, 8) num_threads(g_threads) if (g_threads > 1 && N - k > 256)
      for (int j = k + 1; j < N; ++j)
        for (int i = j; i < N; ++i) A[IDX(i, j, N)] = A[IDX(i, j, N)] - l0[i] * w0[j];
      for (int i = k + 1; i < N; ++i) A[IDX(i, k, N)] = l0[i];
      k += 1;
    } else {
      double a = A[IDX(k, k, N)], b = A[IDX(k + 1, k, N)], c = A[IDX(k + 1, k + 1, N)];
      double det = a * c - b * b;
      dd[k] = a; dd[k + 1] = c; ds[k] = b;
      ipiv[k] = -(kp + 1);
      ipiv[k + 1] = -(kp + 1);
      /* L rows = [w0 w1] * inv([[a b];[b c]]) by Cramer's rule */
      for (int i = k + 2; i < N; ++i) {
        double x = A[IDX(i, k, N)], y = A[IDX(i, k + 1, N)];
        w0[i] = x; w1[i] = y;
        l0[i] = (x * c - y * b) / det;
        l1[i] = (y * a - x * b) / det;
      }
      /* rank-2 update: A -= [l0 l1] [w0 w1]' */
#pragma omp parallel for schedule(dynamic, 8) num_threads(g_threads) if (g_threads > 1 && N - k > 256)
      for (int j = k + 2; j < N; ++j)
        for (int i = j; i < N; ++i)
          A[IDX(i, j, N)] = A[IDX(i, j, N)] - (l0[i] * w0[j] + l1[i] * w1[j]);
      for (int i = k + 2; i < N; ++i) { A[IDX(i, k, N)] = l0[i]; A[IDX(i, k + 1, N)] = l1[i]; }
      A[IDX(k + 1, k, N)] = 0.0; /* belongs to D, not to L */
      k += 2;
    }
  }
  free(w0); free(w1); free(l0); free(l1);
  return info;
}

/* Inertia from the block-diagonal D (Sec. 2.3 and Sylvester's law of inertia):
 * a 1x1 pivot counts by its sign; every 2x2 block that Bunch-Kaufman selects
 * has a negative determinant (|a c| < alpha^2 b^2 < b^2) and so counts (1,0,1). */
void or_inertia(int32_t N, const int32_t *ipiv, const double *dd, const double *ds,
                int32_t out[3]) {
  (void)ds;
  out[0] = out[1] = out[2] = 0;
  for (int k = 0; k < N;) {
    if (ipiv[k] > 0) {
      if (dd[k] > 0.0) out[0]++;
      else if (dd[k] < 0.0) out[2]++;
      else out[1]++;
      k += 1;
    } else {
      out[0]++; out[2]++;
      k += 2;
    }
  }
}

int or_ldl_solve(int32_t N, const double *L, const int32_t *ipiv, const double *dd,
                 const double *ds, double *b) {
  int status = 0;
  /* b <- P' b : interchanges in pivot order */
  for (int k = 0; k < N;) {
    if (ipiv[k] > 0) {
      int kp = ipiv[k] - 1;
      if (kp != k) swap_d(&b[k], &b[kp]);
      k += 1;
    } else {
      int kp = -ipiv[k] - 1;
      if (kp != k + 1) swap_d(&b[k + 1], &b[kp]);
      k += 2;
    }
  }
  /* L y = b (unit lower) */
  for (int j = 0; j < N; ++j)
    for (int i = j + 1; i < N; ++i) b[i] = b[i] - L[IDX(i, j, N)] * b[j];
  /* D z = y */
  for (int k = 0; k < N;) {
    if (ipiv[k] > 0) {
      if (dd[k] == 0.0) status = 1;
      b[k] = b[k] / dd[k];
      k += 1;
    } else {
      double a = dd[k], c = dd[k + 1], s = ds[k];
      double det = a * c - s * s;
      double y0 = b[k], y1 = b[k + 1];
      b[k] = (c * y0 - s * y1) / det;
      b[k + 1] = (a * y1 - s * y0) / det;
      k += 2;
    }
  }
  /* L' x = z */
  for (int j = N - 1; j >= 0; --j) {
    double t = b[j];
    for (int i = j + 1; i < N; ++i) t = t - L[IDX(i, j, N)] * b[i];
    b[j] = t;
  }
  /* x <- P x : interchanges in reverse pivot order */
  int *start = (int *)malloc(sizeof(int) * (size_t)(N > 0 ? N : 1));
  int np = 0;
  for (int k = 0; k < N;) { start[np++] = k; k += (ipiv[k] > 0) ? 1 : 2; }
  for (int t = np - 1; t >= 0; --t) {
    int k = start[t];
    if (ipiv[k] > 0) {
      int kp = ipiv[k] - 1;
      if (kp != k) swap_d(&b[k], &b[kp]);
    } else {
      int kp = -ipiv[k] - 1;
      if (kp != k + 1) swap_d(&b[k + 1], &b[kp]);
    }
  }
  free(start);
  return status;
}

/* ======================================================================== */
/* Full KKT operator of eq. (linsys4x4) restricted to equality constraints. */
/* ======================================================================== */

/* out += blockdiag(Wb) u (each block's full symmetric matrix, rows in
 * ascending column order) */
static void blk_matvec_add(const orq_problem *P, const double *u, double *out) {
  int64_t off = 0;
  for (int b = 0; b < P->nblk; ++b) {
    const int k0 = P->bp[b], sz = P->bp[b + 1] - k0;
    const double *Q = P->Wb + off;
    for (int i = 0; i < sz; ++i) {
      double t = out[k0 + i];
      for (int j = 0; j < sz; ++j) t = t + ((i >= j) ? Q[IDX(i, j, sz)] : Q[IDX(j, i, sz)]) * u[k0 + j];
      out[k0 + i] = t;
    }
    off += (int64_t)sz * sz;
  }
}

/* blockdiag(Wb) u in a new array of n_s entries (zeros without blocks) */
static double *blk_product(const orq_problem *P, const double *u) {
  double *o = (double *)calloc((size_t)(P->n_s > 0 ? P->n_s : 1), sizeof(double));
  blk_matvec_add(P, u, o);
  return o;
}

/* acc += the row sums of |blockdiag(Wb)| off the diagonal; diag = the
 * blocks' diagonal entries (left untouched without blocks) */
static void blk_absrow_add(const orq_problem *P, double *acc, double *diag) {
  int64_t off = 0;
  for (int b = 0; b < P->nblk; ++b) {
    const int k0 = P->bp[b], sz = P->bp[b + 1] - k0;
    const double *Q = P->Wb + off;
    for (int i = 0; i < sz; ++i) {
      diag[k0 + i] = Q[IDX(i, i, sz)];
      for (int j = 0; j < sz; ++j)
        if (i != j) acc[k0 + i] += fabs((i > j) ? Q[IDX(i, j, sz)] : Q[IDX(j, i, sz)]);
    }
    off += (int64_t)sz * sz;
  }
}

void or_kkt_matvec(const orq_problem *P, const double *sigma_d, const double *dsbase,
                   double dw, double dc, const double *dx_d, const double *dx_s,
                   const double *dy, double *o_d, double *o_s, double *o_y) {
  or_kkt_matvec_dcv(P, sigma_d, dsbase, dw, dc, NULL, dx_d, dx_s, dy, o_d, o_s, o_y);
}

void or_kkt_matvec_dcv(const orq_problem *P, const double *sigma_d, const double *dsbase,
                       double dw, double dc, const double *dcv, const double *dx_d,
                       const double *dx_s, const double *dy, double *o_d, double *o_s,
                       double *o_y) {
  const int nd = P->n_d, ns = P->n_s, m = P->m;
  for (int i = 0; i < nd; ++i) {
    double t = 0.0;
    for (int j = 0; j < nd; ++j) {
      double h = (i >= j) ? P->H[IDX(i, j, nd)] : P->H[IDX(j, i, nd)];
      t = t + h * dx_d[j];
    }
    t = t + (sigma_d[i] + dw) * dx_d[i];
    for (int r = 0; r < m; ++r) t = t + P->Jd[IDX(r, i, m)] * dy[r];
    o_d[i] = t;
  }
  for (int k = 0; k < ns; ++k) o_s[k] = (dsbase[k] + dw) * dx_s[k];
  blk_matvec_add(P, dx_s, o_s);
  for (int r = 0; r < m; ++r)
    for (int a = P->rp[r]; a < P->rp[r + 1]; ++a) o_s[P->ci[a]] = o_s[P->ci[a]] + P->v[a] * dy[r];
  for (int r = 0; r < m; ++r) {
    double t = 0.0;
    for (int j = 0; j < nd; ++j) t = t + P->Jd[IDX(r, j, m)] * dx_d[j];
    for (int a = P->rp[r]; a < P->rp[r + 1]; ++a) t = t + P->v[a] * dx_s[P->ci[a]];
    t = t - dc * dy[r];
    if (dcv) t = t - dcv[r] * dy[r];
    o_y[r] = t;
  }
}

double or_kkt_norm_inf(const orq_problem *P, const double *sigma_d, const double *dsbase,
                       double dw, double dc) {
  return or_kkt_norm_inf_dcv(P, sigma_d, dsbase, dw, dc, NULL);
}

double or_kkt_norm_inf_dcv(const orq_problem *P, const double *sigma_d, const double *dsbase,
                           double dw, double dc, const double *dcv) {
  const int nd = P->n_d, ns = P->n_s, m = P->m;
  double best = 0.0;
  for (int i = 0; i < nd; ++i) {
    double t = 0.0;
    for (int j = 0; j < nd; ++j) {
      double h = (i >= j) ? P->H[IDX(i, j, nd)] : P->H[IDX(j, i, nd)];
      if (i == j) h = h + sigma_d[i] + dw;
      t += fabs(h);
    }
    for (int r = 0; r < m; ++r) t += fabs(P->Jd[IDX(r, i, m)]);
    best = fmax(best, t);
  }
  double *col = (double *)calloc((size_t)(ns > 0 ? ns : 1), sizeof(double));
  for (int r = 0; r < m; ++r)
    for (int a = P->rp[r]; a < P->rp[r + 1]; ++a) col[P->ci[a]] += fabs(P->v[a]);
  double *bd = (double *)calloc((size_t)(ns > 0 ? ns : 1), sizeof(double));
  blk_absrow_add(P, col, bd);
  for (int k = 0; k < ns; ++k) best = fmax(best, fabs((bd[k] + dsbase[k]) + dw) + col[k]);
  free(bd);
  free(col);
  for (int r = 0; r < m; ++r) {
    double t = fabs(dc) + (dcv ? fabs(dcv[r]) : 0.0);
    for (int j = 0; j < nd; ++j) t += fabs(P->Jd[IDX(r, j, m)]);
    for (int a = P->rp[r]; a < P->rp[r + 1]; ++a) t += fabs(P->v[a]);
    best = fmax(best, t);
  }
  return best;
}

/* ======================================================================== */
/* Factor objects, the inertia-correction loop, solve and refinement.       */
/* ======================================================================== */

or_factor *or_factor_new(const orq_problem *P) {
  or_factor *F = (or_factor *)calloc(1, sizeof(or_factor));
  int N = P->n_d + P->m;
  F->N = N;
  size_t nn = (size_t)N * (size_t)N;
  F->L = (double *)malloc(sizeof(double) * (nn > 0 ? nn : 1));
  F->dd = (double *)malloc(sizeof(double) * (size_t)(N > 0 ? N : 1));
  F->ds = (double *)malloc(sizeof(double) * (size_t)(N > 0 ? N : 1));
  F->ipiv = (int32_t *)malloc(sizeof(int32_t) * (size_t)(N > 0 ? N : 1));
  F->inv_d = (double *)malloc(sizeof(double) * (size_t)(P->n_s > 0 ? P->n_s : 1));
  const int64_t bw = or_blk_words(P);
  F->lblk = (double *)calloc((size_t)(bw > 0 ? bw : 1), sizeof(double));
  F->dcv = (double *)calloc((size_t)(P->m > 0 ? P->m : 1), sizeof(double));
  F->sig_h = NULL;
  return F;
}

void or_factor_free(or_factor *F) {
  if (!F) return;
  free(F->L); free(F->dd); free(F->ds); free(F->ipiv); free(F->inv_d); free(F->lblk);
  free(F->dcv); free(F);
}

void or_ineq_dcv(const orq_problem *P, const double *sig_h, double dw, double *dcv) {
  const int mE = P->m - P->m_I;
  for (int r = 0; r < P->m; ++r) dcv[r] = (r < mE) ? 0.0 : 1.0 / (sig_h[r - mE] + dw);
}

void or_factor_set_slack(or_factor *F, const double *sig_h) { F->sig_h = sig_h; }

/* the (4,4) diagonal of F's current system, or NULL when it has none */
static const double *fac_dcv(const orq_problem *P, const or_factor *F) {
  return (F->sig_h && P->m_I > 0) ? F->dcv : NULL;
}

void or_factor_once(const orq_problem *P, const double *sigma_d, const double *dsbase,
                    double dw, double dc, or_factor *F) {
  F->dw = dw;
  F->dc = dc;
  /* the slack block's D_h carries the same shift dw as the Hessian blocks */
  if (F->sig_h && P->m_I > 0) or_ineq_dcv(P, F->sig_h, dw, F->dcv);
  or_condense_dcv(P, sigma_d, dsbase, dw, dc, fac_dcv(P, F), F->L, F->inv_d, F->lblk);
  F->info = or_bk(F->N, F->L, F->ipiv, F->dd, F->ds, NULL);
  or_inertia(F->N, F->ipiv, F->dd, F->ds, F->inertia);
}

static int inertia_ok(const orq_problem *P, const or_factor *F) {
  return F->inertia[0] == P->n_d && F->inertia[1] == 0 && F->inertia[2] == P->m;
}

int or_factor_inertia(const orq_problem *P, const double *sigma_d, const double *dsbase,
                      double mu, double *dw_last, double dw_max, or_factor *F) {
  /* Waechter & Biegler (2006), Algorithm IC, with their constants. */
  const double dw_min = 1e-20, dw0 = 1e-4, kw_minus = 1.0 / 3.0, kw_plus = 8.0,
               kw_plus_bar = 100.0, dc_bar = 1e-8, kappa_c = 0.25;
  F->trials = 1;
  or_factor_once(P, sigma_d, dsbase, 0.0, 0.0, F);
  if (inertia_ok(P, F)) return 0;
  double dc = (F->inertia[1] > 0) ? dc_bar * pow(mu, kappa_c) : 0.0;
  double dw = (*dw_last == 0.0) ? dw0 : fmax(dw_min, kw_minus * *dw_last);
  for (;;) {
    F->trials++;
    or_factor_once(P, sigma_d, dsbase, dw, dc, F);
    if (inertia_ok(P, F)) { *dw_last = dw; return 0; }
    dw = (*dw_last == 0.0) ? kw_plus_bar * dw : kw_plus * dw;
    if (dw > dw_max) return 2;
  }
}

int or_newton_solve(const orq_problem *P, const or_factor *F, const double *r_d,
                    const double *r_s, const double *r_y, double *dx_d, double *dx_s,
                    double *dy) {
  const int nd = P->n_d, m = P->m, N = nd + m;
  double *z = (double *)malloc(sizeof(double) * (size_t)(N > 0 ? N : 1));
  for (int i = 0; i < nd; ++i) z[i] = r_d[i];
  or_rhs_condense(P, F->inv_d, F->lblk, r_s, r_y, z + nd);
  int st = or_ldl_solve(N, F->L, F->ipiv, F->dd, F->ds, z);
  for (int i = 0; i < nd; ++i) dx_d[i] = z[i];
  for (int i = 0; i < m; ++i) dy[i] = z[nd + i];
  or_backsub(P, F->inv_d, F->lblk, r_s, dy, dx_s);
  free(z);
  return st;
}

static double amax(int64_t n, const double *v) {
  double t = 0.0;
  for (int64_t i = 0; i < n; ++i) t = fmax(t, fabs(v[i]));
  return t;
}

int or_newton_refine(const orq_problem *P, const or_factor *F, const double *sigma_d,
                     const double *dsbase, const double *r_d, const double *r_s,
                     const double *r_y, double *dx_d, double *dx_s, double *dy,
                     int32_t max_steps, double eta_tol, double *eta_out) {
  const int nd = P->n_d, ns = P->n_s, m = P->m;
  size_t nt = (size_t)nd + (size_t)ns + (size_t)m;
  double *buf = (double *)malloc(sizeof(double) * (nt * 4 + 1));
  double *res = buf, *cor = buf + nt, *prev = buf + 2 * nt, *kx = buf + 3 * nt;
  or_newton_solve(P, F, r_d, r_s, r_y, dx_d, dx_s, dy);
  double nK = or_kkt_norm_inf_dcv(P, sigma_d, dsbase, F->dw, F->dc, fac_dcv(P, F));
  double nr = fmax(amax(nd, r_d), fmax(amax(ns, r_s), amax(m, r_y)));
  double eta_prev = INFINITY;
  int steps = 0;
  double eta = 0.0;
  for (;;) {
    or_kkt_matvec_dcv(P, sigma_d, dsbase, F->dw, F->dc, fac_dcv(P, F), dx_d, dx_s, dy, kx,
                      kx + nd, kx + nd + ns);
    for (int i = 0; i < nd; ++i) res[i] = r_d[i] - kx[i];
    for (int i = 0; i < ns; ++i) res[nd + i] = r_s[i] - kx[nd + i];
    for (int i = 0; i < m; ++i) res[nd + ns + i] = r_y[i] - kx[nd + ns + i];
    double nx = fmax(amax(nd, dx_d), fmax(amax(ns, dx_s), amax(m, dy)));
    double den = nK * nx + nr;
    eta = (den > 0.0) ? amax((int64_t)nt, res) / den : 0.0;
    if (steps > 0 && !(eta < eta_prev)) {
      /* no decrease: keep the previous iterate */
      memcpy(dx_d, prev, sizeof(double) * (size_t)nd);
      memcpy(dx_s, prev + nd, sizeof(double) * (size_t)ns);
      memcpy(dy, prev + nd + ns, sizeof(double) * (size_t)m);
      eta = eta_prev;
      break;
    }
    if (eta <= eta_tol || steps >= max_steps) break;
    memcpy(prev, dx_d, sizeof(double) * (size_t)nd);
    memcpy(prev + nd, dx_s, sizeof(double) * (size_t)ns);
    memcpy(prev + nd + ns, dy, sizeof(double) * (size_t)m);
    eta_prev = eta;
    or_newton_solve(P, F, res, res + nd, res + nd + ns, cor, cor + nd, cor + nd + ns);
    for (int i = 0; i < nd; ++i) dx_d[i] = dx_d[i] + cor[i];
    for (int i = 0; i < ns; ++i) dx_s[i] = dx_s[i] + cor[nd + i];
    for (int i = 0; i < m; ++i) dy[i] = dy[i] + cor[nd + ns + i];
    steps++;
  }
  if (eta_out) *eta_out = eta;
  free(buf);
  return steps;
}

/* ======================================================================== */
/* IPM vector quantities (K1/K2).                                           */
/* ======================================================================== */

/* The primal vector of the IPM: the n variables, then one slack per
 * inequality row; its bounds are [xl; hl] and [xu; hu]. */
static int nx_of(const orq_problem *P) { return P->n_d + P->n_s + P->m_I; }
static double lo_of(const orq_problem *P, int i) {
  const int n = P->n_d + P->n_s;
  return (i < n) ? P->xl[i] : P->hl[i - n];
}
static double up_of(const orq_problem *P, int i) {
  const int n = P->n_d + P->n_s;
  return (i < n) ? P->xu[i] : P->hu[i - n];
}

/* gradient of f over [x; d]: the objective does not depend on the slacks */
static void grad_f(const orq_problem *P, const double *x, double *gf) {
  const int nd = P->n_d, ns = P->n_s, n = nd + ns;
  for (int r = 0; r < P->m_I; ++r) gf[n + r] = 0.0;
  for (int i = 0; i < nd; ++i) {
    double t = 0.0;
    for (int j = 0; j < nd; ++j) {
      double h = (i >= j) ? P->H[IDX(i, j, nd)] : P->H[IDX(j, i, nd)];
      t = t + h * x[j];
    }
    gf[i] = t + P->c[i];
  }
  for (int k = 0; k < ns; ++k) gf[nd + k] = P->w[k] * x[nd + k] + P->g[k];
  blk_matvec_add(P, x + nd, gf + nd);
}

/* c(x, d) = J x - [b; d]: equality rows against b, inequality rows against
 * their slack d = x[n + r - m_E] */
static void constr(const orq_problem *P, const double *x, double *cx) {
  const int nd = P->n_d, m = P->m, n = nd + P->n_s, mE = m - P->m_I;
  for (int r = 0; r < m; ++r) {
    double t = 0.0;
    for (int j = 0; j < nd; ++j) t = t + P->Jd[IDX(r, j, m)] * x[j];
    for (int a = P->rp[r]; a < P->rp[r + 1]; ++a) t = t + P->v[a] * x[nd + P->ci[a]];
    cx[r] = t - ((r < mE) ? P->b[r] : x[n + r - mE]);
  }
}

/* out = (Jacobian of c)' y over [x; d]: J' y, then -y_h (the slack column
 * of an inequality row is -1) */
static void jac_t(const orq_problem *P, const double *y, double *out) {
  const int nd = P->n_d, ns = P->n_s, m = P->m, mE = m - P->m_I;
  for (int r = 0; r < P->m_I; ++r) out[nd + ns + r] = -y[mE + r];
  for (int j = 0; j < nd; ++j) {
    double t = 0.0;
    for (int r = 0; r < m; ++r) t = t + P->Jd[IDX(r, j, m)] * y[r];
    out[j] = t;
  }
  for (int k = 0; k < ns; ++k) out[nd + k] = 0.0;
  for (int r = 0; r < m; ++r)
    for (int a = P->rp[r]; a < P->rp[r + 1]; ++a) out[nd + P->ci[a]] = out[nd + P->ci[a]] + P->v[a] * y[r];
}

void or_sigma_rhs(const orq_problem *P, const double *x, const double *y, const double *zl,
                  const double *zu, double mu, double *sigma, double *r_x, double *r_y) {
  const int n = nx_of(P), m = P->m;
  double *gf = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
  double *jy = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
  grad_f(P, x, gf);
  jac_t(P, y, jy);
  for (int i = 0; i < n; ++i) {
    double s = 0.0, gb = gf[i] + jy[i];
    const double lo = lo_of(P, i), up = up_of(P, i);
    if (isfinite(lo)) {
      double sl = x[i] - lo;
      s = s + zl[i] / sl;
      gb = gb - mu / sl;
    }
    if (isfinite(up)) {
      double su = up - x[i];
      s = s + zu[i] / su;
      gb = gb + mu / su;
    }
    sigma[i] = s;
    r_x[i] = -gb;
  }
  double *cx = (double *)malloc(sizeof(double) * (size_t)(m > 0 ? m : 1));
  constr(P, x, cx);
  for (int r = 0; r < m; ++r) r_y[r] = -cx[r];
  free(cx); free(gf); free(jy);
}

double or_ftb(int64_t n, const double *v, const double *dv, double tau) {
  double a = 1.0;
  for (int64_t i = 0; i < n; ++i)
    if (dv[i] < 0.0) a = fmin(a, -tau * v[i] / dv[i]);
  return a;
}

double or_opt_error(const orq_problem *P, const double *x, const double *y,
                    const double *zl, const double *zu, double mu, double parts[6]) {
  const int n = nx_of(P), m = P->m;
  const double s_max = 100.0;
  double *gf = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
  double *jy = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
  double *cx = (double *)malloc(sizeof(double) * (size_t)(m > 0 ? m : 1));
  grad_f(P, x, gf);
  jac_t(P, y, jy);
  constr(P, x, cx);
  double dual = 0.0, cl = 0.0, cu = 0.0, z1 = 0.0, y1 = 0.0;
  int nz = 0;
  for (int i = 0; i < n; ++i) {
    double r = gf[i] + jy[i];
    const double lo = lo_of(P, i), up = up_of(P, i);
    if (isfinite(lo)) {
      r = r - zl[i];
      cl = fmax(cl, fabs((x[i] - lo) * zl[i] - mu));
      z1 += fabs(zl[i]);
      nz++;
    }
    if (isfinite(up)) {
      r = r + zu[i];
      cu = fmax(cu, fabs((up - x[i]) * zu[i] - mu));
      z1 += fabs(zu[i]);
      nz++;
    }
    dual = fmax(dual, fabs(r));
  }
  double prim = 0.0;
  for (int r = 0; r < m; ++r) { prim = fmax(prim, fabs(cx[r])); y1 += fabs(y[r]); }
  double sd = (m + nz > 0) ? fmax(s_max, (y1 + z1) / (double)(m + nz)) / s_max : 1.0;
  double sc = (nz > 0) ? fmax(s_max, z1 / (double)nz) / s_max : 1.0;
  if (parts) {
    parts[0] = dual; parts[1] = prim; parts[2] = cl; parts[3] = cu; parts[4] = sd; parts[5] = sc;
  }
  free(gf); free(jy); free(cx);
  return fmax(fmax(dual / sd, prim), fmax(cl, cu) / sc);
}

double or_objective(const orq_problem *P, const double *x) {
  const int nd = P->n_d, ns = P->n_s;
  double f = 0.0;
  for (int i = 0; i < nd; ++i) {
    double t = 0.0;
    for (int j = 0; j < nd; ++j) {
      double h = (i >= j) ? P->H[IDX(i, j, nd)] : P->H[IDX(j, i, nd)];
      t = t + h * x[j];
    }
    f = f + x[i] * (0.5 * t + P->c[i]);
  }
  double *wbx = blk_product(P, x + nd);
  for (int k = 0; k < ns; ++k) {
    double xs = x[nd + k];
    f = f + xs * (0.5 * (P->w[k] * xs + wbx[k]) + P->g[k]);
  }
  free(wbx);
  return f;
}

double or_barrier(const orq_problem *P, const double *x, double mu) {
  const int n = nx_of(P);
  double lg = 0.0;
  for (int i = 0; i < n; ++i) {
    const double lo = lo_of(P, i), up = up_of(P, i);
    if (isfinite(lo)) lg = lg + log(x[i] - lo);
    if (isfinite(up)) lg = lg + log(up - x[i]);
  }
  return or_objective(P, x) - mu * lg;
}

/* Rounding scale of phi_mu at x: the sum of the magnitudes of the terms
 * or_barrier adds up.  Its evaluation error is a small multiple of
 * DBL_EPSILON times this, however much the terms cancel. */
static double barrier_scale(const orq_problem *P, const double *x, double mu) {
  const int nd = P->n_d, ns = P->n_s, n = nx_of(P);
  double a = 0.0;
  for (int i = 0; i < nd; ++i) {
    double t = 0.0;
    for (int j = 0; j < nd; ++j) {
      double h = (i >= j) ? P->H[IDX(i, j, nd)] : P->H[IDX(j, i, nd)];
      t = t + h * x[j];
    }
    a = a + fabs(x[i] * (0.5 * t + P->c[i]));
  }
  double *wbx = blk_product(P, x + nd);
  for (int k = 0; k < ns; ++k) {
    double xs = x[nd + k];
    a = a + fabs(xs * (0.5 * (P->w[k] * xs + wbx[k]) + P->g[k]));
  }
  free(wbx);
  for (int i = 0; i < n; ++i) {
    const double lo = lo_of(P, i), up = up_of(P, i);
    if (isfinite(lo)) a = a + mu * fabs(log(x[i] - lo));
    if (isfinite(up)) a = a + mu * fabs(log(up - x[i]));
  }
  return a;
}

double or_theta(const orq_problem *P, const double *x) {
  double *cx = (double *)malloc(sizeof(double) * (size_t)(P->m > 0 ? P->m : 1));
  constr(P, x, cx);
  double t = 0.0;
  for (int r = 0; r < P->m; ++r) t += fabs(cx[r]);
  free(cx);
  return t;
}

/* ======================================================================== */
/* Filter line-search IPM (Sec. 2.1).                                        */
/* ======================================================================== */

typedef struct { double th, ph; } fentry;

/* Start point of a warm start (a reading of our own; the paper has no warm
 * start): the proposed x_d and y; x_s from the stationarity of the separable
 * sparse block without bound multipliers, x_s = -(g + J_s' y) / w where
 * w > 0 (else 0); every x_i then projected into the interior of its bounds by
 * the same kappa_1/kappa_2 rule as the cold start.  Bound multipliers: the
 * centred z_l = mu0 / (x - l), z_u = mu0 / (u - x) on finite bounds (0
 * otherwise), plus the part of the dual residual r = grad f(x) + J' y that
 * the bound can carry (stationarity of the Lagrangian asks z_l - z_u = r):
 * r_i > 0 is added to z_l,i when l_i is finite, -r_i > 0 to z_u,i when u_i is
 * finite. */
static void push_inside(double l, double u, double *xi);
static void init_slacks(const orq_problem *P, double *x);

static void warm_point(const orq_problem *P, const double *xd0, const double *y0, double mu0,
                       double *x, double *y, double *zl, double *zu) {
  const int nd = P->n_d, ns = P->n_s, m = P->m, n = nd + ns, nx = nx_of(P);
  const double kappa1 = 1e-2, kappa2 = 1e-2;
  double *jty = (double *)calloc((size_t)(ns > 0 ? ns : 1), sizeof(double));
  /* J_s' y, accumulated over rows in ascending order for every column */
  for (int r = 0; r < m; ++r)
    for (int a = P->rp[r]; a < P->rp[r + 1]; ++a) jty[P->ci[a]] = jty[P->ci[a]] + P->v[a] * y0[r];
  for (int i = 0; i < n; ++i) {
    double xi;
    if (i < nd) xi = xd0[i];
    else {
      const double wi = P->w[i - nd];
      xi = (wi > 0.0) ? -(P->g[i - nd] + jty[i - nd]) / wi : 0.0;
    }
    double l = P->xl[i], u = P->xu[i];
    int hl = isfinite(l), hu = isfinite(u);
    if (hl && hu) {
      double pl = fmin(kappa1 * fmax(1.0, fabs(l)), kappa2 * (u - l));
      double pu = fmin(kappa1 * fmax(1.0, fabs(u)), kappa2 * (u - l));
      xi = fmin(fmax(xi, l + pl), u - pu);
    } else if (hl) {
      xi = fmax(xi, l + kappa1 * fmax(1.0, fabs(l)));
    } else if (hu) {
      xi = fmin(xi, u - kappa1 * fmax(1.0, fabs(u)));
    }
    x[i] = xi;
    zl[i] = hl ? mu0 / (xi - l) : 0.0;
    zu[i] = hu ? mu0 / (u - xi) : 0.0;
  }
  /* slacks: the rows' values pushed inside their bounds, centred multipliers */
  init_slacks(P, x);
  for (int i = n; i < nx; ++i) {
    const double l = lo_of(P, i), u = up_of(P, i);
    zl[i] = isfinite(l) ? mu0 / (x[i] - l) : 0.0;
    zu[i] = isfinite(u) ? mu0 / (u - x[i]) : 0.0;
  }
  double *gf = (double *)calloc((size_t)(nx > 0 ? nx : 1), sizeof(double));
  double *jt = (double *)calloc((size_t)(nx > 0 ? nx : 1), sizeof(double));
  grad_f(P, x, gf);
  jac_t(P, y0, jt);
  for (int i = 0; i < nx; ++i) {
    const double r = gf[i] + jt[i];
    if (r > 0.0 && isfinite(lo_of(P, i))) zl[i] = zl[i] + r;
    if (r < 0.0 && isfinite(up_of(P, i))) zu[i] = zu[i] - r;
  }
  for (int r = 0; r < m; ++r) y[r] = y0[r];
  free(gf);
  free(jt);
  free(jty);
}

/* The tests of the line search that compare barrier values (Armijo, and
 * sufficient progress in phi) allow ten machine epsilons of the reference
 * iterate's rounding scale of phi (barrier_scale): near a solution the
 * decrease they ask for falls below the rounding error of phi itself, and
 * an exact comparison would reject full Newton steps on rounding noise. */
static int le_tol(double lhs, double rhs, double base) {
  return lhs - rhs <= 10.0 * DBL_EPSILON * fabs(base);
}

static int ipm_from(const orq_problem *P, const or_ipm_opts *o, const double *xd0,
                    const double *y0, double mu0_warm, double *x, double *y, double *zl,
                    double *zu, int32_t *iters, or_ipm_trace *trace);

int or_ipm(const orq_problem *P, const or_ipm_opts *o, double *x, double *y, double *zl,
           double *zu, int32_t *iters, or_ipm_trace *trace) {
  return ipm_from(P, o, NULL, NULL, 0.0, x, y, zl, zu, iters, trace);
}

int or_ipm_warm(const orq_problem *P, const or_ipm_opts *o, const double *xd0, const double *y0,
                double mu0, double *x, double *y, double *zl, double *zu, int32_t *iters,
                or_ipm_trace *trace) {
  /* the completed start point solves a diagonal sparse block (see warm_point) */
  if (P->nblk > 0) { *iters = 0; return 8; }
  return ipm_from(P, o, xd0, y0, mu0, x, y, zl, zu, iters, trace);
}

/* x pushed into the interior of [l, u] (Waechter & Biegler's kappa_1 = kappa_2
 * = 1e-2 rule; infinite bounds impose nothing) */
static void push_inside(double l, double u, double *xi) {
  const double kappa1 = 1e-2, kappa2 = 1e-2;
  const int hl = isfinite(l), hu = isfinite(u);
  if (hl && hu) {
    double pl = fmin(kappa1 * fmax(1.0, fabs(l)), kappa2 * (u - l));
    double pu = fmin(kappa1 * fmax(1.0, fabs(u)), kappa2 * (u - l));
    *xi = fmin(fmax(*xi, l + pl), u - pu);
  } else if (hl) {
    *xi = fmax(*xi, l + kappa1 * fmax(1.0, fabs(l)));
  } else if (hu) {
    *xi = fmin(*xi, u - kappa1 * fmax(1.0, fabs(u)));
  }
}

/* slack of each inequality row: its value (J x)_r at the start, pushed
 * inside [hl_r, hu_r] */
static void init_slacks(const orq_problem *P, double *x) {
  const int nd = P->n_d, m = P->m, n = nd + P->n_s, mE = m - P->m_I;
  for (int r = mE; r < m; ++r) {
    double t = 0.0;
    for (int j = 0; j < nd; ++j) t = t + P->Jd[IDX(r, j, m)] * x[j];
    for (int a = P->rp[r]; a < P->rp[r + 1]; ++a) t = t + P->v[a] * x[nd + P->ci[a]];
    push_inside(P->hl[r - mE], P->hu[r - mE], &t);
    x[n + r - mE] = t;
  }
}

/* The Newton direction for the factored system F (Sec. 2.1, eq. (linsys4x4)
 * with the slack step eliminated, then Sec. 2.2's condensed solve):
 *  - the inequality rows' right-hand side gains D_h^{-1} r_d, r_d being the
 *    slacks' part of r_x (ry2 is scratch of m entries);
 *  - [dx; dy] from the condensed solve refined on the full system;
 *  - the slack step from its row D_h dd - dy_h = r_d: dd = D_h^{-1}(r_d + dy_h);
 *  - the bound-multiplier steps from the linearised complementarity
 *    (x - l) dzl + zl dx = mu - (x - l) zl and (u - x) dzu - zu dx = mu - (u - x) zu. */
static void step_direction(const orq_problem *P, const or_factor *F, const double *x,
                           const double *zl, const double *zu, double mu, const double *sig,
                           const double *dsb, const double *rx, const double *ry,
                           int refine_steps, double *ry2, double *dx, double *dy, double *dzl,
                           double *dzu) {
  const int nd = P->n_d, m = P->m, n = nx_of(P), nv = nd + P->n_s, mE = m - P->m_I;
  for (int r = 0; r < m; ++r) ry2[r] = ry[r];
  for (int r = mE; r < m; ++r) ry2[r] = ry[r] + F->dcv[r] * rx[nv + r - mE];
  double eta = 0.0;
  or_newton_refine(P, F, sig, dsb, rx, rx + nd, ry2, dx, dx + nd, dy, refine_steps, 1e-14, &eta);
  for (int r = mE; r < m; ++r) dx[nv + r - mE] = F->dcv[r] * (rx[nv + r - mE] + dy[r]);
  for (int i = 0; i < n; ++i) {
    const double lo = lo_of(P, i), up = up_of(P, i);
    dzl[i] = 0.0; dzu[i] = 0.0;
    if (isfinite(lo)) {
      double sl = x[i] - lo;
      dzl[i] = mu / sl - zl[i] - (zl[i] / sl) * dx[i];
    }
    if (isfinite(up)) {
      double su = up - x[i];
      dzu[i] = mu / su - zu[i] + (zu[i] / su) * dx[i];
    }
  }
}

int or_newton_direction(const orq_problem *P, const double *x, const double *y, const double *zl,
                        const double *zu, double mu, int32_t refine_steps, double *dx,
                        double *dy, double *dzl, double *dzu) {
  const int nd = P->n_d, ns = P->n_s, m = P->m, n = nx_of(P);
  const size_t nb = (size_t)(n > 0 ? n : 1), mb = (size_t)(m > 0 ? m : 1);
  double *sig = (double *)malloc(sizeof(double) * nb);
  double *rx = (double *)malloc(sizeof(double) * nb);
  double *ry = (double *)malloc(sizeof(double) * mb);
  double *ry2 = (double *)malloc(sizeof(double) * mb);
  double *dsb = (double *)malloc(sizeof(double) * (size_t)(ns > 0 ? ns : 1));
  or_factor *F = or_factor_new(P);
  or_factor_set_slack(F, P->m_I > 0 ? sig + nd + ns : NULL);
  or_sigma_rhs(P, x, y, zl, zu, mu, sig, rx, ry);
  for (int k = 0; k < ns; ++k) dsb[k] = P->w[k] + sig[nd + k];
  double dw_last = 0.0;
  const int st = or_factor_inertia(P, sig, dsb, mu, &dw_last, 1e20, F);
  if (st == 0)
    step_direction(P, F, x, zl, zu, mu, sig, dsb, rx, ry, refine_steps, ry2, dx, dy, dzl, dzu);
  or_factor_free(F);
  free(sig); free(rx); free(ry); free(ry2); free(dsb);
  return st;
}

static int ipm_from(const orq_problem *P, const or_ipm_opts *o, const double *xd0,
                    const double *y0, double mu0_warm, double *x, double *y, double *zl,
                    double *zu, int32_t *iters, or_ipm_trace *trace) {
  const int nd = P->n_d, ns = P->n_s, m = P->m, n = nx_of(P), nv = nd + ns;
  /* Waechter & Biegler (2006) defaults */
  const double tau_min = 0.99, kappa_eps = 10.0, kappa_mu = 0.2, theta_mu = 1.5;
  const double kappa_sigma = 1e10, gamma_theta = 1e-5, gamma_phi = 1e-8, delta = 1.0;
  const double s_theta = 1.1, s_phi = 2.3, eta_phi = 1e-8, gamma_alpha = 0.05;
  int status = 6;

  /* start point: x = 0 pushed into the interior of its bounds, each slack
   * its row's value pushed inside the row's bounds, y = 0, z = 1 */
  for (int i = 0; i < n; ++i) {
    double l = lo_of(P, i), u = up_of(P, i), xi = 0.0;
    push_inside(l, u, &xi);
    x[i] = xi;
    zl[i] = isfinite(l) ? 1.0 : 0.0;
    zu[i] = isfinite(u) ? 1.0 : 0.0;
  }
  init_slacks(P, x);
  for (int r = 0; r < m; ++r) y[r] = 0.0;
  double mu = o->mu0;
  if (xd0) {
    warm_point(P, xd0, y0, mu0_warm, x, y, zl, zu);
    mu = mu0_warm;
  }
  double tau = fmax(tau_min, 1.0 - mu), dw_last = 0.0;
  double th0 = or_theta(P, x);
  double theta_max = 1e4 * fmax(1.0, th0), theta_min = 1e-4 * fmax(1.0, th0);
  fentry *filt = (fentry *)malloc(sizeof(fentry) * (size_t)(o->max_iter + 1));
  int nf = 0;

  const size_t nb = (size_t)(n > 0 ? n : 1), mb = (size_t)(m > 0 ? m : 1);
  double *sig = (double *)malloc(sizeof(double) * nb);
  double *rx = (double *)malloc(sizeof(double) * nb);
  double *ry = (double *)malloc(sizeof(double) * mb);
  double *ry2 = (double *)malloc(sizeof(double) * mb);
  double *dsb = (double *)malloc(sizeof(double) * (size_t)(ns > 0 ? ns : 1));
  double *dx = (double *)malloc(sizeof(double) * nb);
  double *dy = (double *)malloc(sizeof(double) * mb);
  double *dzl = (double *)malloc(sizeof(double) * nb);
  double *dzu = (double *)malloc(sizeof(double) * nb);
  double *xt = (double *)malloc(sizeof(double) * nb);
  double *gf = (double *)malloc(sizeof(double) * nb);
  or_factor *F = or_factor_new(P);
  /* the slack barrier diagonal Sigma_h sits after the variables' in sig */
  or_factor_set_slack(F, P->m_I > 0 ? sig + nv : NULL);

  int it = 0;
  for (it = 0; it < o->max_iter; ++it) {
    double E0 = or_opt_error(P, x, y, zl, zu, 0.0, NULL);
    if (!isfinite(E0)) { status = 7; break; }
    if (trace) { memset(&trace[it], 0, sizeof(or_ipm_trace)); trace[it].E0 = E0; }
    if (E0 <= o->tol) { status = 4; break; }
    /* barrier update while the barrier subproblem is solved to kappa_eps*mu */
    while (or_opt_error(P, x, y, zl, zu, mu, NULL) <= kappa_eps * mu) {
      double mnew = fmax(o->tol / 10.0, fmin(kappa_mu * mu, pow(mu, theta_mu)));
      if (!(mnew < mu)) break;
      mu = mnew;
      tau = fmax(tau_min, 1.0 - mu);
      nf = 0;
    }
    /* Newton system */
    or_sigma_rhs(P, x, y, zl, zu, mu, sig, rx, ry);
    for (int k = 0; k < ns; ++k) dsb[k] = P->w[k] + sig[nd + k];
    int fst = or_factor_inertia(P, sig, dsb, mu, &dw_last, o->dw_max, F);
    if (trace) {
      trace[it].mu = mu; trace[it].dw = F->dw; trace[it].dc = F->dc; trace[it].trials = F->trials;
      memcpy(trace[it].inertia, F->inertia, sizeof(F->inertia));
    }
    if (fst != 0) { status = 2; break; }
    step_direction(P, F, x, zl, zu, mu, sig, dsb, rx, ry, o->refine_steps, ry2, dx, dy, dzl, dzu);
    /* fraction to the boundary for slacks and bound multipliers */
    double a_pr = 1.0, a_du = 1.0;
    for (int i = 0; i < n; ++i) {
      const double lo = lo_of(P, i), up = up_of(P, i);
      if (isfinite(lo)) {
        double sl = x[i] - lo;
        if (dx[i] < 0.0) a_pr = fmin(a_pr, -tau * sl / dx[i]);
        if (dzl[i] < 0.0) a_du = fmin(a_du, -tau * zl[i] / dzl[i]);
      }
      if (isfinite(up)) {
        double su = up - x[i];
        if (-dx[i] < 0.0) a_pr = fmin(a_pr, -tau * su / (-dx[i]));
        if (dzu[i] < 0.0) a_du = fmin(a_du, -tau * zu[i] / dzu[i]);
      }
    }
    /* backtracking filter line search */
    double th = or_theta(P, x), ph = or_barrier(P, x, mu), phs = barrier_scale(P, x, mu);
    grad_f(P, x, gf);
    double gphi = 0.0;
    for (int i = 0; i < n; ++i) {
      double gi = gf[i];
      const double lo = lo_of(P, i), up = up_of(P, i);
      if (isfinite(lo)) gi = gi - mu / (x[i] - lo);
      if (isfinite(up)) gi = gi + mu / (up - x[i]);
      gphi = gphi + gi * dx[i];
    }
    double amin;
    if (gphi < 0.0) {
      amin = fmin(gamma_theta, gamma_phi * th / (-gphi));
      if (th <= theta_min) amin = fmin(amin, delta * pow(th, s_theta) / pow(-gphi, s_phi));
      amin = gamma_alpha * amin;
    } else {
      amin = gamma_alpha * gamma_theta;
    }
    double alpha = a_pr;
    int accepted = 0, augment = 1, nbt = 0;
    double tht = 0.0, pht = 0.0;
    for (;;) {
      for (int i = 0; i < n; ++i) xt[i] = x[i] + alpha * dx[i];
      tht = or_theta(P, xt);
      pht = or_barrier(P, xt, mu);
      int ok = isfinite(tht) && isfinite(pht);
      int infilt = !ok || tht >= theta_max;
      for (int f = 0; f < nf && !infilt; ++f)
        if (tht >= filt[f].th && pht >= filt[f].ph) infilt = 1;
      if (!infilt) {
        int sw = gphi < 0.0 && alpha * pow(-gphi, s_phi) > delta * pow(th, s_theta);
        int armijo = le_tol(pht - ph, eta_phi * alpha * gphi, phs);
        if (th <= theta_min && sw) {
          if (armijo) accepted = 1;
        } else if (tht <= (1.0 - gamma_theta) * th || le_tol(pht - ph, -gamma_phi * th, phs)) {
          accepted = 1;
        }
        if (accepted) augment = !(sw && armijo);
      }
      if (accepted) break;
      alpha = 0.5 * alpha;
      nbt++;
      if (alpha < amin) break;
    }
    if (trace) {
      trace[it].theta = th; trace[it].phi = ph; trace[it].alpha_pr = alpha;
      trace[it].alpha_du = a_du; trace[it].backtracks = nbt;
    }
    if (!accepted) { status = 5; break; }
    if (augment) {
      filt[nf].th = (1.0 - gamma_theta) * th;
      filt[nf].ph = ph - gamma_phi * th;
      nf++;
    }
    for (int i = 0; i < n; ++i) x[i] = xt[i];
    for (int r = 0; r < m; ++r) y[r] = y[r] + alpha * dy[r];
    for (int i = 0; i < n; ++i) {
      const double lo = lo_of(P, i), up = up_of(P, i);
      if (isfinite(lo)) {
        double z = zl[i] + a_du * dzl[i], sl = x[i] - lo;
        zl[i] = fmax(fmin(z, kappa_sigma * mu / sl), mu / (kappa_sigma * sl));
      }
      if (isfinite(up)) {
        double z = zu[i] + a_du * dzu[i], su = up - x[i];
        zu[i] = fmax(fmin(z, kappa_sigma * mu / su), mu / (kappa_sigma * su));
      }
    }
  }
  *iters = it;
  or_factor_free(F);
  free(filt); free(sig); free(rx); free(ry); free(ry2); free(dsb); free(dx); free(dy);
  free(dzl); free(dzu); free(xt); free(gf);
  return status;
}

/* ======================================================================== */
/* General NLP through an external model (the model objects of Sec. 2.3's   */
/* end: Jacobians and Hessians supplied by the modeling layer), with the    */
/* filter line search's second-order correction and feasibility restoration */
/* (the Waechter & Biegler method Sec. 2.1 names).                          */
/* ======================================================================== */

/* c(x) residual over the rows: c_r (equality rows, target 0), h_r - d_r
 * (inequality rows against their slack); returns theta = ||.||_1 */
static double nlp_resid(const orq_problem *P, const or_nlp_model *M, const double *x,
                        double *res) {
  const int m = P->m, n = P->n_d + P->n_s, mE = m - P->m_I;
  M->constraints(M->ctx, x, res);
  double t = 0.0;
  for (int r = 0; r < m; ++r) {
    if (r >= mE) res[r] = res[r] - x[n + r - mE];
    t += fabs(res[r]);
  }
  return t;
}

/* sum of log-slacks over the finite bounds of [x; d], and its magnitude sum */
static double nlp_logs(const orq_problem *P, const double *x, double *absum) {
  const int nx = nx_of(P);
  double lg = 0.0, a = 0.0;
  for (int i = 0; i < nx; ++i) {
    const double lo = lo_of(P, i), up = up_of(P, i);
    if (isfinite(lo)) { const double t = log(x[i] - lo); lg = lg + t; a = a + fabs(t); }
    if (isfinite(up)) { const double t = log(up - x[i]); lg = lg + t; a = a + fabs(t); }
  }
  if (absum) *absum = a;
  return lg;
}

/* scaled optimality error from gf (objective gradient over [x; d]), jy
 * (J' y over [x; d]) and res (constraint residual) */
static double nlp_error(const orq_problem *P, const double *x, const double *y,
                        const double *zl, const double *zu, double mu, const double *gf,
                        const double *jy, const double *res) {
  const int n = nx_of(P), m = P->m;
  const double s_max = 100.0;
  double dual = 0.0, cl = 0.0, cu = 0.0, z1 = 0.0, y1 = 0.0, prim = 0.0;
  int nz = 0;
  for (int i = 0; i < n; ++i) {
    double r = gf[i] + jy[i];
    const double lo = lo_of(P, i), up = up_of(P, i);
    if (isfinite(lo)) { r = r - zl[i]; cl = fmax(cl, fabs((x[i] - lo) * zl[i] - mu)); z1 += fabs(zl[i]); nz++; }
    if (isfinite(up)) { r = r + zu[i]; cu = fmax(cu, fabs((up - x[i]) * zu[i] - mu)); z1 += fabs(zu[i]); nz++; }
    if (!isfinite(r)) return NAN;
    dual = fmax(dual, fabs(r));
  }
  for (int r = 0; r < m; ++r) { prim = fmax(prim, fabs(res[r])); y1 += fabs(y[r]); }
  double sd = (m + nz > 0) ? fmax(s_max, (y1 + z1) / (double)(m + nz)) / s_max : 1.0;
  double sc = (nz > 0) ? fmax(s_max, z1 / (double)nz) / s_max : 1.0;
  return fmax(fmax(dual / sd, prim), fmax(cl, cu) / sc);
}

/* objective gradient over [x; d] (the slacks carry none) */
static void nlp_grad(const orq_problem *P, const or_nlp_model *M, const double *x, double *gf) {
  const int n = P->n_d + P->n_s, nx = nx_of(P);
  M->gradient(M->ctx, x, gf);
  for (int i = n; i < nx; ++i) gf[i] = 0.0;
}

/* largest primal step in (0, 1] keeping [x; d] + a dx at least (1 - tau) of
 * every slack to its finite bounds */
static double nlp_ftb(const orq_problem *P, const double *x, const double *dx, double tau) {
  const int nx = nx_of(P);
  double a = 1.0;
  for (int i = 0; i < nx; ++i) {
    const double lo = lo_of(P, i), up = up_of(P, i);
    if (isfinite(lo) && dx[i] < 0.0) a = fmin(a, -tau * (x[i] - lo) / dx[i]);
    if (isfinite(up) && -dx[i] < 0.0) a = fmin(a, -tau * (up - x[i]) / (-dx[i]));
  }
  return a;
}

typedef struct {
  double th_max, th_min;
  fentry *filt;
  int nf;
} nlp_filter;

static int nlp_in_filter(const nlp_filter *F, double th, double ph) {
  if (!(isfinite(th) && isfinite(ph)) || th >= F->th_max) return 1;
  for (int f = 0; f < F->nf; ++f)
    if (th >= F->filt[f].th && ph >= F->filt[f].ph) return 1;
  return 0;
}

/* the acceptance tests of one trial point (th_t, ph_t) against the current
 * (th, ph) with step alpha; *augment receives whether the filter grows */
static int nlp_accept(const nlp_filter *F, double th, double ph, double phs, double gphi,
                      double alpha, double th_t, double ph_t, int *augment) {
  const double gamma_theta = 1e-5, gamma_phi = 1e-8, delta = 1.0, s_theta = 1.1, s_phi = 2.3;
  const double eta_phi = 1e-8;
  if (nlp_in_filter(F, th_t, ph_t)) return 0;
  const int sw = gphi < 0.0 && alpha * pow(-gphi, s_phi) > delta * pow(th, s_theta);
  const int armijo = le_tol(ph_t - ph, eta_phi * alpha * gphi, phs);
  int acc = 0;
  if (th <= F->th_min && sw) {
    if (armijo) acc = 1;
  } else if (th_t <= (1.0 - gamma_theta) * th || le_tol(ph_t - ph, -gamma_phi * th, phs)) {
    acc = 1;
  }
  if (acc) *augment = !(sw && armijo);
  return acc;
}

/* Newton step of the factored system F for the right-hand side (rx, ry) of
 * the barrier problem at x, with the slack step eliminated as in
 * step_direction: dx over [x; d], dy; the bound-multiplier steps when dzl is
 * given */
static void nlp_step(const orq_problem *W, const or_factor *F, const double *x, const double *zl,
                     const double *zu, double mu, const double *sig, const double *dsb,
                     const double *rx, const double *ry, int refine_steps, double *ry2,
                     double *dx, double *dy, double *dzl, double *dzu) {
  step_direction(W, F, x, zl, zu, mu, sig, dsb, rx, ry, refine_steps, ry2, dx, dy, dzl, dzu);
}

/* Feasibility restoration (our reading of the phase Waechter & Biegler
 * describe): from x_R, Gauss-Newton-type barrier steps on
 *   min  zeta/2 ||D_R (x - x_R)||^2 - mu sum log(slacks)   s.t.  c(x) = 0
 * (zeta = sqrt(mu), D_R = diag(min(1, 1/|x_R|)), no constraint curvature,
 * bound multipliers centred at mu / slack), each step cut to the boundary
 * fraction and backtracked until theta decreases by 1e-4 alpha theta; the
 * phase ends when theta <= 0.9 theta(x_R) and (theta, phi) is acceptable to
 * the filter.  Returns the restoration iterations, or -1 (failure). */
static int nlp_restore(const orq_problem *P, const or_nlp_model *M, orq_problem *W,
                       const nlp_filter *Flt, double mu, double tau, int refine_steps,
                       double *x, double *y, double *zl, double *zu, or_factor *F,
                       double *work) {
  const int nd = P->n_d, ns = P->n_s, m = P->m, n = nd + ns, nx = nx_of(P);
  const size_t nb = (size_t)(nx > 0 ? nx : 1), mb = (size_t)(m > 0 ? m : 1);
  double *xR = work, *dr = xR + nb, *sig = dr + nb, *rx = sig + nb, *dx = rx + nb;
  double *xt = dx + nb, *jy = xt + nb, *dzl = jy + nb, *dzu = dzl + nb;
  double *res = dzu + nb, *ry = res + mb, *ry2 = ry + mb, *dy = ry2 + mb, *yr = dy + mb;
  double *dsb = yr + mb;  /* n_s <= nb entries */
  const double zeta = sqrt(mu);
  for (int i = 0; i < nx; ++i) {
    xR[i] = x[i];
    dr[i] = fmin(1.0, 1.0 / fabs(x[i]));
  }
  for (int r = 0; r < m; ++r) yr[r] = 0.0;
  const double thR = nlp_resid(P, M, x, res);
  double dw_last = 0.0;
  /* the factor's slack block follows this phase's barrier diagonal */
  or_factor_set_slack(F, P->m_I > 0 ? sig + n : NULL);
  for (int k = 0; k < 30; ++k) {
    const double th = nlp_resid(P, M, x, res);
    if (k > 0 && th <= 0.9 * thR) {
      double ab = 0.0;
      const double ph = M->objective(M->ctx, x) - mu * nlp_logs(P, x, &ab);
      if (!nlp_in_filter(Flt, th, ph)) {
        /* leave with centred bound multipliers */
        for (int i = 0; i < nx; ++i) {
          const double lo = lo_of(P, i), up = up_of(P, i);
          zl[i] = isfinite(lo) ? mu / (x[i] - lo) : 0.0;
          zu[i] = isfinite(up) ? mu / (up - x[i]) : 0.0;
        }
        return k;
      }
    }
    M->jacobian(M->ctx, x, (double *)W->Jd, (double *)W->v);
    /* proximal Hessian zeta D_R^2 (no constraint curvature) */
    double *H = (double *)W->H, *w = (double *)W->w;
    for (int j = 0; j < nd; ++j)
      for (int i = 0; i < nd; ++i) H[IDX(i, j, nd)] = (i == j) ? zeta * dr[i] * dr[i] : 0.0;
    for (int k2 = 0; k2 < ns; ++k2) w[k2] = zeta * dr[nd + k2] * dr[nd + k2];
    jac_t(W, yr, jy);
    for (int i = 0; i < nx; ++i) {
      double s = 0.0, gb = zeta * dr[i] * dr[i] * (x[i] - xR[i]) + jy[i];
      const double lo = lo_of(P, i), up = up_of(P, i);
      if (isfinite(lo)) { const double sl = x[i] - lo; s = s + (mu / sl) / sl; gb = gb - mu / sl; }
      if (isfinite(up)) { const double su = up - x[i]; s = s + (mu / su) / su; gb = gb + mu / su; }
      sig[i] = s;
      rx[i] = -gb;
      zl[i] = isfinite(lo) ? mu / (x[i] - lo) : 0.0;
      zu[i] = isfinite(up) ? mu / (up - x[i]) : 0.0;
    }
    for (int r = 0; r < m; ++r) ry[r] = -res[r];
    for (int k2 = 0; k2 < ns; ++k2) dsb[k2] = w[k2] + sig[nd + k2];
    if (or_factor_inertia(W, sig, dsb, mu, &dw_last, 1e20, F) != 0) return -1;
    nlp_step(W, F, x, zl, zu, mu, sig, dsb, rx, ry, refine_steps, ry2, dx, dy, dzl, dzu);
    double a = nlp_ftb(P, x, dx, tau);
    for (;;) {
      for (int i = 0; i < nx; ++i) xt[i] = x[i] + a * dx[i];
      const double tht = nlp_resid(P, M, xt, res);
      if (isfinite(tht) && tht <= (1.0 - 1e-4 * a) * th) break;
      a = 0.5 * a;
      if (a < 1e-12) return -1;
    }
    for (int i = 0; i < nx; ++i) x[i] = xt[i];
    for (int r = 0; r < m; ++r) yr[r] = yr[r] + a * dy[r];
  }
  return -1;
}

int or_nlp_ipm(const orq_problem *P, const or_nlp_model *M, const or_ipm_opts *o,
               int32_t force_resto, double *x, double *y, double *zl, double *zu,
               int32_t *iters, or_ipm_trace *trace, or_nlp_stats *stats) {
  const int nd = P->n_d, ns = P->n_s, m = P->m, n = nd + ns, nx = nx_of(P);
  const double tau_min = 0.99, kappa_eps = 10.0, kappa_mu = 0.2, theta_mu = 1.5;
  const double kappa_sigma = 1e10, gamma_theta = 1e-5, gamma_phi = 1e-8, delta = 1.0;
  const double s_theta = 1.1, s_phi = 2.3, gamma_alpha = 0.05, kappa_soc = 0.99;
  const int p_max = 4;
  int status = 6;
  const size_t nb = (size_t)(nx > 0 ? nx : 1), mb = (size_t)(m > 0 ? m : 1);
  /* the working problem: P's pattern and bounds, the model's current values */
  orq_problem W = *P;
  double *Hb = (double *)calloc((size_t)(nd > 0 ? nd * nd : 1), sizeof(double));
  double *Jdb = (double *)calloc((size_t)(m * nd > 0 ? m * nd : 1), sizeof(double));
  double *vb = (double *)calloc((size_t)(P->rp[m] > 0 ? P->rp[m] : 1), sizeof(double));
  double *wb = (double *)calloc((size_t)(ns > 0 ? ns : 1), sizeof(double));
  W.H = Hb; W.Jd = Jdb; W.v = vb; W.w = wb; W.nblk = 0;
  double *buf = (double *)calloc(24 * nb + 12 * mb, sizeof(double));
  double *gf = buf, *jy = gf + nb, *sig = jy + nb, *rx = sig + nb, *dx = rx + nb;
  double *dzl = dx + nb, *dzu = dzl + nb, *xt = dzu + nb, *xs = xt + nb, *dxs = xs + nb;
  double *dzs = dxs + nb, *dzs2 = dzs + nb;
  double *rwork = dzs2 + nb;  /* restoration: 10 nb + 5 mb */
  double *res = rwork + 10 * nb + 5 * mb, *ry = res + mb, *ry2 = ry + mb, *dy = ry2 + mb;
  double *dys = dy + mb, *csoc = dys + mb;
  double *dsb = (double *)calloc((size_t)(ns > 0 ? ns : 1), sizeof(double));
  fentry *filt = (fentry *)malloc(sizeof(fentry) * (size_t)(o->max_iter + 2));
  or_factor *F = or_factor_new(P);
  or_factor_set_slack(F, P->m_I > 0 ? sig + n : NULL);
  or_nlp_stats st0 = {0, 0, 0, 0};

  /* start point: x = 0 pushed inside its bounds, the inequality rows' slacks
   * their values pushed inside [hl, hu], y = 0, z = 1 */
  for (int i = 0; i < n; ++i) {
    double xi = 0.0;
    push_inside(P->xl[i], P->xu[i], &xi);
    x[i] = xi;
  }
  M->constraints(M->ctx, x, res);
  for (int r = m - P->m_I; r < m; ++r) {
    double t = res[r];
    push_inside(P->hl[r - (m - P->m_I)], P->hu[r - (m - P->m_I)], &t);
    x[n + r - (m - P->m_I)] = t;
  }
  for (int i = 0; i < nx; ++i) {
    zl[i] = isfinite(lo_of(P, i)) ? 1.0 : 0.0;
    zu[i] = isfinite(up_of(P, i)) ? 1.0 : 0.0;
  }
  for (int r = 0; r < m; ++r) y[r] = 0.0;
  double mu = o->mu0, tau = fmax(tau_min, 1.0 - mu), dw_last = 0.0;
  const double th0 = nlp_resid(P, M, x, res);
  nlp_filter Flt = {1e4 * fmax(1.0, th0), 1e-4 * fmax(1.0, th0), filt, 0};

  int it = 0;
  for (it = 0; it < o->max_iter; ++it) {
    nlp_grad(P, M, x, gf);
    const double th_x = nlp_resid(P, M, x, res);
    M->jacobian(M->ctx, x, Jdb, vb);
    jac_t(&W, y, jy);
    const double E0 = nlp_error(P, x, y, zl, zu, 0.0, gf, jy, res);
    if (trace) { memset(&trace[it], 0, sizeof(or_ipm_trace)); trace[it].E0 = E0; }
    if (!isfinite(E0)) { status = 7; break; }
    if (E0 <= o->tol) { status = 4; break; }
    while (nlp_error(P, x, y, zl, zu, mu, gf, jy, res) <= kappa_eps * mu) {
      const double mnew = fmax(o->tol / 10.0, fmin(kappa_mu * mu, pow(mu, theta_mu)));
      if (!(mnew < mu)) break;
      mu = mnew;
      tau = fmax(tau_min, 1.0 - mu);
      Flt.nf = 0;
    }
    M->hessian(M->ctx, x, y, Hb, wb);
    int wbad = 0;
    for (int k = 0; k < ns; ++k) wbad |= !(wb[k] >= 0.0);
    if (wbad) { status = 9; break; }
    /* barrier diagonal and Newton right-hand side over [x; d] */
    for (int i = 0; i < nx; ++i) {
      double s = 0.0, gb = gf[i] + jy[i];
      const double lo = lo_of(P, i), up = up_of(P, i);
      if (isfinite(lo)) { const double sl = x[i] - lo; s = s + zl[i] / sl; gb = gb - mu / sl; }
      if (isfinite(up)) { const double su = up - x[i]; s = s + zu[i] / su; gb = gb + mu / su; }
      sig[i] = s;
      rx[i] = -gb;
    }
    for (int r = 0; r < m; ++r) ry[r] = -res[r];
    for (int k = 0; k < ns; ++k) dsb[k] = wb[k] + sig[nd + k];
    const int fst = or_factor_inertia(&W, sig, dsb, mu, &dw_last, o->dw_max, F);
    if (trace) {
      trace[it].mu = mu; trace[it].dw = F->dw; trace[it].dc = F->dc; trace[it].trials = F->trials;
      memcpy(trace[it].inertia, F->inertia, sizeof(F->inertia));
    }
    if (fst != 0) { status = 2; break; }
    nlp_step(&W, F, x, zl, zu, mu, sig, dsb, rx, ry, o->refine_steps, ry2, dx, dy, dzl, dzu);
    /* fraction to the boundary */
    double a_pr = nlp_ftb(P, x, dx, tau), a_du = 1.0;
    for (int i = 0; i < nx; ++i) {
      if (isfinite(lo_of(P, i)) && dzl[i] < 0.0) a_du = fmin(a_du, -tau * zl[i] / dzl[i]);
      if (isfinite(up_of(P, i)) && dzu[i] < 0.0) a_du = fmin(a_du, -tau * zu[i] / dzu[i]);
    }
    /* merit values at x */
    double labs = 0.0;
    const double fx = M->objective(M->ctx, x);
    const double th = th_x, ph = fx - mu * nlp_logs(P, x, &labs);
    const double phs = fabs(fx) + mu * labs;
    double gphi = 0.0;
    for (int i = 0; i < nx; ++i) {
      double gi = gf[i];
      const double lo = lo_of(P, i), up = up_of(P, i);
      if (isfinite(lo)) gi = gi - mu / (x[i] - lo);
      if (isfinite(up)) gi = gi + mu / (up - x[i]);
      gphi = gphi + gi * dx[i];
    }
    double amin;
    if (gphi < 0.0) {
      amin = fmin(gamma_theta, gamma_phi * th / (-gphi));
      if (th <= Flt.th_min) amin = fmin(amin, delta * pow(th, s_theta) / pow(-gphi, s_phi));
      amin = gamma_alpha * amin;
    } else {
      amin = gamma_alpha * gamma_theta;
    }
    double alpha = a_pr, alpha_y = a_pr;
    int accepted = 0, augment = 1, nbt = 0, soc = 0;
    const double *xacc = xt;
    for (;;) {
      for (int i = 0; i < nx; ++i) xt[i] = x[i] + alpha * dx[i];
      double la = 0.0;
      const double tht = nlp_resid(P, M, xt, csoc);
      const double pht = M->objective(M->ctx, xt) - mu * nlp_logs(P, xt, &la);
      if (nlp_accept(&Flt, th, ph, phs, gphi, alpha, tht, pht, &augment)) {
        accepted = 1;
        xacc = xt;
        break;
      }
      /* second-order correction on the first trial when theta did not drop */
      if (nbt == 0 && tht >= th) {
        double th_old = tht, a_soc = alpha;
        /* c_soc = alpha c(x) + c(x + alpha dx) */
        for (int r = 0; r < m; ++r) csoc[r] = alpha * res[r] + csoc[r];
        for (int p = 0; p < p_max; ++p) {
          st0.soc_trials++;
          for (int r = 0; r < m; ++r) ry[r] = -csoc[r];
          nlp_step(&W, F, x, zl, zu, mu, sig, dsb, rx, ry, o->refine_steps, ry2, dxs, dys, dzs,
                   dzs2);
          a_soc = nlp_ftb(P, x, dxs, tau);
          for (int i = 0; i < nx; ++i) xs[i] = x[i] + a_soc * dxs[i];
          double lb = 0.0;
          const double ths = nlp_resid(P, M, xs, ry2);
          const double phs_t = M->objective(M->ctx, xs) - mu * nlp_logs(P, xs, &lb);
          if (nlp_accept(&Flt, th, ph, phs, gphi, alpha, ths, phs_t, &augment)) {
            accepted = 1;
            soc = 1;
            xacc = xs;
            st0.soc_accepted++;
            break;
          }
          if (!(ths <= kappa_soc * th_old)) break;
          th_old = ths;
          for (int r = 0; r < m; ++r) csoc[r] = a_soc * csoc[r] + ry2[r];
        }
        if (accepted) break;
      }
      alpha = 0.5 * alpha;
      nbt++;
      if (alpha < amin || nbt >= 200) break;
    }
    if (trace) {
      trace[it].theta = th; trace[it].phi = ph; trace[it].alpha_pr = soc ? a_pr : alpha;
      trace[it].alpha_du = a_du; trace[it].backtracks = nbt; trace[it].soc = soc;
    }
    if (!accepted || it == force_resto) {
      /* the iterate that enters restoration joins the filter */
      filt[Flt.nf].th = (1.0 - gamma_theta) * th;
      filt[Flt.nf].ph = ph - gamma_phi * th;
      Flt.nf++;
      const int k = nlp_restore(P, M, &W, &Flt, mu, tau, o->refine_steps, x, y, zl, zu, F, rwork);
      or_factor_set_slack(F, P->m_I > 0 ? sig + n : NULL);
      st0.resto_calls++;
      if (trace) trace[it].resto = (k >= 0) ? k : -1;
      if (k < 0) { status = 5; break; }
      st0.resto_iters += k;
      continue;
    }
    if (augment) {
      filt[Flt.nf].th = (1.0 - gamma_theta) * th;
      filt[Flt.nf].ph = ph - gamma_phi * th;
      Flt.nf++;
    }
    alpha_y = soc ? a_pr : alpha;
    for (int i = 0; i < nx; ++i) x[i] = xacc[i];
    for (int r = 0; r < m; ++r) y[r] = y[r] + alpha_y * dy[r];
    for (int i = 0; i < nx; ++i) {
      const double lo = lo_of(P, i), up = up_of(P, i);
      if (isfinite(lo)) {
        const double z = zl[i] + a_du * dzl[i], sl = x[i] - lo;
        zl[i] = fmax(fmin(z, kappa_sigma * mu / sl), mu / (kappa_sigma * sl));
      }
      if (isfinite(up)) {
        const double z = zu[i] + a_du * dzu[i], su = up - x[i];
        zu[i] = fmax(fmin(z, kappa_sigma * mu / su), mu / (kappa_sigma * su));
      }
    }
  }
  *iters = it;
  if (stats) *stats = st0;
  or_factor_free(F);
  free(filt); free(buf); free(dsb); free(Hb); free(Jdb); free(vb); free(wb);
  return status;
}

/* ---- the nonlinear test family (separable, A1 and A2 hold) --------------- */
/* f(x) = 0.5 x_d'H x_d + c'x_d + sum_k (0.5 w_k x_k^2 + g_k x_k + e_k (exp(x_k) - x_k))
 * c_r(x) = (J_d x_d)_r + (J_s x_s)_r + sum_j Q_rj x_d,j^2 - b_r  (equality rows)
 * h_r(x) = the same without b_r                                   (inequality rows)
 * with P's H, c, w, g, J_d, J_s, b and the family's Q (m x n_d) and e (n_s). */
typedef struct {
  const orq_problem *P;
  const double *Q, *e;
} nlp_test;

static double nt_f(void *ctx, const double *x) {
  const nlp_test *T = (const nlp_test *)ctx;
  const orq_problem *P = T->P;
  const int nd = P->n_d, ns = P->n_s;
  double f = or_objective(P, x);
  for (int k = 0; k < ns; ++k) f = f + T->e[k] * (exp(x[nd + k]) - x[nd + k]);
  return f;
}
static void nt_g(void *ctx, const double *x, double *g) {
  const nlp_test *T = (const nlp_test *)ctx;
  const orq_problem *P = T->P;
  const int nd = P->n_d, ns = P->n_s;
  for (int i = 0; i < nd; ++i) {
    double t = 0.0;
    for (int j = 0; j < nd; ++j) {
      double h = (i >= j) ? P->H[IDX(i, j, nd)] : P->H[IDX(j, i, nd)];
      t = t + h * x[j];
    }
    g[i] = t + P->c[i];
  }
  for (int k = 0; k < ns; ++k)
    g[nd + k] = P->w[k] * x[nd + k] + P->g[k] + T->e[k] * (exp(x[nd + k]) - 1.0);
}
static void nt_c(void *ctx, const double *x, double *c) {
  const nlp_test *T = (const nlp_test *)ctx;
  const orq_problem *P = T->P;
  const int nd = P->n_d, m = P->m, mE = m - P->m_I;
  for (int r = 0; r < m; ++r) {
    double t = 0.0;
    for (int j = 0; j < nd; ++j) t = t + P->Jd[IDX(r, j, m)] * x[j];
    for (int a = P->rp[r]; a < P->rp[r + 1]; ++a) t = t + P->v[a] * x[nd + P->ci[a]];
    for (int j = 0; j < nd; ++j) t = t + T->Q[IDX(r, j, m)] * (x[j] * x[j]);
    c[r] = (r < mE) ? t - P->b[r] : t;
  }
}
static void nt_j(void *ctx, const double *x, double *Jd, double *v) {
  const nlp_test *T = (const nlp_test *)ctx;
  const orq_problem *P = T->P;
  const int nd = P->n_d, m = P->m;
  for (int j = 0; j < nd; ++j)
    for (int r = 0; r < m; ++r)
      Jd[IDX(r, j, m)] = P->Jd[IDX(r, j, m)] + 2.0 * T->Q[IDX(r, j, m)] * x[j];
  for (int a = 0; a < P->rp[m]; ++a) v[a] = P->v[a];
}
static void nt_h(void *ctx, const double *x, const double *y, double *H, double *w) {
  const nlp_test *T = (const nlp_test *)ctx;
  const orq_problem *P = T->P;
  const int nd = P->n_d, ns = P->n_s, m = P->m;
  for (int j = 0; j < nd; ++j)
    for (int i = 0; i < nd; ++i) H[IDX(i, j, nd)] = P->H[IDX(i, j, nd)];
  for (int j = 0; j < nd; ++j) {
    double t = 0.0;
    for (int r = 0; r < m; ++r) t = t + y[r] * (2.0 * T->Q[IDX(r, j, m)]);
    H[IDX(j, j, nd)] = H[IDX(j, j, nd)] + t;
  }
  for (int k = 0; k < ns; ++k) w[k] = P->w[k] + T->e[k] * exp(x[nd + k]);
}

int or_nlp_test_ipm(const orq_problem *P, const double *Q, const double *e,
                    const or_ipm_opts *o, int32_t force_resto, double *x, double *y,
                    double *zl, double *zu, int32_t *iters, or_ipm_trace *trace,
                    or_nlp_stats *stats) {
  nlp_test T = {P, Q, e};
  or_nlp_model M = {&T, nt_f, nt_g, nt_c, nt_j, nt_h};
  return or_nlp_ipm(P, &M, o, force_resto, x, y, zl, zu, iters, trace, stats);
}

/* the test family's model at x (for finite-difference pins): f, gradient
 * (n), constraints (m), Jacobian values (J_d m x n_d, J_s nnz) and the
 * Lagrangian Hessian at (x, y) (H n_d x n_d, w n_s) */
double or_nlp_test_eval(const orq_problem *P, const double *Q, const double *e, const double *x,
                        const double *y, double *g, double *c, double *Jd, double *v,
                        double *H, double *w) {
  nlp_test T = {P, Q, e};
  nt_g(&T, x, g);
  nt_c(&T, x, c);
  nt_j(&T, x, Jd, v);
  nt_h(&T, x, y, H, w);
  return nt_f(&T, x);
}
