// IPM vector and matrix-vector kernels (Sec. 2.1 and Sec. 2.3, kernel
// classes K1 and K2): dense GEMV with H and J_d, sparse products with J_s
// and J_s', the barrier diagonal and Newton right-hand side, multiplier
// directions, fraction to the boundary, optimality error, merit functions and
// the step update.  All reductions use a fixed tree (per-block partials in a
// fixed order, then one workgroup over the partials), so results are
// bitwise reproducible run to run.
#include "internal.hpp"
#include "vec.hpp"

namespace mds {
namespace {

inline unsigned grid1(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

// y = beta*y + A x,  A rows x cols (column-major, lda).  Workgroup = 64 rows x
// 16 column groups; partial sums combined in a fixed order.
__global__ __launch_bounds__(1024) void k_gemv_n(int rows, int cols, const double *__restrict__ A,
                                                 int lda, const double *__restrict__ x,
                                                 double beta, double *__restrict__ y) {
  __shared__ double part[16][65];
  const int r = threadIdx.x & 63, g = threadIdx.x >> 6;
  const int i = blockIdx.x * 64 + r;
  double s = 0.0;
  if (i < rows)
    for (int j = g; j < cols; j += 16) s = fma(A[(size_t)i + (size_t)j * lda], x[j], s);
  part[g][r] = s;
  __syncthreads();
  if (g == 0 && i < rows) {
    double t = 0.0;
    for (int q = 0; q < 16; ++q) t += part[q][r];
    y[i] = (beta == 0.0) ? t : fma(beta, y[i], t);
  }
}

// y = beta*y + A' x: one wave per column.
__global__ __launch_bounds__(256) void k_gemv_t(int rows, int cols, const double *__restrict__ A,
                                                int lda, const double *__restrict__ x,
                                                double beta, double *__restrict__ y) {
  const int lane = threadIdx.x & 63;
  const int j = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (j >= cols) return;
  double s = 0.0;
  for (int i = lane; i < rows; i += 64) s = fma(A[(size_t)i + (size_t)j * lda], x[i], s);
  s = wave_sum(s);
  if (lane == 0) y[j] = (beta == 0.0) ? s : fma(beta, y[j], s);
}

__global__ void k_spmv_csr(int rows, const int32_t *__restrict__ rp,
                           const int32_t *__restrict__ ci, const double *__restrict__ v,
                           const double *__restrict__ x, double beta, double *__restrict__ y) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= rows) return;
  double s = (beta == 0.0) ? 0.0 : beta * y[i];
  for (int a = rp[i]; a < rp[i + 1]; ++a) s = fma(v[a], x[ci[a]], s);
  y[i] = s;
}

__global__ void k_spmv_csc(int cols, const int32_t *__restrict__ cptr,
                           const int32_t *__restrict__ crow, const double *__restrict__ cval,
                           const double *__restrict__ x, double beta, double *__restrict__ y) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= cols) return;
  double s = (beta == 0.0) ? 0.0 : beta * y[k];
  for (int e = cptr[k]; e < cptr[k + 1]; ++e) s = fma(cval[e], x[crow[e]], s);
  y[k] = s;
}

}  // namespace

void launch_gemv_n(hipStream_t s, int rows, int cols, const double *A, int lda,
                   const double *x, double beta, double *y) {
  if (rows <= 0) return;
  k_gemv_n<<<grid1(rows, 64), 1024, 0, s>>>(rows, cols, A, lda, x, beta, y);
}

void launch_gemv_t(hipStream_t s, int rows, int cols, const double *A, int lda,
                   const double *x, double beta, double *y) {
  if (cols <= 0) return;
  k_gemv_t<<<grid1(cols, 4), 256, 0, s>>>(rows, cols, A, lda, x, beta, y);
}

void launch_spmv_csr(hipStream_t s, int rows, const int32_t *rp, const int32_t *ci,
                     const double *v, const double *x, double beta, double *y) {
  if (rows <= 0) return;
  k_spmv_csr<<<grid1(rows, 256), 256, 0, s>>>(rows, rp, ci, v, x, beta, y);
}

void launch_spmv_csc(hipStream_t s, int cols, const int32_t *cptr, const int32_t *crow,
                     const double *cval, const double *x, double beta, double *y) {
  if (cols <= 0) return;
  k_spmv_csc<<<grid1(cols, 256), 256, 0, s>>>(cols, cptr, crow, cval, x, beta, y);
}

}  // namespace mds
