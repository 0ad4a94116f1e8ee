// FP64 kernels of the GMRES-based refinement (Krylov basis products and
// updates).  Reductions are deterministic: each of kDotBlocks blocks sums a
// fixed chunk in a fixed tree, and the host adds the per-block partials in
// block order.
#include "internal.hpp"
#include "vec.hpp"

namespace mds {
namespace {

constexpr int kDotThreads = 256;

// partial[c * kDotBlocks + b] = sum over block b's chunk of V[:, c] . w
__global__ __launch_bounds__(kDotThreads) void k_dots(int64_t n, int ncol,
                                                     const double *__restrict__ V, int64_t ldv,
                                                     const double *__restrict__ w,
                                                     double *__restrict__ partial) {
  __shared__ double sh[kDotThreads / 64];
  const int b = blockIdx.x, c = blockIdx.y, tid = threadIdx.x;
  const int64_t chunk = (n + kDotBlocks - 1) / kDotBlocks;
  const int64_t lo = (int64_t)b * chunk, hi = (lo + chunk < n) ? lo + chunk : n;
  const double *v = V + (int64_t)c * ldv;
  double acc = 0.0;
  for (int64_t i = lo + tid; i < hi; i += kDotThreads) acc = fma(v[i], w[i], acc);
  acc = wave_sum(acc);
  if ((tid & 63) == 0) sh[tid >> 6] = acc;
  __syncthreads();
  if (tid == 0) {
    double t = sh[0];
    for (int q = 1; q < kDotThreads / 64; ++q) t += sh[q];
    partial[(int64_t)c * kDotBlocks + b] = t;
  }
}

// w -= sum_j coef[j] V[:, j]
__global__ void k_sub_cols(int64_t n, int ncol, const double *__restrict__ V, int64_t ldv,
                           const double *__restrict__ coef, double *__restrict__ w) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double acc = w[i];
  for (int j = 0; j < ncol; ++j) acc = fma(-coef[j], V[i + (int64_t)j * ldv], acc);
  w[i] = acc;
}

// x += sum_j coef[j] Z[:, j]
__global__ void k_add_cols(int64_t n, int ncol, const double *__restrict__ Z, int64_t ldz,
                           const double *__restrict__ coef, double *__restrict__ x) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double acc = x[i];
  for (int j = 0; j < ncol; ++j) acc = fma(coef[j], Z[i + (int64_t)j * ldz], acc);
  x[i] = acc;
}

__global__ void k_scale(int64_t n, double alpha, const double *__restrict__ w,
                        double *__restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = alpha * w[i];
}

inline unsigned g256(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

void launch_dots(hipStream_t s, int64_t n, int ncol, const double *V, int64_t ldv,
                 const double *w, double *partial) {
  k_dots<<<dim3(kDotBlocks, (unsigned)ncol), kDotThreads, 0, s>>>(n, ncol, V, ldv, w, partial);
}

void launch_sub_cols(hipStream_t s, int64_t n, int ncol, const double *V, int64_t ldv,
                     const double *coef, double *w) {
  if (n > 0) k_sub_cols<<<g256(n), 256, 0, s>>>(n, ncol, V, ldv, coef, w);
}

void launch_add_cols(hipStream_t s, int64_t n, int ncol, const double *Z, int64_t ldz,
                     const double *coef, double *x) {
  if (n > 0) k_add_cols<<<g256(n), 256, 0, s>>>(n, ncol, Z, ldz, coef, x);
}

void launch_scale(hipStream_t s, int64_t n, double alpha, const double *w, double *out) {
  if (n > 0) k_scale<<<g256(n), 256, 0, s>>>(n, alpha, w, out);
}

}  // namespace mds
