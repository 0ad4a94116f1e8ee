// Warm-start model: a multilayer perceptron in0 -> h -> h -> out with GELU
// (exact, erf form) after the two hidden layers and a linear skip path from
// the input to the output (Y = H2 W2 + b2 + X Ws), trained by mean-squared
// error with Adam, all in own HIP kernels.  Training products run on FP32
// MFMA (v_mfma_f32_16x16x4f32); inference can run on BF16 MFMA with FP32
// accumulation (v_mfma_f32_16x16x16bf16_1k).  Row-major activations
// (batch x features), weights W[l] as (in x out) row-major.
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "internal.hpp"

namespace mds {
namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef short s4 __attribute__((ext_vector_type(4)));

constexpr int GT = 64;  // output tile (rows x cols) per workgroup of 256 threads

__device__ inline short bf16_rne(float x) {
  const uint32_t u = __float_as_uint(x);
  return (short)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}

// C(i, j) = sum_k A(i, k) B(k, j) [+ bias(j)] [GELU], A(i,k) = A[i*sai + k*sak],
// B(k,j) = B[k*sbk + j*sbj], C row-major with ldc.  Optionally stores the
// pre-activation in Z.  MODE 0: FP32 MFMA; MODE 1: BF16 MFMA, FP32 accumulate.
template <int MODE>
__global__ __launch_bounds__(256) void k_gemm(int M, int N, int K, const float *__restrict__ A,
                                              int64_t sai, int64_t sak,
                                              const float *__restrict__ B, int64_t sbk,
                                              int64_t sbj, const float *__restrict__ bias,
                                              float *__restrict__ Z, float *__restrict__ C,
                                              int64_t ldc, int gelu, int accumulate) {
  const int i0 = blockIdx.y * GT, j0 = blockIdx.x * GT;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int wi = i0 + (wv >> 1) * 32, wj = j0 + (wv & 1) * 32;
  const int l16 = lane & 15, l4 = lane >> 4;
  f4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = f4{0.f, 0.f, 0.f, 0.f};
  if (MODE == 0) {
    for (int k0 = 0; k0 < K; k0 += 4) {
      const int k = k0 + l4;
      float av[2], bv[2];
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        const int i = wi + a * 16 + l16;
        av[a] = (i < M && k < K) ? A[i * sai + k * sak] : 0.f;
      }
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        const int j = wj + b * 16 + l16;
        bv[b] = (j < N && k < K) ? B[k * sbk + j * sbj] : 0.f;
      }
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
          acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[a], bv[b], acc[a][b], 0, 0, 0);
    }
  } else {
    for (int k0 = 0; k0 < K; k0 += 16) {
      s4 av[2], bv[2];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int k = k0 + 4 * l4 + e;
#pragma unroll
        for (int a = 0; a < 2; ++a) {
          const int i = wi + a * 16 + l16;
          av[a][e] = bf16_rne((i < M && k < K) ? A[i * sai + k * sak] : 0.f);
        }
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          const int j = wj + b * 16 + l16;
          bv[b][e] = bf16_rne((j < N && k < K) ? B[k * sbk + j * sbj] : 0.f);
        }
      }
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
          acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av[a], bv[b], acc[a][b], 0, 0, 0);
    }
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        // 16 x 16 FP32-accumulating MFMA result: lane l, register r holds
        // row 4 (l / 16) + r, column l % 16
        const int i = wi + a * 16 + 4 * l4 + r;
        const int j = wj + b * 16 + l16;
        if (i < M && j < N) {
          float v = acc[a][b][r];
          if (accumulate) v += C[i * ldc + j];
          if (bias) v += bias[j];
          if (Z) Z[i * ldc + j] = v;
          if (gelu) v = 0.5f * v * (1.0f + erff(v * 0.70710678118654752f));
          C[i * ldc + j] = v;
        }
      }
}

// dZ = dC * GELU'(Z)
__global__ void k_gelu_bwd(int64_t n, const float *__restrict__ Z, const float *__restrict__ dC,
                           float *__restrict__ dZ) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const float z = Z[e];
  const float cdf = 0.5f * (1.0f + erff(z * 0.70710678118654752f));
  const float pdf = 0.39894228040143268f * expf(-0.5f * z * z);
  dZ[e] = dC[e] * (cdf + z * pdf);
}

// db(j) = sum_i dZ(i, j), one thread per column, rows in order
__global__ void k_colsum(int M, int N, const float *__restrict__ dZ, float *__restrict__ db) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= N) return;
  float s = 0.f;
  for (int i = 0; i < M; ++i) s += dZ[(int64_t)i * N + j];
  db[j] = s;
}

// dY = (2 / (M N)) (Y - T); per-block partial sums of (Y - T)^2
__global__ void k_mse(int64_t n, const float *__restrict__ Y, const float *__restrict__ T,
                      float scale, float *__restrict__ dY, double *__restrict__ part) {
  __shared__ double sh[4];
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double s = 0.0;
  if (e < n) {
    const float d = Y[e] - T[e];
    dY[e] = scale * d;
    s = (double)d * (double)d;
  }
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

__global__ void k_adam(int64_t n, float *__restrict__ w, const float *__restrict__ g,
                       float *__restrict__ m, float *__restrict__ v, float lr, float b1, float b2,
                       float c1, float c2, float eps) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const float ge = g[e];
  const float me = b1 * m[e] + (1.f - b1) * ge;
  const float ve = b2 * v[e] + (1.f - b2) * ge * ge;
  m[e] = me;
  v[e] = ve;
  w[e] -= lr * (me / c1) / (sqrtf(ve / c2) + eps);
}

inline unsigned g256(int64_t n) { return (unsigned)((n + 255) / 256); }

void gemm(hipStream_t s, int mode, int M, int N, int K, const float *A, int64_t sai, int64_t sak,
          const float *B, int64_t sbk, int64_t sbj, const float *bias, float *Z, float *C,
          int64_t ldc, int gelu, int accumulate) {
  dim3 grid((unsigned)((N + GT - 1) / GT), (unsigned)((M + GT - 1) / GT));
  if (mode == 1)
    k_gemm<1><<<grid, 256, 0, s>>>(M, N, K, A, sai, sak, B, sbk, sbj, bias, Z, C, ldc, gelu,
                                   accumulate);
  else
    k_gemm<0><<<grid, 256, 0, s>>>(M, N, K, A, sai, sak, B, sbk, sbj, bias, Z, C, ldc, gelu,
                                   accumulate);
}

}  // namespace
}  // namespace mds

using namespace mds;

struct mds_mlp {
  hipStream_t stream = nullptr;
  int d[4] = {0, 0, 0, 0};  // in, h, h, out
  int max_batch = 0;
  int64_t step = 0;
  // parameters and Adam state (device, FP32): W0 b0 W1 b1 W2 b2 Ws contiguous
  float *param = nullptr, *grad = nullptr, *m1 = nullptr, *m2 = nullptr;
  int64_t nparam = 0;
  int64_t off_w[3] = {0, 0, 0}, off_b[3] = {0, 0, 0}, off_s = 0;
  // activations: A0 (input copy not needed), Z1, H1, Z2, H2, Y; gradients dH, dZ
  float *z[3] = {nullptr, nullptr, nullptr}, *h[3] = {nullptr, nullptr, nullptr};
  float *dA = nullptr, *dB = nullptr;
  double *part = nullptr;
};

extern "C" {

size_t mds_mlp_workspace_bytes(const int32_t dims[4], int32_t max_batch) {
  if (!dims || max_batch <= 0) return 0;
  for (int i = 0; i < 4; ++i)
    if (dims[i] <= 0 || dims[i] > (1 << 20)) return 0;
  const int64_t np = (int64_t)dims[0] * dims[1] + dims[1] + (int64_t)dims[1] * dims[2] + dims[2] +
                     (int64_t)dims[2] * dims[3] + dims[3] + (int64_t)dims[0] * dims[3];
  const int64_t wmax = std::max(std::max(dims[1], dims[2]), std::max(dims[3], dims[0]));
  const int64_t act = (int64_t)max_batch * (dims[1] + dims[2] + dims[3]);
  const int64_t nblk = ((int64_t)max_batch * dims[3] + 255) / 256;
  return (size_t)(4 * (4 * np + 2 * act + 2 * (int64_t)max_batch * wmax) + 8 * nblk + 4096);
}

int mds_mlp_create(mds_mlp **out, const int32_t dims[4], int32_t max_batch, void *stream,
                   void *workspace, size_t bytes) {
  if (!out || !dims || !workspace) return MDS_ENULL;
  *out = nullptr;
  const size_t need = mds_mlp_workspace_bytes(dims, max_batch);
  if (need == 0) return MDS_EDIMS;
  if (bytes < need || ((uintptr_t)workspace & 255) != 0) return MDS_EWORKSPACE;
  mds_mlp *M = new (std::nothrow) mds_mlp();
  if (!M) return MDS_EINVAL;
  M->stream = (hipStream_t)stream;
  for (int i = 0; i < 4; ++i) M->d[i] = dims[i];
  M->max_batch = max_batch;
  int64_t o = 0;
  for (int l = 0; l < 3; ++l) {
    M->off_w[l] = o;
    o += (int64_t)dims[l] * dims[l + 1];
    M->off_b[l] = o;
    o += dims[l + 1];
  }
  M->off_s = o;
  o += (int64_t)dims[0] * dims[3];
  M->nparam = o;
  float *p = (float *)workspace;
  M->param = p;
  p += o;
  M->grad = p;
  p += o;
  M->m1 = p;
  p += o;
  M->m2 = p;
  p += o;
  for (int l = 0; l < 3; ++l) {
    M->z[l] = p;
    p += (int64_t)max_batch * dims[l + 1];
    M->h[l] = p;
    p += (int64_t)max_batch * dims[l + 1];
  }
  const int64_t wmax = std::max(std::max(dims[1], dims[2]), std::max(dims[3], dims[0]));
  M->dA = p;
  p += (int64_t)max_batch * wmax;
  M->dB = p;
  p += (int64_t)max_batch * wmax;
  M->part = (double *)(((uintptr_t)p + 7) & ~(uintptr_t)7);
  if (hipMemsetAsync(M->m1, 0, 8 * (size_t)o, M->stream) != hipSuccess ||
      hipStreamSynchronize(M->stream) != hipSuccess) {
    delete M;
    return MDS_EHIP;
  }
  *out = M;
  return MDS_OK;
}

void mds_mlp_destroy(mds_mlp *M) { delete M; }

int32_t mds_mlp_param_count(const mds_mlp *M) { return M ? (int32_t)M->nparam : 0; }

// params: W0 (in x h) b0 W1 (h x h) b1 W2 (h x out) b2 Ws (in x out),
// row-major, FP32, host
int mds_mlp_set_params(mds_mlp *M, const float *params_host) {
  if (!M || !params_host) return MDS_ENULL;
  if (hipMemcpyAsync(M->param, params_host, 4 * (size_t)M->nparam, hipMemcpyHostToDevice,
                     M->stream) != hipSuccess ||
      hipMemsetAsync(M->m1, 0, 8 * (size_t)M->nparam, M->stream) != hipSuccess ||
      hipStreamSynchronize(M->stream) != hipSuccess)
    return MDS_EHIP;
  M->step = 0;
  return MDS_OK;
}

int mds_mlp_get_params(const mds_mlp *M, float *params_host) {
  if (!M || !params_host) return MDS_ENULL;
  if (hipMemcpyAsync(params_host, M->param, 4 * (size_t)M->nparam, hipMemcpyDeviceToHost,
                     M->stream) != hipSuccess ||
      hipStreamSynchronize(M->stream) != hipSuccess)
    return MDS_EHIP;
  return MDS_OK;
}

// Y (batch x out, device) = MLP(X (batch x in, device)); precision MDS_FP32
// or MDS_BF16.  Async.
int mds_mlp_forward(mds_mlp *M, const float *X, int32_t batch, int32_t precision, float *Y) {
  if (!M || !X || !Y) return MDS_ENULL;
  if (batch <= 0 || batch > M->max_batch) return MDS_EDIMS;
  if (precision != MDS_FP32 && precision != MDS_BF16) return MDS_EINVAL;
  const int mode = (precision == MDS_BF16) ? 1 : 0;
  const float *in = X;
  for (int l = 0; l < 3; ++l) {
    const int K = M->d[l], N = M->d[l + 1];
    float *outp = (l == 2) ? Y : M->h[l];
    gemm(M->stream, mode, batch, N, K, in, K, 1, M->param + M->off_w[l], N, 1,
         M->param + M->off_b[l], M->z[l], outp, N, l < 2 ? 1 : 0, 0);
    in = outp;
  }
  // skip path: Y += X Ws
  gemm(M->stream, mode, batch, M->d[3], M->d[0], X, M->d[0], 1, M->param + M->off_s, M->d[3], 1,
       nullptr, nullptr, Y, M->d[3], 0, 1);
  return hipGetLastError() == hipSuccess ? MDS_OK : MDS_EHIP;
}

// One Adam step on the mean-squared error of MLP(X) against T (both device,
// batch rows).  Writes the loss (mean over batch x out) to *loss_host when
// non-NULL.  Synchronizes.
int mds_mlp_train_step(mds_mlp *M, const float *X, const float *T, int32_t batch, float lr,
                       double *loss_host) {
  if (!M || !X || !T) return MDS_ENULL;
  if (batch <= 0 || batch > M->max_batch) return MDS_EDIMS;
  hipStream_t s = M->stream;
  const int *d = M->d;
  float *Yout = M->h[2];
  int st = mds_mlp_forward(M, X, batch, MDS_FP32, Yout);
  if (st != MDS_OK) return st;
  const int64_t ny = (int64_t)batch * d[3];
  const unsigned nblk = g256(ny);
  float *dY = M->dA;
  k_mse<<<nblk, 256, 0, s>>>(ny, Yout, T, 2.0f / (float)ny, dY, M->part);
  // skip path: dWs = X' dY  (in x out)
  gemm(s, 0, d[0], d[3], batch, X, 1, d[0], dY, d[3], 1, nullptr, nullptr, M->grad + M->off_s, d[3],
       0, 0);
  // backward through the three layers
  float *dcur = dY;  // gradient w.r.t. the layer output (after activation)
  for (int l = 2; l >= 0; --l) {
    const int K = d[l], N = d[l + 1];
    float *dZ = dcur;
    if (l < 2) {
      float *tmp = (dcur == M->dA) ? M->dB : M->dA;
      k_gelu_bwd<<<g256((int64_t)batch * N), 256, 0, s>>>((int64_t)batch * N, M->z[l], dcur, tmp);
      dZ = tmp;
    }
    const float *Ain = (l == 0) ? X : M->h[l - 1];
    // dW = Ain' dZ  (K x N)
    gemm(s, 0, K, N, batch, Ain, 1, K, dZ, N, 1, nullptr, nullptr, M->grad + M->off_w[l], N, 0, 0);
    k_colsum<<<g256(N), 256, 0, s>>>(batch, N, dZ, M->grad + M->off_b[l]);
    if (l > 0) {
      // dH_{l-1} = dZ W'  (batch x K)
      float *dprev = (dZ == M->dA) ? M->dB : M->dA;
      gemm(s, 0, batch, K, N, dZ, N, 1, M->param + M->off_w[l], 1, N, nullptr, nullptr, dprev, K,
           0, 0);
      dcur = dprev;
    }
  }
  M->step += 1;
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = 1.f - powf(b1, (float)M->step), c2 = 1.f - powf(b2, (float)M->step);
  k_adam<<<g256(M->nparam), 256, 0, s>>>(M->nparam, M->param, M->grad, M->m1, M->m2, lr, b1, b2,
                                         c1, c2, 1e-8f);
  if (hipGetLastError() != hipSuccess) return MDS_EHIP;
  if (loss_host) {
    std::vector<double> part(nblk);
    if (hipMemcpyAsync(part.data(), M->part, 8 * (size_t)nblk, hipMemcpyDeviceToHost, s) !=
            hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return MDS_EHIP;
    double t = 0.0;
    for (unsigned b = 0; b < nblk; ++b) t += part[b];
    *loss_host = t / (double)ny;
  } else if (hipStreamSynchronize(s) != hipSuccess) {
    return MDS_EHIP;
  }
  return MDS_OK;
}

// Gradient of the last train step (FP32, host, same layout as the params).
int mds_mlp_get_grad(const mds_mlp *M, float *grad_host) {
  if (!M || !grad_host) return MDS_ENULL;
  if (hipMemcpyAsync(grad_host, M->grad, 4 * (size_t)M->nparam, hipMemcpyDeviceToHost,
                     M->stream) != hipSuccess ||
      hipStreamSynchronize(M->stream) != hipSuccess)
    return MDS_EHIP;
  return MDS_OK;
}

}  // extern "C"
