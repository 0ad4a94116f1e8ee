// Solve with the blocked Bunch-Kaufman factor (Sec. 2.3).
//
// The factor is  M = P_1 L_1 P_2 L_2 ... D ... L_2' P_2' L_1' P_1'  at panel
// granularity: panel b interchanged rows only inside its own columns, so
// each panel's interchanges are applied to the right-hand side just before
// that panel's columns are eliminated (forward), and undone right after its
// columns are back-substituted (backward):
//   forward,  panel b: z <- P_b' z; z[k0:k1] <- L11^{-1} z[k0:k1];
//                      z[k1:] -= L21 z[k0:k1]
//   diagonal:          z <- D^{-1} z  (1x1 and 2x2 blocks, Cramer's rule)
//   backward, panel b: z[k0:k1] -= L21' z[k1:]; z[k0:k1] <- L11^{-T} z[k0:k1];
//                      z <- P_b z
// One workgroup walks the panels in order; the vector lives in LDS when it
// fits (N <= 6144) and in global memory otherwise.
#include "internal.hpp"

namespace mds {
namespace {

constexpr int NT = 1024;
constexpr int NW = NT / 64;
constexpr int kLdsMaxN = 6144;

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

constexpr int kStage = 34;  // diagonal blocks up to this width are staged in LDS

template <bool kLds>
__global__ __launch_bounds__(NT) void k_ldl_solve(int N, const double *__restrict__ M0,
                                                  const double *__restrict__ M1, int pingpong,
                                                  const double *__restrict__ dd,
                                                  const double *__restrict__ ds,
                                                  const int32_t *__restrict__ ipiv,
                                                  const int32_t *__restrict__ blk,
                                                  const int32_t *__restrict__ panel_k0,
                                                  const FacState *__restrict__ st,
                                                  double *__restrict__ zg) {
  extern __shared__ double s_dyn[];
  __shared__ double s_zc[kMaxNb + 2];
  __shared__ double s_part[kMaxNb + 2][NW];
  __shared__ double s_L[kStage][kStage + 1];  // diagonal block of the panel, [row][col]
  __shared__ int s_piv[kMaxNb + 2], s_blk[kMaxNb + 2];
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const size_t ld = (size_t)N;
  double *z = kLds ? s_dyn : zg;
  if (kLds) {
    for (int i = tid; i < N; i += NT) z[i] = zg[i];
    __syncthreads();
  }
  const int np = st->npanel;

  // ---- forward --------------------------------------------------------------
  for (int b = 0; b < np; ++b) {
    const int k0 = panel_k0[b], k1 = panel_k0[b + 1], w = k1 - k0;
    const double *__restrict__ M = (pingpong && (b & 1) == 0) ? M1 : M0;
    const bool staged = (w <= kStage);
    if (tid < w) {
      s_piv[tid] = ipiv[k0 + tid];
      s_blk[tid] = blk[k0 + tid];
    }
    if (staged)
      for (int e = tid; e < w * w; e += NT) {
        const int r = e % w, c = e / w;
        s_L[r][c] = (r > c) ? M[(size_t)(k0 + r) + (size_t)(k0 + c) * ld] : 0.0;
      }
    __syncthreads();
    if (wid == 0) {
      if (lane == 0) {
        for (int t = 0; t < w;) {
          const int k = k0 + t;
          if (s_blk[t] == 1) {
            const int kp = s_piv[t] - 1;
            if (kp != k) {
              const double x = z[k], y = z[kp];
              z[k] = y;
              z[kp] = x;
            }
            t += 1;
          } else {
            const int kp = -s_piv[t] - 1;
            if (kp != k + 1) {
              const double x = z[k + 1], y = z[kp];
              z[k + 1] = y;
              z[kp] = x;
            }
            t += 2;
          }
        }
      }
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      if (staged) {
        // unit-lower triangle of the panel: lane t owns z[k0 + t]
        double zt = (lane < w) ? z[k0 + lane] : 0.0;
        for (int c = 0; c < w; ++c) {
          const double zc = __shfl(zt, c);
          if (lane > c && lane < w) zt = fma(-s_L[lane][c], zc, zt);
        }
        if (lane < w) {
          z[k0 + lane] = zt;
          s_zc[lane] = zt;
        }
      } else if (lane == 0) {
        for (int c = 0; c < w; ++c) {
          const double zc = z[k0 + c];
          for (int i = c + 1; i < w; ++i)
            z[k0 + i] = fma(-M[(size_t)(k0 + i) + (size_t)(k0 + c) * ld], zc, z[k0 + i]);
        }
        for (int c = 0; c < w; ++c) s_zc[c] = z[k0 + c];
      }
    }
    __syncthreads();
    for (int i = k1 + tid; i < N; i += NT) {
      double a = z[i];
      for (int t = 0; t < w; ++t) a = fma(-M[(size_t)i + (size_t)(k0 + t) * ld], s_zc[t], a);
      z[i] = a;
    }
    __syncthreads();
  }

  // ---- block diagonal -------------------------------------------------------
  for (int k = tid; k < N; k += NT) {
    const int bk = blk[k];
    if (bk == 1) {
      z[k] = z[k] / dd[k];
    } else if (bk == 2) {
      const double a = dd[k], c = dd[k + 1], s = ds[k];
      const double det = a * c - s * s;
      const double y0 = z[k], y1 = z[k + 1];
      z[k] = (c * y0 - s * y1) / det;
      z[k + 1] = (a * y1 - s * y0) / det;
    }
  }
  __syncthreads();

  // ---- backward -------------------------------------------------------------
  for (int b = np - 1; b >= 0; --b) {
    const int k0 = panel_k0[b], k1 = panel_k0[b + 1], w = k1 - k0;
    const double *__restrict__ M = (pingpong && (b & 1) == 0) ? M1 : M0;
    const bool staged = (w <= kStage);
    for (int t = 0; t < w; ++t) {
      double a = 0.0;
      for (int i = k1 + tid; i < N; i += NT) a = fma(M[(size_t)i + (size_t)(k0 + t) * ld], z[i], a);
      a = wave_sum(a);
      if (lane == 0) s_part[t][wid] = a;
    }
    if (tid < w) {
      s_piv[tid] = ipiv[k0 + tid];
      s_blk[tid] = blk[k0 + tid];
    }
    if (staged)
      for (int e = tid; e < w * w; e += NT) {
        const int r = e % w, c = e / w;
        s_L[r][c] = (r > c) ? M[(size_t)(k0 + r) + (size_t)(k0 + c) * ld] : 0.0;
      }
    __syncthreads();
    if (wid == 0) {
      if (staged) {
        // z[k0:k1] -= dots, then the unit-upper triangle L11' backwards:
        // lane t owns z[k0 + t]
        double zt = 0.0;
        if (lane < w) {
          double sdot = 0.0;
          for (int q = 0; q < NW; ++q) sdot += s_part[lane][q];
          zt = z[k0 + lane] - sdot;
        }
        for (int c = w - 1; c >= 0; --c) {
          // finalize x_c, then remove its contribution from the rows above
          const double xc = __shfl(zt, c);
          if (lane < c) zt = fma(-s_L[c][lane], xc, zt);
        }
        if (lane < w) z[k0 + lane] = zt;
      } else if (lane == 0) {
        for (int t = 0; t < w; ++t) {
          double sdot = 0.0;
          for (int q = 0; q < NW; ++q) sdot += s_part[t][q];
          z[k0 + t] -= sdot;
        }
        for (int c = w - 1; c >= 0; --c) {
          double a = z[k0 + c];
          for (int i = c + 1; i < w; ++i)
            a = fma(-M[(size_t)(k0 + i) + (size_t)(k0 + c) * ld], z[k0 + i], a);
          z[k0 + c] = a;
        }
      }
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      if (lane == 0) {
        // undo this panel's interchanges in reverse order
        int starts[kMaxNb + 2];
        int ns = 0;
        for (int t = 0; t < w;) {
          starts[ns++] = t;
          t += (s_blk[t] == 1) ? 1 : 2;
        }
        for (int e = ns - 1; e >= 0; --e) {
          const int t = starts[e], k = k0 + t;
          if (s_blk[t] == 1) {
            const int kp = s_piv[t] - 1;
            if (kp != k) {
              const double x = z[k], y = z[kp];
              z[k] = y;
              z[kp] = x;
            }
          } else {
            const int kp = -s_piv[t] - 1;
            if (kp != k + 1) {
              const double x = z[k + 1], y = z[kp];
              z[k + 1] = y;
              z[kp] = x;
            }
          }
        }
      }
    }
    __syncthreads();
  }
  if (kLds) {
    for (int i = tid; i < N; i += NT) zg[i] = z[i];
  }
}

}  // namespace

void launch_ldl_solve(hipStream_t s, int N, const double *M0, const double *M1, int pingpong,
                      const double *dd, const double *ds, const int32_t *ipiv,
                      const int32_t *blk, const int32_t *panel_k0, const FacState *st,
                      double *z) {
  if (N <= 0) return;
  if (N <= kLdsMaxN) {
    k_ldl_solve<true><<<1, NT, sizeof(double) * (size_t)N, s>>>(N, M0, M1, pingpong, dd, ds,
                                                                  ipiv, blk, panel_k0, st, z);
  } else {
    k_ldl_solve<false><<<1, NT, 0, s>>>(N, M0, M1, pingpong, dd, ds, ipiv, blk, panel_k0, st,
                                        z);
  }
}

}  // namespace mds
