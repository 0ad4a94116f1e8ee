// Device-side reduction helpers shared by the vector kernels.
#pragma once

#include <hip/hip_runtime.h>

namespace mds {

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

__device__ inline double wave_max(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off));
  return v;
}

// Eight-slot block reduction for 256-thread workgroups: slots 0-3 are
// maxima, slots 4-7 are sums.  Thread 0 writes the block's record to out[0..7].
__device__ inline void block_reduce8(double (&v)[8], double *out) {
  __shared__ double sh[4][8];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int s = 0; s < 8; ++s) v[s] = (s < 4) ? wave_max(v[s]) : wave_sum(v[s]);
  if (lane == 0)
#pragma unroll
    for (int s = 0; s < 8; ++s) sh[wid][s] = v[s];
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int s = 0; s < 8; ++s) {
      double t = sh[0][s];
      for (int q = 1; q < 4; ++q) t = (s < 4) ? fmax(t, sh[q][s]) : t + sh[q][s];
      out[s] = t;
    }
  }
}

}  // namespace mds
