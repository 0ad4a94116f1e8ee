// Standard-form factor and the multi-workgroup LDL' solve (Sec. 2.3).
//
// The blocked factorization leaves each panel's multipliers in that panel's
// own row order: later panels' interchanges are not applied to the columns
// of earlier panels.  Before the first solve after a factorization:
//  1. k_std_sweep (one workgroup) walks the panels backwards composing the
//     interchanges.  h_b maps a row position in panel b's frame to its final
//     position; h_{b-1} = h_b o T_b where T_b applies panel b's transpositions
//     in pivot order, so on the array h they are applied as swaps in reverse
//     pivot order.  h_b is stored for the rows past panel b; the last map is
//     the permutation of the factorization: P M P' = L D L' with
//     (P v)[h(x)] = v[x].
//  2. k_std_apply (one workgroup per column) moves the rows of each column
//     that lie past its panel to their final positions through h_b.  The
//     column is staged in LDS, so the result may overwrite the first buffer
//     in place.
// The solve is then P -> L^{-1} -> D^{-1} -> L^{-T} -> P'.  Each triangular
// solve runs one workgroup per 64-row block: block i accumulates the products
// of its rows of L with the solutions of the blocks it depends on, as their
// per-block flags (stamped with a per-solve epoch kept in device memory)
// appear, then solves its diagonal block and publishes its own flag.  A
// block's dependencies all have smaller launch indices, so every awaited
// block has been dispatched before its dependants; waits are bounded by a
// wall-clock limit and set an error word instead of hanging.
#include "internal.hpp"
#include "wave.hpp"

namespace mds {
namespace {

constexpr int SW = 1024;  // sweep workgroup
constexpr int AT = 1024;  // standard-form copy workgroup (one column)
constexpr int BS = 64;    // triangular-solve block (one wave's rows)
constexpr int TB = 256;   // triangular-solve workgroup: 4 waves
constexpr int NR = 4;     // dependency blocks consumed per batch
constexpr unsigned long long kWaitTicks = 1ull << 26;  // ~0.7 s of the 100 MHz clock

__global__ __launch_bounds__(SW) void k_std_sweep(int N, const int32_t *__restrict__ ipiv,
                                                  const int32_t *__restrict__ blk,
                                                  const int32_t *__restrict__ panel_k0,
                                                  const FacState *__restrict__ st,
                                                  int32_t *__restrict__ hmap,
                                                  int32_t *__restrict__ perm,
                                                  int32_t *__restrict__ colpanel) {
  extern __shared__ int s_h[];
  __shared__ int s_p[kMaxNb + 2], s_q[kMaxNb + 2];
  static_assert(kMaxNb + 1 <= 128, "a panel's pivot entries fit two per lane of one wave");
  const int tid = threadIdx.x;
  const int np = st->npanel;
  for (int x = tid; x < N; x += SW) s_h[x] = x;
  // panel b's bounds and pivot entries are loaded one panel ahead, so that
  // their memory latency overlaps the previous panel's work
  int k1 = 0, k0 = 0, bk = 0, iv = 0;
  if (np > 0) {
    k1 = panel_k0[np];
    k0 = panel_k0[np - 1];
    if (tid < k1 - k0) {
      bk = blk[k0 + tid];
      iv = ipiv[k0 + tid];
    }
  }
  __syncthreads();
  for (int b = np - 1; b >= 0; --b) {
    int k0n = 0, bkn = 0, ivn = 0;
    if (b > 0) {
      k0n = panel_k0[b - 1];
      if (tid < k0 - k0n) {
        bkn = blk[k0n + tid];
        ivn = ipiv[k0n + tid];
      }
    }
    int32_t *hb = hmap + (size_t)b * N;
    for (int x = k1 + tid; x < N; x += SW) hb[x] = s_h[x];
    for (int c = k0 + tid; c < k1; c += SW) colpanel[c] = b;
    // the panel's transpositions in pivot order, read in parallel: entry k
    // gives (k, q) for a 1x1 pivot, (k + 1, q) for the first row of a 2x2
    // one and nothing for its second row
    if (tid < k1 - k0) {
      const int k = k0 + tid;
      s_p[tid] = (bk == 1) ? k : (bk == 2) ? k + 1 : -1;
      s_q[tid] = (bk == 1) ? iv - 1 : -iv - 1;
    }
    __syncthreads();
    // wave 0 holds entries e and e + 64 in lane e and applies only those that
    // move a row, in reverse pivot order, taking their positions from the
    // lanes that hold them (one LDS read per lane instead of two per entry)
    if (tid < 64) {
      const int w = k1 - k0;
      int p0 = -1, q0 = 0, p1 = -1, q1 = 0;
      if (tid < w) {
        p0 = s_p[tid];
        q0 = s_q[tid];
      }
      if (tid + 64 < w) {
        p1 = s_p[tid + 64];
        q1 = s_q[tid + 64];
      }
      unsigned long long m = __ballot(p1 >= 0 && p1 != q1);
      while (m) {
        const int e = 63 - __clzll((long long)m);
        m &= ~(1ull << e);
        const int pe = wave::lane_read(p1, e), qe = wave::lane_read(q1, e);
        if (tid == 0) {
          const int x = s_h[pe];
          s_h[pe] = s_h[qe];
          s_h[qe] = x;
        }
      }
      m = __ballot(p0 >= 0 && p0 != q0);
      while (m) {
        const int e = 63 - __clzll((long long)m);
        m &= ~(1ull << e);
        const int pe = wave::lane_read(p0, e), qe = wave::lane_read(q0, e);
        if (tid == 0) {
          const int x = s_h[pe];
          s_h[pe] = s_h[qe];
          s_h[qe] = x;
        }
      }
    }
    __syncthreads();
    k1 = k0;
    k0 = k0n;
    bk = bkn;
    iv = ivn;
  }
  for (int x = tid; x < N; x += SW) perm[x] = s_h[x];
}

// Column c: rows c+1 .. k1-1 (inside its panel) stay, rows x >= k1 go to
// hb[x].  Reads column c from the buffer its panel wrote and writes column c
// of Lstd; no other workgroup touches column c of either buffer.
__global__ __launch_bounds__(AT) void k_std_apply(int N, const double *M0, const double *M1,
                                                   int pingpong,
                                                   const int32_t *__restrict__ panel_k0,
                                                   const int32_t *__restrict__ colpanel,
                                                   const int32_t *__restrict__ hmap,
                                                   double *Lstd) {
  extern __shared__ double s_col[];
  const int c = blockIdx.x, tid = threadIdx.x;
  const int b = colpanel[c];
  const int k1 = panel_k0[b + 1];
  const double *src = (pingpong && (b & 1) == 0) ? M1 : M0;
  const size_t co = (size_t)c * (size_t)N;
  const int32_t *hb = hmap + (size_t)b * N;
  // a column takes up to N * 8 B of LDS, so one workgroup may hold a whole
  // compute unit: 1024 threads with four loads each in flight keep enough
  // reads outstanding for the copy to run at memory speed
  for (int x = k1 + tid; x < N; x += 4 * AT) {
    double v[4];
    int h[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int y = x + u * AT;
      if (y < N) {
        v[u] = src[co + y];
        h[u] = hb[y];
      }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int y = x + u * AT;
      if (y < N) s_col[h[u] - k1] = v[u];
    }
  }
  // rows inside the panel: fewer than kMaxNb of them
  const int x0 = c + 1 + tid;
  const double vin = (tid < kMaxNb && x0 < k1) ? src[co + x0] : 0.0;
  __syncthreads();
  if (tid < kMaxNb && x0 < k1) Lstd[co + x0] = vin;
  for (int y = k1 + tid; y < N; y += AT) Lstd[co + y] = s_col[y - k1];
}

// z[h(x)] = v[x]; also advances the solve epoch
__global__ void k_perm_scatter(int N, const int32_t *__restrict__ perm,
                               const double *__restrict__ v, double *__restrict__ z,
                               int32_t *epoch) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x == 0) epoch[0] = epoch[0] + 1;
  if (x < N) z[perm[x]] = v[x];
}

// v[x] = z[h(x)]
__global__ void k_perm_gather(int N, const int32_t *__restrict__ perm,
                              const double *__restrict__ z, double *__restrict__ v) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x < N) v[x] = z[perm[x]];
}

// D^{-1}: 1x1 pivots divide, 2x2 pivots [a s; s c] by Cramer's rule
__global__ void k_diag_solve(int N, const double *__restrict__ dd, const double *__restrict__ ds,
                             const int32_t *__restrict__ blk, double *__restrict__ z) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= N) return;
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

__device__ inline int ld_flag(const int32_t *f) {
  return __hip_atomic_load(f, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ inline double ld_sol(const double *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Thread 0: wait for flag[j] (dependencies are consumed in direction dir),
// then count how many of the following blocks are also ready (NR at most,
// stopping before jend).  Returns 0 on timeout.
__device__ int wait_ready(const int32_t *flags, int j, int jend, int dir, int epoch,
                          int32_t *err) {
  const unsigned long long t0 = wall_clock64();
  while (ld_flag(&flags[j]) != epoch) {
    if (wall_clock64() - t0 > kWaitTicks) {
      __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return 0;
    }
    __builtin_amdgcn_s_sleep(2);
  }
  int nr = 1;
  while (nr < NR && j + dir * nr != jend && ld_flag(&flags[j + dir * nr]) == epoch) ++nr;
  return nr;
}

// Forward L y = z (unit lower triangular, standard form), in place on z.
// Workgroup i owns rows [64 i, 64 i + 64): lane r its row, wave g a quarter
// of each dependency block's 64 columns.
__global__ __launch_bounds__(TB) void k_trsv_fwd(int N, const double *__restrict__ L, double *z,
                                                 int32_t *flags, const int32_t *epoch_p,
                                                 int32_t *err) {
  __shared__ double s_part[4][BS];
  __shared__ double s_d[BS][BS + 1];
  __shared__ int s_nr;
  const int i = blockIdx.x, tid = threadIdx.x, r = tid & 63, g = tid >> 6;
  const int r0 = i * BS, row = r0 + r;
  const bool live = row < N;
  const size_t ld = (size_t)N;
  const int epoch = *epoch_p;
  for (int e = tid; e < BS * BS; e += TB) {
    const int rr = e & 63, cc = e >> 6;
    s_d[rr][cc] = (rr > cc && r0 + rr < N) ? L[(size_t)(r0 + rr) + (size_t)(r0 + cc) * ld] : 0.0;
  }
  // this row's right-hand side: only this workgroup writes it, at its end
  const double zrow = live ? z[row] : 0.0;
  double acc = 0.0;
  // L of the next dependency block does not depend on the flags: it is
  // loaded before the wait, so that the last link of the chain (block i - 1)
  // finds it in registers
  double pf[16];
  if (i > 0) {
#pragma unroll
    for (int t = 0; t < 16; ++t) pf[t] = live ? L[(size_t)row + (size_t)(g * 16 + t) * ld] : 0.0;
  }
  for (int j = 0; j < i;) {
    if (tid == 0) s_nr = wait_ready(flags, j, i, 1, epoch, err);
    __syncthreads();
    const int nr = s_nr;
    __syncthreads();
    if (nr == 0) return;
    double lv[NR][16], yv[NR];
#pragma unroll
    for (int u = 0; u < NR; ++u) {
      if (u < nr) {
        const int c0 = (j + u) * BS + g * 16;
        yv[u] = (r < 16) ? ld_sol(&z[c0 + r]) : 0.0;
#pragma unroll
        for (int t = 0; t < 16; ++t)
          lv[u][t] = (u == 0) ? pf[t] : (live ? L[(size_t)row + (size_t)(c0 + t) * ld] : 0.0);
      }
    }
    j += nr;
    if (j < i) {
#pragma unroll
      for (int t = 0; t < 16; ++t)
        pf[t] = live ? L[(size_t)row + (size_t)(j * BS + g * 16 + t) * ld] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < NR; ++u) {
      if (u < nr) {
#pragma unroll
        for (int t = 0; t < 16; ++t) acc = fma(-lv[u][t], wave::lane_read(yv[u], t), acc);
      }
    }
  }
  s_part[g][r] = acc;
  __syncthreads();
  if (g == 0) {
    double v = zrow;
    v += (s_part[0][r] + s_part[1][r]) + (s_part[2][r] + s_part[3][r]);
    for (int c = 0; c < BS - 1; ++c) {
      const double yc = wave::lane_read(v, c);
      if (r > c) v = fma(-s_d[r][c], yc, v);
    }
    if (live) __hip_atomic_store(&z[row], v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __threadfence();
    if (r == 0) __hip_atomic_store(&flags[i], epoch, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// Backward L' x = z, in place.  Launch index b handles block i = nblk-1-b.
// Lane r takes row q0 + r of a dependency block (contiguous in a column of
// L), wave g the 16 columns r0 + 16 g + t of this block; the 64 lane partial
// sums of every column are reduced through LDS at the end.
__global__ __launch_bounds__(TB) void k_trsv_bwd(int N, int nblk, const double *__restrict__ L,
                                                 double *z, int32_t *flags,
                                                 const int32_t *epoch_p, int32_t *err) {
  __shared__ double s_red[BS][BS + 1];
  __shared__ double s_d[BS][BS + 1];
  __shared__ int s_nr;
  const int i = nblk - 1 - (int)blockIdx.x, tid = threadIdx.x, r = tid & 63, g = tid >> 6;
  const int r0 = i * BS;
  const size_t ld = (size_t)N;
  const int epoch = *epoch_p;
  for (int e = tid; e < BS * BS; e += TB) {
    const int rr = e & 63, cc = e >> 6;
    s_d[rr][cc] = (rr > cc && r0 + rr < N) ? L[(size_t)(r0 + rr) + (size_t)(r0 + cc) * ld] : 0.0;
  }
  const int cbase = r0 + g * 16;  // this wave's 16 columns of the block
  // this row's right-hand side: only this workgroup writes it, at its end
  const double zrow = (r0 + r < N) ? z[r0 + r] : 0.0;
  double acc[16];
#pragma unroll
  for (int t = 0; t < 16; ++t) acc[t] = 0.0;
  // L of the next dependency block (row q of it, this wave's 16 columns) is
  // loaded before the wait, as in the forward solve
  double pf[16];
  if (nblk - 1 > i) {
    const int q = (nblk - 1) * BS + r;
#pragma unroll
    for (int t = 0; t < 16; ++t) {
      const int c = cbase + t;
      pf[t] = (q < N && c < N) ? L[(size_t)q + (size_t)c * ld] : 0.0;
    }
  }
  for (int j = nblk - 1; j > i;) {
    if (tid == 0) s_nr = wait_ready(flags, j, i, -1, epoch, err);
    __syncthreads();
    const int nr = s_nr;
    __syncthreads();
    if (nr == 0) return;
    double xv[NR], lv[NR][16];
#pragma unroll
    for (int u = 0; u < NR; ++u) {
      if (u < nr) {
        const int q = (j - u) * BS + r;
        const bool ok = q < N;
        xv[u] = ok ? ld_sol(&z[q]) : 0.0;
#pragma unroll
        for (int t = 0; t < 16; ++t) {
          const int c = cbase + t;
          lv[u][t] = (u == 0) ? pf[t] : ((ok && c < N) ? L[(size_t)q + (size_t)c * ld] : 0.0);
        }
      }
    }
    j -= nr;
    if (j > i) {
      const int q = j * BS + r;
#pragma unroll
      for (int t = 0; t < 16; ++t) {
        const int c = cbase + t;
        pf[t] = (q < N && c < N) ? L[(size_t)q + (size_t)c * ld] : 0.0;
      }
    }
#pragma unroll
    for (int u = 0; u < NR; ++u) {
      if (u < nr) {
#pragma unroll
        for (int t = 0; t < 16; ++t) acc[t] = fma(-lv[u][t], xv[u], acc[t]);
      }
    }
  }
#pragma unroll
  for (int t = 0; t < 16; ++t) s_red[g * 16 + t][r] = acc[t];
  __syncthreads();
  if (g == 0) {
    const int row = r0 + r;
    const bool live = row < N;
    double s = 0.0;
    for (int k = 0; k < BS; ++k) s += s_red[r][k];
    double v = (live ? zrow : 0.0) + s;
    // unit upper L11': last row first
    for (int c = BS - 1; c > 0; --c) {
      const double xc = wave::lane_read(v, c);
      if (r < c) v = fma(-s_d[c][r], xc, v);
    }
    if (live) __hip_atomic_store(&z[row], v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __threadfence();
    if (r == 0) __hip_atomic_store(&flags[i], epoch, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
  }
}

inline unsigned grid1(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

int std_max_n() { return 160 * 1024 / 8; }
int std_solve_blocks(int N) { return (N + BS - 1) / BS; }

hipError_t std_prepare() {
  hipError_t e = hipFuncSetAttribute((const void *)k_std_apply,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute((const void *)k_std_sweep, hipFuncAttributeMaxDynamicSharedMemorySize,
                             128 * 1024);
}

void launch_std_form(hipStream_t s, int N, const double *M0, const double *M1, int pingpong,
                     const int32_t *ipiv, const int32_t *blk, const int32_t *panel_k0,
                     const FacState *st, int32_t *hmap, int32_t *perm, int32_t *colpanel,
                     double *Lstd) {
  if (N <= 0) return;
  k_std_sweep<<<1, SW, sizeof(int32_t) * (size_t)N, s>>>(N, ipiv, blk, panel_k0, st, hmap, perm,
                                                         colpanel);
  k_std_apply<<<(unsigned)N, AT, sizeof(double) * (size_t)N, s>>>(N, M0, M1, pingpong, panel_k0,
                                                                    colpanel, hmap, Lstd);
}

void launch_std_solve(hipStream_t s, int N, const double *Lstd, const double *dd,
                      const double *ds, const int32_t *blk, const int32_t *perm, const double *v,
                      double *z, double *out, int32_t *trsv) {
  if (N <= 0) return;
  const int nblk = std_solve_blocks(N);
  int32_t *epoch = trsv, *err = trsv + 1, *ff = trsv + 4, *fb = trsv + 4 + nblk;
  k_perm_scatter<<<grid1(N, 256), 256, 0, s>>>(N, perm, v, z, epoch);
  k_trsv_fwd<<<(unsigned)nblk, TB, 0, s>>>(N, Lstd, z, ff, epoch, err);
  k_diag_solve<<<grid1(N, 256), 256, 0, s>>>(N, dd, ds, blk, z);
  k_trsv_bwd<<<(unsigned)nblk, TB, 0, s>>>(N, nblk, Lstd, z, fb, epoch, err);
  k_perm_gather<<<grid1(N, 256), 256, 0, s>>>(N, perm, z, out);
}

}  // namespace mds
