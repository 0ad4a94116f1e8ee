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
// tagged solution words (stamped with a per-solve epoch kept in device
// memory) appear, then solves its diagonal block and publishes its own.  A
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

// Solved values are published as tagged words: the double of row x goes
// out as two 64-bit words (its low and its high half, each with the phase's
// tag in the upper 32 bits), stored with relaxed single-copy-atomic stores.
// A consumer polls the words themselves: matching tags mean the payload is
// this phase's value, so no flag, fence or second round trip is needed.  The
// tag is 2 epoch + phase (0 forward, 1 backward) and the epoch grows with
// every solve, so words left by an earlier phase or solve never match.
__device__ inline void pub_sol(uint64_t *tw, int x, double v, uint32_t tag) {
  const uint64_t b = (uint64_t)__double_as_longlong(v), hi = (uint64_t)tag << 32;
  __hip_atomic_store(&tw[2 * (size_t)x], hi | (b & 0xffffffffull), __ATOMIC_RELAXED,
                     __HIP_MEMORY_SCOPE_AGENT);
  __hip_atomic_store(&tw[2 * (size_t)x + 1], hi | (b >> 32), __ATOMIC_RELAXED,
                     __HIP_MEMORY_SCOPE_AGENT);
}

__device__ inline bool try_sol(const uint64_t *tw, int x, uint32_t tag, double &v) {
  const uint64_t w0 = __hip_atomic_load(&tw[2 * (size_t)x], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const uint64_t w1 =
      __hip_atomic_load(&tw[2 * (size_t)x + 1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  v = __longlong_as_double((long long)((w1 << 32) | (w0 & 0xffffffffull)));
  return (uint32_t)(w0 >> 32) == tag && (uint32_t)(w1 >> 32) == tag;
}

// Called by every lane of a wave: each lane with need waits for the value of
// row x.  Bounded by the wall clock: on expiry the error word is set and
// false returned (the caller then ends without publishing, so its consumers
// expire too and the grid drains).
__device__ bool wait_sol(const uint64_t *tw, int x, bool need, uint32_t tag, double &v,
                         int32_t *err) {
  bool ok = need ? try_sol(tw, x, tag, v) : true;
  if (__ballot(!ok) == 0) return true;
  const unsigned long long t0 = wall_clock64();
  for (;;) {
    __builtin_amdgcn_s_sleep(1);
    if (!ok) ok = try_sol(tw, x, tag, v);
    if (__ballot(!ok) == 0) return true;
    if (wall_clock64() - t0 > kWaitTicks) {
      __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return false;
    }
  }
}

// Forward L y = z (unit lower triangular, standard form), in place on z.
// Workgroup i owns rows [64 i, 64 i + 64): lane r its row, wave g a quarter
// of each dependency block's 64 columns (lanes 0..15 wait for those 16
// solved values).  Each wave walks the dependency blocks on its own; the
// L of the next block does not depend on the solved values and is loaded
// before the wait, so the last link of the chain (block i - 1) finds it in
// registers.
__global__ __launch_bounds__(TB) void k_trsv_fwd(int N, const double *__restrict__ L, double *z,
                                                 uint64_t *tw, const int32_t *epoch_p,
                                                 int32_t *err) {
  __shared__ double s_part[4][BS];
  __shared__ double s_d[BS][BS + 1];
  __shared__ int s_bad;
  const int i = blockIdx.x, tid = threadIdx.x, r = tid & 63, g = tid >> 6;
  const int r0 = i * BS, row = r0 + r;
  const bool live = row < N;
  const size_t ld = (size_t)N;
  const uint32_t tag = 2u * (uint32_t)*epoch_p;
  if (tid == 0) s_bad = 0;
  for (int e = tid; e < BS * BS; e += TB) {
    const int rr = e & 63, cc = e >> 6;
    s_d[rr][cc] = (rr > cc && r0 + rr < N) ? L[(size_t)(r0 + rr) + (size_t)(r0 + cc) * ld] : 0.0;
  }
  // this row's right-hand side: only this workgroup writes it, at its end
  const double zrow = live ? z[row] : 0.0;
  double acc = 0.0, pf[16];
  bool bad = false;
  if (i > 0) {
#pragma unroll
    for (int t = 0; t < 16; ++t) pf[t] = live ? L[(size_t)row + (size_t)(g * 16 + t) * ld] : 0.0;
  }
  for (int j = 0; j < i; ++j) {
    double yv = 0.0;
    if (!wait_sol(tw, j * BS + g * 16 + r, r < 16, tag, yv, err)) {
      bad = true;
      break;
    }
    double lv[16];
#pragma unroll
    for (int t = 0; t < 16; ++t) lv[t] = pf[t];
    if (j + 1 < i) {
#pragma unroll
      for (int t = 0; t < 16; ++t)
        pf[t] = live ? L[(size_t)row + (size_t)((j + 1) * BS + g * 16 + t) * ld] : 0.0;
    }
#pragma unroll
    for (int t = 0; t < 16; ++t) acc = fma(-lv[t], wave::lane_read(yv, t), acc);
  }
  s_part[g][r] = acc;
  __syncthreads();  // s_bad was cleared before the loop
  if (bad && r == 0) s_bad = 1;
  __syncthreads();
  if (s_bad) return;
  if (g == 0) {
    double v = zrow;
    v += (s_part[0][r] + s_part[1][r]) + (s_part[2][r] + s_part[3][r]);
    for (int c = 0; c < BS - 1; ++c) {
      const double yc = wave::lane_read(v, c);
      if (r > c) v = fma(-s_d[r][c], yc, v);
    }
    if (live) {
      z[row] = v;
      pub_sol(tw, row, v, tag);
    }
  }
}

// Backward L' x = z, in place.  Launch index b handles block i = nblk-1-b.
// Lane r takes row q0 + r of a dependency block (contiguous in a column of
// L) and waits for its solved value, wave g the 16 columns r0 + 16 g + t of
// this block; the 64 lane partial sums of every column are reduced through
// LDS at the end.
__global__ __launch_bounds__(TB) void k_trsv_bwd(int N, int nblk, const double *__restrict__ L,
                                                 double *z, uint64_t *tw,
                                                 const int32_t *epoch_p, int32_t *err) {
  __shared__ double s_red[BS][BS + 1];
  __shared__ double s_d[BS][BS + 1];
  __shared__ int s_bad;
  const int i = nblk - 1 - (int)blockIdx.x, tid = threadIdx.x, r = tid & 63, g = tid >> 6;
  const int r0 = i * BS;
  const size_t ld = (size_t)N;
  const uint32_t tag = 2u * (uint32_t)*epoch_p + 1u;
  if (tid == 0) s_bad = 0;
  for (int e = tid; e < BS * BS; e += TB) {
    const int rr = e & 63, cc = e >> 6;
    s_d[rr][cc] = (rr > cc && r0 + rr < N) ? L[(size_t)(r0 + rr) + (size_t)(r0 + cc) * ld] : 0.0;
  }
  const int cbase = r0 + g * 16;  // this wave's 16 columns of the block
  // this row's right-hand side: only this workgroup writes it, at its end
  const double zrow = (r0 + r < N) ? z[r0 + r] : 0.0;
  double acc[16], pf[16];
#pragma unroll
  for (int t = 0; t < 16; ++t) acc[t] = 0.0;
  bool bad = false;
  if (nblk - 1 > i) {
    const int q = (nblk - 1) * BS + r;
#pragma unroll
    for (int t = 0; t < 16; ++t) {
      const int c = cbase + t;
      pf[t] = (q < N && c < N) ? L[(size_t)q + (size_t)c * ld] : 0.0;
    }
  }
  for (int j = nblk - 1; j > i; --j) {
    const int q = j * BS + r;
    double xq = 0.0;
    if (!wait_sol(tw, q, q < N, tag, xq, err)) {
      bad = true;
      break;
    }
    double lv[16];
#pragma unroll
    for (int t = 0; t < 16; ++t) lv[t] = pf[t];
    if (j - 1 > i) {
      const int qn = (j - 1) * BS + r;
#pragma unroll
      for (int t = 0; t < 16; ++t) {
        const int c = cbase + t;
        pf[t] = (qn < N && c < N) ? L[(size_t)qn + (size_t)c * ld] : 0.0;
      }
    }
#pragma unroll
    for (int t = 0; t < 16; ++t) acc[t] = fma(-lv[t], xq, acc[t]);
  }
#pragma unroll
  for (int t = 0; t < 16; ++t) s_red[g * 16 + t][r] = acc[t];
  __syncthreads();  // s_bad was cleared before the loop
  if (bad && r == 0) s_bad = 1;
  __syncthreads();
  if (s_bad) return;
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
    if (live) {
      z[row] = v;
      pub_sol(tw, row, v, tag);
    }
  }
}

inline unsigned grid1(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

int std_max_n() { return 160 * 1024 / 8; }
int std_solve_blocks(int N) { return (N + BS - 1) / BS; }
// epoch, error word, two pad words, then two tagged words per row
size_t std_trsv_bytes(int N) { return 16 + 16 * (size_t)(N > 0 ? N : 0); }

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
  int32_t *epoch = trsv, *err = trsv + 1;
  uint64_t *tw = reinterpret_cast<uint64_t *>(trsv + 4);
  k_perm_scatter<<<grid1(N, 256), 256, 0, s>>>(N, perm, v, z, epoch);
  k_trsv_fwd<<<(unsigned)nblk, TB, 0, s>>>(N, Lstd, z, tw, epoch, err);
  k_diag_solve<<<grid1(N, 256), 256, 0, s>>>(N, dd, ds, blk, z);
  k_trsv_bwd<<<(unsigned)nblk, TB, 0, s>>>(N, nblk, Lstd, z, tw, epoch, err);
  k_perm_gather<<<grid1(N, 256), 256, 0, s>>>(N, perm, z, out);
}

}  // namespace mds
