// Mixed-precision factorization helpers.  The low-precision factorization
// works on the equilibrated S M S (S = diag(1/sqrt(row max |M|))), which has
// the inertia of M and entries of comparable size, so FP32/BF16 rounding is
// relative to each row's scale; the solve undoes S on both sides.
//
// Mixed-precision trailing update of the blocked Bunch-Kaufman factorization:
// the trailing matrix is stored in FP32 and the rank-w product L21 W21' runs
// on FP32 MFMA (v_mfma_f32_16x16x4f32) or on BF16 MFMA with FP32 accumulation
// (v_mfma_f32_16x16x16bf16_1k).  The panel (pivot search, D blocks, L and W)
// stays FP64: L and W are rounded to the product's input type here.  As in
// the FP64 update, the un-updated entry is read through the panel's index
// map from the lower triangle of one buffer and the lower tile of the result
// is written to the other.
#include <algorithm>

#include "internal.hpp"
#include "tile_order.hpp"

namespace mds {
namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef short s4 __attribute__((ext_vector_type(4)));

constexpr int TT = 64;
constexpr int TSL = 48;        // panel columns staged in LDS per chunk (multiple of 16)
constexpr int TSL1 = TSL + 1;  // odd row stride of the staged panels
constexpr int TSTL = TT * TSL / 256;  // staged entries per thread and panel
constexpr int kTrailingLpGrid = kTileGrid;  // persistent form: 512 workgroups (2 per CU at <= 196 VGPRs)
static_assert(TT * TSL % 256 == 0, "staging");
static_assert(TT == kNearCols, "the near strip is one tile column");

// round-to-nearest-even FP32 -> BF16 (finite inputs)
__device__ inline short to_bf16(float x) {
  const uint32_t u = __float_as_uint(x);
  return (short)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}

__device__ inline float bf16_to_f32(short h) { return __uint_as_float(((uint32_t)(uint16_t)h) << 16); }

// MODE 1: FP32 products; MODE 2: BF16 products; MODE 3: split BF16 products,
// each FP32 operand v = hi + lo with hi = bf16(v), lo = bf16(v - hi), and
// a b ~ hi_a hi_b + hi_a lo_b + lo_a hi_b (three BF16 MFMAs, FP32
// accumulation; the dropped lo lo term is 2^-16 relative).  256 threads per 64 x 64
// lower tile; wave w computes the 32 x 32 quarter (c rows wc.., i columns wi..)
// of D[c][i] = sum_t W[c, t] L[i, t] as 2 x 2 MFMA blocks of 16 x 16.
template <int MODE>
__global__ __launch_bounds__(256) void k_trailing_lp(int N, int nb, const double *__restrict__ W,
                                                     const float *X, float *Y,
                                                     const double *__restrict__ Lsrc,
                                                     const int32_t *__restrict__ src,
                                                     const FacState *__restrict__ st,
                                                     const int32_t *__restrict__ panel_k0,
                                                     int slot) {
  // the staged panels (FP32: W rows c0.., L rows i0..)
  __shared__ float s_buf[2 * TT * TSL1];
  float *s_w = s_buf, *s_l = s_buf + TT * TSL1;
  if (slot >= st->npanel) return;
  const int k0 = panel_k0[slot], kend = panel_k0[slot + 1];
  if (kend >= N || kend <= k0 || kend - k0 > nb + 1) return;
  const int jw = kend - k0;
  const int nt = (N - kend + TT - 1) / TT;
  const int x = blockIdx.x;
  int ti = (int)((sqrt(8.0 * (double)x + 1.0) - 1.0) * 0.5);
  while ((ti + 1) * (ti + 2) / 2 <= x) ++ti;
  while (ti * (ti + 1) / 2 > x) --ti;
  const int tj = x - ti * (ti + 1) / 2;
  if (ti >= nt) return;
  const int i0 = kend + ti * TT, c0 = kend + tj * TT;
  const size_t ld = (size_t)N;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int wc = c0 + (wv & 1) * 32, wi = i0 + (wv >> 1) * 32;
  const int l16 = lane & 15, l4 = lane >> 4;

  const bool diag = (ti == tj);
  // the entries this lane updates, loaded before the product loop so that
  // their memory latency overlaps it (FP32-accumulating MFMA result: lane l,
  // register r holds row 4 (l / 16) + r, column l % 16)
  int si[2], sc[2][4];
#pragma unroll
  for (int b = 0; b < 2; ++b) {
    const int i = wi + b * 16 + l16;
    si[b] = (i < N) ? (src ? src[i] : i) : 0;
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int c = wc + a * 16 + 4 * l4 + r;
      sc[a][r] = (c < N) ? (src ? src[c] : c) : 0;
    }
  float xv[2][2][4];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int c = wc + a * 16 + 4 * l4 + r;
        const int i = wi + b * 16 + l16;
        const int pi = si[b], pc = sc[a][r];  // physical row and column
        xv[a][b][r] = (c < N && i < N && (!diag || i >= c))
                          ? X[(pi >= pc) ? (size_t)pi + (size_t)pc * ld : (size_t)pc + (size_t)pi * ld]
                          : 0.f;
      }

  f4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = f4{0.f, 0.f, 0.f, 0.f};

  // panel columns in chunks of TSL, rounded to FP32 once while staging; every
  // load of a chunk is issued before the LDS stores (one memory latency per
  // chunk instead of one per product step)
  for (int tb = 0; tb < jw; tb += TSL) {
    const int tw = min(TSL, jw - tb);
    if (tb > 0) __syncthreads();  // the previous chunk has been read
    double vw[TSTL], vl[TSTL];
#pragma unroll
    for (int u = 0; u < TSTL; ++u) {
      const int e = tid + 256 * u, r = e & (TT - 1), t = e >> 6;
      const int c = c0 + r, i = i0 + r;
      vw[u] = (t < tw && c < N) ? W[(size_t)c + (size_t)(tb + t) * ld] : 0.0;
      vl[u] = (t < tw && i < N) ? Lsrc[(size_t)i + (size_t)(k0 + tb + t) * ld] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < TSTL; ++u) {
      const int e = tid + 256 * u, r = e & (TT - 1), t = e >> 6;
      s_w[r * TSL1 + t] = (float)vw[u];
      s_l[r * TSL1 + t] = (float)vl[u];
    }
    __syncthreads();
    const float *wr[2], *lr[2];  // this lane's rows of the staged panels
#pragma unroll
    for (int a = 0; a < 2; ++a) wr[a] = s_w + (wc - c0 + a * 16 + l16) * TSL1;
#pragma unroll
    for (int b = 0; b < 2; ++b) lr[b] = s_l + (wi - i0 + b * 16 + l16) * TSL1;
    if (MODE == 1) {
      for (int t0 = 0; t0 < tw; t0 += 4) {
        const int t = t0 + l4;  // < TSL; entries past tw are zero
        float av[2], bv[2];
#pragma unroll
        for (int a = 0; a < 2; ++a) av[a] = wr[a][t];
#pragma unroll
        for (int b = 0; b < 2; ++b) bv[b] = lr[b][t];
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
          for (int b = 0; b < 2; ++b)
            acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[a], bv[b], acc[a][b], 0, 0, 0);
      }
    } else if (MODE == 3) {
      for (int t0 = 0; t0 < tw; t0 += 16) {
        s4 ah[2], al[2], bh[2], bl[2];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int t = t0 + 4 * l4 + e;  // < TSL
#pragma unroll
          for (int a = 0; a < 2; ++a) {
            const float v = wr[a][t];
            const short h = to_bf16(v);
            ah[a][e] = h;
            al[a][e] = to_bf16(v - bf16_to_f32(h));
          }
#pragma unroll
          for (int b = 0; b < 2; ++b) {
            const float v = lr[b][t];
            const short h = to_bf16(v);
            bh[b][e] = h;
            bl[b][e] = to_bf16(v - bf16_to_f32(h));
          }
        }
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
          for (int b = 0; b < 2; ++b) {
            acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(al[a], bh[b], acc[a][b], 0, 0, 0);
            acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah[a], bl[b], acc[a][b], 0, 0, 0);
            acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah[a], bh[b], acc[a][b], 0, 0, 0);
          }
      }
    } else {
      for (int t0 = 0; t0 < tw; t0 += 16) {
        s4 av[2], bv[2];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int t = t0 + 4 * l4 + e;  // < TSL
#pragma unroll
          for (int a = 0; a < 2; ++a) av[a][e] = to_bf16(wr[a][t]);
#pragma unroll
          for (int b = 0; b < 2; ++b) bv[b][e] = to_bf16(lr[b][t]);
        }
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
          for (int b = 0; b < 2; ++b)
            acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av[a], bv[b], acc[a][b], 0, 0, 0);
      }
    }
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int c = wc + a * 16 + 4 * l4 + r;
        const int i = wi + b * 16 + l16;
        if (c < N && i < N && (!diag || i >= c)) Y[(size_t)i + (size_t)c * ld] = xv[a][b][r] - acc[a][b][r];
      }
}

// Persistent form of k_trailing_lp for panels of at most TSL - 1 columns
// (one staging chunk): a grid of a few workgroups per compute unit walks the
// tiles, loading the next tile's entries and panel rows while it computes
// the current one.  Per entry the arithmetic is the one of k_trailing_lp.
__device__ inline void lp_load(int i0, int c0, bool diag, int N, int kend, int k0, int jw,
                               const double *__restrict__ W, const float *X,
                               const double *__restrict__ Lsrc, const int32_t *__restrict__ src,
                               float (&xv)[2][2][4], double (&vw)[TSTL], double (&vl)[TSTL]) {
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int l16 = lane & 15, l4 = lane >> 4;
  const size_t ld = (size_t)N;
  const int wc = c0 + (wv & 1) * 32, wi = i0 + (wv >> 1) * 32;
  int si[2], sc[2][4];
#pragma unroll
  for (int b = 0; b < 2; ++b) {
    const int i = wi + b * 16 + l16;
    si[b] = (i < N) ? (src ? src[i] : i) : 0;
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int c = wc + a * 16 + 4 * l4 + r;
      sc[a][r] = (c < N) ? (src ? src[c] : c) : 0;
    }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int c = wc + a * 16 + 4 * l4 + r;
        const int i = wi + b * 16 + l16;
        const int pi = si[b], pc = sc[a][r];  // physical row and column
        xv[a][b][r] = (c < N && i < N && (!diag || i >= c))
                          ? X[(pi >= pc) ? (size_t)pi + (size_t)pc * ld : (size_t)pc + (size_t)pi * ld]
                          : 0.f;
      }
#pragma unroll
  for (int u = 0; u < TSTL; ++u) {
    const int e = tid + 256 * u, r = e & (TT - 1), t = e >> 6;
    const int c = c0 + r, i = i0 + r;
    vw[u] = (t < jw && c < N) ? W[(size_t)c + (size_t)t * ld] : 0.0;
    vl[u] = (t < jw && i < N) ? Lsrc[(size_t)i + (size_t)(k0 + t) * ld] : 0.0;
  }
}

template <int MODE>
__global__ __launch_bounds__(256) void k_trailing_lp_ps(int N, int nb,
                                                        const double *__restrict__ W,
                                                        const float *X, float *Y,
                                                        const double *__restrict__ Lsrc,
                                                        const int32_t *__restrict__ src,
                                                        const FacState *__restrict__ st,
                                                        const int32_t *__restrict__ panel_k0,
                                                        int slot, int part) {
  __shared__ float s_buf[2 * TT * TSL1];
  float *s_w = s_buf, *s_l = s_buf + TT * TSL1;
  if (slot >= st->npanel) return;
  const int k0 = panel_k0[slot], kend = panel_k0[slot + 1];
  if (kend >= N || kend <= k0 || kend - k0 > nb + 1 || kend - k0 > TSL) return;
  const int jw = kend - k0;
  const int nt = (N - kend + TT - 1) / TT;
  // the super-tile order needs a grid that is a multiple of the XCD count;
  // the near strip (part 1) is one tile column.  As the look-ahead's rest of
  // the update it measured 146.0 against 150.4 ms per N = 16384
  // factorization in the row-major order
  const bool xcd = part != 1 && gridDim.x % kXcds == 0;
  const long nslots = part_slots(part, nt, xcd);
  const size_t ld = (size_t)N;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int l16 = lane & 15, l4 = lane >> 4;
  // first slot of this workgroup that holds a tile (order of tile_order.hpp)
  long x = blockIdx.x;
  int ti = 0, tj = 0;
  while (x < nslots && !part_tile(part, x, nt, xcd, ti, tj)) x += gridDim.x;
  if (x >= nslots) return;
  float xn[2][2][4];
  double vwn[TSTL], vln[TSTL];
  lp_load(kend + ti * TT, kend + tj * TT, ti == tj, N, kend, k0, jw, W, X, Lsrc, src, xn, vwn, vln);
  while (x < nslots) {
    const int i0 = kend + ti * TT, c0 = kend + tj * TT;
    const bool diag = (ti == tj);
    const int wc = c0 + (wv & 1) * 32, wi = i0 + (wv >> 1) * 32;
    float xv[2][2][4];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int r = 0; r < 4; ++r) xv[a][b][r] = xn[a][b][r];
    __syncthreads();  // the previous tile is done with the staging buffer
#pragma unroll
    for (int u = 0; u < TSTL; ++u) {
      const int e = tid + 256 * u, r = e & (TT - 1), t = e >> 6;
      s_w[r * TSL1 + t] = (float)vwn[u];
      s_l[r * TSL1 + t] = (float)vln[u];
    }
    __syncthreads();
    // the next slot that holds a tile, its loads in flight during this one
    long xnext = x + gridDim.x;
    int tin = 0, tjn = 0;
    while (xnext < nslots && !part_tile(part, xnext, nt, xcd, tin, tjn)) xnext += gridDim.x;
    if (xnext < nslots)
      lp_load(kend + tin * TT, kend + tjn * TT, tin == tjn, N, kend, k0, jw, W, X, Lsrc, src, xn,
              vwn, vln);
    f4 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) acc[a][b] = f4{0.f, 0.f, 0.f, 0.f};
    const float *wr[2], *lr[2];
#pragma unroll
    for (int a = 0; a < 2; ++a) wr[a] = s_w + (wc - c0 + a * 16 + l16) * TSL1;
#pragma unroll
    for (int b = 0; b < 2; ++b) lr[b] = s_l + (wi - i0 + b * 16 + l16) * TSL1;
    if (MODE == 1) {
      for (int t0 = 0; t0 < jw; t0 += 4) {
        const int t = t0 + l4;
        float av[2], bv[2];
#pragma unroll
        for (int a = 0; a < 2; ++a) av[a] = wr[a][t];
#pragma unroll
        for (int b = 0; b < 2; ++b) bv[b] = lr[b][t];
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
          for (int b = 0; b < 2; ++b)
            acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[a], bv[b], acc[a][b], 0, 0, 0);
      }
    } else if (MODE == 3) {
      for (int t0 = 0; t0 < jw; t0 += 16) {
        s4 ah[2], al[2], bh[2], bl[2];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int t = t0 + 4 * l4 + e;
#pragma unroll
          for (int a = 0; a < 2; ++a) {
            const float v = wr[a][t];
            const short h = to_bf16(v);
            ah[a][e] = h;
            al[a][e] = to_bf16(v - bf16_to_f32(h));
          }
#pragma unroll
          for (int b = 0; b < 2; ++b) {
            const float v = lr[b][t];
            const short h = to_bf16(v);
            bh[b][e] = h;
            bl[b][e] = to_bf16(v - bf16_to_f32(h));
          }
        }
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
          for (int b = 0; b < 2; ++b) {
            acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(al[a], bh[b], acc[a][b], 0, 0, 0);
            acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah[a], bl[b], acc[a][b], 0, 0, 0);
            acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah[a], bh[b], acc[a][b], 0, 0, 0);
          }
      }
    } else {
      for (int t0 = 0; t0 < jw; t0 += 16) {
        s4 av[2], bv[2];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int t = t0 + 4 * l4 + e;
#pragma unroll
          for (int a = 0; a < 2; ++a) av[a][e] = to_bf16(wr[a][t]);
#pragma unroll
          for (int b = 0; b < 2; ++b) bv[b][e] = to_bf16(lr[b][t]);
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
          const int c = wc + a * 16 + 4 * l4 + r;
          const int i = wi + b * 16 + l16;
          if (c < N && i < N && (!diag || i >= c)) Y[(size_t)i + (size_t)c * ld] = xv[a][b][r] - acc[a][b][r];
        }
    x = xnext;
    ti = tin;
    tj = tjn;
  }
}

// Symmetric equilibration s_j = 1 / sqrt(max_i |M_ij|) (1 for a zero
// column): one wave per column of the full symmetric M, so the column maximum
// is the row maximum.
__global__ void k_row_scale(int N, const double *__restrict__ M, double *__restrict__ s) {
  const int lane = threadIdx.x & 63;
  const int j = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (j >= N) return;
  double mx = 0.0;
  for (int i = lane; i < N; i += 64) mx = fmax(mx, fabs(M[(size_t)i + (size_t)j * N]));
  for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off));
  if (lane == 0) s[j] = (mx > 0.0 && isfinite(mx)) ? 1.0 / sqrt(mx) : 1.0;
}

// b = (float)(s_i a_ij s_j), rounded once from FP64
__global__ void k_to_f32_scaled(int N, const double *__restrict__ a, const double *__restrict__ s,
                                float *__restrict__ b) {
  const int64_t n = (int64_t)N * N;
  const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = i0; e < n; e += stride) {
    const int i = (int)(e % N), j = (int)(e / N);
    b[e] = (float)((s[i] * a[e]) * s[j]);
  }
}

// v = s .* v
__global__ void k_vscale(int n, const double *__restrict__ s, double *__restrict__ v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) v[i] = s[i] * v[i];
}

}  // namespace

void launch_trailing_lp(hipStream_t s, int mode, int N, int nb, long rem, int slot,
                        const double *W, const float *X, float *Y, const double *Lsrc,
                        const int32_t *src, const FacState *st, const int32_t *panel_k0) {
  if (rem <= 0) return;
  const long nt = (rem + TT - 1) / TT;
  const long tiles = nt * (nt + 1) / 2;
  if (nb + 1 <= TSL) {
    // persistent: a few workgroups per compute unit walk the tiles
    const unsigned g = (unsigned)std::min(tiles, (long)kTrailingLpGrid);
    if (mode == 2)
      k_trailing_lp_ps<2><<<g, 256, 0, s>>>(N, nb, W, X, Y, Lsrc, src, st, panel_k0, slot, 0);
    else if (mode == 3)
      k_trailing_lp_ps<3><<<g, 256, 0, s>>>(N, nb, W, X, Y, Lsrc, src, st, panel_k0, slot, 0);
    else
      k_trailing_lp_ps<1><<<g, 256, 0, s>>>(N, nb, W, X, Y, Lsrc, src, st, panel_k0, slot, 0);
    return;
  }
  if (mode == 2)
    k_trailing_lp<2><<<(unsigned)tiles, 256, 0, s>>>(N, nb, W, X, Y, Lsrc, src, st, panel_k0, slot);
  else if (mode == 3)
    k_trailing_lp<3><<<(unsigned)tiles, 256, 0, s>>>(N, nb, W, X, Y, Lsrc, src, st, panel_k0, slot);
  else
    k_trailing_lp<1><<<(unsigned)tiles, 256, 0, s>>>(N, nb, W, X, Y, Lsrc, src, st, panel_k0, slot);
}

void launch_trailing_lp_part(hipStream_t s, int mode, int N, int nb, long rem, int slot, int part,
                             int grid, const double *W, const float *X, float *Y,
                             const double *Lsrc, const int32_t *src, const FacState *st,
                             const int32_t *panel_k0) {
  if (rem <= 0 || nb + 1 > TSL) return;
  const long nt = (rem + TT - 1) / TT;
  const long tiles = (part == 1) ? nt : (nt - 1) * nt / 2;
  if (tiles <= 0) return;
  const unsigned g = (unsigned)std::min(tiles, (long)std::max(grid, 1));
  if (mode == 2)
    k_trailing_lp_ps<2><<<g, 256, 0, s>>>(N, nb, W, X, Y, Lsrc, src, st, panel_k0, slot, part);
  else if (mode == 3)
    k_trailing_lp_ps<3><<<g, 256, 0, s>>>(N, nb, W, X, Y, Lsrc, src, st, panel_k0, slot, part);
  else
    k_trailing_lp_ps<1><<<g, 256, 0, s>>>(N, nb, W, X, Y, Lsrc, src, st, panel_k0, slot, part);
}

void launch_equilibrate_f32(hipStream_t s, int N, const double *M, double *scale, float *b) {
  if (N <= 0) return;
  k_row_scale<<<(unsigned)((N + 3) / 4), 256, 0, s>>>(N, M, scale);
  const int64_t n = (int64_t)N * N;
  const int64_t blocks = std::min<int64_t>((n + 255) / 256, 8192);
  k_to_f32_scaled<<<(unsigned)blocks, 256, 0, s>>>(N, M, scale, b);
}

void launch_vscale(hipStream_t s, int n, const double *scale, double *v) {
  if (n > 0) k_vscale<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(n, scale, v);
}

}  // namespace mds
