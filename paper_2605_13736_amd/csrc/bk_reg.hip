// Register-resident Bunch-Kaufman panel kernel (Sec. 2.3): N <= 4096, or the
// last rows of a cooperative factorization; the body is panel::panel_reg_dev.
#include <algorithm>

#include "panel_reg.hpp"

namespace mds {
namespace {

constexpr int TMAX = 512;

template <int T, int R, int NB, typename TX>
__global__ __launch_bounds__(T) void k_bk_panel_reg(int N, int nb, double alpha,
                                                    const TX *__restrict__ X,
                                                    double *__restrict__ Lout,
                                                    int32_t *__restrict__ src_out,
                                                    double *__restrict__ W,
                                                    double *__restrict__ dd,
                                                    double *__restrict__ ds,
                                                    int32_t *__restrict__ ipiv,
                                                    int32_t *__restrict__ blk, FacState *st,
                                                    int32_t *__restrict__ panel_k0) {
  panel::panel_reg_dev<T, R, NB, TX>(N, nb, alpha, X, Lout, src_out, W, dd, ds, ipiv, blk, st,
                                     panel_k0);
}

}  // namespace

// Panel variant for a matrix of order N and a workgroup of T threads: R rows
// per thread with R * T >= N, and the register tile NB chosen so that
// R * NB = 64 doubles of L per thread at T = 512 (VGPR budget 256) and 32 at
// T = 1024 (budget 128).  Workgroups of 64, 128 or 256 threads (one or two
// waves per SIMD at most) take up to 2 rows per thread with nb = 32: for
// small orders fewer waves wait at each barrier of a pivot step.
int bk_reg_rows(int N, int threads) {
  if (threads == 64 || threads == 128 || threads == 256) {
    for (int r = 1; r <= 2; ++r)
      if (N <= r * threads) return r;
    return 0;
  }
  const int T = (threads == 1024) ? 1024 : TMAX;
  const int rmax = (T == 1024) ? 4 : 8;
  for (int r = 1; r <= rmax; r *= 2)
    if (N <= r * T) return r;
  return 0;
}

int bk_reg_nb(int N, int threads) {
  const int r = bk_reg_rows(N, threads);
  if (r == 0) return 0;
  if (threads == 64 || threads == 128 || threads == 256) return 32;
  if (threads == 1024) return 32 / r;
  return (r == 1) ? 32 : 64 / r;
}

template <typename TX>
static void panel_reg(hipStream_t s, int threads, int N, int nb, double alpha, const TX *X,
                      double *Lout, int32_t *src_out, double *W, double *dd, double *ds,
                      int32_t *ipiv, int32_t *blk, FacState *st, int32_t *panel_k0) {
#define MDS_PANEL_REG(T_, R_, NB_)                                                             \
  k_bk_panel_reg<T_, R_, NB_, TX><<<1, T_, 0, s>>>(N, nb, alpha, X, Lout, src_out, W, dd, ds, \
                                                   ipiv, blk, st, panel_k0)
  const int r = bk_reg_rows(N, threads);
  if (threads == 64 || threads == 128 || threads == 256) {
    switch (threads * 10 + r) {
      case 641: MDS_PANEL_REG(64, 1, 32); break;
      case 642: MDS_PANEL_REG(64, 2, 32); break;
      case 1281: MDS_PANEL_REG(128, 1, 32); break;
      case 1282: MDS_PANEL_REG(128, 2, 32); break;
      case 2561: MDS_PANEL_REG(256, 1, 32); break;
      case 2562: MDS_PANEL_REG(256, 2, 32); break;
      default: break;
    }
  } else if (threads == 1024) {
    switch (r) {
      case 1: MDS_PANEL_REG(1024, 1, 32); break;
      case 2: MDS_PANEL_REG(1024, 2, 16); break;
      case 4: MDS_PANEL_REG(1024, 4, 8); break;
      default: break;
    }
  } else {
    switch (r) {
      case 1: MDS_PANEL_REG(TMAX, 1, 32); break;
      case 2: MDS_PANEL_REG(TMAX, 2, 32); break;
      case 4: MDS_PANEL_REG(TMAX, 4, 16); break;
      case 8: MDS_PANEL_REG(TMAX, 8, 8); break;
      default: break;
    }
  }
#undef MDS_PANEL_REG
}

// Tail of a cooperative factorization: once at most 2048 rows remain, one
// workgroup of 512 threads holds them in its registers and a pivot step
// needs no grid-wide exchange.  Measured on KKT systems of the tail's sizes
// (factorization time): 2048 rows, 512 threads x 4 rows with a 16-column
// tile 8.5 ms against 12.6 ms for the cooperative panel (two workgroups)
// and its tail; 1024 rows, 512 x 2 with the 32-column tile 3.4 ms against
// 4.0 for 1024 x 1; 512 rows, 512 x 1 1.55 ms against 1.66 for 256 x 2.
// rows bounds N - k0 from above (the host's slot plan).
int bk_reg_tail_rows() { return 4 * TMAX; }
int bk_reg_tail_nb(int rows) { return (rows > 2 * TMAX) ? 16 : 32; }

template <typename TX>
static void panel_reg_tail(hipStream_t s, int rows, int N, int nb, double alpha, const TX *X,
                           double *Lout, int32_t *src_out, double *W, double *dd, double *ds,
                           int32_t *ipiv, int32_t *blk, FacState *st, int32_t *panel_k0) {
  const int tnb = std::min(nb, bk_reg_tail_nb(rows));
  if (rows <= 256)
    k_bk_panel_reg<256, 1, 32, TX><<<1, 256, 0, s>>>(N, tnb, alpha, X, Lout, src_out, W, dd, ds,
                                                     ipiv, blk, st, panel_k0);
  else if (rows <= TMAX)
    k_bk_panel_reg<TMAX, 1, 32, TX><<<1, TMAX, 0, s>>>(N, tnb, alpha, X, Lout, src_out, W, dd,
                                                       ds, ipiv, blk, st, panel_k0);
  else if (rows <= 2 * TMAX)
    k_bk_panel_reg<TMAX, 2, 32, TX><<<1, TMAX, 0, s>>>(N, tnb, alpha, X, Lout, src_out, W, dd,
                                                       ds, ipiv, blk, st, panel_k0);
  else  // rows beyond 2048 would break the caller's bound: the kernel's guard flags them
    k_bk_panel_reg<TMAX, 4, 16, TX><<<1, TMAX, 0, s>>>(N, tnb, alpha, X, Lout, src_out, W, dd,
                                                       ds, ipiv, blk, st, panel_k0);
}

void launch_bk_panel_reg_tail(hipStream_t s, int rows, int N, int nb, double alpha,
                              const double *X, double *Lout, int32_t *src_out, double *W,
                              double *dd, double *ds, int32_t *ipiv, int32_t *blk, FacState *st,
                              int32_t *panel_k0) {
  panel_reg_tail(s, rows, N, nb, alpha, X, Lout, src_out, W, dd, ds, ipiv, blk, st, panel_k0);
}

void launch_bk_panel_reg_tail(hipStream_t s, int rows, int N, int nb, double alpha,
                              const float *X, double *Lout, int32_t *src_out, double *W,
                              double *dd, double *ds, int32_t *ipiv, int32_t *blk, FacState *st,
                              int32_t *panel_k0) {
  panel_reg_tail(s, rows, N, nb, alpha, X, Lout, src_out, W, dd, ds, ipiv, blk, st, panel_k0);
}

void launch_bk_panel_reg(hipStream_t s, int threads, int N, int nb, double alpha, const double *X,
                         double *Lout, int32_t *src_out, double *W, double *dd, double *ds,
                         int32_t *ipiv, int32_t *blk, FacState *st, int32_t *panel_k0) {
  panel_reg(s, threads, N, nb, alpha, X, Lout, src_out, W, dd, ds, ipiv, blk, st, panel_k0);
}

void launch_bk_panel_reg(hipStream_t s, int threads, int N, int nb, double alpha, const float *X,
                         double *Lout, int32_t *src_out, double *W, double *dd, double *ds,
                         int32_t *ipiv, int32_t *blk, FacState *st, int32_t *panel_k0) {
  panel_reg(s, threads, N, nb, alpha, X, Lout, src_out, W, dd, ds, ipiv, blk, st, panel_k0);
}

}  // namespace mds
