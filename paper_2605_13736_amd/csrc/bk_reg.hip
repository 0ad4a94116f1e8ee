// Register-resident Bunch-Kaufman panel kernel (Sec. 2.3) for N <= 4096; the
// workgroup-level body is panel::panel_reg_dev.
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

// Panel variant for a matrix of order N: 512 threads and R rows per thread
// (R * 512 >= N), with the register tile NB chosen so that R * NB <= 64
// doubles of L per thread.
int bk_reg_rows(int N) {
  for (int r = 1; r <= 8; r *= 2)
    if (N <= r * TMAX) return r;
  return 0;
}

int bk_reg_nb(int N) {
  switch (bk_reg_rows(N)) {
    case 1: return 32;
    case 2: return 32;
    case 4: return 16;
    case 8: return 8;
    default: return 0;
  }
}

template <typename TX>
static void panel_reg(hipStream_t s, int N, int nb, double alpha, const TX *X, double *Lout,
                      int32_t *src_out, double *W, double *dd, double *ds, int32_t *ipiv,
                      int32_t *blk, FacState *st, int32_t *panel_k0) {
#define MDS_PANEL_REG(R_, NB_)                                                                \
  k_bk_panel_reg<TMAX, R_, NB_, TX><<<1, TMAX, 0, s>>>(N, nb, alpha, X, Lout, src_out, W, dd, \
                                                       ds, ipiv, blk, st, panel_k0)
  switch (bk_reg_rows(N)) {
    case 1: MDS_PANEL_REG(1, 32); break;
    case 2: MDS_PANEL_REG(2, 32); break;
    case 4: MDS_PANEL_REG(4, 16); break;
    case 8: MDS_PANEL_REG(8, 8); break;
    default: break;
  }
#undef MDS_PANEL_REG
}

void launch_bk_panel_reg(hipStream_t s, int N, int nb, double alpha, const double *X,
                         double *Lout, int32_t *src_out, double *W, double *dd, double *ds,
                         int32_t *ipiv, int32_t *blk, FacState *st, int32_t *panel_k0) {
  panel_reg(s, N, nb, alpha, X, Lout, src_out, W, dd, ds, ipiv, blk, st, panel_k0);
}

void launch_bk_panel_reg(hipStream_t s, int N, int nb, double alpha, const float *X,
                         double *Lout, int32_t *src_out, double *W, double *dd, double *ds,
                         int32_t *ipiv, int32_t *blk, FacState *st, int32_t *panel_k0) {
  panel_reg(s, N, nb, alpha, X, Lout, src_out, W, dd, ds, ipiv, blk, st, panel_k0);
}

}  // namespace mds
