// Element-wise and reduction kernels of the filter line-search IPM
// (Sec. 2.1; kernel class K1).  Infinite bounds contribute nothing: their
// slacks, barrier terms and multipliers are skipped.
//
// Reductions write one 8-slot record per workgroup (slots 0-3 maxima, 4-7
// sums) into `red`; k_red_final combines the records in block order.  The
// grid size depends only on the vector length, so every sum is evaluated in
// the same order on every run.
#include "internal.hpp"
#include "ipm.hpp"
#include "vec.hpp"

namespace mds {
namespace {

constexpr int RB = 256;

inline unsigned grid1(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

__global__ void k_init_point(int n, int m, const double *__restrict__ xl,
                             const double *__restrict__ xu, double *__restrict__ x,
                             double *__restrict__ y, double *__restrict__ zl,
                             double *__restrict__ zu) {
  const double kappa1 = 1e-2, kappa2 = 1e-2;
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    const double l = xl[i], u = xu[i];
    const bool hl = isfinite(l), hu = isfinite(u);
    double xi = 0.0;
    if (hl && hu) {
      const double pl = fmin(kappa1 * fmax(1.0, fabs(l)), kappa2 * (u - l));
      const double pu = fmin(kappa1 * fmax(1.0, fabs(u)), kappa2 * (u - l));
      xi = fmin(fmax(xi, l + pl), u - pu);
    } else if (hl) {
      xi = fmax(xi, l + kappa1 * fmax(1.0, fabs(l)));
    } else if (hu) {
      xi = fmin(xi, u - kappa1 * fmax(1.0, fabs(u)));
    }
    x[i] = xi;
    zl[i] = hl ? 1.0 : 0.0;
    zu[i] = hu ? 1.0 : 0.0;
  }
  if (i < m) y[i] = 0.0;
}

// Warm start: x_d = xd0, x_s = -(g + J_s' y0) / w (w > 0; else 0), every x_i
// projected into its bounds as in the cold start, y = y0, z = mu0 / slack on
// finite bounds.  J_s' y0 is accumulated per column over its rows in
// ascending order (CSC), as plain multiply-then-add.
__global__ void k_init_warm(int nd, int ns, int m, const double *__restrict__ xl,
                            const double *__restrict__ xu, const double *__restrict__ w,
                            const double *__restrict__ g, const int32_t *__restrict__ cptr,
                            const int32_t *__restrict__ crow, const double *__restrict__ cval,
                            const double *__restrict__ xd0, const double *__restrict__ y0,
                            double mu0, double *__restrict__ x, double *__restrict__ y,
                            double *__restrict__ zl, double *__restrict__ zu) {
  const double kappa1 = 1e-2, kappa2 = 1e-2;
  const int n = nd + ns;
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    double xi;
    if (i < nd) {
      xi = xd0[i];
    } else {
      const int k = i - nd;
      double t = 0.0;
      for (int e = cptr[k]; e < cptr[k + 1]; ++e) t = t + cval[e] * y0[crow[e]];
      const double wk = w[k];
      xi = (wk > 0.0) ? -(g[k] + t) / wk : 0.0;
    }
    const double l = xl[i], u = xu[i];
    const bool hl = isfinite(l), hu = isfinite(u);
    if (hl && hu) {
      const double pl = fmin(kappa1 * fmax(1.0, fabs(l)), kappa2 * (u - l));
      const double pu = fmin(kappa1 * fmax(1.0, fabs(u)), kappa2 * (u - l));
      xi = fmin(fmax(xi, l + pl), u - pu);
    } else if (hl) {
      xi = fmax(xi, l + kappa1 * fmax(1.0, fabs(l)));
    } else if (hu) {
      xi = fmin(xi, u - kappa1 * fmax(1.0, fabs(u)));
    }
    x[i] = xi;
    zl[i] = hl ? mu0 / (xi - l) : 0.0;
    zu[i] = hu ? mu0 / (u - xi) : 0.0;
  }
  if (i < m) y[i] = y0[i];
}

// Warm start, bound multipliers: add to the centred mu0 / s the part of the
// dual residual r = grad f(x) + J'y each finite bound can carry
// (stationarity asks z_l - z_u = r): r > 0 to z_l, -r > 0 to z_u.
__global__ void k_warm_duals(int n, const double *__restrict__ xl, const double *__restrict__ xu,
                             const double *__restrict__ gf, const double *__restrict__ jty,
                             double *__restrict__ zl, double *__restrict__ zu) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double r = gf[i] + jty[i];
  if (r > 0.0 && isfinite(xl[i])) zl[i] = zl[i] + r;
  if (r < 0.0 && isfinite(xu[i])) zu[i] = zu[i] - r;
}

// gf[0:nd] holds H x_d on entry; gradient of f completed in place.
__global__ void k_grad_finish(int nd, int ns, const double *__restrict__ c,
                              const double *__restrict__ w, const double *__restrict__ g,
                              const double *__restrict__ x, double *__restrict__ gf) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nd) gf[i] = gf[i] + c[i];
  else if (i < nd + ns) gf[i] = w[i - nd] * x[i] + g[i - nd];
}

__global__ void k_sigma_rhs(int n, const double *__restrict__ x, const double *__restrict__ zl,
                            const double *__restrict__ zu, const double *__restrict__ xl,
                            const double *__restrict__ xu, const double *__restrict__ gf,
                            const double *__restrict__ jty, double mu,
                            double *__restrict__ sigma, double *__restrict__ rx) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = 0.0, gb = gf[i] + jty[i];
  const double l = xl[i], u = xu[i];
  if (isfinite(l)) {
    const double sl = x[i] - l;
    s = s + zl[i] / sl;
    gb = gb - mu / sl;
  }
  if (isfinite(u)) {
    const double su = u - x[i];
    s = s + zu[i] / su;
    gb = gb + mu / su;
  }
  sigma[i] = s;
  rx[i] = -gb;
}

// cx holds J x on entry; becomes c = J x - [b; d] (equality rows against b,
// inequality rows against their slack d), and r_y = -c.
__global__ void k_constr_finish(int m, int mE, const double *__restrict__ b,
                                const double *__restrict__ d, double *__restrict__ cx,
                                double *__restrict__ ry) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  const double t = cx[i] - ((i < mE) ? b[i] : d[i - mE]);
  cx[i] = t;
  if (ry) ry[i] = -t;
}

// Slack entries of the Lagrangian gradient (Sec. 2, eq. (ineq) turned into
// J_h x - d = 0): the objective does not depend on d, and the slack column
// of the constraint Jacobian is -I, so grad f = 0 and J'y = -y_h there.
// y may be null (gradient only).
__global__ void k_slack_grad(int mI, int mE, const double *__restrict__ y,
                             double *__restrict__ gf_t, double *__restrict__ jty_t) {
  int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= mI) return;
  gf_t[r] = 0.0;
  if (y) jty_t[r] = -y[mE + r];
}

// d = row value of J_h x (in hx) pushed into the interior of [hl, hu] by
// the start point's rule for bounded variables.
__global__ void k_slack_project(int mI, const double *__restrict__ hx,
                                const double *__restrict__ hl, const double *__restrict__ hu,
                                double *__restrict__ d) {
  const double kappa1 = 1e-2, kappa2 = 1e-2;
  int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= mI) return;
  const double l = hl[r], u = hu[r];
  const bool fl = isfinite(l), fu = isfinite(u);
  double v = hx[r];
  if (fl && fu) {
    const double pl = fmin(kappa1 * fmax(1.0, fabs(l)), kappa2 * (u - l));
    const double pu = fmin(kappa1 * fmax(1.0, fabs(u)), kappa2 * (u - l));
    v = fmin(fmax(v, l + pl), u - pu);
  } else if (fl) {
    v = fmax(v, l + kappa1 * fmax(1.0, fabs(l)));
  } else if (fu) {
    v = fmin(v, u - kappa1 * fmax(1.0, fabs(u)));
  }
  d[r] = v;
}

// Warm start of the slacks' multipliers: mu0 / slack on finite bounds.
__global__ void k_slack_duals(int mI, const double *__restrict__ hl,
                              const double *__restrict__ hu, const double *__restrict__ d,
                              double mu0, double *__restrict__ vl, double *__restrict__ vu) {
  int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= mI) return;
  vl[r] = isfinite(hl[r]) ? mu0 / (d[r] - hl[r]) : 0.0;
  vu[r] = isfinite(hu[r]) ? mu0 / (hu[r] - d[r]) : 0.0;
}

// (4,4) block of eq. (linsys4x4) after the slack step is eliminated:
// dcv = 1 / (Sigma_h + dw) on inequality rows, 0 on equality rows.
__global__ void k_ineq_dcv(int m, int mE, const double *__restrict__ sig_h, double dw,
                           double *__restrict__ dcv) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  dcv[i] = (i < mE) ? 0.0 : 1.0 / (sig_h[i - mE] + dw);
}

// Slack step eliminated from the right-hand side: r_y,h += dcv .* r_d.
__global__ void k_ineq_rhs(int mI, int mE, const double *__restrict__ dcv,
                           const double *__restrict__ rd, double *__restrict__ ry) {
  int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= mI) return;
  ry[mE + r] = ry[mE + r] + dcv[mE + r] * rd[r];
}

// Slack step recovered from the multiplier step: dd = dcv .* (r_d + dy_h).
__global__ void k_ineq_step(int mI, int mE, const double *__restrict__ dcv,
                            const double *__restrict__ rd, const double *__restrict__ dy,
                            double *__restrict__ dd) {
  int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= mI) return;
  dd[r] = dcv[mE + r] * (rd[r] + dy[mE + r]);
}

__global__ void k_dsbase(int nd, int ns, const double *__restrict__ w,
                         const double *__restrict__ sig, double *__restrict__ dsb) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < ns) dsb[k] = w[k] + sig[nd + k];
}

__global__ void k_dz(int n, const double *__restrict__ x, const double *__restrict__ zl,
                     const double *__restrict__ zu, const double *__restrict__ xl,
                     const double *__restrict__ xu, const double *__restrict__ dx, double mu,
                     double *__restrict__ dzl, double *__restrict__ dzu) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double a = 0.0, b = 0.0;
  if (isfinite(xl[i])) {
    const double sl = x[i] - xl[i];
    a = mu / sl - zl[i] - (zl[i] / sl) * dx[i];
  }
  if (isfinite(xu[i])) {
    const double su = xu[i] - x[i];
    b = mu / su - zu[i] + (zu[i] / su) * dx[i];
  }
  dzl[i] = a;
  dzu[i] = b;
}

// slot 0: max dual infeasibility, 1: max |J x - b|, 2/3: max complementarity
// (lower/upper), 4: sum |y|, 5: sum of bound multipliers, 6: finite bounds
// PAIR: slot 2 = both complementarity maxima at mu, slot 3 = both at mu = 0
// (E_mu and E_0 from one pass; the maxima are the same numbers either way)
template <bool PAIR>
__global__ __launch_bounds__(RB) void k_red_opt(int n, int m, const double *__restrict__ x,
                                                const double *__restrict__ y,
                                                const double *__restrict__ zl,
                                                const double *__restrict__ zu,
                                                const double *__restrict__ xl,
                                                const double *__restrict__ xu,
                                                const double *__restrict__ gf,
                                                const double *__restrict__ jty,
                                                const double *__restrict__ cx, double mu,
                                                double *__restrict__ red) {
  double v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  const int64_t stride = (int64_t)gridDim.x * RB;
  const int64_t len = (n > m) ? n : m;
  for (int64_t e = (int64_t)blockIdx.x * RB + threadIdx.x; e < len; e += stride) {
    if (e < n) {
      double r = gf[e] + jty[e];
      if (isfinite(xl[e])) {
        r = r - zl[e];
        const double sz = (x[e] - xl[e]) * zl[e];
        if (PAIR) {
          v[2] = fmax(v[2], fabs(sz - mu));
          v[3] = fmax(v[3], fabs(sz - 0.0));
        } else {
          v[2] = fmax(v[2], fabs(sz - mu));
        }
        v[5] += fabs(zl[e]);
        v[6] += 1.0;
      }
      if (isfinite(xu[e])) {
        r = r + zu[e];
        const double sz = (xu[e] - x[e]) * zu[e];
        if (PAIR) {
          v[2] = fmax(v[2], fabs(sz - mu));
          v[3] = fmax(v[3], fabs(sz - 0.0));
        } else {
          v[3] = fmax(v[3], fabs(sz - mu));
        }
        v[5] += fabs(zu[e]);
        v[6] += 1.0;
      }
      v[0] = fmax(v[0], fabs(r));
    }
    if (e < m) {
      v[1] = fmax(v[1], fabs(cx[e]));
      v[4] += fabs(y[e]);
    }
  }
  block_reduce8(v, red + (size_t)blockIdx.x * 8);
}

// slot 4: f(x), 5: sum of log-slacks over the nx bounded entries (the
// variables, then the inequality slacks), 6: theta = ||c||_1, 7: the rounding
// scale of phi_mu = f - mu * (slot 5), the sum of the magnitudes of its terms.
// hx holds H x_d, cx holds c = J x - [b; d].
__global__ __launch_bounds__(RB) void k_red_merit(int nd, int ns, int nx, int m, double mu,
                                                  const double *__restrict__ x,
                                                  const double *__restrict__ hx,
                                                  const double *__restrict__ c,
                                                  const double *__restrict__ w,
                                                  const double *__restrict__ g,
                                                  const double *__restrict__ wbx,
                                                  const double *__restrict__ xl,
                                                  const double *__restrict__ xu,
                                                  const double *__restrict__ cx,
                                                  double *__restrict__ red) {
  double v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  const int n = nd + ns;
  const int64_t stride = (int64_t)gridDim.x * RB;
  const int64_t len = (nx > m) ? nx : m;
  for (int64_t e = (int64_t)blockIdx.x * RB + threadIdx.x; e < len; e += stride) {
    if (e < nd) {
      const double t = x[e] * (0.5 * hx[e] + c[e]);
      v[4] += t;
      v[7] += fabs(t);
    } else if (e < n) {
      const double xs = x[e];
      // with coupling blocks: 0.5 x_s' (diag(w) + blockdiag(Wb)) x_s + g' x_s
      const double t = wbx ? xs * (0.5 * (w[e - nd] * xs + wbx[e - nd]) + g[e - nd])
                           : xs * (0.5 * w[e - nd] * xs + g[e - nd]);
      v[4] += t;
      v[7] += fabs(t);
    }
    if (e < nx) {
      if (isfinite(xl[e])) {
        const double t = log(x[e] - xl[e]);
        v[5] += t;
        v[7] += mu * fabs(t);
      }
      if (isfinite(xu[e])) {
        const double t = log(xu[e] - x[e]);
        v[5] += t;
        v[7] += mu * fabs(t);
      }
    }
    if (e < m) v[6] += fabs(cx[e]);
  }
  block_reduce8(v, red + (size_t)blockIdx.x * 8);
}

// slot 4: grad(phi_mu)' dx
__global__ __launch_bounds__(RB) void k_red_gphi(int n, const double *__restrict__ gf,
                                                 const double *__restrict__ x,
                                                 const double *__restrict__ xl,
                                                 const double *__restrict__ xu,
                                                 const double *__restrict__ dx, double mu,
                                                 double *__restrict__ red) {
  double v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  const int64_t stride = (int64_t)gridDim.x * RB;
  for (int64_t e = (int64_t)blockIdx.x * RB + threadIdx.x; e < n; e += stride) {
    double gi = gf[e];
    if (isfinite(xl[e])) gi = gi - mu / (x[e] - xl[e]);
    if (isfinite(xu[e])) gi = gi + mu / (xu[e] - x[e]);
    v[4] += gi * dx[e];
  }
  block_reduce8(v, red + (size_t)blockIdx.x * 8);
}

// Fraction to the boundary: slot 0 = max of -(step limit) over primal slacks,
// slot 1 = same over bound multipliers (so alpha = min(1, -slot)).
__global__ __launch_bounds__(RB) void k_red_ftb(int n, const double *__restrict__ x,
                                                const double *__restrict__ xl,
                                                const double *__restrict__ xu,
                                                const double *__restrict__ dx,
                                                const double *__restrict__ zl,
                                                const double *__restrict__ zu,
                                                const double *__restrict__ dzl,
                                                const double *__restrict__ dzu, double tau,
                                                double *__restrict__ red) {
  double v[8] = {-1.0, -1.0, 0, 0, 0, 0, 0, 0};
  const int64_t stride = (int64_t)gridDim.x * RB;
  for (int64_t e = (int64_t)blockIdx.x * RB + threadIdx.x; e < n; e += stride) {
    if (isfinite(xl[e])) {
      const double sl = x[e] - xl[e];
      if (dx[e] < 0.0) v[0] = fmax(v[0], -(-tau * sl / dx[e]));
      if (dzl[e] < 0.0) v[1] = fmax(v[1], -(-tau * zl[e] / dzl[e]));
    }
    if (isfinite(xu[e])) {
      const double su = xu[e] - x[e];
      if (-dx[e] < 0.0) v[0] = fmax(v[0], -(-tau * su / (-dx[e])));
      if (dzu[e] < 0.0) v[1] = fmax(v[1], -(-tau * zu[e] / dzu[e]));
    }
  }
  block_reduce8(v, red + (size_t)blockIdx.x * 8);
}

// generic fraction to the boundary of one vector
__global__ __launch_bounds__(RB) void k_red_ftb1(int64_t n, const double *__restrict__ v0,
                                                 const double *__restrict__ dv, double tau,
                                                 double *__restrict__ red) {
  double v[8] = {-1.0, 0, 0, 0, 0, 0, 0, 0};
  const int64_t stride = (int64_t)gridDim.x * RB;
  for (int64_t e = (int64_t)blockIdx.x * RB + threadIdx.x; e < n; e += stride)
    if (dv[e] < 0.0) v[0] = fmax(v[0], -(-tau * v0[e] / dv[e]));
  block_reduce8(v, red + (size_t)blockIdx.x * 8);
}

// alpha = -out[0] (the fraction-to-the-boundary step from the record's max
// slot, which holds the largest -(step limit))
__global__ void k_neg_first(const double *__restrict__ out, double *__restrict__ alpha) {
  if (threadIdx.x == 0) alpha[0] = -out[0];
}

// 256 threads: thread t combines the records t, t + 256, ... in increasing
// order, then a fixed pairwise tree over the threads (max for slots 0-3, sum
// for slots 4-7); the order depends only on nb.
__global__ __launch_bounds__(256) void k_red_final(int nb, const double *__restrict__ red,
                                                   double *__restrict__ out) {
  __shared__ double sh[8][256];
  const int t = threadIdx.x;
#pragma unroll
  for (int s = 0; s < 8; ++s) {
    double v = (s < 4) ? -INFINITY : 0.0;
    for (int b = t; b < nb; b += 256) {
      const double x = red[(size_t)b * 8 + s];
      v = (s < 4) ? fmax(v, x) : v + x;
    }
    sh[s][t] = v;
  }
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w) {
#pragma unroll
      for (int s = 0; s < 8; ++s)
        sh[s][t] = (s < 4) ? fmax(sh[s][t], sh[s][t + w]) : sh[s][t] + sh[s][t + w];
    }
    __syncthreads();
  }
  if (t < 8) out[t] = sh[t][0];
}

__global__ void k_axpy_to(int n, const double *__restrict__ x, const double *__restrict__ dx,
                          double a, double *__restrict__ out) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = x[i] + a * dx[i];
}

__global__ void k_accept(int n, int m, const double *__restrict__ xt, double *__restrict__ x,
                         double *__restrict__ y, const double *__restrict__ dy,
                         double *__restrict__ zl, double *__restrict__ zu,
                         const double *__restrict__ dzl, const double *__restrict__ dzu,
                         const double *__restrict__ xl, const double *__restrict__ xu,
                         double alpha, double alpha_z, double mu) {
  const double kappa_sigma = 1e10;
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    const double xi = xt[i];
    x[i] = xi;
    if (isfinite(xl[i])) {
      const double z = zl[i] + alpha_z * dzl[i], sl = xi - xl[i];
      zl[i] = fmax(fmin(z, kappa_sigma * mu / sl), mu / (kappa_sigma * sl));
    }
    if (isfinite(xu[i])) {
      const double z = zu[i] + alpha_z * dzu[i], su = xu[i] - xi;
      zu[i] = fmax(fmin(z, kappa_sigma * mu / su), mu / (kappa_sigma * su));
    }
  }
  if (i < m) y[i] = y[i] + alpha * dy[i];
}

__global__ void k_copy_scaled(int64_t n, const double *__restrict__ src, double *__restrict__ dst) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[i];
}

// res = r - K d for the full regularised Newton system; kd holds K d.
__global__ void k_sub(int64_t n, const double *__restrict__ a, const double *__restrict__ b,
                      double *__restrict__ out) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = a[i] - b[i];
}

__global__ void k_add_inplace(int64_t n, const double *__restrict__ a, double *__restrict__ out) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = out[i] + a[i];
}

// K d, second block row (x_s): (dsbase + dw) dx_s + J_s' dy, with J_s' dy in o_s.
__global__ void k_kkt_s(int ns, const double *__restrict__ dsb, double dw,
                        const double *__restrict__ dxs, double *__restrict__ o_s) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < ns) o_s[k] = fma(dsb[k] + dw, dxs[k], o_s[k]);
}

// first block row (x_d): o_d = H dx_d + (sigma_d + dw) dx_d + J_d' dy (o_d holds
// H dx_d + J_d' dy on entry)
__global__ void k_kkt_d(int nd, const double *__restrict__ sig, double dw,
                        const double *__restrict__ dxd, double *__restrict__ o_d) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nd) o_d[i] = fma(sig[i] + dw, dxd[i], o_d[i]);
}

// third block row (y): o_y = J dx - dc dy - dcv .* dy (o_y holds J dx on
// entry; dcv, the optional per-row diagonal, may be null)
__global__ void k_kkt_y(int m, double dc, const double *__restrict__ dcv,
                        const double *__restrict__ dy, double *__restrict__ o_y) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m) {
    double o = fma(-dc, dy[i], o_y[i]);
    if (dcv) o = fma(-dcv[i], dy[i], o);
    o_y[i] = o;
  }
}

// slot 0: max |a|, slot 1: max |b|, slot 2: max |c|  (infinity norms)
__global__ __launch_bounds__(RB) void k_red_amax3(int64_t na, const double *__restrict__ a,
                                                  int64_t nb, const double *__restrict__ b,
                                                  int64_t nc, const double *__restrict__ c,
                                                  double *__restrict__ red) {
  double v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  const int64_t stride = (int64_t)gridDim.x * RB;
  int64_t len = na > nb ? na : nb;
  len = len > nc ? len : nc;
  for (int64_t e = (int64_t)blockIdx.x * RB + threadIdx.x; e < len; e += stride) {
    if (e < na) v[0] = fmax(v[0], fabs(a[e]));
    if (e < nb) v[1] = fmax(v[1], fabs(b[e]));
    if (e < nc) v[2] = fmax(v[2], fabs(c[e]));
  }
  block_reduce8(v, red + (size_t)blockIdx.x * 8);
}

// ||K||_inf row sums (the operator norm used in the backward error):
// slot 0 over the x_d rows, slot 1 over the x_s rows, slot 2 over the y rows.
// colsum holds, per x_s column, sum_i |J_s(i,k)|; rowabs_d / rowabs_y the
// absolute row sums of the dense parts (computed by k_absrows).
__global__ __launch_bounds__(RB) void k_red_knorm(int nd, int ns, int m,
                                                  const double *__restrict__ hrow,
                                                  const double *__restrict__ sig, double dw,
                                                  const double *__restrict__ jdcol,
                                                  const double *__restrict__ dsb,
                                                  const double *__restrict__ jscol,
                                                  const double *__restrict__ yrow, double dc,
                                                  const double *__restrict__ dcv,
                                                  double *__restrict__ red) {
  double v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  const int64_t stride = (int64_t)gridDim.x * RB;
  int64_t len = nd > ns ? nd : ns;
  len = len > m ? len : m;
  for (int64_t e = (int64_t)blockIdx.x * RB + threadIdx.x; e < len; e += stride) {
    if (e < nd) v[0] = fmax(v[0], hrow[e] + jdcol[e]);
    if (e < ns) v[1] = fmax(v[1], fabs(dsb[e] + dw) + jscol[e]);
    if (e < m) v[2] = fmax(v[2], yrow[e] + fabs(dc) + (dcv ? fabs(dcv[e]) : 0.0));
  }
  (void)sig;
  block_reduce8(v, red + (size_t)blockIdx.x * 8);
}

// absolute row sums: x_d rows of [H + diag(sig + dw)], |J_d| column sums
// (x_d rows of J_d'), and y rows |J_d| + |J_s|; J_s column sums for x_s rows.
// Row sums of |H + diag(sig) + dw I|.  H is exactly symmetric (checked when
// the problem is set), so row i's sum is column i's: one wave per column,
// reading along the column.
__global__ void k_abs_hrow(int nd, const double *__restrict__ H, const double *__restrict__ sig,
                           double dw, double *__restrict__ out) {
  const int lane = threadIdx.x & 63;
  const int j = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (j >= nd) return;
  double t = 0.0;
  for (int i = lane; i < nd; i += 64) {
    double h = H[(size_t)i + (size_t)j * nd];
    if (i == j) h = h + sig[j] + dw;
    t += fabs(h);
  }
  t = wave_sum(t);
  if (lane == 0) out[j] = t;
}

__global__ void k_abs_jdcol(int m, int nd, const double *__restrict__ Jd,
                            double *__restrict__ out) {
  const int lane = threadIdx.x & 63;
  const int j = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (j >= nd) return;
  double s = 0.0;
  for (int i = lane; i < m; i += 64) s += fabs(Jd[(size_t)i + (size_t)j * m]);
  s = wave_sum(s);
  if (lane == 0) out[j] = s;
}

// Row sums of |[J_d J_s]|: 64 rows per block of 256 threads, the four waves
// take every fourth column, partials combined in wave order.
// 64 rows per workgroup, 16 waves, wave g summing the columns j = g mod 16
// (enough loads in flight for the row sums to stream J_d at memory speed),
// then the 16 partial sums combined in a fixed tree order
__global__ __launch_bounds__(1024) void k_abs_yrow(int m, int nd, const double *__restrict__ Jd,
                                                   const int32_t *__restrict__ rp,
                                                   const double *__restrict__ v,
                                                   double *__restrict__ out) {
  __shared__ double sh[16][64];
  const int lane = threadIdx.x & 63, g = threadIdx.x >> 6;
  const int i = blockIdx.x * 64 + lane;
  double t = 0.0;
  if (i < m)
    for (int j = g; j < nd; j += 16) t += fabs(Jd[(size_t)i + (size_t)j * m]);
  sh[g][lane] = t;
  __syncthreads();
  if (g == 0 && i < m) {
    double q[8];
#pragma unroll
    for (int a = 0; a < 8; ++a) q[a] = sh[2 * a][lane] + sh[2 * a + 1][lane];
    double u = ((q[0] + q[1]) + (q[2] + q[3])) + ((q[4] + q[5]) + (q[6] + q[7]));
    for (int a = rp[i]; a < rp[i + 1]; ++a) u += fabs(v[a]);
    out[i] = u;
  }
}

__global__ void k_abs_jscol(int ns, const int32_t *__restrict__ cptr,
                            const double *__restrict__ cval, double *__restrict__ out) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= ns) return;
  double t = 0.0;
  for (int e = cptr[k]; e < cptr[k + 1]; ++e) t += fabs(cval[e]);
  out[k] = t;
}

inline unsigned red_grid(int64_t len) {
  int64_t g = (len + RB - 1) / RB;
  if (g < 1) g = 1;
  if (g > kRedBlocks) g = kRedBlocks;
  return (unsigned)g;
}

}  // namespace

void ipm_init_point(hipStream_t s, int n, int m, const double *xl, const double *xu, double *x,
                    double *y, double *zl, double *zu) {
  const int len = n > m ? n : m;
  if (len <= 0) return;
  k_init_point<<<grid1(len, 256), 256, 0, s>>>(n, m, xl, xu, x, y, zl, zu);
}

void ipm_init_warm(hipStream_t s, int nd, int ns, int m, const double *xl, const double *xu,
                   const double *w, const double *g, const int32_t *cptr, const int32_t *crow,
                   const double *cval, const double *xd0, const double *y0, double mu0,
                   double *x, double *y, double *zl, double *zu) {
  const int len = (nd + ns) > m ? (nd + ns) : m;
  if (len <= 0) return;
  k_init_warm<<<grid1(len, 256), 256, 0, s>>>(nd, ns, m, xl, xu, w, g, cptr, crow, cval, xd0, y0,
                                              mu0, x, y, zl, zu);
}

void ipm_warm_duals(hipStream_t s, int n, const double *xl, const double *xu, const double *gf,
                    const double *jty, double *zl, double *zu) {
  if (n <= 0) return;
  k_warm_duals<<<grid1(n, 256), 256, 0, s>>>(n, xl, xu, gf, jty, zl, zu);
}

void ipm_grad_finish(hipStream_t s, int nd, int ns, const double *c, const double *w,
                     const double *g, const double *x, double *gf) {
  if (nd + ns <= 0) return;
  k_grad_finish<<<grid1(nd + ns, 256), 256, 0, s>>>(nd, ns, c, w, g, x, gf);
}

void ipm_sigma_rhs(hipStream_t s, int n, const double *x, const double *zl, const double *zu,
                   const double *xl, const double *xu, const double *gf, const double *jty,
                   double mu, double *sigma, double *rx) {
  if (n <= 0) return;
  k_sigma_rhs<<<grid1(n, 256), 256, 0, s>>>(n, x, zl, zu, xl, xu, gf, jty, mu, sigma, rx);
}

void ipm_constr_finish(hipStream_t s, int m, int mE, const double *b, const double *d,
                       double *cx, double *ry) {
  if (m <= 0) return;
  k_constr_finish<<<grid1(m, 256), 256, 0, s>>>(m, mE, b, d, cx, ry);
}

void ipm_slack_grad(hipStream_t s, int mI, int mE, const double *y, double *gf_t, double *jty_t) {
  if (mI <= 0) return;
  k_slack_grad<<<grid1(mI, 256), 256, 0, s>>>(mI, mE, y, gf_t, jty_t);
}

void ipm_slack_project(hipStream_t s, int mI, const double *hx, const double *hl,
                       const double *hu, double *d) {
  if (mI <= 0) return;
  k_slack_project<<<grid1(mI, 256), 256, 0, s>>>(mI, hx, hl, hu, d);
}

void ipm_slack_duals(hipStream_t s, int mI, const double *hl, const double *hu, const double *d,
                     double mu0, double *vl, double *vu) {
  if (mI <= 0) return;
  k_slack_duals<<<grid1(mI, 256), 256, 0, s>>>(mI, hl, hu, d, mu0, vl, vu);
}

void ipm_ineq_dcv(hipStream_t s, int m, int mE, const double *sig_h, double dw, double *dcv) {
  if (m <= 0) return;
  k_ineq_dcv<<<grid1(m, 256), 256, 0, s>>>(m, mE, sig_h, dw, dcv);
}

void ipm_ineq_rhs(hipStream_t s, int mI, int mE, const double *dcv, const double *rd,
                  double *ry) {
  if (mI <= 0) return;
  k_ineq_rhs<<<grid1(mI, 256), 256, 0, s>>>(mI, mE, dcv, rd, ry);
}

void ipm_ineq_step(hipStream_t s, int mI, int mE, const double *dcv, const double *rd,
                   const double *dy, double *dd) {
  if (mI <= 0) return;
  k_ineq_step<<<grid1(mI, 256), 256, 0, s>>>(mI, mE, dcv, rd, dy, dd);
}

void ipm_dsbase(hipStream_t s, int nd, int ns, const double *w, const double *sig, double *dsb) {
  if (ns <= 0) return;
  k_dsbase<<<grid1(ns, 256), 256, 0, s>>>(nd, ns, w, sig, dsb);
}

void ipm_dz(hipStream_t s, int n, const double *x, const double *zl, const double *zu,
            const double *xl, const double *xu, const double *dx, double mu, double *dzl,
            double *dzu) {
  if (n <= 0) return;
  k_dz<<<grid1(n, 256), 256, 0, s>>>(n, x, zl, zu, xl, xu, dx, mu, dzl, dzu);
}

void ipm_red_opt(hipStream_t s, int n, int m, const double *x, const double *y, const double *zl,
                 const double *zu, const double *xl, const double *xu, const double *gf,
                 const double *jty, const double *cx, double mu, double *red, double *out) {
  const unsigned g = red_grid(n > m ? n : m);
  k_red_opt<false><<<g, RB, 0, s>>>(n, m, x, y, zl, zu, xl, xu, gf, jty, cx, mu, red);
  k_red_final<<<1, 256, 0, s>>>((int)g, red, out);
}

void ipm_red_opt_pair(hipStream_t s, int n, int m, const double *x, const double *y,
                      const double *zl, const double *zu, const double *xl, const double *xu,
                      const double *gf, const double *jty, const double *cx, double mu,
                      double *red, double *out) {
  const unsigned g = red_grid(n > m ? n : m);
  k_red_opt<true><<<g, RB, 0, s>>>(n, m, x, y, zl, zu, xl, xu, gf, jty, cx, mu, red);
  k_red_final<<<1, 256, 0, s>>>((int)g, red, out);
}

void ipm_red_merit(hipStream_t s, int nd, int ns, int nx, int m, double mu, const double *x,
                   const double *hx, const double *c, const double *w, const double *g,
                   const double *wbx, const double *xl, const double *xu, const double *cx,
                   double *red, double *out) {
  const unsigned gr = red_grid(nx > m ? nx : m);
  k_red_merit<<<gr, RB, 0, s>>>(nd, ns, nx, m, mu, x, hx, c, w, g, wbx, xl, xu, cx, red);
  k_red_final<<<1, 256, 0, s>>>((int)gr, red, out);
}

void ipm_red_gphi(hipStream_t s, int n, const double *gf, const double *x, const double *xl,
                  const double *xu, const double *dx, double mu, double *red, double *out) {
  const unsigned g = red_grid(n);
  k_red_gphi<<<g, RB, 0, s>>>(n, gf, x, xl, xu, dx, mu, red);
  k_red_final<<<1, 256, 0, s>>>((int)g, red, out);
}

void ipm_red_ftb(hipStream_t s, int n, const double *x, const double *xl, const double *xu,
                 const double *dx, const double *zl, const double *zu, const double *dzl,
                 const double *dzu, double tau, double *red, double *out) {
  const unsigned g = red_grid(n);
  k_red_ftb<<<g, RB, 0, s>>>(n, x, xl, xu, dx, zl, zu, dzl, dzu, tau, red);
  k_red_final<<<1, 256, 0, s>>>((int)g, red, out);
}

void ipm_red_ftb1(hipStream_t s, int64_t n, const double *v, const double *dv, double tau,
                  double *red, double *out) {
  const unsigned g = red_grid(n);
  k_red_ftb1<<<g, RB, 0, s>>>(n, v, dv, tau, red);
  k_red_final<<<1, 256, 0, s>>>((int)g, red, out);
}

void ipm_ftb1_to_device(hipStream_t s, int64_t n, const double *v, const double *dv, double tau,
                        double *red, double *out, double *alpha) {
  ipm_red_ftb1(s, n, v, dv, tau, red, out);
  k_neg_first<<<1, 64, 0, s>>>(out, alpha);
}

void ipm_red_amax3(hipStream_t s, int64_t na, const double *a, int64_t nb, const double *b,
                   int64_t nc, const double *c, double *red, double *out) {
  int64_t len = na > nb ? na : nb;
  len = len > nc ? len : nc;
  const unsigned g = red_grid(len);
  k_red_amax3<<<g, RB, 0, s>>>(na, a, nb, b, nc, c, red);
  k_red_final<<<1, 256, 0, s>>>((int)g, red, out);
}

void ipm_axpy_to(hipStream_t s, int n, const double *x, const double *dx, double a, double *out) {
  if (n <= 0) return;
  k_axpy_to<<<grid1(n, 256), 256, 0, s>>>(n, x, dx, a, out);
}

void ipm_accept(hipStream_t s, int n, int m, const double *xt, double *x, double *y,
                const double *dy, double *zl, double *zu, const double *dzl, const double *dzu,
                const double *xl, const double *xu, double alpha, double alpha_z, double mu) {
  const int len = n > m ? n : m;
  if (len <= 0) return;
  k_accept<<<grid1(len, 256), 256, 0, s>>>(n, m, xt, x, y, dy, zl, zu, dzl, dzu, xl, xu, alpha,
                                           alpha_z, mu);
}

void vec_copy(hipStream_t s, int64_t n, const double *src, double *dst) {
  if (n <= 0) return;
  k_copy_scaled<<<grid1(n, 256), 256, 0, s>>>(n, src, dst);
}

void vec_sub(hipStream_t s, int64_t n, const double *a, const double *b, double *out) {
  if (n <= 0) return;
  k_sub<<<grid1(n, 256), 256, 0, s>>>(n, a, b, out);
}

void vec_add_inplace(hipStream_t s, int64_t n, const double *a, double *out) {
  if (n <= 0) return;
  k_add_inplace<<<grid1(n, 256), 256, 0, s>>>(n, a, out);
}

__global__ void k_check_nonneg(int64_t n, const double *__restrict__ v, int32_t *bad) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && !(v[i] >= 0.0 && v[i] < INFINITY)) atomicOr(bad, 1);
}

void check_nonneg(hipStream_t s, int64_t n, const double *v, int32_t *bad) {
  if (n > 0) k_check_nonneg<<<grid1(n, 256), 256, 0, s>>>(n, v, bad);
}

// inequality bounds (eq. (ineq)): hl < hu, no NaN, at least one finite
__global__ void k_check_ineq_bounds(int mI, const double *__restrict__ hl,
                                    const double *__restrict__ hu, int32_t *bad) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= mI) return;
  const double l = hl[r], u = hu[r];
  if (!(l < u) || (!isfinite(l) && !isfinite(u))) atomicOr(bad, 1);
}

void check_ineq_bounds(hipStream_t s, int mI, const double *hl, const double *hu, int32_t *bad) {
  if (mI > 0) k_check_ineq_bounds<<<grid1(mI, 256), 256, 0, s>>>(mI, hl, hu, bad);
}

void kkt_finish(hipStream_t s, int nd, int ns, int m, const double *sig, const double *dsb,
                double dw, double dc, const double *dcv, const double *dxd, const double *dxs,
                const double *dy, double *od, double *os, double *oy) {
  if (nd > 0) k_kkt_d<<<grid1(nd, 256), 256, 0, s>>>(nd, sig, dw, dxd, od);
  if (ns > 0) k_kkt_s<<<grid1(ns, 256), 256, 0, s>>>(ns, dsb, dw, dxs, os);
  if (m > 0) k_kkt_y<<<grid1(m, 256), 256, 0, s>>>(m, dc, dcv, dy, oy);
}

void kkt_norm_parts(hipStream_t s, int nd, int ns, int m, const double *H, const double *sig,
                    double dw, const double *Jd, const int32_t *rp, const double *v,
                    const int32_t *cptr, const double *cval, const double *dsb, double dc,
                    const double *dcv, double *hrow, double *jdcol, double *yrow, double *jscol,
                    double *red, double *out, const SBlk *sb) {
  if (nd > 0) {
    k_abs_hrow<<<grid1(nd, 4), 256, 0, s>>>(nd, H, sig, dw, hrow);
    k_abs_jdcol<<<grid1(nd, 4), 256, 0, s>>>(m, nd, Jd, jdcol);
  }
  if (m > 0) k_abs_yrow<<<grid1(m, 64), 1024, 0, s>>>(m, nd, Jd, rp, v, yrow);
  if (ns > 0) k_abs_jscol<<<grid1(ns, 256), 256, 0, s>>>(ns, cptr, cval, jscol);
  if (sb && sb->nblk > 0 && ns > 0) {
    // coupling blocks: their off-diagonal row sums join J_s's column sums,
    // their diagonal joins dsbase
    sblk_absrow(s, *sb, ns, dsb, jscol, sb->tmp2);
    dsb = sb->tmp2;
  }
  int64_t len = nd > ns ? nd : ns;
  len = len > m ? len : m;
  const unsigned g = red_grid(len);
  k_red_knorm<<<g, RB, 0, s>>>(nd, ns, m, hrow, sig, dw, jdcol, dsb, jscol, yrow, dc, dcv, red);
  k_red_final<<<1, 256, 0, s>>>((int)g, red, out);
}

}  // namespace mds
