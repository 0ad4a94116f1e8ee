// A built-in model of the general-NLP interface (mds_nlp_model): the
// separable nonlinear family on an MDS problem's data, for tests and the
// benchmark.  The model objects of Sec. 2 are the modeling layer's (the end
// of Sec. 2.3); this one keeps A1 (no x_d / x_s cross terms) and A2 (a
// nonnegative diagonal sparse Hessian):
//   f(x)   = 0.5 x_d'H x_d + c'x_d + sum_k (0.5 w_k x_k^2 + g_k x_k
//            + e_k (exp(x_k) - x_k))                       (x_k = x_s,k)
//   row r  = (J_d x_d)_r + (J_s x_s)_r + sum_j Q_rj x_d,j^2 (- b_r on the
//            equality rows)
// so J_d(x) = J_d + 2 Q diag(x_d), J_s is constant, and the Hessian of
// f + y'c is H + diag(2 Q'y) on the dense block and w + e exp(x_s) on the
// sparse one.
#include <new>

#include "internal.hpp"
#include "vec.hpp"

struct mds_sep_model {
  hipStream_t stream = nullptr;
  int nd = 0, ns = 0, m = 0, mE = 0;
  int64_t nnz = 0;
  const double *H = nullptr, *c = nullptr, *w = nullptr, *g = nullptr, *Jd = nullptr;
  const double *Jsv = nullptr, *b = nullptr, *Q = nullptr, *e = nullptr;
  const int32_t *rp = nullptr, *ci = nullptr;
  double *red = nullptr;  // kRedBlocks * 8 partial sums, then 8 final
};

namespace mds {
namespace {

constexpr int RB = 256;
inline unsigned grid1(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

// partial sums of f: slot 4 of one 8-slot record per workgroup
__global__ __launch_bounds__(RB) void k_sep_f(int nd, int ns, const double *__restrict__ H,
                                              const double *__restrict__ c,
                                              const double *__restrict__ w,
                                              const double *__restrict__ g,
                                              const double *__restrict__ e,
                                              const double *__restrict__ x,
                                              double *__restrict__ red) {
  double v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  const int n = nd + ns;
  for (int i = blockIdx.x * RB + threadIdx.x; i < n; i += gridDim.x * RB) {
    if (i < nd) {
      double t = 0.0;
      for (int j = 0; j < nd; ++j) t = t + H[(size_t)i + (size_t)j * nd] * x[j];
      v[4] += x[i] * (0.5 * t + c[i]);
    } else {
      const int k = i - nd;
      const double xs = x[i];
      v[4] += xs * (0.5 * w[k] * xs + g[k]) + e[k] * (exp(xs) - xs);
    }
  }
  block_reduce8(v, red + (size_t)blockIdx.x * 8);
}

__global__ void k_sep_f_final(int nb, const double *__restrict__ red, double *__restrict__ out) {
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int b = 0; b < nb; ++b) t = t + red[(size_t)b * 8 + 4];
    out[0] = t;
  }
}

__global__ void k_sep_grad(int nd, int ns, const double *__restrict__ H,
                           const double *__restrict__ c, const double *__restrict__ w,
                           const double *__restrict__ g, const double *__restrict__ e,
                           const double *__restrict__ x, double *__restrict__ gf) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nd) {
    double t = 0.0;
    for (int j = 0; j < nd; ++j) t = t + H[(size_t)i + (size_t)j * nd] * x[j];
    gf[i] = t + c[i];
  } else if (i < nd + ns) {
    const int k = i - nd;
    gf[i] = w[k] * x[i] + g[k] + e[k] * (exp(x[i]) - 1.0);
  }
}

__global__ void k_sep_cons(int nd, int m, int mE, const double *__restrict__ Jd,
                           const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                           const double *__restrict__ v, const double *__restrict__ Q,
                           const double *__restrict__ b, const double *__restrict__ x,
                           double *__restrict__ out) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= m) return;
  double t = 0.0;
  for (int j = 0; j < nd; ++j) t = t + Jd[(size_t)r + (size_t)j * m] * x[j];
  for (int a = rp[r]; a < rp[r + 1]; ++a) t = t + v[a] * x[nd + ci[a]];
  for (int j = 0; j < nd; ++j) t = t + Q[(size_t)r + (size_t)j * m] * (x[j] * x[j]);
  out[r] = (r < mE) ? t - b[r] : t;
}

__global__ void k_sep_jac(int nd, int m, int64_t nnz, const double *__restrict__ Jd0,
                          const double *__restrict__ Q, const double *__restrict__ v0,
                          const double *__restrict__ x, double *__restrict__ Jd,
                          double *__restrict__ v) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t md = (int64_t)m * nd;
  if (e < md) {
    const int j = (int)(e / m);
    Jd[e] = Jd0[e] + 2.0 * Q[e] * x[j];
  } else if (e < md + nnz) {
    v[e - md] = v0[e - md];
  }
}

// dense block: H + diag(sum_r y_r 2 Q_rj) (column j of H per thread block
// row); sparse block: w + e exp(x_s)
__global__ void k_sep_hess(int nd, int ns, int m, const double *__restrict__ H0,
                           const double *__restrict__ Q, const double *__restrict__ w0,
                           const double *__restrict__ e, const double *__restrict__ x,
                           const double *__restrict__ y, double *__restrict__ H,
                           double *__restrict__ w) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t dd = (int64_t)nd * nd;
  if (t < dd) {
    const int i = (int)(t % nd), j = (int)(t / nd);
    double h = H0[t];
    if (i == j) {
      double s = 0.0;
      for (int r = 0; r < m; ++r) s = s + y[r] * (2.0 * Q[(size_t)r + (size_t)j * m]);
      h = h + s;
    }
    H[t] = h;
  } else if (t < dd + ns) {
    const int k = (int)(t - dd);
    w[k] = w0[k] + e[k] * exp(x[nd + k]);
  }
}

int sep_objective(void *ctx, const double *x, double *f_host) {
  mds_sep_model *M = static_cast<mds_sep_model *>(ctx);
  const int64_t n = (int64_t)M->nd + M->ns;
  unsigned nb = grid1(n > 0 ? n : 1, RB);
  if (nb > (unsigned)kRedBlocks) nb = kRedBlocks;
  k_sep_f<<<nb, RB, 0, M->stream>>>(M->nd, M->ns, M->H, M->c, M->w, M->g, M->e, x, M->red);
  k_sep_f_final<<<1, 64, 0, M->stream>>>((int)nb, M->red, M->red + (size_t)kRedBlocks * 8);
  if (hipMemcpyAsync(f_host, M->red + (size_t)kRedBlocks * 8, 8, hipMemcpyDeviceToHost,
                     M->stream) != hipSuccess ||
      hipStreamSynchronize(M->stream) != hipSuccess)
    return 1;
  return 0;
}

int sep_gradient(void *ctx, const double *x, double *g) {
  mds_sep_model *M = static_cast<mds_sep_model *>(ctx);
  const int n = M->nd + M->ns;
  if (n > 0) k_sep_grad<<<grid1(n, 256), 256, 0, M->stream>>>(M->nd, M->ns, M->H, M->c, M->w,
                                                                M->g, M->e, x, g);
  return hipGetLastError() == hipSuccess ? 0 : 1;
}

int sep_constraints(void *ctx, const double *x, double *c) {
  mds_sep_model *M = static_cast<mds_sep_model *>(ctx);
  if (M->m > 0)
    k_sep_cons<<<grid1(M->m, 256), 256, 0, M->stream>>>(M->nd, M->m, M->mE, M->Jd, M->rp, M->ci,
                                                         M->Jsv, M->Q, M->b, x, c);
  return hipGetLastError() == hipSuccess ? 0 : 1;
}

int sep_jacobian(void *ctx, const double *x, double *Jd, double *v) {
  mds_sep_model *M = static_cast<mds_sep_model *>(ctx);
  const int64_t tot = (int64_t)M->m * M->nd + M->nnz;
  if (tot > 0)
    k_sep_jac<<<grid1(tot, 256), 256, 0, M->stream>>>(M->nd, M->m, M->nnz, M->Jd, M->Q, M->Jsv,
                                                       x, Jd, v);
  return hipGetLastError() == hipSuccess ? 0 : 1;
}

int sep_hessian(void *ctx, const double *x, const double *y, double *H, double *w) {
  mds_sep_model *M = static_cast<mds_sep_model *>(ctx);
  const int64_t tot = (int64_t)M->nd * M->nd + M->ns;
  if (tot > 0)
    k_sep_hess<<<grid1(tot, 256), 256, 0, M->stream>>>(M->nd, M->ns, M->m, M->H, M->Q, M->w,
                                                        M->e, x, y, H, w);
  return hipGetLastError() == hipSuccess ? 0 : 1;
}

// ---- helpers of the IPM's NLP mode -------------------------------------------
__global__ void k_gather_i(int64_t n, const int32_t *__restrict__ map, const double *__restrict__ src,
                           double *__restrict__ dst) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q < n) dst[q] = src[map[q]];
}

// out = a * u + v (out may be u or v)
__global__ void k_axpby(int n, double a, const double *u, const double *v, double *out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = a * u[i] + v[i];
}

// restoration: x_R = x, D_R = min(1, 1 / |x|)
__global__ void k_resto_init(int n, const double *__restrict__ x, double *__restrict__ xr,
                             double *__restrict__ dr) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    xr[i] = x[i];
    dr[i] = fmin(1.0, 1.0 / fabs(x[i]));
  }
}

// restoration Hessian: H = diag(zeta D_R,d^2), w = zeta D_R,s^2
__global__ void k_resto_hess(int nd, int ns, double zeta, const double *__restrict__ dr,
                             double *__restrict__ H, double *__restrict__ w) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t dd = (int64_t)nd * nd;
  if (t < dd) {
    const int i = (int)(t % nd), j = (int)(t / nd);
    H[t] = (i == j) ? zeta * dr[i] * dr[i] : 0.0;
  } else if (t < dd + ns) {
    const int k = (int)(t - dd);
    w[k] = zeta * dr[nd + k] * dr[nd + k];
  }
}

// restoration Newton system over [x; d]: bound multipliers centred at
// mu / slack, Sigma = sum (mu / s) / s, r_x = -(zeta D_R^2 (x - x_R) + J'y
// - mu / (x - l) + mu / (u - x))
__global__ void k_resto_rhs(int n, double zeta, double mu, const double *__restrict__ x,
                            const double *__restrict__ xr, const double *__restrict__ dr,
                            const double *__restrict__ jty, const double *__restrict__ xl,
                            const double *__restrict__ xu, double *__restrict__ sig,
                            double *__restrict__ rx, double *__restrict__ zl,
                            double *__restrict__ zu) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = 0.0, gb = zeta * dr[i] * dr[i] * (x[i] - xr[i]) + jty[i];
  double a = 0.0, b = 0.0;
  if (isfinite(xl[i])) {
    const double sl = x[i] - xl[i];
    s = s + (mu / sl) / sl;
    gb = gb - mu / sl;
    a = mu / sl;
  }
  if (isfinite(xu[i])) {
    const double su = xu[i] - x[i];
    s = s + (mu / su) / su;
    gb = gb + mu / su;
    b = mu / su;
  }
  sig[i] = s;
  rx[i] = -gb;
  zl[i] = a;
  zu[i] = b;
}

// bound multipliers centred at mu / slack (0 on infinite bounds)
__global__ void k_center_z(int n, double mu, const double *__restrict__ x,
                           const double *__restrict__ xl, const double *__restrict__ xu,
                           double *__restrict__ zl, double *__restrict__ zu) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  zl[i] = isfinite(xl[i]) ? mu / (x[i] - xl[i]) : 0.0;
  zu[i] = isfinite(xu[i]) ? mu / (xu[i] - x[i]) : 0.0;
}

// flag = 1 when an entry of w is negative or NaN
__global__ void k_check_nonneg(int n, const double *__restrict__ w, int32_t *__restrict__ flag) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && !(w[i] >= 0.0)) atomicOr(flag, 1);
}

}  // namespace

void nlp_check_nonneg(hipStream_t s, int n, const double *w, int32_t *flag) {
  if (n > 0) k_check_nonneg<<<grid1(n, 256), 256, 0, s>>>(n, w, flag);
}
void nlp_gather(hipStream_t s, int64_t n, const int32_t *map, const double *src, double *dst) {
  if (n > 0) k_gather_i<<<grid1(n, 256), 256, 0, s>>>(n, map, src, dst);
}
void nlp_axpby(hipStream_t s, int n, double a, const double *u, const double *v, double *out) {
  if (n > 0) k_axpby<<<grid1(n, 256), 256, 0, s>>>(n, a, u, v, out);
}
void nlp_resto_init(hipStream_t s, int n, const double *x, double *xr, double *dr) {
  if (n > 0) k_resto_init<<<grid1(n, 256), 256, 0, s>>>(n, x, xr, dr);
}
void nlp_resto_hess(hipStream_t s, int nd, int ns, double zeta, const double *dr, double *H,
                    double *w) {
  const int64_t t = (int64_t)nd * nd + ns;
  if (t > 0) k_resto_hess<<<grid1(t, 256), 256, 0, s>>>(nd, ns, zeta, dr, H, w);
}
void nlp_resto_rhs(hipStream_t s, int n, double zeta, double mu, const double *x, const double *xr,
                   const double *dr, const double *jty, const double *xl, const double *xu,
                   double *sig, double *rx, double *zl, double *zu) {
  if (n > 0)
    k_resto_rhs<<<grid1(n, 256), 256, 0, s>>>(n, zeta, mu, x, xr, dr, jty, xl, xu, sig, rx, zl, zu);
}
void nlp_center_z(hipStream_t s, int n, double mu, const double *x, const double *xl,
                  const double *xu, double *zl, double *zu) {
  if (n > 0) k_center_z<<<grid1(n, 256), 256, 0, s>>>(n, mu, x, xl, xu, zl, zu);
}

}  // namespace mds

extern "C" {

size_t mds_sep_model_workspace_bytes(void) {
  return 8 * ((size_t)mds::kRedBlocks * 8 + 8);
}

int mds_sep_model_create(mds_sep_model **out, const mds_dims *dims, const mds_problem *p,
                         const double *Q, const double *e, void *stream, void *workspace,
                         size_t bytes, mds_nlp_model *model_out) {
  if (!out || !dims || !p || !model_out || !workspace) return MDS_ENULL;
  *out = nullptr;
  if (dims->n_d < 0 || dims->n_s < 0 || dims->m < 0 || dims->m_I < 0 || dims->m_I > dims->m)
    return MDS_EDIMS;
  if (bytes < mds_sep_model_workspace_bytes() || ((uintptr_t)workspace & 255) != 0)
    return MDS_EWORKSPACE;
  if ((dims->n_d > 0 && (!p->H || !p->c)) || (dims->n_s > 0 && (!p->w || !p->g || !e)) ||
      (dims->m > 0 && dims->n_d > 0 && (!p->J_d || !Q)) || !p->Js_rowptr ||
      (dims->nnz_s > 0 && (!p->Js_col || !p->Js_val)) || (dims->m - dims->m_I > 0 && !p->b))
    return MDS_ENULL;
  mds_sep_model *M = new (std::nothrow) mds_sep_model();
  if (!M) return MDS_EINVAL;
  M->stream = (hipStream_t)stream;
  M->nd = dims->n_d;
  M->ns = dims->n_s;
  M->m = dims->m;
  M->mE = dims->m - dims->m_I;
  M->nnz = dims->nnz_s;
  M->H = p->H;
  M->c = p->c;
  M->w = p->w;
  M->g = p->g;
  M->Jd = p->J_d;
  M->Jsv = p->Js_val;
  M->b = p->b;
  M->rp = p->Js_rowptr;
  M->ci = p->Js_col;
  M->Q = Q;
  M->e = e;
  M->red = (double *)workspace;
  model_out->ctx = M;
  model_out->objective = mds::sep_objective;
  model_out->gradient = mds::sep_gradient;
  model_out->constraints = mds::sep_constraints;
  model_out->jacobian = mds::sep_jacobian;
  model_out->hessian = mds::sep_hessian;
  *out = M;
  return MDS_OK;
}

void mds_sep_model_destroy(mds_sep_model *M) { delete M; }

}  // extern "C"
