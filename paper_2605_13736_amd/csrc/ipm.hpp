// Launchers of the IPM vector kernels (ipm.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "internal.hpp"

namespace mds {

void ipm_init_point(hipStream_t s, int n, int m, const double *xl, const double *xu, double *x,
                    double *y, double *zl, double *zu);
void ipm_init_warm(hipStream_t s, int nd, int ns, int m, const double *xl, const double *xu,
                   const double *w, const double *g, const int32_t *cptr, const int32_t *crow,
                   const double *cval, const double *xd0, const double *y0, double mu0,
                   double *x, double *y, double *zl, double *zu);
// zl, zu += the bound-carried parts of r = gf + jty (warm start)
void ipm_warm_duals(hipStream_t s, int n, const double *xl, const double *xu, const double *gf,
                    const double *jty, double *zl, double *zu);
void ipm_grad_finish(hipStream_t s, int nd, int ns, const double *c, const double *w,
                     const double *g, const double *x, double *gf);
void ipm_sigma_rhs(hipStream_t s, int n, const double *x, const double *zl, const double *zu,
                   const double *xl, const double *xu, const double *gf, const double *jty,
                   double mu, double *sigma, double *rx);
// cx: J x on entry, c = J x - [b; d] on exit; ry (may be null) = -c
void ipm_constr_finish(hipStream_t s, int m, int mE, const double *b, const double *d,
                       double *cx, double *ry);
// inequality slacks: gradient entries (gf = 0, J'y = -y_h; y may be null),
// start value (row value pushed inside [hl, hu]), the (4,4) diagonal
// dcv = 1/(Sigma_h + dw) (0 on the mE equality rows), the rhs update
// r_y,h += dcv .* r_d and the slack step dd = dcv .* (r_d + dy_h)
void ipm_slack_grad(hipStream_t s, int mI, int mE, const double *y, double *gf_t, double *jty_t);
void ipm_slack_project(hipStream_t s, int mI, const double *hx, const double *hl,
                       const double *hu, double *d);
void ipm_slack_duals(hipStream_t s, int mI, const double *hl, const double *hu, const double *d,
                     double mu0, double *vl, double *vu);
void ipm_ineq_dcv(hipStream_t s, int m, int mE, const double *sig_h, double dw, double *dcv);
void ipm_ineq_rhs(hipStream_t s, int mI, int mE, const double *dcv, const double *rd,
                  double *ry);
void ipm_ineq_step(hipStream_t s, int mI, int mE, const double *dcv, const double *rd,
                   const double *dy, double *dd);
void ipm_dsbase(hipStream_t s, int nd, int ns, const double *w, const double *sig, double *dsb);
void ipm_dz(hipStream_t s, int n, const double *x, const double *zl, const double *zu,
            const double *xl, const double *xu, const double *dx, double mu, double *dzl,
            double *dzu);
void ipm_red_opt(hipStream_t s, int n, int m, const double *x, const double *y, const double *zl,
                 const double *zu, const double *xl, const double *xu, const double *gf,
                 const double *jty, const double *cx, double mu, double *red, double *out);
// as ipm_red_opt, but slot 2 holds max(lower, upper) complementarity at mu
// and slot 3 the same at mu = 0
void ipm_red_opt_pair(hipStream_t s, int n, int m, const double *x, const double *y, const double *zl,
                 const double *zu, const double *xl, const double *xu, const double *gf,
                 const double *jty, const double *cx, double mu, double *red, double *out);
// wbx (may be null): blockdiag(Wb) x_s, the coupling blocks' part of the
// sparse Hessian times x_s
void ipm_red_merit(hipStream_t s, int nd, int ns, int nx, int m, double mu, const double *x,
                   const double *hx, const double *c, const double *w, const double *g,
                   const double *wbx, const double *xl, const double *xu, const double *cx,
                   double *red, double *out);
void ipm_red_gphi(hipStream_t s, int n, const double *gf, const double *x, const double *xl,
                  const double *xu, const double *dx, double mu, double *red, double *out);
void ipm_red_ftb(hipStream_t s, int n, const double *x, const double *xl, const double *xu,
                 const double *dx, const double *zl, const double *zu, const double *dzl,
                 const double *dzu, double tau, double *red, double *out);
void ipm_red_ftb1(hipStream_t s, int64_t n, const double *v, const double *dv, double tau,
                  double *red, double *out);
// ipm_red_ftb1, then alpha[0] (device) = the step; red holds kRedBlocks
// records of 8 doubles and out 8 doubles, written before they are read
void ipm_ftb1_to_device(hipStream_t s, int64_t n, const double *v, const double *dv, double tau,
                        double *red, double *out, double *alpha);
void ipm_red_amax3(hipStream_t s, int64_t na, const double *a, int64_t nb, const double *b,
                   int64_t nc, const double *c, double *red, double *out);
void ipm_axpy_to(hipStream_t s, int n, const double *x, const double *dx, double a, double *out);
void ipm_accept(hipStream_t s, int n, int m, const double *xt, double *x, double *y,
                const double *dy, double *zl, double *zu, const double *dzl, const double *dzu,
                const double *xl, const double *xu, double alpha, double alpha_z, double mu);
void vec_copy(hipStream_t s, int64_t n, const double *src, double *dst);
void vec_sub(hipStream_t s, int64_t n, const double *a, const double *b, double *out);
void vec_add_inplace(hipStream_t s, int64_t n, const double *a, double *out);
void kkt_finish(hipStream_t s, int nd, int ns, int m, const double *sig, const double *dsb,
                double dw, double dc, const double *dcv, const double *dxd, const double *dxs,
                const double *dy, double *od, double *os, double *oy);
// *bad |= 1 when some v[i] is negative or not finite
void check_nonneg(hipStream_t s, int64_t n, const double *v, int32_t *bad);
// *bad |= 1 unless hl < hu with at least one of them finite, for every row
void check_ineq_bounds(hipStream_t s, int mI, const double *hl, const double *hu, int32_t *bad);
void kkt_norm_parts(hipStream_t s, int nd, int ns, int m, const double *H, const double *sig,
                    double dw, const double *Jd, const int32_t *rp, const double *v,
                    const int32_t *cptr, const double *cval, const double *dsb, double dc,
                    const double *dcv, double *hrow, double *jdcol, double *yrow, double *jscol,
                    double *red, double *out, const SBlk *sb);

}  // namespace mds
