/*
 * cpc_oracle.c — plain FP64 CPU oracle for the partition-and-combine
 * maximum-pseudo-likelihood (MPL) copula estimator of Wei, Kim & Conlon,
 * "Parallel Computing for Copula Parameter Estimation with Big Data:
 * A Simulation Study" (arXiv:1609.05530).
 *
 * TEST INFRASTRUCTURE. This file is the reference the GPU library is checked
 * against. Only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg may load it; the product path never does. It shares no
 * code with the GPU library and deliberately uses different algorithms:
 *   - ranks by a comparison sort (qsort) instead of a radix sort;
 *   - the normal quantile by safeguarded Newton on libm erfc instead of a
 *     rational approximation;
 *   - every derivative of the log density by forward-mode automatic
 *     differentiation (hyper-dual numbers) of ONE written-out log density per
 *     family, instead of hand-derived derivative formulas;
 *   - the maximiser by a 65-point grid, uniform in Kendall's tau, followed by
 *     a bracketed Newton polish, instead of a Spearman-started Newton solve.
 * Everything is IEEE double, no fast-math.
 *
 * Paper map (section / equation of arXiv:1609.05530):
 *   eq. (5)              density as the mixed partial of the copula
 *   eq. (8), (10), (11)  Gaussian, Frank, Gumbel copulas
 *   eq. (12)             normalised ranks u = r / (N + 1)
 *   eq. (13)             pseudo log-likelihood, maximised numerically (Sec. 2.3)
 *   Sec. 2.3             asymptotic variance after Genest, Ghoudi & Rivest (1995)
 *   eq. (14)             partition of the rows into M disjoint subsets
 *   eq. (15), (16)       inverse-variance weighted combination
 */
#include "cpc_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* ------------------------------------------------------------------------ */
/* Hyper-dual numbers: x = v + d1*e1 + d2*e2 + d12*e1*e2 with e1^2 = e2^2 = 0.
 * Evaluating f on (theta + e1, ...) and (... + e2) gives f, df/da, df/db and
 * d2f/da db exactly (up to rounding), so every derivative the method needs is
 * the derivative of the same written-out log density.                       */
typedef struct { double v, d1, d2, d12; } hd;

static hd hd_c(double c) { hd r = {c, 0.0, 0.0, 0.0}; return r; }
static hd hd_add(hd a, hd b) { hd r = {a.v + b.v, a.d1 + b.d1, a.d2 + b.d2, a.d12 + b.d12}; return r; }
static hd hd_sub(hd a, hd b) { hd r = {a.v - b.v, a.d1 - b.d1, a.d2 - b.d2, a.d12 - b.d12}; return r; }
static hd hd_neg(hd a) { hd r = {-a.v, -a.d1, -a.d2, -a.d12}; return r; }
static hd hd_scale(hd a, double s) { hd r = {a.v * s, a.d1 * s, a.d2 * s, a.d12 * s}; return r; }
static hd hd_addc(hd a, double c) { a.v += c; return a; }
static hd hd_mul(hd a, hd b) {
  hd r;
  r.v = a.v * b.v;
  r.d1 = a.d1 * b.v + a.v * b.d1;
  r.d2 = a.d2 * b.v + a.v * b.d2;
  r.d12 = a.d12 * b.v + a.d1 * b.d2 + a.d2 * b.d1 + a.v * b.d12;
  return r;
}
/* chain rule for a scalar function with value f, first and second derivative */
static hd hd_chain(hd a, double f, double fp, double fpp) {
  hd r;
  r.v = f;
  r.d1 = fp * a.d1;
  r.d2 = fp * a.d2;
  r.d12 = fp * a.d12 + fpp * a.d1 * a.d2;
  return r;
}
static hd hd_exp(hd a) { double e = exp(a.v); return hd_chain(a, e, e, e); }
static hd hd_expm1(hd a) { double e = exp(a.v); return hd_chain(a, expm1(a.v), e, e); }
static hd hd_log(hd a) { return hd_chain(a, log(a.v), 1.0 / a.v, -1.0 / (a.v * a.v)); }
static hd hd_log1p(hd a) {
  double w = 1.0 + a.v;
  return hd_chain(a, log1p(a.v), 1.0 / w, -1.0 / (w * w));
}
static hd hd_inv(hd a) {
  double i = 1.0 / a.v;
  return hd_chain(a, i, -i * i, 2.0 * i * i * i);
}
static hd hd_div(hd a, hd b) { return hd_mul(a, hd_inv(b)); }
static hd hd_sqr(hd a) { return hd_mul(a, a); }

/* ------------------------------------------------------------------------ */
/* Standard normal quantile (needed by eq. (8): z = Phi^{-1}(u)).
 * Safeguarded Newton on Phi(z) = 0.5 erfc(-z/sqrt 2), computed from the
 * smaller of p and 1-p so the tail keeps full relative accuracy.            */
static double phi_pdf(double z) { return exp(-0.5 * z * z) / sqrt(2.0 * M_PI); }
static double Phi_cdf(double z) { return 0.5 * erfc(-z / sqrt(2.0)); }

double or_qnorm(double p, double omp) {
  if (!(p > 0.0)) return -INFINITY;
  if (!(omp > 0.0)) return INFINITY;
  if (p == omp) return 0.0;
  if (p > omp) return -or_qnorm(omp, p); /* Phi^{-1}(p) = -Phi^{-1}(1-p) */
  /* here p < 1/2 so z < 0, where Phi is convex and increasing */
  double lo = -40.0, hi = 0.0;
  double z = -sqrt(-2.0 * log(p));
  if (!(z > lo && z < hi)) z = 0.5 * (lo + hi);
  for (int it = 0; it < 200; ++it) {
    double f = Phi_cdf(z) - p;
    if (f > 0.0) hi = z; else lo = z;
    double zn = z - f / phi_pdf(z);
    if (!(zn > lo && zn < hi)) zn = 0.5 * (lo + hi);
    double dz = fabs(zn - z);
    z = zn;
    if (dz <= 2e-16 * fabs(z) || hi - lo <= 2e-16 * fabs(z)) break;
  }
  return z;
}

/* z = Phi^{-1}(p) as a hyper-dual: dz/dp = 1/phi(z), d2z/dp2 = z/phi(z)^2 */
static hd hd_qnorm(hd p, hd omp) {
  double z = or_qnorm(p.v, omp.v);
  double ph = phi_pdf(z);
  return hd_chain(p, z, 1.0 / ph, z / (ph * ph));
}

/* ------------------------------------------------------------------------ */
/* Log copula densities, eq. (5) applied to eq. (8), (10), (11).
 * Arguments carry u and 1-u (and v, 1-v) separately: both are exact
 * rationals of the integer ranks, and 1-u near 1 would lose digits.        */

/* Gaussian, eq. (8): the bivariate normal density with correlation rho divided
 * by the product of its standard normal margins, at z_j = Phi^{-1}(u_j). */
static hd logc_gaussian(hd rho, hd u, hd omu, hd v, hd omv) {
  hd z1 = hd_qnorm(u, omu), z2 = hd_qnorm(v, omv);
  hd one_m_r2 = hd_mul(hd_addc(hd_neg(rho), 1.0), hd_addc(rho, 1.0)); /* (1-rho)(1+rho) */
  hd quad = hd_sub(hd_mul(hd_sqr(rho), hd_add(hd_sqr(z1), hd_sqr(z2))),
                   hd_scale(hd_mul(rho, hd_mul(z1, z2)), 2.0));
  return hd_sub(hd_scale(hd_log(one_m_r2), -0.5), hd_div(quad, hd_scale(one_m_r2, 2.0)));
}

/* Frank, eq. (10). Its mixed partial is
 *   c = theta (1 - e^-theta) e^{-theta(u+v)} / D^2,
 *   D = (1 - e^-theta) - (1 - e^{-theta u})(1 - e^{-theta v}).
 * For theta > 0 the same D is a(1-b) + b(1 - e^{-theta(1-v)}) with
 * a = e^{-theta u}, b = e^{-theta v}: a sum of positive terms (no cancellation).
 * Negative theta uses c(u, v; theta) = c(u, 1-v; -theta). Near theta = 0 the
 * density tends to 1 (independence); there the Taylor series in theta is used. */
static hd logc_frank_series(hd th, hd u, hd omu, hd v, hd omv) {
  hd A = hd_mul(u, omu), B = hd_mul(v, omv); /* u(1-u), v(1-v) */
  hd su = hd_sub(u, omu), sv = hd_sub(v, omv); /* 2u-1, 2v-1 */
  hd AB = hd_mul(A, B);
  hd c1 = hd_scale(hd_mul(su, sv), 0.5);
  hd c2 = hd_addc(AB, -1.0 / 24.0);
  hd c3 = hd_scale(hd_mul(AB, hd_mul(su, sv)), 1.0 / 6.0);
  hd c4 = hd_addc(hd_sub(hd_scale(hd_sqr(AB), 0.5), hd_scale(hd_mul(AB, hd_add(A, B)), 1.0 / 12.0)),
                  1.0 / 2880.0);
  hd c5 = hd_scale(hd_mul(hd_mul(AB, hd_mul(su, sv)),
                          hd_addc(hd_sub(hd_scale(AB, 36.0), hd_scale(hd_add(A, B), 3.0)), -1.0)),
                   1.0 / 360.0);
  /* Horner in theta: theta (c1 + theta (c2 + theta (c3 + theta (c4 + theta c5)))) */
  hd acc = hd_add(c4, hd_mul(th, c5));
  acc = hd_add(c3, hd_mul(th, acc));
  acc = hd_add(c2, hd_mul(th, acc));
  acc = hd_add(c1, hd_mul(th, acc));
  return hd_mul(th, acc);
}

static hd logc_frank(hd th, hd u, hd omu, hd v, hd omv) {
  if (th.v < 0.0) return logc_frank(hd_neg(th), u, omu, omv, v);
  if (th.v < 3e-3) return logc_frank_series(th, u, omu, v, omv);
  hd a = hd_exp(hd_neg(hd_mul(th, u)));
  hd b = hd_exp(hd_neg(hd_mul(th, v)));
  hd one_m_b = hd_neg(hd_expm1(hd_neg(hd_mul(th, v))));
  hd one_m_eomv = hd_neg(hd_expm1(hd_neg(hd_mul(th, omv))));
  hd D = hd_add(hd_mul(a, one_m_b), hd_mul(b, one_m_eomv));
  hd E = hd_neg(hd_expm1(hd_neg(th))); /* 1 - e^-theta */
  hd r = hd_add(hd_log(th), hd_log(E));
  r = hd_sub(r, hd_mul(th, hd_add(u, v)));
  return hd_sub(r, hd_scale(hd_log(D), 2.0));
}

/* Gumbel, eq. (11): with x = -ln u, y = -ln v, A = x^theta + y^theta,
 *   c = C(u,v) (xy)^{theta-1} / (uv) * A^{1/theta - 2} * (A^{1/theta} + theta - 1).
 * log A is formed as theta*max(ln x, ln y) + log1p(e^{theta (min - max)}),
 * which equals ln(x^theta + y^theta) without overflow or underflow. */
static hd logc_gumbel(hd th, hd u, hd omu, hd v, hd omv) {
  hd x = (u.v < 0.5) ? hd_neg(hd_log(u)) : hd_neg(hd_log1p(hd_neg(omu)));
  hd y = (v.v < 0.5) ? hd_neg(hd_log(v)) : hd_neg(hd_log1p(hd_neg(omv)));
  hd lx = hd_log(x), ly = hd_log(y);
  hd lM = (lx.v >= ly.v) ? lx : ly;
  hd lm = (lx.v >= ly.v) ? ly : lx;
  hd LA = hd_add(hd_mul(th, lM), hd_log1p(hd_exp(hd_mul(th, hd_sub(lm, lM)))));
  hd inv_th = hd_inv(th);
  hd w = hd_exp(hd_mul(LA, inv_th)); /* A^{1/theta} */
  hd r = hd_neg(w);
  r = hd_add(r, hd_mul(hd_addc(th, -1.0), hd_add(lx, ly)));
  r = hd_add(r, hd_add(x, y));
  r = hd_add(r, hd_mul(hd_addc(inv_th, -2.0), LA));
  r = hd_add(r, hd_log(hd_add(w, hd_addc(th, -1.0))));
  return r;
}

static hd logc(int32_t family, hd th, hd u, hd omu, hd v, hd omv) {
  switch (family) {
    case OR_GAUSSIAN: return logc_gaussian(th, u, omu, v, omv);
    case OR_FRANK: return logc_frank(th, u, omu, v, omv);
    default: return logc_gumbel(th, u, omu, v, omv);
  }
}

/* seeds: which = 0 -> (theta, theta): v, d1 = l_theta, d12 = l_theta,theta
 *        which = 1 -> (theta, u):     d12 = l_theta,u
 *        which = 2 -> (theta, v):     d12 = l_theta,v                       */
static hd logc_seeded(int32_t family, double th, double u, double omu, double v, double omv,
                      int which) {
  hd T = {th, 1.0, (which == 0) ? 1.0 : 0.0, 0.0};
  hd U = {u, 0.0, (which == 1) ? 1.0 : 0.0, 0.0};
  hd OU = {omu, 0.0, (which == 1) ? -1.0 : 0.0, 0.0};
  hd V = {v, 0.0, (which == 2) ? 1.0 : 0.0, 0.0};
  hd OV = {omv, 0.0, (which == 2) ? -1.0 : 0.0, 0.0};
  return logc(family, T, U, OU, V, OV);
}

static double logc_value(int32_t family, double th, double u, double omu, double v, double omv) {
  return logc(family, hd_c(th), hd_c(u), hd_c(omu), hd_c(v), hd_c(omv)).v;
}

void or_logc_derivs(int32_t family, double theta, const double* u, const double* omu,
                    const double* v, const double* omv, int64_t n, double* out) {
  for (int64_t i = 0; i < n; ++i) {
    hd a = logc_seeded(family, theta, u[i], omu[i], v[i], omv[i], 0);
    hd b = logc_seeded(family, theta, u[i], omu[i], v[i], omv[i], 1);
    hd c = logc_seeded(family, theta, u[i], omu[i], v[i], omv[i], 2);
    out[5 * i + 0] = a.v;
    out[5 * i + 1] = a.d1;
    out[5 * i + 2] = a.d12;
    out[5 * i + 3] = b.d12;
    out[5 * i + 4] = c.d12;
  }
}

/* ------------------------------------------------------------------------ */
/* Kendall's tau and Spearman's rho (used for the tau-uniform search grid and
 * checked against the values printed in Sec. 2.5). Debye functions
 * D_k(x) = k x^-k int_0^x t^k / (e^t - 1) dt by adaptive Simpson.          */
static double debye_f(double t, int k) {
  if (t == 0.0) return (k == 1) ? 1.0 : 0.0;
  return pow(t, (double)k) / expm1(t);
}
static double asimpson_debye(double a, double b, double fa, double fm, double fb, double whole,
                             double eps, int k, int depth) {
  double m = 0.5 * (a + b), lm = 0.5 * (a + m), rm = 0.5 * (m + b);
  double flm = debye_f(lm, k), frm = debye_f(rm, k);
  double left = (m - a) / 6.0 * (fa + 4.0 * flm + fm);
  double right = (b - m) / 6.0 * (fm + 4.0 * frm + fb);
  double delta = left + right - whole;
  if (depth <= 0 || fabs(delta) <= 15.0 * eps) return left + right + delta / 15.0;
  return asimpson_debye(a, m, fa, flm, fm, left, 0.5 * eps, k, depth - 1) +
         asimpson_debye(m, b, fm, frm, fb, right, 0.5 * eps, k, depth - 1);
}
double or_debye(int32_t k, double x) {
  if (x == 0.0) return 1.0;
  double fa = debye_f(0.0, k), fb = debye_f(x, k), fm = debye_f(0.5 * x, k);
  double whole = x / 6.0 * (fa + 4.0 * fm + fb);
  double integral = asimpson_debye(0.0, x, fa, fm, fb, whole, 1e-15 * fabs(x) + 1e-300, k, 50);
  return (double)k / pow(x, (double)k) * integral;
}

static double gumbel_cdf(double u, double v, double th) {
  if (u <= 0.0 || v <= 0.0) return 0.0;
  if (u >= 1.0) return v;
  if (v >= 1.0) return u;
  double x = -log(u), y = -log(v);
  return exp(-pow(pow(x, th) + pow(y, th), 1.0 / th));
}
/* nested adaptive Simpson for int int C(u,v) du dv (Gumbel Spearman rho) */
typedef struct { double th, u; } gum_ctx;
static double gum_inner_f(double v, const gum_ctx* c) { return gumbel_cdf(c->u, v, c->th); }
static double asimpson_inner(double a, double b, double fa, double fm, double fb, double whole,
                             double eps, const gum_ctx* c, int depth) {
  double m = 0.5 * (a + b), lm = 0.5 * (a + m), rm = 0.5 * (m + b);
  double flm = gum_inner_f(lm, c), frm = gum_inner_f(rm, c);
  double left = (m - a) / 6.0 * (fa + 4.0 * flm + fm);
  double right = (b - m) / 6.0 * (fm + 4.0 * frm + fb);
  double delta = left + right - whole;
  if (depth <= 0 || fabs(delta) <= 15.0 * eps) return left + right + delta / 15.0;
  return asimpson_inner(a, m, fa, flm, fm, left, 0.5 * eps, c, depth - 1) +
         asimpson_inner(m, b, fm, frm, fb, right, 0.5 * eps, c, depth - 1);
}
static double gum_outer_f(double u, double th) {
  gum_ctx c = {th, u};
  double fa = gum_inner_f(0.0, &c), fb = gum_inner_f(1.0, &c), fm = gum_inner_f(0.5, &c);
  return asimpson_inner(0.0, 1.0, fa, fm, fb, (fa + 4.0 * fm + fb) / 6.0, 1e-12, &c, 40);
}
static double asimpson_outer(double a, double b, double fa, double fm, double fb, double whole,
                             double eps, double th, int depth) {
  double m = 0.5 * (a + b), lm = 0.5 * (a + m), rm = 0.5 * (m + b);
  double flm = gum_outer_f(lm, th), frm = gum_outer_f(rm, th);
  double left = (m - a) / 6.0 * (fa + 4.0 * flm + fm);
  double right = (b - m) / 6.0 * (fm + 4.0 * frm + fb);
  double delta = left + right - whole;
  if (depth <= 0 || fabs(delta) <= 15.0 * eps) return left + right + delta / 15.0;
  return asimpson_outer(a, m, fa, flm, fm, left, 0.5 * eps, th, depth - 1) +
         asimpson_outer(m, b, fm, frm, fb, right, 0.5 * eps, th, depth - 1);
}

double or_tau(int32_t family, double th) {
  switch (family) {
    case OR_GAUSSIAN: return 2.0 / M_PI * asin(th);
    case OR_FRANK:
      if (fabs(th) < 1e-6) return th / 9.0;
      return 1.0 - 4.0 / th * (1.0 - or_debye(1, th));
    default: return 1.0 - 1.0 / th;
  }
}

double or_rho_s(int32_t family, double th) {
  switch (family) {
    case OR_GAUSSIAN: return 6.0 / M_PI * asin(0.5 * th);
    case OR_FRANK:
      if (fabs(th) < 1e-6) return th / 6.0;
      return 1.0 - 12.0 / th * (or_debye(1, th) - or_debye(2, th));
    default: {
      double fa = gum_outer_f(0.0, th), fb = gum_outer_f(1.0, th), fm = gum_outer_f(0.5, th);
      double I = asimpson_outer(0.0, 1.0, fa, fm, fb, (fa + 4.0 * fm + fb) / 6.0, 1e-10, th, 30);
      return 12.0 * I - 3.0;
    }
  }
}

/* ------------------------------------------------------------------------ */
/* Search box per family (reading of the parameter ranges of eq. (8), (10),
 * (11): Gaussian open interval (-1, 1), Frank nonzero real, Gumbel >= 1).   */
static double box_lo(int32_t f) { return f == OR_GAUSSIAN ? -(1.0 - 1e-9) : (f == OR_FRANK ? -200.0 : 1.0); }
static double box_hi(int32_t f) { return f == OR_GAUSSIAN ? (1.0 - 1e-9) : (f == OR_FRANK ? 200.0 : 100.0); }

#define OR_GRID 65
static double g_grid[3][OR_GRID];
static int g_grid_ready[3];

static double tau_inverse(int32_t f, double tau) {
  if (f == OR_GAUSSIAN) return sin(0.5 * M_PI * tau);
  if (f == OR_GUMBEL) return 1.0 / (1.0 - tau);
  double lo = box_lo(f), hi = box_hi(f); /* Frank: tau is increasing in theta */
  for (int it = 0; it < 200; ++it) {
    double m = 0.5 * (lo + hi);
    if (or_tau(f, m) < tau) lo = m; else hi = m;
    if (hi - lo <= 1e-14 * (1.0 + fabs(m))) break;
  }
  return 0.5 * (lo + hi);
}

static void ensure_grid(int32_t f) {
  int ready;
#pragma omp atomic read
  ready = g_grid_ready[f];
  if (ready) return;
#pragma omp critical(or_grid)
  {
    if (!g_grid_ready[f]) {
      double t0 = or_tau(f, box_lo(f)), t1 = or_tau(f, box_hi(f));
      for (int j = 0; j < OR_GRID; ++j) {
        double t = t0 + (t1 - t0) * (double)j / (double)(OR_GRID - 1);
        double th = (j == 0) ? box_lo(f) : (j == OR_GRID - 1 ? box_hi(f) : tau_inverse(f, t));
        g_grid[f][j] = th;
      }
#pragma omp atomic write
      g_grid_ready[f] = 1;
    }
  }
}

/* ------------------------------------------------------------------------ */
/* Ranks, eq. (12), with N read as the subset size: R_i = 2 * rank_i.
 * AVERAGE ties: R_i = 2 #{x_j < x_i} + #{x_j = x_i} + 1.
 * FIRST ties:   R_i = 2 (#{x_j < x_i} + #{j < i : x_j = x_i} + 1).
 * -0 and +0 compare equal.                                                   */
typedef struct { double v; int64_t i; } vi_pair;
static int cmp_vi(const void* pa, const void* pb) {
  const vi_pair* a = (const vi_pair*)pa;
  const vi_pair* b = (const vi_pair*)pb;
  if (a->v < b->v) return -1;
  if (a->v > b->v) return 1;
  return (a->i < b->i) ? -1 : (a->i > b->i);
}

void or_ranks(const double* x, int64_t n, int32_t ties, int64_t* R) {
  if (n <= 0) return;
  vi_pair* p = (vi_pair*)malloc((size_t)n * sizeof(vi_pair));
  for (int64_t i = 0; i < n; ++i) { p[i].v = x[i]; p[i].i = i; }
  qsort(p, (size_t)n, sizeof(vi_pair), cmp_vi);
  int64_t i = 0;
  while (i < n) {
    int64_t j = i;
    while (j + 1 < n && p[j + 1].v == p[i].v) ++j;
    int64_t L = j - i + 1;
    for (int64_t k = i; k <= j; ++k)
      R[p[k].i] = (ties == OR_TIES_FIRST) ? 2 * (k + 1) : 2 * i + L + 1;
    i = j + 1;
  }
  free(p);
}

/* ------------------------------------------------------------------------ */
/* Per-subset working data: pseudo-observations as exact rationals. */
typedef struct {
  int64_t n;
  double *u, *omu, *v, *omv;
} pobs;

static double loglik_at(int32_t f, const pobs* P, double th) {
  double s = 0.0;
  for (int64_t i = 0; i < P->n; ++i) s += logc_value(f, th, P->u[i], P->omu[i], P->v[i], P->omv[i]);
  return s;
}
static void score_hess_at(int32_t f, const pobs* P, double th, double* s, double* h) {
  double a = 0.0, b = 0.0;
  for (int64_t i = 0; i < P->n; ++i) {
    hd r = logc_seeded(f, th, P->u[i], P->omu[i], P->v[i], P->omv[i], 0);
    a += r.d1;
    b += r.d12;
  }
  *s = a;
  *h = b;
}

/* Maximise eq. (13) numerically (Sec. 2.3): grid, then bracketed Newton. */
static void maximise(int32_t f, const pobs* P, const or_options* o, double* theta, int32_t* status,
                     int32_t* iters) {
  ensure_grid(f);
  const double* g = g_grid[f];
  int jb = 0;
  double lb = -INFINITY;
  for (int j = 0; j < OR_GRID; ++j) {
    double l = loglik_at(f, P, g[j]);
    if (l > lb) { lb = l; jb = j; }
  }
  *iters = 0;
  if (f == OR_GUMBEL && jb == 0) {
    double s, h;
    score_hess_at(f, P, 1.0, &s, &h);
    if (s <= 0.0) { *theta = 1.0; *status = OR_BOUNDARY_NATURAL; return; }
  }
  double lo = g[jb > 0 ? jb - 1 : 0], hi = g[jb < OR_GRID - 1 ? jb + 1 : OR_GRID - 1];
  double th = g[jb];
  int conv = 0;
  for (int it = 1; it <= o->max_iter; ++it) {
    double s, h;
    score_hess_at(f, P, th, &s, &h);
    *iters = it;
    if (s > 0.0) lo = th; else hi = th;
    double tn = (h < 0.0) ? th - s / h : NAN;
    if (!(tn > lo && tn < hi)) tn = 0.5 * (lo + hi);
    double d = fabs(tn - th);
    th = tn;
    if (d <= o->tol * (1.0 + fabs(th)) || hi - lo <= o->tol * (1.0 + fabs(th))) { conv = 1; break; }
  }
  *theta = th;
  *status = conv ? OR_OK : OR_NOCONV;
  double e0 = box_lo(f), e1 = box_hi(f);
  if (conv && fabs(th - e1) <= 1e-9 * (1.0 + fabs(e1))) { *theta = e1; *status = OR_BOUNDARY_BOX; }
  if (conv && fabs(th - e0) <= 1e-9 * (1.0 + fabs(e0))) {
    *theta = e0;
    *status = (f == OR_GUMBEL) ? OR_BOUNDARY_NATURAL : OR_BOUNDARY_BOX;
  }
}

/* ------------------------------------------------------------------------ */
/* Asymptotic variance of the MPL estimator after Genest, Ghoudi & Rivest
 * (1995) (Sec. 2.3), plug-in form at theta:
 *   s_i  = dl/dtheta (u_i, v_i),  g1_i = d2l/dtheta du,  g2_i = d2l/dtheta dv
 *   W1_i = (1/n) sum_{l : u_l >= u_i} g1_l,   W2_i likewise in v
 *   psi_i = s_i + W1_i + W2_i
 *   nu = (1/n) sum (psi_i - mean psi)^2,  beta = (1/n) sum s_i^2
 *   var(theta_hat) = nu / (n beta^2)            (GGR)
 *                 or 1 / (n beta)               (inverse information)       */
static void suffix_by_rank(const int64_t* R, const double* g, int64_t n, double* W) {
  vi_pair* p = (vi_pair*)malloc((size_t)n * sizeof(vi_pair));
  double* S = (double*)malloc((size_t)(n + 1) * sizeof(double));
  for (int64_t i = 0; i < n; ++i) { p[i].v = (double)R[i]; p[i].i = i; }
  qsort(p, (size_t)n, sizeof(vi_pair), cmp_vi);
  S[n] = 0.0;
  for (int64_t k = n - 1; k >= 0; --k) S[k] = S[k + 1] + g[p[k].i];
  int64_t i = 0;
  while (i < n) { /* all members of a tie group see the sum from the group's first member */
    int64_t j = i;
    while (j + 1 < n && p[j + 1].v == p[i].v) ++j;
    for (int64_t k = i; k <= j; ++k) W[p[k].i] = S[i] / (double)n;
    i = j + 1;
  }
  free(S);
  free(p);
}

double or_ggr(const int64_t* R1, const int64_t* R2, int64_t n, int32_t family, double theta,
              int32_t var_method, double* psi_out) {
  double *s = (double*)malloc((size_t)n * sizeof(double) * 5);
  double *g1 = s + n, *g2 = s + 2 * n, *W1 = s + 3 * n, *W2 = s + 4 * n;
  double den = 2.0 * ((double)n + 1.0);
  for (int64_t i = 0; i < n; ++i) {
    double u = (double)R1[i] / den, omu = (den - (double)R1[i]) / den;
    double v = (double)R2[i] / den, omv = (den - (double)R2[i]) / den;
    hd a = logc_seeded(family, theta, u, omu, v, omv, 1);
    hd b = logc_seeded(family, theta, u, omu, v, omv, 2);
    s[i] = a.d1;
    g1[i] = a.d12;
    g2[i] = b.d12;
  }
  suffix_by_rank(R1, g1, n, W1);
  suffix_by_rank(R2, g2, n, W2);
  double mpsi = 0.0, beta = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    double psi = s[i] + W1[i] + W2[i];
    mpsi += psi;
    beta += s[i] * s[i];
    if (psi_out) {
      psi_out[4 * i + 0] = s[i];
      psi_out[4 * i + 1] = W1[i];
      psi_out[4 * i + 2] = W2[i];
      psi_out[4 * i + 3] = psi;
    }
  }
  mpsi /= (double)n;
  beta /= (double)n;
  double nu = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    double d = s[i] + W1[i] + W2[i] - mpsi;
    nu += d * d;
  }
  nu /= (double)n;
  free(s);
  if (var_method == OR_VAR_INVINFO) return 1.0 / ((double)n * beta);
  return nu / ((double)n * beta * beta);
}

/* ------------------------------------------------------------------------ */
void or_default_options(or_options* o) {
  o->ties = OR_TIES_AVERAGE;
  o->var = OR_VAR_GGR;
  o->max_iter = 100;
  o->pad = 0;
  o->tol = 1e-13;
  o->n_min = 2;
}

/* One subset through Sec. 2.3: ranks (eq. 12), maximise eq. (13), variance. */
void or_fit_subset(const double* x, const double* y, int64_t n, int32_t family,
                   const or_options* opt, or_subset* out) {
  or_options o;
  if (opt) o = *opt; else or_default_options(&o);
  int64_t n_min = o.n_min < 2 ? 2 : o.n_min;
  out->theta = NAN; out->var = NAN; out->loglik = NAN; out->score = NAN;
  out->n = n; out->iters = 0; out->status = OR_OK;
  if (n < n_min) { out->status = OR_DEGENERATE; return; }
  for (int64_t i = 0; i < n; ++i)
    if (!isfinite(x[i]) || !isfinite(y[i])) { out->status = OR_NONFINITE; return; }
  int same_x = 1, same_y = 1;
  for (int64_t i = 1; i < n; ++i) {
    if (x[i] != x[0]) same_x = 0;
    if (y[i] != y[0]) same_y = 0;
  }
  if (same_x || same_y) { out->status = OR_DEGENERATE; return; }

  int64_t* R1 = (int64_t*)malloc((size_t)n * 2 * sizeof(int64_t));
  int64_t* R2 = R1 + n;
  or_ranks(x, n, o.ties, R1);
  or_ranks(y, n, o.ties, R2);
  pobs P;
  P.n = n;
  P.u = (double*)malloc((size_t)n * 4 * sizeof(double));
  P.omu = P.u + n; P.v = P.u + 2 * n; P.omv = P.u + 3 * n;
  double den = 2.0 * ((double)n + 1.0); /* u = r/(n+1) = R / (2(n+1)) */
  for (int64_t i = 0; i < n; ++i) {
    P.u[i] = (double)R1[i] / den;
    P.omu[i] = (den - (double)R1[i]) / den;
    P.v[i] = (double)R2[i] / den;
    P.omv[i] = (den - (double)R2[i]) / den;
  }
  double th;
  int32_t st, it;
  maximise(family, &P, &o, &th, &st, &it);
  out->theta = th;
  out->status = st;
  out->iters = it;
  out->loglik = loglik_at(family, &P, th);
  double s, h;
  score_hess_at(family, &P, th, &s, &h);
  out->score = s;
  if (st == OR_OK || st == OR_BOUNDARY_NATURAL) {
    double var = or_ggr(R1, R2, n, family, th, o.var, NULL);
    out->var = var;
    if (!(var > 0.0) || !isfinite(var)) out->status = OR_BADVAR;
  }
  free(P.u);
  free(R1);
}

/* eq. (15) / (16): theta = sum w_m theta_m / sum w_m with w_m = 1 / sigma_m^2,
 * over the usable subsets of each group (status OK or BOUNDARY_NATURAL). */
void or_combine(const or_subset* sub, const int64_t* group_offsets, int64_t G, or_combined* comb) {
  for (int64_t g = 0; g < G; ++g) {
    double sw = 0.0, swt = 0.0;
    int64_t used = 0, total = group_offsets[g + 1] - group_offsets[g];
    for (int64_t m = group_offsets[g]; m < group_offsets[g + 1]; ++m) {
      int32_t st = sub[m].status;
      if (st != OR_OK && st != OR_BOUNDARY_NATURAL) continue;
      double w = 1.0 / sub[m].var;
      sw += w;
      swt += w * sub[m].theta;
      ++used;
    }
    comb[g].n_used = used;
    comb[g].n_excluded = total - used;
    comb[g].pad = 0;
    if (used > 0) {
      comb[g].theta = swt / sw;
      comb[g].var_combined = 1.0 / sw;
      comb[g].status = 0;
    } else {
      comb[g].theta = NAN;
      comb[g].var_combined = NAN;
      comb[g].status = 1;
    }
  }
}

int32_t or_num_threads(int32_t requested) {
#ifdef _OPENMP
  return requested > 0 ? requested : omp_get_max_threads();
#else
  (void)requested;
  return 1;
#endif
}

/* eq. (14): rows [offsets[m], offsets[m+1]) form subset m; each subset is an
 * independent MPL fit (Sec. 2.4), then eq. (15) per group of subsets. */
void or_fit(const double* x, const double* y, const int64_t* offsets, int64_t K,
            const int64_t* group_offsets, int64_t G, const int32_t* family_per_group,
            const or_options* opt, int32_t nthreads, or_subset* out, or_combined* comb) {
  int32_t* fam = (int32_t*)malloc((size_t)(K > 0 ? K : 1) * sizeof(int32_t));
  for (int64_t g = 0; g < G; ++g)
    for (int64_t m = group_offsets[g]; m < group_offsets[g + 1]; ++m) fam[m] = family_per_group[g];
  for (int32_t f = 0; f < 3; ++f) ensure_grid(f);
  int32_t nt = or_num_threads(nthreads);
  (void)nt;
#pragma omp parallel for schedule(dynamic, 1) num_threads(nt)
  for (int64_t m = 0; m < K; ++m)
    or_fit_subset(x + offsets[m], y + offsets[m], offsets[m + 1] - offsets[m], fam[m], opt, &out[m]);
  or_combine(out, group_offsets, G, comb);
  free(fam);
}
