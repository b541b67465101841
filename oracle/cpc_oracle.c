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
  /* the interval is cut into pieces of length at most 4 before the adaptive
   * rule sees it: over [0, x] at once, the first samples of a long interval
   * (x ~ 200) all fall where t^k / (e^t - 1) has died away and the rule stops
   * on an estimate near zero. The integrand has one sign on each piece, so
   * the target error is relative to the piece's integral (for x < 0 it grows
   * like |t|^k, and an absolute target falls below its rounding) */
  const int pieces = (int)ceil(fabs(x) / 4.0);
  double integral = 0.0;
  for (int p = 0; p < pieces; ++p) {
    const double a = x * p / pieces, b = x * (p + 1) / pieces;
    double fa = debye_f(a, k), fb = debye_f(b, k), fm = debye_f(0.5 * (a + b), k);
    double whole = (b - a) / 6.0 * (fa + 4.0 * fm + fb);
    integral += asimpson_debye(a, b, fa, fm, fb, whole, 1e-15 * fabs(whole) + 1e-300, k, 50);
  }
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

/* ======================================================================== */
/* Simulation inputs (Sec. 2.5: data simulated from the copula itself) from a
 * counter-based generator, so that any row can be drawn independently and
 * the GPU sampler can be compared with this one value by value.
 *
 * Philox4x32-10 (Salmon, Moraes, Dror & Shaw, "Parallel random numbers: as
 * easy as 1, 2, 3", SC 2011): a 4 x 32-bit counter and a 2 x 32-bit key,
 * ten rounds of two 32 x 32 -> 64-bit multiplications (multipliers
 * 0xD2511F53 and 0xCD9E8D57) with the key bumped by the Weyl constants
 * 0x9E3779B9 and 0xBB67AE85 between rounds.                                 */
void or_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4]) {
  uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
  uint32_t k0 = key_in[0], k1 = key_in[1];
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    c0 = hi1 ^ c1 ^ k0;
    c1 = lo1;
    c2 = hi0 ^ c3 ^ k1;
    c3 = lo0;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* A uniform on the open interval from two words: k = the 20 low bits of a
 * above the 32 bits of b (52 bits), u = (k + 1/2) 2^-52 and 1 - u =
 * (2^52 - k - 1/2) 2^-52, both exact.                                       */
static void uniform_pair(uint32_t a, uint32_t b, double* u, double* omu) {
  const uint64_t k = ((uint64_t)(a & 0xFFFFFu) << 32) | (uint64_t)b;
  *u = ((double)k + 0.5) * 0x1p-52;
  *omu = (4503599627370496.0 - (double)k - 0.5) * 0x1p-52;
}

/* The uniforms of row `row` of a stream keyed by `seed`: block `blk` is the
 * generator at counter (row low word, row high word, blk, 0).               */
static void row_uniforms(uint64_t seed, int64_t row, uint32_t blk, double u[2], double omu[2]) {
  const uint32_t ctr[4] = {(uint32_t)(uint64_t)row, (uint32_t)((uint64_t)row >> 32), blk, 0u};
  const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  uint32_t w[4];
  or_philox4x32_10(ctr, key, w);
  uniform_pair(w[0], w[1], &u[0], &omu[0]);
  uniform_pair(w[2], w[3], &u[1], &omu[1]);
}

/* An exponential variate -log(u), from 1 - u where u is near 1. */
static double exp_variate(double u, double omu) { return (u < 0.5) ? -log(u) : -log1p(-omu); }

/* Phi^{-1}(exp(-t)) (a margin of the Marshall-Olkin construction): the upper
 * tail through 1 - e^{-t} = -expm1(-t) when e^{-t} > 1/2; t is capped at
 * 700 (e^{-700} ~ 1e-304) so that e^{-t} stays a normal double.             */
static double qnorm_exp_neg(double t) {
  if (t > 700.0) t = 700.0;
  return or_qnorm(exp(-t), -expm1(-t));
}

/* Row i of n pairs (x, y) with N(0,1) margins whose copula is the family's
 * (eq. 8, 10, 11) at theta; row0 + i is the generator row.
 *  Gaussian: z1 = Phi^{-1}(u1), z2 = Phi^{-1}(u2), x = z1,
 *            y = rho z1 + sqrt(1 - rho^2) z2 (Cholesky factor of the
 *            correlation matrix).
 *  Frank:    u, and v from dC/du (u, v) = w solved in closed form:
 *            e^{-theta v} = ((1-w) e^{-theta u} + w e^{-theta}) / (w + (1-w) e^{-theta u}),
 *            i.e. v = u - D / theta, 1 - v = (1 - u) + D / theta with
 *            D = log1p(w expm1(-theta (1-u))) - log1p((1-w) expm1(-theta u))
 *            (theta = 0: v = w); v and 1 - v are kept in [2^-1000, 1 - 2^-53].
 *  Gumbel:   Marshall-Olkin: S positive stable with Laplace transform
 *            exp(-s^alpha), alpha = 1/theta, by Kanter's representation
 *            S = sin(alpha T) / sin(T)^(1/alpha) * (sin((1-alpha) T) / W)^((1-alpha)/alpha)
 *            with T ~ U(0, pi), W ~ Exp(1) (formed in logarithms); then
 *            U_j = exp(-(E_j / S)^alpha) with E_j ~ Exp(1).
 *  The margin of a uniform takes the tail of the smaller of u and 1 - u.     */
void or_sample(int32_t family, double theta, uint64_t seed, int64_t row0, int64_t n, double* x, double* y) {
  for (int64_t i = 0; i < n; ++i) {
    const int64_t row = row0 + i;
    double u[2], omu[2];
    row_uniforms(seed, row, 0u, u, omu);
    if (family == OR_GAUSSIAN) {
      const double z1 = or_qnorm(u[0], omu[0]), z2 = or_qnorm(u[1], omu[1]);
      x[i] = z1;
      y[i] = theta * z1 + sqrt((1.0 - theta) * (1.0 + theta)) * z2;
    } else if (family == OR_FRANK) {
      double v = u[1], omv = omu[1];
      if (theta != 0.0) {
        const double D = log1p(u[1] * expm1(-theta * omu[0])) - log1p(omu[1] * expm1(-theta * u[0]));
        v = u[0] - D / theta;
        omv = omu[0] + D / theta;
      }
      v = fmin(fmax(v, 0x1p-1000), 1.0 - 0x1p-53);
      omv = fmin(fmax(omv, 0x1p-1000), 1.0 - 0x1p-53);
      x[i] = or_qnorm(u[0], omu[0]);
      y[i] = or_qnorm(v, omv);
    } else {
      double s[2], oms[2];
      row_uniforms(seed, row, 1u, s, oms);
      const double E1 = exp_variate(u[0], omu[0]), E2 = exp_variate(u[1], omu[1]);
      const double alpha = 1.0 / theta;
      double logS = 0.0;
      if (theta != 1.0) {
        const double T = M_PI * s[0];
        const double W = exp_variate(s[1], oms[1]);
        logS = log(sin(alpha * T)) - log(sin(T)) / alpha +
               (1.0 - alpha) / alpha * (log(sin((1.0 - alpha) * T)) - log(W));
      }
      const double t1 = exp(alpha * (log(E1) - logS)), t2 = exp(alpha * (log(E2) - logS));
      x[i] = qnorm_exp_neg(t1);
      y[i] = qnorm_exp_neg(t2);
    }
  }
}

/* ======================================================================== */
/* Sec. 2.6, eq. (19)-(20): distances between the copula densities at two
 * parameter values, over the unit square, in normal-score coordinates
 * u = Phi(s), v = Phi(t):  int int f(c(u, v)) du dv = int int f(c(Phi(s),
 * Phi(t))) phi(s) phi(t) ds dt. The corners of the square move to infinity,
 * where the transformed integrands decay, and the box |s|, |t| <= Lbox is
 * integrated by composite Gauss-Legendre rules (m nodes on each of `panels`
 * equal panels per axis; the nodes by Newton's method on the Legendre
 * polynomial P_m). |c_a - c_b| has a kink where the densities cross: on each
 * line s = const the inner integral of |c_a - c_b| is split at the crossings
 * (located by bisection between sample points where the difference changes
 * sign) and each piece integrated by the same rule. out[0] = int |c_a - c_b|,
 * out[1] = int c_a, out[2] = int (c_a - c_b)^2, out[3] = int c_a^2, so that
 * eq. (19) is out[0] / out[1] and eq. (20) is sqrt(out[2] / out[3]).        */
static void gauss_legendre(int m, double* xn, double* wn) {
  for (int i = 0; i < m; ++i) {
    double z = cos(M_PI * (i + 0.75) / (m + 0.5)), dp = 0.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= m; ++k) {
        const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = m * (z * p1 - p0) / (z * z - 1.0);
      const double dz = p1 / dp;
      z -= dz;
      if (fabs(dz) < 1e-16) break;
    }
    xn[i] = z;
    wn[i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

static double density_at(int32_t family, double theta, double u, double omu, double v, double omv) {
  return exp(logc_value(family, theta, u, omu, v, omv));
}

typedef struct {
  int32_t family;
  double ta, tb, u, omu; /* the line s = const: u = Phi(s) */
} dd_line;

/* c_a - c_b at normal score t on the line */
static double dd_diff(const dd_line* L, double t) {
  const double v = Phi_cdf(t), omv = Phi_cdf(-t);
  return density_at(L->family, L->ta, L->u, L->omu, v, omv) - density_at(L->family, L->tb, L->u, L->omu, v, omv);
}

/* int_a^b |c_a - c_b| phi(t) dt on the line by the m-point rule */
static double dd_abs_piece(const dd_line* L, double a, double b, int m, const double* xn, const double* wn) {
  double acc = 0.0;
  for (int k = 0; k < m; ++k) {
    const double t = 0.5 * (a + b) + 0.5 * (b - a) * xn[k];
    acc += 0.5 * (b - a) * wn[k] * fabs(dd_diff(L, t)) * phi_pdf(t);
  }
  return acc;
}

void or_density_distance(int32_t family, double theta_a, double theta_b, double Lbox, int32_t panels, int32_t m,
                         double out[4]) {
  double xn[64], wn[64];
  if (m > 64) m = 64;
  gauss_legendre(m, xn, wn);
  const int64_t N = (int64_t)panels * m;
  double* s = (double*)malloc(sizeof(double) * (size_t)N);
  double* w = (double*)malloc(sizeof(double) * (size_t)N);
  double* u = (double*)malloc(sizeof(double) * (size_t)N);
  double* omu = (double*)malloc(sizeof(double) * (size_t)N);
  const double h = 2.0 * Lbox / panels;
  for (int p = 0; p < panels; ++p)
    for (int k = 0; k < m; ++k) {
      const int64_t j = (int64_t)p * m + k;
      s[j] = -Lbox + h * (p + 0.5 * (xn[k] + 1.0));
      w[j] = 0.5 * h * wn[k] * phi_pdf(s[j]);
      u[j] = Phi_cdf(s[j]);
      omu[j] = Phi_cdf(-s[j]);
    }
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
#pragma omp parallel for schedule(dynamic, 4) reduction(+ : acc[:4])
  for (int64_t i = 0; i < N; ++i) {
    const dd_line L = {family, theta_a, theta_b, u[i], omu[i]};
    double row[4] = {0.0, 0.0, 0.0, 0.0};
    double d[64 + 2], t[64 + 2];
    for (int p = 0; p < panels; ++p) {
      /* samples of the difference along the panel: its ends and the nodes */
      const double a = -Lbox + h * p, b = a + h;
      int ns = 0;
      int change = 0;
      t[ns] = a;
      d[ns++] = (theta_b == theta_a) ? 0.0 : dd_diff(&L, a);
      for (int k = 0; k < m; ++k) {
        const int64_t j = (int64_t)p * m + k;
        const double ca = density_at(family, theta_a, u[i], omu[i], u[j], omu[j]);
        const double cb = (theta_b == theta_a) ? ca : density_at(family, theta_b, u[i], omu[i], u[j], omu[j]);
        const double dd = ca - cb;
        row[1] += ca * w[j];
        row[2] += dd * dd * w[j];
        row[3] += ca * ca * w[j];
        t[ns] = s[j];
        d[ns++] = dd;
      }
      t[ns] = b;
      d[ns++] = (theta_b == theta_a) ? 0.0 : dd_diff(&L, b);
      for (int q = 1; q < ns; ++q)
        if ((d[q - 1] < 0.0 && d[q] > 0.0) || (d[q - 1] > 0.0 && d[q] < 0.0)) change = 1;
      if (!change) {
        for (int k = 0; k < m; ++k) row[0] += fabs(d[k + 1]) * w[(int64_t)p * m + k];
        continue;
      }
      /* split the panel at every crossing and integrate the pieces */
      double lo = a;
      for (int q = 1; q < ns; ++q) {
        if (!((d[q - 1] < 0.0 && d[q] > 0.0) || (d[q - 1] > 0.0 && d[q] < 0.0))) continue;
        double x0 = t[q - 1], x1 = t[q], f0 = d[q - 1];
        for (int it = 0; it < 200 && x1 - x0 > 1e-15 * (1.0 + fabs(x0)); ++it) {
          const double xm = 0.5 * (x0 + x1), fm = dd_diff(&L, xm);
          if ((fm < 0.0) == (f0 < 0.0)) { x0 = xm; f0 = fm; } else { x1 = xm; }
        }
        const double root = 0.5 * (x0 + x1);
        row[0] += dd_abs_piece(&L, lo, root, m, xn, wn);
        lo = root;
      }
      row[0] += dd_abs_piece(&L, lo, b, m, xn, wn);
    }
    for (int k = 0; k < 4; ++k) acc[k] += row[k] * w[i];
  }
  for (int k = 0; k < 4; ++k) out[k] = acc[k];
  free(s); free(w); free(u); free(omu);
}

/* ======================================================================== */
/* The inversion of Spearman's rho (Sec. 2.3 names it beside the pseudo-
 * likelihood): rho_S of the subset's ranks, theta with rho_S(theta) = rho_S
 * hat (closed form for the Gaussian, bisection on the Debye-function form
 * for Frank and on the quadrature form for Gumbel), and the asymptotic
 * variance of this moment estimator by the same plug-in sandwich as the
 * pseudo-likelihood's (Genest, Ghoudi & Rivest 1995): with
 * J(u, v) = 12 (u - 1/2)(v - 1/2), psi_i = J_i + W1(u_i) + W2(v_i),
 * W1(u_i) = (1/n) sum over u_l >= u_i of dJ/du (u_l, v_l), likewise W2, and
 * sigma^2 = var(psi) / (n rho_S'(theta)^2).                                 */

/* rho_S hat from doubled ranks: 12 / (n (n^2 - 1)) sum (r1 - (n+1)/2)(r2 - (n+1)/2) */
double or_spearman(const int64_t* R1, const int64_t* R2, int64_t n) {
  long double s = 0.0L;
  for (int64_t i = 0; i < n; ++i) s += (long double)((R1[i] - (n + 1)) * (R2[i] - (n + 1)));
  const double dn = (double)n;
  return 3.0 * (double)s / (dn * (dn * dn - 1.0));
}

/* d rho_S / d theta by a central difference of or_rho_s (closed form for the
 * Gaussian) */
static double rho_s_slope(int32_t f, double th) {
  if (f == OR_GAUSSIAN) return 3.0 / (M_PI * sqrt(1.0 - 0.25 * th * th));
  const double h = 1e-4 * (1.0 + fabs(th));
  if (f == OR_GUMBEL && th - h < 1.0) {
    /* at the edge of the parameter space: the one-sided derivative, by the
     * second-order forward difference (-3 f(a) + 4 f(a + h) - f(a + 2h)) / 2h */
    const double a = th;
    return (-3.0 * or_rho_s(f, a) + 4.0 * or_rho_s(f, a + h) - or_rho_s(f, a + 2.0 * h)) / (2.0 * h);
  }
  return (or_rho_s(f, th + h) - or_rho_s(f, th - h)) / (2.0 * h);
}

/* theta with rho_S(theta) = r: status 0, 1 (Gumbel at theta = 1, r <= 0) or
 * 2 (at the family's search box edge) */
double or_spearman_theta(int32_t f, double r, int32_t* status) {
  *status = OR_OK;
  if (f == OR_GAUSSIAN) {
    const double th = 2.0 * sin(M_PI * r / 6.0);
    if (fabs(th) >= 1.0 - 1e-9) { *status = OR_BOUNDARY_BOX; return th > 0 ? 1.0 - 1e-9 : -(1.0 - 1e-9); }
    return th;
  }
  double lo = box_lo(f), hi = box_hi(f);
  if (f == OR_GUMBEL && r <= 0.0) { *status = OR_BOUNDARY_NATURAL; return 1.0; }
  double flo = or_rho_s(f, lo) - r, fhi = or_rho_s(f, hi) - r;
  if (flo >= 0.0) { *status = OR_BOUNDARY_BOX; return lo; }
  if (fhi <= 0.0) { *status = OR_BOUNDARY_BOX; return hi; }
  /* rho_S increases in theta: the root stays bracketed by [lo, hi];
   * regula falsi with the Illinois halving of the retained end, bisection
   * where the secant point leaves the bracket */
  double m = lo, prev = hi;
  int side = 0;
  for (int it = 0; it < 200; ++it) {
    m = (lo * fhi - hi * flo) / (fhi - flo);
    if (!(m > lo && m < hi)) m = 0.5 * (lo + hi);
    const double fm = or_rho_s(f, m) - r;
    if (fm == 0.0 || fabs(m - prev) <= 1e-13 * (1.0 + fabs(m)) || hi - lo <= 1e-12 * (1.0 + fabs(lo))) break;
    prev = m;
    if (fm < 0.0) {
      lo = m; flo = fm;
      if (side == -1) fhi *= 0.5;
      side = -1;
    } else {
      hi = m; fhi = fm;
      if (side == 1) flo *= 0.5;
      side = 1;
    }
  }
  return m;
}

/* Variance of the Spearman-inversion estimate at theta (from the doubled
 * ranks; the suffix sums by a sort of the rows by rank, ties taking the
 * group's sum over u_l >= u_i). Returns var(psi) in *nu. */
double or_spearman_var(const int64_t* R1, const int64_t* R2, int64_t n, int32_t f, double theta, double* nu) {
  const double den = 2.0 * (n + 1.0);
  double* g1 = (double*)malloc(sizeof(double) * (size_t)n);
  double* g2 = (double*)malloc(sizeof(double) * (size_t)n);
  double* W1 = (double*)malloc(sizeof(double) * (size_t)n);
  double* W2 = (double*)malloc(sizeof(double) * (size_t)n);
  for (int64_t i = 0; i < n; ++i) {
    g1[i] = 12.0 * ((double)R2[i] / den - 0.5); /* dJ/du = 12 (v - 1/2) */
    g2[i] = 12.0 * ((double)R1[i] / den - 0.5); /* dJ/dv = 12 (u - 1/2) */
  }
  suffix_by_rank(R1, g1, n, W1);
  suffix_by_rank(R2, g2, n, W2);
  double sp = 0.0, sq = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    const double J = 12.0 * ((double)R1[i] / den - 0.5) * ((double)R2[i] / den - 0.5);
    const double psi = J + W1[i] + W2[i]; /* (the suffix sums are already means) */
    sp += psi;
    sq += psi * psi;
  }
  free(g1); free(g2); free(W1); free(W2);
  const double m = sp / n;
  *nu = sq / n - m * m;
  const double b = rho_s_slope(f, theta);
  return *nu / (n * b * b);
}

/* The Spearman-inversion estimate of one subset from its doubled ranks:
 * out->theta, out->var, out->loglik = rho_S hat, out->score = rho_S(theta) -
 * rho_S hat, out->status (DEGENERATE below n_min rows or for a margin of one
 * value). */
void or_spearman_fit_ranks(const int64_t* R1, const int64_t* R2, int64_t n, int32_t family, int64_t n_min,
                           or_subset* out) {
  out->theta = NAN; out->var = NAN; out->loglik = NAN; out->score = NAN;
  out->n = n; out->iters = 0; out->status = OR_OK;
  if (n < (n_min < 2 ? 2 : n_min)) { out->status = OR_DEGENERATE; return; }
  int same1 = 1, same2 = 1;
  for (int64_t i = 1; i < n; ++i) {
    if (R1[i] != R1[0]) same1 = 0;
    if (R2[i] != R2[0]) same2 = 0;
  }
  if (same1 || same2) { out->status = OR_DEGENERATE; return; }
  const double r = or_spearman(R1, R2, n);
  int32_t st;
  const double th = or_spearman_theta(family, r, &st);
  out->theta = th;
  out->status = st;
  out->loglik = r;
  out->score = or_rho_s(family, th) - r;
  if (st == OR_OK || st == OR_BOUNDARY_NATURAL) {
    double nu;
    const double v = or_spearman_var(R1, R2, n, family, th, &nu);
    out->var = v;
    if (!(v > 0.0) || !isfinite(v)) out->status = OR_BADVAR;
  }
}

/* ======================================================================== */
/* The inversion of Kendall's tau (Sec. 2.3 names it with Spearman's rho):
 * tau hat = (concordant - discordant pairs) / (n (n - 1) / 2), a pair tied
 * in either margin counting as neither; theta with tau(theta) = tau hat
 * (closed forms for the Gaussian, sin(pi tau / 2), and for Gumbel,
 * 1 / (1 - tau); for Frank the Debye form of tau solved by regula falsi);
 * tau hat is a U-statistic of degree two with kernel
 * sign(r1_i - r1_l) sign(r2_i - r2_l), so var(tau hat) ~ 4 var(k1) / n with
 * k1_i = S_i / (n - 1), S_i = sum over l != i of that kernel, and the
 * estimate's variance is var(tau hat) / tau'(theta)^2.                      */

static int sgn64(int64_t d) { return (d > 0) - (d < 0); }

/* S_i of every row, by all pairs */
void or_kendall_rows(const int64_t* R1, const int64_t* R2, int64_t n, int64_t* S) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    int64_t s = 0;
    for (int64_t l = 0; l < n; ++l) s += sgn64(R1[i] - R1[l]) * sgn64(R2[i] - R2[l]);
    S[i] = s;
  }
}

/* tau hat of doubled ranks (all pairs) */
double or_kendall(const int64_t* R1, const int64_t* R2, int64_t n) {
  if (n < 2) return NAN;
  int64_t* S = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
  or_kendall_rows(R1, R2, n, S);
  int64_t t = 0;
  for (int64_t i = 0; i < n; ++i) t += S[i];
  free(S);
  return (double)t / ((double)n * (double)(n - 1));
}

/* d tau / d theta: Gaussian 2 / (pi sqrt(1 - theta^2)); Gumbel 1 / theta^2;
 * Frank, from tau = 1 - (4 / theta)(1 - D1(theta)) and
 * D1'(x) = -D1(x) / x + 1 / (e^x - 1): 4 (1 - D1) / theta^2 + 4 D1' / theta,
 * by its series 1/9 - theta^2 / 300 + theta^4 / 10584 below |theta| = 1e-2 */
double or_tau_slope(int32_t f, double th) {
  if (f == OR_GAUSSIAN) return 2.0 / (M_PI * sqrt(1.0 - th * th));
  if (f == OR_GUMBEL) return 1.0 / (th * th);
  if (fabs(th) < 1e-2) {
    const double t2 = th * th;
    return 1.0 / 9.0 - t2 / 300.0 + t2 * t2 / 10584.0;
  }
  const double d1 = or_debye(1, th);
  const double dd1 = -d1 / th + 1.0 / expm1(th);
  return 4.0 * (1.0 - d1) / (th * th) + 4.0 * dd1 / th;
}

/* theta with tau(theta) = t: status 0, 1 (Gumbel at theta = 1, t <= 0) or 2
 * (at the family's search box edge) */
double or_kendall_theta(int32_t f, double t, int32_t* status) {
  *status = OR_OK;
  const double lo0 = box_lo(f), hi0 = box_hi(f);
  if (f == OR_GAUSSIAN) {
    const double th = sin(0.5 * M_PI * t);
    if (th <= lo0) { *status = OR_BOUNDARY_BOX; return lo0; }
    if (th >= hi0) { *status = OR_BOUNDARY_BOX; return hi0; }
    return th;
  }
  if (f == OR_GUMBEL) {
    if (t <= 0.0) { *status = OR_BOUNDARY_NATURAL; return 1.0; }
    if (t >= 1.0 - 1.0 / hi0) { *status = OR_BOUNDARY_BOX; return hi0; }
    return 1.0 / (1.0 - t);
  }
  double lo = lo0, hi = hi0;
  double flo = or_tau(f, lo) - t, fhi = or_tau(f, hi) - t;
  if (flo >= 0.0) { *status = OR_BOUNDARY_BOX; return lo; }
  if (fhi <= 0.0) { *status = OR_BOUNDARY_BOX; return hi; }
  /* tau increases in theta: regula falsi with the Illinois halving, bisection
   * where the secant point leaves the bracket */
  double m = lo, prev = hi;
  int side = 0;
  for (int it = 0; it < 200; ++it) {
    m = (lo * fhi - hi * flo) / (fhi - flo);
    if (!(m > lo && m < hi)) m = 0.5 * (lo + hi);
    const double fm = or_tau(f, m) - t;
    if (fm == 0.0 || fabs(m - prev) <= 1e-13 * (1.0 + fabs(m)) || hi - lo <= 1e-12 * (1.0 + fabs(lo))) break;
    prev = m;
    if (fm < 0.0) {
      lo = m; flo = fm;
      if (side == -1) fhi *= 0.5;
      side = -1;
    } else {
      hi = m; fhi = fm;
      if (side == 1) flo *= 0.5;
      side = 1;
    }
  }
  return m;
}

/* Variance of the Kendall-inversion estimate at theta; var(k1) in *zeta and
 * tau hat in *tau_hat */
double or_kendall_var(const int64_t* R1, const int64_t* R2, int64_t n, int32_t f, double theta, double* zeta,
                      double* tau_hat) {
  int64_t* S = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
  or_kendall_rows(R1, R2, n, S);
  int64_t tot = 0;
  for (int64_t i = 0; i < n; ++i) tot += S[i];
  const double th = (double)tot / ((double)n * (double)(n - 1));
  double q = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    const double k1 = (double)S[i] / (double)(n - 1) - th;
    q += k1 * k1;
  }
  free(S);
  *tau_hat = th;
  *zeta = q / (double)n;
  const double b = or_tau_slope(f, theta);
  return 4.0 * *zeta / ((double)n * b * b);
}

/* One subset from its doubled ranks: out->loglik = tau hat, out->score =
 * tau(theta) - tau hat (statuses as for Spearman's rho) */
void or_kendall_fit_ranks(const int64_t* R1, const int64_t* R2, int64_t n, int32_t family, int64_t n_min,
                          or_subset* out) {
  out->theta = NAN; out->var = NAN; out->loglik = NAN; out->score = NAN;
  out->n = n; out->iters = 0; out->status = OR_OK;
  if (n < (n_min < 2 ? 2 : n_min)) { out->status = OR_DEGENERATE; return; }
  int same1 = 1, same2 = 1;
  for (int64_t i = 1; i < n; ++i) {
    if (R1[i] != R1[0]) same1 = 0;
    if (R2[i] != R2[0]) same2 = 0;
  }
  if (same1 || same2) { out->status = OR_DEGENERATE; return; }
  const double t = or_kendall(R1, R2, n);
  int32_t st;
  const double th = or_kendall_theta(family, t, &st);
  out->theta = th;
  out->status = st;
  out->loglik = t;
  out->score = or_tau(family, th) - t;
  if (st == OR_OK || st == OR_BOUNDARY_NATURAL) {
    double zeta, t2;
    const double v = or_kendall_var(R1, R2, n, family, th, &zeta, &t2);
    out->var = v;
    if (!(v > 0.0) || !isfinite(v)) out->status = OR_BADVAR;
  }
}
