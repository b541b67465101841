// solver.h — per-subset maximisation of the pseudo log-likelihood (eq. 13 of
// arXiv:1609.05530, "maximised numerically", Sec. 2.3): a safeguarded Newton
// iteration on the score with a bracket that shrinks on the sign of the
// score, started from the Spearman correlation of the subset's ranks. All of
// it is FP64 and runs on one thread per subset; the score and Hessian it
// consumes are the workgroup's sums over the subset's rows.
#pragma once

#include "cpc_device.h"

namespace cpc {

struct NewtonState {
  double theta, lo, hi, prev_step;
  int32_t it, status, done, flags;  // flags: bit 0 lower box edge evaluated, bit 1 upper,
                                    // bit 2 the previous step was a plain Newton step
};

// Starting value from Spearman's rho of the ranks (Sec. 2.3 names the
// inversion of Spearman's rho among the estimators; here it only seeds the
// iteration). Gaussian: rho = 2 sin(pi rho_S / 6). Frank: 6 rho_S / sqrt(1 -
// rho_S^2), a close fit to the inverse of Frank's rho_S(theta) over the
// family's range. Gumbel: tau from the Gaussian relation, theta = 1/(1 - tau).
__device__ inline double start_theta(int fam, double rho_s) {
  const double pi = 3.14159265358979323846;
  double r = fmin(fmax(rho_s, -0.999999), 0.999999);
  if (fam == FAM_GAUSSIAN) {
    double t = 2.0 * sin(pi * r / 6.0);
    return fmin(fmax(t, -0.999), 0.999);
  }
  if (fam == FAM_FRANK) {
    double t = 6.0 * r / sqrt(1.0 - r * r);
    if (fabs(t) < 1e-6) t = (t < 0.0) ? -1e-6 : 1e-6;
    return fmin(fmax(t, -150.0), 150.0);
  }
  const double rho = 2.0 * sin(pi * r / 6.0);
  const double tau = 2.0 / pi * asin(fmin(fmax(rho, -1.0), 1.0));
  if (tau <= 0.0) return 1.0;
  return fmin(1.0 / (1.0 - tau), 80.0);
}

__device__ inline void newton_init(NewtonState& st, int fam, double theta0) {
  st.theta = theta0;
  st.lo = box_lo(fam);
  st.hi = box_hi(fam);
  st.prev_step = INFINITY;
  st.it = 0;
  st.status = ST_OK;
  st.done = 0;
  st.flags = (theta0 <= st.lo) ? 1 : 0;
}

__device__ inline void newton_snap(NewtonState& st, int fam) {
  const double bl = box_lo(fam), bh = box_hi(fam);
  if (fabs(st.theta - bh) <= 1e-9 * (1.0 + fabs(bh))) {
    st.theta = bh;
    st.status = ST_BOUNDARY_BOX;
  } else if (fabs(st.theta - bl) <= 1e-9 * (1.0 + fabs(bl))) {
    st.theta = bl;
    st.status = (fam == FAM_GUMBEL) ? ST_BOUNDARY_NATURAL : ST_BOUNDARY_BOX;
  }
}

// One Newton step from the score S and Hessian H at st.theta.
//   S2   : sum of squared per-row scores (sets the rounding-noise floor)
//   tol  : stop when |step| <= tol (1 + |theta|)
//   noise: relative rounding error of one row's score (0 disables the test)
__device__ inline void newton_update(NewtonState& st, int fam, double S, double H, double S2,
                                     double tol, double noise, int max_iter) {
  st.it += 1;
  const double bl = box_lo(fam), bh = box_hi(fam);
  const double th = st.theta;
  if (!isfinite(S) || !isfinite(H)) {  // cannot happen for ranks inside (0,1); keep the subset flagged
    st.status = ST_NOCONV;
    st.done = 1;
    return;
  }
  // a maximum on the boundary: the score points out of the box at an edge
  if (th <= bl && S <= 0.0) {
    st.theta = bl;
    st.status = (fam == FAM_GUMBEL) ? ST_BOUNDARY_NATURAL : ST_BOUNDARY_BOX;
    st.done = 1;
    return;
  }
  if (th >= bh && S >= 0.0) {
    st.theta = bh;
    st.status = ST_BOUNDARY_BOX;
    st.done = 1;
    return;
  }
  if (S > 0.0) st.lo = th; else st.hi = th;
  if (noise > 0.0 && fabs(S) <= noise * sqrt(S2)) {  // the score is zero within rounding
    st.done = 1;
    newton_snap(st, fam);
    return;
  }
  double tn = (H < 0.0) ? th - S / H : NAN;
  bool newton = true;  // tn is the plain Newton step
  if (!(tn > st.lo && tn < st.hi)) {
    newton = false;
    if (!(tn > st.lo) && st.lo == bl && !(st.flags & 1)) {
      tn = bl;
      st.flags |= 1;
    } else if (!(tn < st.hi) && st.hi == bh && !(st.flags & 2)) {
      tn = bh;
      st.flags |= 2;
    } else {
      tn = 0.5 * (st.lo + st.hi);
    }
  }
  const double step = fabs(tn - th);
  const bool edge = (tn == bl) || (tn == bh);
  const double scale = 1.0 + fabs(th);
  // FP32 rows: once the steps stop shrinking below 1e-6 the iteration sits on
  // the rounding noise of the score and further passes change nothing
  const bool stalled = noise > 1e-10 && st.it >= 3 && step > 0.5 * st.prev_step && step <= 1e-6 * scale;
  // Quadratic convergence: the error after this step is about C step^2 with
  // C ~ step / prev_step^2 when the last two steps were plain Newton steps;
  // once that prediction is a tenth of the tolerance the confirming pass
  // is skipped.
  const bool predicted = newton && (st.flags & 4) && step <= 0.1 * st.prev_step &&
                         step * step * step <= 0.1 * tol * scale * st.prev_step * st.prev_step;
  if (!edge && (step <= tol * scale || (st.hi - st.lo) <= tol * scale || stalled || predicted)) {
    st.theta = tn;
    st.done = 1;
    newton_snap(st, fam);
    return;
  }
  st.prev_step = step;
  st.flags = newton ? (st.flags | 4) : (st.flags & ~4);
  st.theta = tn;
  if (st.it >= max_iter) {
    st.status = ST_NOCONV;
    st.done = 1;
  }
}

// Gaussian: the whole solve on the sufficient statistics (no row passes);
// `it` then reports the single pass over the rows.
__device__ inline void gauss_solve(NewtonState& st, double n, double Sp, double Sm, double tol) {
  while (!st.done) {
    double S, H;
    gauss_score_hess(st.theta, n, Sp, Sm, S, H);
    newton_update(st, FAM_GAUSSIAN, S, H, 0.0, tol, 0.0, 200);
  }
  st.it = 1;
}

}  // namespace cpc
