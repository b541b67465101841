// row_eval.h — per-subset constants and per-row evaluation of the pseudo
// log-likelihood terms (eq. 13 of arXiv:1609.05530) from doubled ranks, in
// the arithmetic the kernels use. Shared by the GPU kernels and the host-only
// test shim, so the branch decisions (FP32 rows vs FP64 rows near family
// boundaries, the Frank reflection and series) are the same code in both.
//
// Kernels hoist the family and the FP32/FP64 decision out of their row loops
// and call the family-specific functions (frank_*, gumbel_*, gauss_*) with a
// fixed arithmetic type; row_sh / row_full below are the dispatching wrappers.
#pragma once

#include "family_math.h"

namespace cpc {

enum Family { FAM_GAUSSIAN = 0, FAM_FRANK = 1, FAM_GUMBEL = 2 };

// Rows switch from FP32 to FP64 arithmetic (in the FP32-compensated mode)
// where the FP32 forms lose digits: Frank near independence or far out
// (e^{-theta} leaves FP32 range), Gaussian with |rho| near 1, and Gumbel
// next to its natural boundary theta = 1. There the sign of the summed
// score at theta = 1 decides between the boundary estimate and an interior
// one (an integer status), so it is taken in the oracle's precision; the
// FP32 forms themselves stay accurate to ~2e-8 absolute down to
// theta = 1.001 (the factor theta - 1 is formed in FP64). Near Frank
// independence the log-likelihood is flat (mean d2l/dtheta2 ~ -0.03 at
// theta = 0.1), so a rounding bias of one FP32 ulp in the per-row score
// moves the root by ~2e-6 absolute: FP64 rows below |theta| = 0.5 keep the
// estimate within 1e-5 relative (4e-6 measured worst case above it).
constexpr double FRANK_F32_MIN_ABS = 0.5;
constexpr double FRANK_F32_MAX_ABS = 50.0;
constexpr double GAUSS_F32_MAX_ABS = 0.99;
constexpr double GUMBEL_F32_MIN = 1.01;

// FP64 rows of an FP32-compensated solve at theta (the bands above).
CPC_HD bool rows_in_fp64(int fam, double theta) {
  if (fam == FAM_FRANK) return fabs(theta) < FRANK_F32_MIN_ABS || fabs(theta) > FRANK_F32_MAX_ABS;
  if (fam == FAM_GUMBEL) return theta < GUMBEL_F32_MIN;
  return fabs(theta) > GAUSS_F32_MAX_ABS;
}

// Search box per family (the parameter ranges of eq. 8, 10 and 11).
CPC_HD double box_lo(int fam) { return fam == FAM_GAUSSIAN ? -(1.0 - 1e-9) : (fam == FAM_FRANK ? -200.0 : 1.0); }
CPC_HD double box_hi(int fam) { return fam == FAM_GAUSSIAN ? (1.0 - 1e-9) : (fam == FAM_FRANK ? 200.0 : 100.0); }

template <typename CT>
struct Consts {
  int fam;
  bool use_d;  // (FP32 kernels) evaluate rows in double
  bool neg;    // Frank with theta < 0: reflected
  double theta;
  FrankConst<CT> fk;
  GumbelConst<CT> gk;
  GaussConst<CT> gc;
};

template <typename CT>
CPC_HD Consts<CT> make_consts(int fam, double theta) {
  Consts<CT> c;
  c.fam = fam;
  c.theta = theta;
  c.neg = false;
  c.use_d = sizeof(CT) == 4 && rows_in_fp64(fam, theta);
  if (fam == FAM_FRANK) {
    const double a = fabs(theta);
    c.neg = theta < 0.0;
    c.fk = frank_const<CT>(a > 0.0 ? a : 1.0);  // the FP32 forms only see |theta| >= 0.5
  } else if (fam == FAM_GUMBEL) {
    c.gk = gumbel_const<CT>(theta);
  } else {
    c.gc = gauss_const<CT>(theta);
  }
  return c;
}

// ---------------------------------------------------------------------------
// Frank rows. In double: reflection and series inside frank_row_d. In float:
// the FP32 forms of family_math.h (|theta| within [0.5, 50]).
// FORM (FP32 only): 1 scaled form, 0 direct form, -1 chosen per call (the
// kernels choose once per subset and pass it down); 2 (variance rows only)
// the scaled form near theta = 0, l without its per-subset constant.
template <typename CT, int FORM = -1>
CPC_HD void frank_rsh(const Consts<CT>& c, uint32_t R1, uint32_t R2, uint32_t twon1, CT inv, CT& s,
                      CT& h) {
  const PObs<CT> p = pobs<CT>(R1, twon1, inv), q = pobs<CT>(R2, twon1, inv);
  if constexpr (sizeof(CT) == 8) {
    double l, g1, g2;
    frank_row_d(c.theta, p.u, p.omu, q.u, q.omu, l, s, h, g1, g2);
  } else {
    const CT v = c.neg ? q.omu : q.u, omv = c.neg ? q.u : q.omu;
    CT ss;
    frank_sh<CT, FORM>(c.fk, p.u, v, omv, ss, h);
    s = c.neg ? -ss : ss;
  }
}
template <typename CT, int FORM = -1>
CPC_HD void frank_rfull(const Consts<CT>& c, uint32_t R1, uint32_t R2, uint32_t twon1, CT inv, CT& l,
                        CT& s, CT& g1, CT& g2) {
  const PObs<CT> p = pobs<CT>(R1, twon1, inv), q = pobs<CT>(R2, twon1, inv);
  if constexpr (sizeof(CT) == 8) {
    double h;
    frank_row_d(c.theta, p.u, p.omu, q.u, q.omu, l, s, h, g1, g2);
  } else {
    const CT v = c.neg ? q.omu : q.u, omv = c.neg ? q.u : q.omu;
    CT ll, ss, gg1, gg2;
    frank_full<CT, FORM>(c.fk, p.u, v, omv, ll, ss, gg1, gg2);
    l = (FORM == 2) ? ll : ll + (CT)c.fk.logthE;  // (FORM 2: the constant is the caller's)
    s = c.neg ? -ss : ss;
    g1 = c.neg ? -gg1 : gg1;
    g2 = gg2;
  }
}

// Gumbel rows: lx = log(-log u), ly = log(-log v) (theta-free, may be cached).
template <typename CT>
CPC_HD void gumbel_lxy(uint32_t R1, uint32_t R2, uint32_t twon1, CT inv, CT& lx, CT& ly) {
  const PObs<CT> p = pobs<CT>(R1, twon1, inv), q = pobs<CT>(R2, twon1, inv);
  lx = gumbel_lx(p.u, p.omu);
  ly = gumbel_lx(q.u, q.omu);
}
template <typename CT>
CPC_HD void gumbel_rfull(const Consts<CT>& c, uint32_t R1, uint32_t R2, uint32_t twon1, CT inv, CT lx,
                         CT ly, CT& l, CT& s, CT& g1, CT& g2) {
  const PObs<CT> p = pobs<CT>(R1, twon1, inv), q = pobs<CT>(R2, twon1, inv);
  gumbel_full(c.gk, lx, ly, p.u, q.u, l, s, g1, g2);
}

// Gaussian rows: z = Phi^{-1}(u) by AS 241.
template <typename CT>
CPC_HD void gauss_z(uint32_t R1, uint32_t R2, uint32_t twon1, CT& z1, CT& z2) {
  z1 = qnorm_rank<CT>(R1, twon1);
  z2 = qnorm_rank<CT>(R2, twon1);
}
template <typename CT>
CPC_HD void gauss_rfull(const Consts<CT>& c, CT z1, CT z2, CT& l, CT& s, CT& g1, CT& g2) {
  gauss_row(c.gc, z1, z2, l, s, g1, g2);
  l -= (CT)c.gc.half_log_omr2;
}
// per-row d2l/drho2 (the solve uses the sufficient statistics instead)
template <typename CT>
CPC_HD CT gauss_rh(double r, CT z1, CT z2) {
  const double omr = 1.0 - r, opr = 1.0 + r, omr2 = omr * opr;
  const double a = (double)z1 + (double)z2, d = (double)z1 - (double)z2;
  return (CT)((1.0 + r * r) / (omr2 * omr2) - 0.5 * a * a / (opr * opr * opr) - 0.5 * d * d / (omr * omr * omr));
}

// ---------------------------------------------------------------------------
// Dispatching wrappers (any family; FP64 escalation inside). Used by the
// adjoint kernel and the host test shim.
template <typename CT>
CPC_HD void row_lshf(const Consts<CT>& c, uint32_t R1, uint32_t R2, uint32_t twon1, CT& l, CT& s, CT& h,
                     CT& g1, CT& g2) {
  if (sizeof(CT) == 4 && c.use_d) {
    const Consts<double> cd = make_consts<double>(c.fam, c.theta);
    double ld, sd, hd, g1d, g2d;
    row_lshf<double>(cd, R1, R2, twon1, ld, sd, hd, g1d, g2d);
    l = (CT)ld; s = (CT)sd; h = (CT)hd; g1 = (CT)g1d; g2 = (CT)g2d;
    return;
  }
  const CT inv = (CT)1 / (CT)twon1;
  if (c.fam == FAM_FRANK) {
    CT s2;
    frank_rfull(c, R1, R2, twon1, inv, l, s, g1, g2);
    frank_rsh(c, R1, R2, twon1, inv, s2, h);
  } else if (c.fam == FAM_GUMBEL) {
    CT lx, ly, s2;
    gumbel_lxy(R1, R2, twon1, inv, lx, ly);
    gumbel_rfull(c, R1, R2, twon1, inv, lx, ly, l, s, g1, g2);
    gumbel_sh(c.gk, lx, ly, s2, h);
  } else {
    CT z1, z2;
    gauss_z(R1, R2, twon1, z1, z2);
    gauss_rfull(c, z1, z2, l, s, g1, g2);
    h = gauss_rh<CT>(c.theta, z1, z2);
  }
}

}  // namespace cpc
