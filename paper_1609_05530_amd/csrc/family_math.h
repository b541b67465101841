// family_math.h — per-row log copula density, score, Hessian and mixed
// partials for the three one-parameter families of arXiv:1609.05530,
// Sec. 2.2: Gaussian (eq. 8), Frank (eq. 10), Gumbel (eq. 11); the density of
// each is eq. (5) applied to its copula. The pseudo log-likelihood eq. (13)
// is the sum of `l` over the rows of a subset; its theta-derivatives drive
// the Newton solve and, with the u- and v-mixed partials, the asymptotic
// variance of Sec. 2.3.
//
// Every function is __host__ __device__ and templated on the arithmetic type
// (float for the FP32 row path, double for the FP64 path), so the same code
// is compiled into the GPU kernels and into a host-only shim used by unit
// tests. The derivative formulas are derived by hand from the closed-form
// densities and rearranged to avoid cancellation; the FP64 CPU oracle uses
// automatic differentiation instead and shares nothing with this file.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cmath>

#define CPC_HD __host__ __device__ __forceinline__

namespace cpc {

// FP32 exp and reciprocal of the row paths. In GPU code they go straight to
// the transcendental units: exp(x) = 2^t 2^e with t = fl(x log2 e) and the
// rounding error e = x log2 e - t recovered by two FMAs (log2 e split into a
// float head and tail), 2^t by v_exp_f32 and 2^e by 1 + e ln 2 (|e| <= 2^-17
// for the bounded arguments the rows pass); 1/x by v_rcp_f32. Both are within
// a few ulp, far inside what the FP32 rows tolerate, at a third of the
// instructions of the correctly rounded library routines. The host build
// (used only by unit tests of the formulas) calls libm.
CPC_HD float m_exp(float x) {
#if defined(__HIP_DEVICE_COMPILE__)
  constexpr float kL2E = 1.44269502162933349609375f;  // float(log2 e)
  constexpr float kL2ELo = 1.925963033500011e-08f;     // log2 e - kL2E
  constexpr float kLn2 = 0.693147182464599609375f;
  const float t = x * kL2E;
  const float e = fmaf(x, kL2ELo, fmaf(x, kL2E, -t));
  const float r = __builtin_amdgcn_exp2f(t);
  return fmaf(r, e * kLn2, r);
#else
  return expf(x);
#endif
}
CPC_HD double m_exp(double x) { return exp(x); }
CPC_HD float m_log(float x) { return logf(x); }
CPC_HD double m_log(double x) { return log(x); }
CPC_HD float m_log1p(float x) { return log1pf(x); }
CPC_HD double m_log1p(double x) { return log1p(x); }
CPC_HD float m_expm1(float x) { return expm1f(x); }
CPC_HD double m_expm1(double x) { return expm1(x); }
CPC_HD float m_sqrt(float x) { return sqrtf(x); }
CPC_HD double m_sqrt(double x) { return sqrt(x); }
CPC_HD float m_rcp(float x) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_amdgcn_rcpf(x);
#else
  return 1.0f / x;
#endif
}
CPC_HD double m_rcp(double x) { return 1.0 / x; }
CPC_HD float m_abs(float x) { return fabsf(x); }
CPC_HD double m_abs(double x) { return fabs(x); }

// --------------------------------------------------------------------------
// Pseudo-observations from doubled ranks (eq. 12 with N read as the subset
// size n): u = R / (2(n+1)) and 1 - u = (2(n+1) - R) / (2(n+1)), both from
// exact integers.
template <typename T>
struct PObs {
  T u, omu;
};
template <typename T>
CPC_HD PObs<T> pobs(uint32_t R, uint32_t twon1, T inv_twon1) {
  PObs<T> p;
  p.u = (T)R * inv_twon1;
  p.omu = (T)(twon1 - R) * inv_twon1;
  return p;
}

// --------------------------------------------------------------------------
// Standard normal quantile by Wichura's algorithm AS 241 (Applied Statistics
// 37, 1988): rational approximations in three regions. PPND16 (about 1e-16
// relative) for double, PPND7 (about 1e-7) for float. The argument is the
// doubled rank R with p = R / twon1; the central variable q = p - 1/2 and the
// tail variable min(p, 1-p) are formed from integers, so the tails keep full
// relative accuracy.
// PPND16 from the central variable q = p - 1/2 and the tail probability
// min(p, 1 - p) (each formed exactly by the caller).
CPC_HD double qnorm_ppnd16_qt(double q, double tail) {
  if (fabs(q) <= 0.425) {
    const double r = 0.180625 - q * q;
    const double num = (((((((2.5090809287301226727e3 * r + 3.3430575583588128105e4) * r +
                              6.7265770927008700853e4) * r + 4.5921953931549871457e4) * r +
                            1.3731693765509461125e4) * r + 1.9715909503065514427e3) * r +
                          1.3314166789178437745e2) * r + 3.3871328727963666080e0);
    const double den = (((((((5.2264952788528545610e3 * r + 2.8729085735721942674e4) * r +
                              3.9307895800092710610e4) * r + 2.1213794301586595867e4) * r +
                            5.3941960214247511077e3) * r + 6.8718700749205790830e2) * r +
                          4.2313330701600911252e1) * r + 1.0);
    return q * num / den;
  }
  double r = sqrt(-log(tail));
  double z;
  if (r <= 5.0) {
    r -= 1.6;
    z = (((((((7.74545014278341407640e-4 * r + 2.27238449892691845833e-2) * r +
              2.41780725177450611770e-1) * r + 1.27045825245236838258e0) * r +
            3.64784832476320460504e0) * r + 5.76949722146069140550e0) * r +
          4.63033784615654529590e0) * r + 1.42343711074968357734e0) /
        (((((((1.05075007164441684324e-9 * r + 5.47593808499534494600e-4) * r +
              1.51986665636164571966e-2) * r + 1.48103976427480074590e-1) * r +
            6.89767334985100004550e-1) * r + 1.67638483018380384940e0) * r +
          2.05319162663775882187e0) * r + 1.0);
  } else {
    r -= 5.0;
    z = (((((((2.01033439929228813265e-7 * r + 2.71155556874348757815e-5) * r +
              1.24266094738807843860e-3) * r + 2.65321895265761230930e-2) * r +
            2.96560571828504891230e-1) * r + 1.78482653991729133580e0) * r +
          5.46378491116411436990e0) * r + 6.65790464350110377720e0) /
        (((((((2.04426310338993978564e-15 * r + 1.42151175831644588870e-7) * r +
              1.84631831751005468180e-5) * r + 7.86869131145613259100e-4) * r +
            1.48753612908506148525e-2) * r + 1.36929880922735805310e-1) * r +
          5.99832206555887937690e-1) * r + 1.0);
  }
  return (q < 0.0) ? -z : z;
}
CPC_HD double qnorm_ppnd16(int64_t R, int64_t twon1) {
  const double inv = 1.0 / (double)twon1;
  const double q = (double)(2 * R - twon1) * 0.5 * inv;  // p - 1/2
  const int64_t m = (2 * R < twon1) ? R : (twon1 - R);
  return qnorm_ppnd16_qt(q, (double)m * inv);
}
// Phi^{-1}(p) given p and 1 - p (each exact), from the smaller tail.
CPC_HD double qnorm_p(double p, double omp) {
  if (p == omp) return 0.0;
  return p < omp ? qnorm_ppnd16_qt(p - 0.5, p) : qnorm_ppnd16_qt(0.5 - omp, omp);
}

CPC_HD float qnorm_ppnd7(int64_t R, int64_t twon1) {
  const float inv = 1.0f / (float)twon1;
  const float q = (float)(2 * R - twon1) * 0.5f * inv;
  if (fabsf(q) <= 0.425f) {
    const float r = 0.180625f - q * q;
    return q * (((59.109374720f * r + 159.29113202f) * r + 50.434271938f) * r + 3.3871327179f) *
           m_rcp(((67.187563600f * r + 78.757757664f) * r + 17.895169469f) * r + 1.0f);
  }
  const int64_t m = (2 * R < twon1) ? R : (twon1 - R);
  float r = sqrtf(-logf((float)m * inv));
  float z;
  if (r <= 5.0f) {
    r -= 1.6f;
    z = (((0.17023821103f * r + 1.3067284816f) * r + 2.7568153900f) * r + 1.4234372777f) *
        m_rcp((0.12021132975f * r + 0.73700164250f) * r + 1.0f);
  } else {
    r -= 5.0f;
    z = (((0.017337203997f * r + 0.42868294337f) * r + 3.0812263860f) * r + 6.6579051150f) *
        m_rcp((0.012258202635f * r + 0.24197894225f) * r + 1.0f);
  }
  return (q < 0.0f) ? -z : z;
}

template <typename T>
CPC_HD T qnorm_rank(int64_t R, int64_t twon1);
template <>
CPC_HD float qnorm_rank<float>(int64_t R, int64_t twon1) { return qnorm_ppnd7(R, twon1); }
template <>
CPC_HD double qnorm_rank<double>(int64_t R, int64_t twon1) { return qnorm_ppnd16(R, twon1); }

// --------------------------------------------------------------------------
// Gaussian copula, eq. (8). With z1, z2 the normal scores, a = z1 + z2 and
// d = z1 - z2, the log density is
//   l = -1/2 log(1 - r^2) + r a^2 / (4 (1 + r)) - r d^2 / (4 (1 - r)),
// and (no cancellation as |r| -> 1)
//   dl/dr        = r / (1 - r^2) + a^2 / (4 (1 + r)^2) - d^2 / (4 (1 - r)^2)
//   d2l/dr du1   = [a / (2 (1 + r)^2) - d / (2 (1 - r)^2)] / phi(z1)
//   d2l/dr du2   = [a / (2 (1 + r)^2) + d / (2 (1 - r)^2)] / phi(z2).
// The subset solve only needs S+ = sum a^2 and S- = sum d^2.
template <typename T>
struct GaussConst {
  T r_omr2;     // r / (1 - r^2)
  T cA, cD;     // 1 / (4 (1 + r)^2), 1 / (4 (1 - r)^2)
  T lA, lD;     // r / (4 (1 + r)), r / (4 (1 - r))
  double half_log_omr2;
};
CPC_HD void gauss_const_d(double r, double& r_omr2, double& cA, double& cD, double& lA, double& lD,
                          double& hl) {
  const double omr = 1.0 - r, opr = 1.0 + r;
  r_omr2 = r / (omr * opr);
  cA = 0.25 / (opr * opr);
  cD = 0.25 / (omr * omr);
  lA = 0.25 * r / opr;
  lD = 0.25 * r / omr;
  hl = 0.5 * (log1p(-r) + log1p(r));
}
template <typename T>
CPC_HD GaussConst<T> gauss_const(double r) {
  double a, b, c, d, e, f;
  gauss_const_d(r, a, b, c, d, e, f);
  GaussConst<T> k;
  k.r_omr2 = (T)a; k.cA = (T)b; k.cD = (T)c; k.lA = (T)d; k.lD = (T)e; k.half_log_omr2 = f;
  return k;
}
// Per row (l without the -1/2 log(1 - r^2) constant): l, s, g1, g2.
template <typename T>
CPC_HD void gauss_row(const GaussConst<T>& k, T z1, T z2, T& l, T& s, T& g1, T& g2) {
  const T a = z1 + z2, d = z1 - z2;
  const T a2 = a * a, d2 = d * d;
  l = k.lA * a2 - k.lD * d2;
  s = k.r_omr2 + k.cA * a2 - k.cD * d2;
  // 1 / phi(z) = sqrt(2 pi) exp(z^2 / 2)
  const T s2pi = (T)2.5066282746310002;
  const T ia = (T)2 * k.cA * a, id = (T)2 * k.cD * d;
  g1 = (ia - id) * s2pi * m_exp((T)0.5 * z1 * z1);
  g2 = (ia + id) * s2pi * m_exp((T)0.5 * z2 * z2);
}
// Score and Hessian of eq. (13) from the sufficient statistics (FP64).
CPC_HD void gauss_score_hess(double r, double n, double Sp, double Sm, double& S, double& H) {
  const double omr = 1.0 - r, opr = 1.0 + r, omr2 = omr * opr;
  S = n * r / omr2 + 0.25 * (Sp / (opr * opr) - Sm / (omr * omr));
  H = n * (1.0 + r * r) / (omr2 * omr2) - 0.5 * (Sp / (opr * opr * opr) + Sm / (omr * omr * omr));
}
CPC_HD double gauss_loglik(double r, double n, double Sp, double Sm) {
  return -0.5 * n * (log1p(-r) + log1p(r)) + 0.25 * r * (Sp / (1.0 + r) - Sm / (1.0 - r));
}

// --------------------------------------------------------------------------
// Frank copula, eq. (10), for theta > 0 (negative theta by the reflection
// c(u, v; theta) = c(u, 1 - v; -theta), applied by the caller). With
// a = e^{-theta u}, b = e^{-theta v}, e = e^{-theta}, E = 1 - e:
//   c = theta E e^{-theta (u + v)} / D^2,
//   D = E - (1 - a)(1 - b) = a (1 - b) + b (1 - e^{-theta (1 - v)}) > 0,
//   l = log(theta E) - theta (u + v) - 2 log D.
// Writing D' = dD/dtheta and D'' = d2D/dtheta2,
//   D'  = e - u a (1 - b) - v b (1 - a)
//   D'' = -e + u^2 a (1 - b) - 2 u v a b + v^2 b (1 - a)
//   dl/dtheta   = 1/theta + e/E - (u + v) - 2 D'/D
//   d2l/dtheta2 = -1/theta^2 - e/E - (e/E)^2 - 2 D''/D + 2 (D'/D)^2
//   d2l/dtheta du = -1 - 2 (D'_u / D - D' D_u / D^2),
//     D_u = -theta a (1 - b),  D'_u = -a (1 - theta u)(1 - b) - theta v a b,
// and symmetrically in v.
template <typename T>
struct FrankConst {
  T th, e, C1, C2;  // theta (> 0), e^{-theta}, 1/theta + e/E, -1/theta^2 - e/E - (e/E)^2
  T Eh, iEh, psi;   // E/theta, theta/E, (E/theta - e)/theta (scaled form, small theta)
  T ith;            // 1/theta
  double logthE;    // log(theta E)
  double logth;     // log(theta)
};
template <typename T>
CPC_HD FrankConst<T> frank_const(double th) {
  const double e = exp(-th), E = -expm1(-th), r = e / E;
  FrankConst<T> k;
  k.th = (T)th;
  k.e = (T)e;
  k.C1 = (T)(1.0 / th + r);
  k.C2 = (T)(-1.0 / (th * th) - r - r * r);
  k.Eh = (T)(E / th);
  k.iEh = (T)(th / E);
  k.psi = (T)((E - th * e) / (th * th));
  k.ith = (T)(1.0 / th);
  k.logthE = log(th * E);
  k.logth = log(th);
  return k;
}

// In FP32 and for theta below FRANK_SCALED_BELOW the score is evaluated in a
// scaled form without the 1/theta terms that otherwise cancel: with
// Ah = (1 - a)/theta, Bh = (1 - b)/theta, Eh = E/theta,
// psi = (Eh - e)/theta and Dh = D/theta = Eh - theta Ah Bh,
//   dl/dtheta = (Eh psi - Ah Bh (Eh + e)) / (Eh Dh) - (u + v) + 2 (u a Bh + v b Ah) / Dh.
constexpr double FRANK_SCALED_BELOW = 2.0;

// 1 - e^{-x} and related terms: FP64 uses expm1 throughout; FP32 forms 1 - a
// from a (absolute error of one rounding, which is all D needs since every
// term of D is non-negative).
template <typename T>
struct FrankTerms {
  T a, b, Am, Bm, D, iD, Dp, r1;
};
template <typename T>
CPC_HD FrankTerms<T> frank_terms(const FrankConst<T>& k, T u, T v, T omv) {
  FrankTerms<T> t;
  const T th = k.th;
  t.a = m_exp(-th * u);
  t.b = m_exp(-th * v);
  T Tm;
  if constexpr (sizeof(T) == 8) {
    t.Am = -m_expm1(-th * u);
    t.Bm = -m_expm1(-th * v);
    Tm = -m_expm1(-th * omv);
  } else {
    (void)omv;
    t.Am = (T)1 - t.a;
    t.Bm = (T)1 - t.b;
    Tm = (T)1 - k.e * m_rcp(t.b);  // 1 - e^{-theta (1 - v)}
  }
  t.D = t.a * t.Bm + t.b * Tm;
  t.iD = m_rcp(t.D);
  t.Dp = k.e - u * t.a * t.Bm - v * t.b * t.Am;
  t.r1 = t.Dp * t.iD;
  return t;
}
// Newton pass: score and Hessian per row. FORM: 1 the scaled form (FP32,
// theta below FRANK_SCALED_BELOW), 0 the direct form, -1 chosen here.
template <typename T, int FORM = -1>
CPC_HD void frank_sh(const FrankConst<T>& k, T u, T v, T omv, T& s, T& h) {
  const bool scaled = FORM == 1 || (FORM == -1 && sizeof(T) == 4 && k.th < (T)FRANK_SCALED_BELOW);
  if (scaled) {
    const T th = k.th;
    const T Ah = -m_expm1(-th * u) * k.ith, Bh = -m_expm1(-th * v) * k.ith;
    const T a = (T)1 - th * Ah, b = (T)1 - th * Bh;
    const T iDh = m_rcp(k.Eh - th * Ah * Bh);
    const T P = u * a * Bh + v * b * Ah;
    s = (k.Eh * k.psi - Ah * Bh * (k.Eh + k.e)) * k.iEh * iDh - (u + v) + (T)2 * P * iDh;
    const T ith = k.ith;
    const T r1 = (k.e - th * P) * iDh * ith;
    const T r2 = (-k.e + th * (u * u * a * Bh + v * v * b * Ah) - (T)2 * u * v * a * b) * iDh * ith;
    h = k.C2 - (T)2 * r2 + (T)2 * r1 * r1;
    return;
  }
  const FrankTerms<T> t = frank_terms(k, u, v, omv);
  const T Dpp = -k.e + u * u * t.a * t.Bm - (T)2 * u * v * t.a * t.b + v * v * t.b * t.Am;
  const T r2 = Dpp * t.iD;
  s = k.C1 - (u + v) - (T)2 * t.r1;
  h = k.C2 - (T)2 * r2 + (T)2 * t.r1 * t.r1;
}
// Adjoint pass: l (without log(theta E)), score and Hessian from one D.
template <typename T, int FORM = -1>
CPC_HD void frank_lsh(const FrankConst<T>& k, T u, T v, T omv, T& l, T& s, T& h) {
  const bool scaled = FORM == 1 || (FORM == -1 && sizeof(T) == 4 && k.th < (T)FRANK_SCALED_BELOW);
  const T th = k.th;
  if (scaled) {
    const T Ah = -m_expm1(-th * u) * k.ith, Bh = -m_expm1(-th * v) * k.ith;
    const T a = (T)1 - th * Ah, b = (T)1 - th * Bh;
    const T Dh = k.Eh - th * Ah * Bh;
    const T iDh = m_rcp(Dh);
    const T P = u * a * Bh + v * b * Ah;
    l = -th * (u + v) - (T)2 * ((T)k.logth + m_log(Dh));
    s = (k.Eh * k.psi - Ah * Bh * (k.Eh + k.e)) * k.iEh * iDh - (u + v) + (T)2 * P * iDh;
    const T ith = k.ith;
    const T r1 = (k.e - th * P) * iDh * ith;
    const T r2 = (-k.e + th * (u * u * a * Bh + v * v * b * Ah) - (T)2 * u * v * a * b) * iDh * ith;
    h = k.C2 - (T)2 * r2 + (T)2 * r1 * r1;
    return;
  }
  const FrankTerms<T> t = frank_terms(k, u, v, omv);
  const T Dpp = -k.e + u * u * t.a * t.Bm - (T)2 * u * v * t.a * t.b + v * v * t.b * t.Am;
  l = -th * (u + v) - (T)2 * m_log(t.D);
  s = k.C1 - (u + v) - (T)2 * t.r1;
  h = k.C2 - (T)2 * Dpp * t.iD + (T)2 * t.r1 * t.r1;
}
// Variance pass: l (without log(theta E)), score, d2l/dtheta du, d2l/dtheta dv.
// FORM 2 (FP32, theta near 0): the scaled form with l written as
// -theta (u + v) - 2 log1p(-theta Ah Bh / Eh), which is O(theta) and keeps its
// relative accuracy; the caller adds the per-subset constant log(theta / E)
// (the rest of -2 log(theta Dh) + log(theta E)) in FP64.
template <typename T, int FORM = -1>
CPC_HD void frank_full(const FrankConst<T>& k, T u, T v, T omv, T& l, T& s, T& g1, T& g2) {
  const T th = k.th;
  const bool scaled = FORM >= 1 || (FORM == -1 && sizeof(T) == 4 && k.th < (T)FRANK_SCALED_BELOW);
  if (scaled) {
    const T Ah = -m_expm1(-th * u) * k.ith, Bh = -m_expm1(-th * v) * k.ith;
    const T a = (T)1 - th * Ah, b = (T)1 - th * Bh;
    const T Dh = k.Eh - th * Ah * Bh;
    const T iDh = m_rcp(Dh);
    const T P = u * a * Bh + v * b * Ah;
    if constexpr (FORM == 2)
      l = -th * (u + v) - (T)2 * m_log1p(-th * Ah * Bh * k.iEh);
    else
      l = -th * (u + v) - (T)2 * ((T)k.logth + m_log(Dh));
    s = (k.Eh * k.psi - Ah * Bh * (k.Eh + k.e)) * k.iEh * iDh - (u + v) + (T)2 * P * iDh;
    const T r1t = (k.e - th * P) * iDh;  // theta D'/D
    const T ab = a * b;
    g1 = (T)-1 - (T)2 * (-a * ((T)1 - th * u) * Bh - v * ab + r1t * a * Bh) * iDh;
    g2 = (T)-1 - (T)2 * (-b * ((T)1 - th * v) * Ah - u * ab + r1t * b * Ah) * iDh;
    return;
  }
  const FrankTerms<T> t = frank_terms(k, u, v, omv);
  l = -th * (u + v) - (T)2 * m_log(t.D);
  s = k.C1 - (u + v) - (T)2 * t.r1;
  const T Du = -th * t.a * t.Bm;
  const T Dv = -th * t.b * t.Am;
  const T ab = t.a * t.b;
  const T Dpu = -t.a * ((T)1 - th * u) * t.Bm - th * v * ab;
  const T Dpv = -t.b * ((T)1 - th * v) * t.Am - th * u * ab;
  g1 = (T)-1 - (T)2 * (Dpu - t.r1 * Du) * t.iD;
  g2 = (T)-1 - (T)2 * (Dpv - t.r1 * Dv) * t.iD;
}

// Near theta = 0 (|theta| < FRANK_SERIES_BELOW) the density tends to 1 and
// the closed form cancels; there l is the Taylor series in theta through
// theta^5, with A = u(1-u), B = v(1-v), su = 2u - 1, sv = 2v - 1:
//   c1 = su sv / 2, c2 = A B - 1/24, c3 = A B su sv / 6,
//   c4 = (A B)^2 / 2 - A B (A + B) / 12 + 1/2880,
//   c5 = A B su sv (36 A B - 3 A - 3 B - 1) / 360.
// Valid for either sign of theta (no reflection).
constexpr double FRANK_SERIES_BELOW = 3e-3;

CPC_HD void frank_series(double th, double u, double omu, double v, double omv, double& l,
                         double& s, double& h, double& g1, double& g2) {
  const double A = u * omu, B = v * omv, su = u - omu, sv = v - omv, AB = A * B;
  const double c1 = 0.5 * su * sv;
  const double c2 = AB - 1.0 / 24.0;
  const double c3 = AB * su * sv / 6.0;
  const double c4 = 0.5 * AB * AB - AB * (A + B) / 12.0 + 1.0 / 2880.0;
  const double P = 36.0 * AB - 3.0 * A - 3.0 * B - 1.0;
  const double c5 = AB * su * sv * P / 360.0;
  // u-derivatives (dA/du = -su, d su/du = 2)
  const double c1u = sv;
  const double c2u = -su * B;
  const double c3u = B * sv * (2.0 * A - su * su) / 6.0;
  const double c4u = -su * (A * B * B - (2.0 * A * B + B * B) / 12.0);
  const double c5u = sv * B * ((2.0 * A - su * su) * P - A * su * su * (36.0 * B - 3.0)) / 360.0;
  const double c1v = su;
  const double c2v = -sv * A;
  const double c3v = A * su * (2.0 * B - sv * sv) / 6.0;
  const double c4v = -sv * (B * A * A - (2.0 * A * B + A * A) / 12.0);
  const double c5v = su * A * ((2.0 * B - sv * sv) * P - B * sv * sv * (36.0 * A - 3.0)) / 360.0;
  const double t = th;
  l = t * (c1 + t * (c2 + t * (c3 + t * (c4 + t * c5))));
  s = c1 + t * (2.0 * c2 + t * (3.0 * c3 + t * (4.0 * c4 + t * 5.0 * c5)));
  h = 2.0 * c2 + t * (6.0 * c3 + t * (12.0 * c4 + t * 20.0 * c5));
  g1 = c1u + t * (2.0 * c2u + t * (3.0 * c3u + t * (4.0 * c4u + t * 5.0 * c5u)));
  g2 = c1v + t * (2.0 * c2v + t * (3.0 * c3v + t * (4.0 * c4v + t * 5.0 * c5v)));
}

// Frank row in double for any theta (reflection and series included).
// Returns l (full log density), s, h, g1, g2.
CPC_HD void frank_row_d(double th, double u, double omu, double v, double omv, double& l,
                        double& s, double& h, double& g1, double& g2) {
  if (fabs(th) < FRANK_SERIES_BELOW) {
    frank_series(th, u, omu, v, omv, l, s, h, g1, g2);
    return;
  }
  const bool neg = th < 0.0;
  const double vv = neg ? omv : v, ovv = neg ? v : omv;
  const FrankConst<double> k = frank_const<double>(fabs(th));
  double ll, ss, gg1, gg2, hh, s2;
  frank_full(k, u, vv, ovv, ll, ss, gg1, gg2);
  frank_sh(k, u, vv, ovv, s2, hh);
  l = ll + k.logthE;
  s = neg ? -ss : ss;
  h = hh;
  g1 = neg ? -gg1 : gg1;
  g2 = gg2;
}

// --------------------------------------------------------------------------
// Gumbel copula, eq. (11), theta >= 1. With x = -log u, y = -log v,
// lx = log x, ly = log y, lM = max(lx, ly), lm = min, dl = lM - lm,
// delta = theta dl, q = e^{-delta}, A = x^theta + y^theta:
//   log A = theta lM + log(1 + q),   w = A^{1/theta},
//   c = C(u, v) (xy)^{theta-1} / (uv) A^{1/theta - 2} (w + theta - 1),
//   l = -w + (theta-1)(lx + ly) + x + y + (1/theta - 2) log A + log(w + theta - 1).
// With H = q delta / (1 + q) + log(1 + q) >= 0 (= log A - theta R1, where R1
// is the x^theta / A-weighted mean of lx, ly) and V = q dl^2 / (1 + q)^2:
//   g1 = d(log A / theta)/dtheta = -H / theta^2,
//   g2 = d2(log A / theta)/dtheta2 = V / theta + 2 H / theta^3,
//   w_t = w g1,  w_tt = w (g1^2 + g2),  den = w + theta - 1,
//   dl/dtheta   = -w_t - dl (1 - q)/(1 + q) - H / theta^2 + (w_t + 1) / den
//   d2l/dtheta2 = -w_tt + w_tt / den - ((w_t + 1)/den)^2 + 2 H / theta^3 + (1/theta - 2) V.
// Mixed partials via d lx / du = -1 / (x u):
//   d(dl/dtheta)/d lx = -dwx + 1 - px/theta + (1/theta - 2)(px + theta px py (lx - ly))
//                        + dwx / den - (w_t + 1) w px / den^2,
//   dwx = w px g1 + w px py (lx - ly),  px = x^theta / A,  py = 1 - px.
template <typename T>
struct GumbelConst {
  T th, thm1, ith, ith2, ith3;  // theta, theta - 1 (formed in double: w + (theta - 1) keeps w's digits)
};
template <typename T>
CPC_HD GumbelConst<T> gumbel_const(double th) {
  GumbelConst<T> k;
  k.th = (T)th;
  k.thm1 = (T)(th - 1.0);
  k.ith = (T)(1.0 / th);
  k.ith2 = (T)(1.0 / (th * th));
  k.ith3 = (T)(1.0 / (th * th * th));
  return k;
}
// lx = log(-log u) from the doubled rank (u near 1 through log1p(-(1 - u))).
template <typename T>
CPC_HD T gumbel_lx(T u, T omu) {
  const T x = (u < (T)0.5) ? -m_log(u) : -m_log1p(-omu);
  return m_log(x);
}
template <typename T>
struct GumbelTerms {
  T lM, lm, dl, q, ip, H, LA, V, w, g1, g2, wt, wtt, iden;
};
template <typename T>
CPC_HD GumbelTerms<T> gumbel_terms(const GumbelConst<T>& k, T lx, T ly) {
  GumbelTerms<T> t;
  t.lM = lx > ly ? lx : ly;
  t.lm = lx > ly ? ly : lx;
  t.dl = t.lM - t.lm;
  const T delta = k.th * t.dl;
  t.q = m_exp(-delta);
  t.ip = m_rcp((T)1 + t.q);
  const T l1q = m_log((T)1 + t.q);
  t.H = t.q * delta * t.ip + l1q;
  t.LA = k.th * t.lM + l1q;
  t.V = t.q * t.ip * t.ip * t.dl * t.dl;
  t.w = m_exp(t.LA * k.ith);
  t.g1 = -t.H * k.ith2;
  t.g2 = t.V * k.ith + (T)2 * t.H * k.ith3;
  t.wt = t.w * t.g1;
  t.wtt = t.w * (t.g1 * t.g1 + t.g2);
  t.iden = m_rcp(t.w + k.thm1);
  return t;
}
template <typename T>
CPC_HD void gumbel_sh(const GumbelConst<T>& k, T lx, T ly, T& s, T& h) {
  const GumbelTerms<T> t = gumbel_terms(k, lx, ly);
  const T a = (t.wt + (T)1) * t.iden;
  s = -t.wt - t.dl * ((T)1 - t.q) * t.ip - t.H * k.ith2 + a;
  h = -t.wtt + t.wtt * t.iden - a * a + (T)2 * t.H * k.ith3 + (k.ith - (T)2) * t.V;
}
// Adjoint pass: l, score and Hessian from one set of terms.
template <typename T>
CPC_HD void gumbel_lsh(const GumbelConst<T>& k, T lx, T ly, T& l, T& s, T& h) {
  const GumbelTerms<T> t = gumbel_terms(k, lx, ly);
  const T a = (t.wt + (T)1) * t.iden;
  s = -t.wt - t.dl * ((T)1 - t.q) * t.ip - t.H * k.ith2 + a;
  h = -t.wtt + t.wtt * t.iden - a * a + (T)2 * t.H * k.ith3 + (k.ith - (T)2) * t.V;
  l = -t.w + k.thm1 * (lx + ly) + m_exp(lx) + m_exp(ly) + (k.ith - (T)2) * t.LA + m_log(t.w + k.thm1);
}
// Variance pass: l, s, g1 = d2l/dtheta du, g2 = d2l/dtheta dv.
template <typename T>
CPC_HD void gumbel_full(const GumbelConst<T>& k, T lx, T ly, T u, T v, T& l, T& s, T& g1, T& g2) {
  const GumbelTerms<T> t = gumbel_terms(k, lx, ly);
  const T a = (t.wt + (T)1) * t.iden;
  s = -t.wt - t.dl * ((T)1 - t.q) * t.ip - t.H * k.ith2 + a;
  const T x = m_exp(lx), y = m_exp(ly);
  l = -t.w + k.thm1 * (lx + ly) + x + y + (k.ith - (T)2) * t.LA + m_log(t.w + k.thm1);
  const bool xmax = lx > ly;
  const T px = xmax ? t.ip : t.q * t.ip;
  const T py = xmax ? t.q * t.ip : t.ip;
  const T dxy = lx - ly;
  const T pxy = px * py;
  const T wp = t.w * pxy * dxy;
  const T dwx = t.w * px * t.g1 + wp;
  const T dwy = t.w * py * t.g1 - wp;
  const T c = k.ith - (T)2;
  const T z = (t.wt + (T)1) * t.w * t.iden * t.iden;
  const T dsx = -dwx + (T)1 - px * k.ith + c * (px + k.th * pxy * dxy) + dwx * t.iden - z * px;
  const T dsy = -dwy + (T)1 - py * k.ith + c * (py - k.th * pxy * dxy) + dwy * t.iden - z * py;
  // d lx / du = -1 / (x u)
  g1 = -dsx * m_rcp(x * u);
  g2 = -dsy * m_rcp(y * v);
}

}  // namespace cpc
