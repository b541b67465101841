// k_sample.hip — simulation inputs drawn on the device (Sec. 2.5 of
// arXiv:1609.05530: the data are simulated from the copula itself, eq. 8,
// 10 and 11, here with N(0, 1) margins). Every row is an independent draw
// of a counter-based generator, so a launch needs no state, any row range
// can be drawn on its own, and results do not depend on the launch shape.
//
// Generator: Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC 2011), counter
// (row low word, row high word, block, 0), key (seed low word, seed high
// word). Two uniforms per block: 52 random bits k, u = (k + 1/2) 2^-52 and
// 1 - u formed exactly from k. One thread per row, grid-stride; FP64
// arithmetic, the result stored as FP64 or rounded to FP32.
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace cpc {

namespace {

struct U2 {
  double u[2], omu[2];
};

__device__ __forceinline__ U2 philox_uniforms(uint64_t seed, uint64_t row, uint32_t blk) {
  uint32_t c0 = (uint32_t)row, c1 = (uint32_t)(row >> 32), c2 = blk, c3 = 0u;
  uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint32_t lo0 = 0xD2511F53u * c0, hi0 = __umulhi(0xD2511F53u, c0);
    const uint32_t lo1 = 0xCD9E8D57u * c2, hi1 = __umulhi(0xCD9E8D57u, c2);
    const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  U2 r;
  const uint64_t ka = ((uint64_t)(c0 & 0xFFFFFu) << 32) | c1;
  const uint64_t kb = ((uint64_t)(c2 & 0xFFFFFu) << 32) | c3;
  r.u[0] = ((double)ka + 0.5) * 0x1p-52;
  r.omu[0] = (4503599627370496.0 - (double)ka - 0.5) * 0x1p-52;
  r.u[1] = ((double)kb + 0.5) * 0x1p-52;
  r.omu[1] = (4503599627370496.0 - (double)kb - 0.5) * 0x1p-52;
  return r;
}

// -log(u) for u ~ U(0, 1): from 1 - u where u is near 1.
__device__ __forceinline__ double neg_log(double u, double omu) { return u < 0.5 ? -log(u) : -log1p(-omu); }

// Phi^{-1}(e^{-t}): the upper tail from 1 - e^{-t} = -expm1(-t); t at most
// 700 (e^{-700} ~ 1e-304, a normal double).
__device__ __forceinline__ double qnorm_exp_neg(double t) {
  t = fmin(t, 700.0);
  return qnorm_p(exp(-t), -expm1(-t));
}

template <typename OT>
__global__ void __launch_bounds__(256) k_sample(int fam, double theta, uint64_t seed, int64_t row0, int64_t n,
                                                OT* __restrict__ x, OT* __restrict__ y) {
  const double pi = 3.141592653589793;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t row = (uint64_t)(row0 + i);
    const U2 a = philox_uniforms(seed, row, 0u);
    double xv, yv;
    if (fam == FAM_GAUSSIAN) {
      // Cholesky factor of [[1, rho], [rho, 1]] applied to two N(0, 1) draws
      const double z1 = qnorm_p(a.u[0], a.omu[0]), z2 = qnorm_p(a.u[1], a.omu[1]);
      xv = z1;
      yv = theta * z1 + sqrt((1.0 - theta) * (1.0 + theta)) * z2;
    } else if (fam == FAM_FRANK) {
      // dC/du (u, v) = w solved for v: e^{-theta v} = ((1 - w) e^{-theta u} +
      // w e^{-theta}) / (w + (1 - w) e^{-theta u}), written as
      // v = u - D / theta and 1 - v = (1 - u) + D / theta
      double v = a.u[1], omv = a.omu[1];
      if (theta != 0.0) {
        const double D = log1p(a.u[1] * expm1(-theta * a.omu[0])) - log1p(a.omu[1] * expm1(-theta * a.u[0]));
        v = a.u[0] - D / theta;
        omv = a.omu[0] + D / theta;
      }
      v = fmin(fmax(v, 0x1p-1000), 1.0 - 0x1p-53);
      omv = fmin(fmax(omv, 0x1p-1000), 1.0 - 0x1p-53);
      xv = qnorm_p(a.u[0], a.omu[0]);
      yv = qnorm_p(v, omv);
    } else {
      // Marshall-Olkin: a positive stable frailty S (Laplace transform
      // exp(-s^alpha), alpha = 1/theta) by Kanter's representation, in
      // logarithms; U_j = exp(-(E_j / S)^alpha) with E_j ~ Exp(1)
      const U2 b = philox_uniforms(seed, row, 1u);
      const double e1 = neg_log(a.u[0], a.omu[0]), e2 = neg_log(a.u[1], a.omu[1]);
      const double alpha = 1.0 / theta;
      double logS = 0.0;
      if (theta != 1.0) {
        const double T = pi * b.u[0];
        const double W = neg_log(b.u[1], b.omu[1]);
        logS = log(sin(alpha * T)) - log(sin(T)) / alpha + (1.0 - alpha) / alpha * (log(sin((1.0 - alpha) * T)) - log(W));
      }
      xv = qnorm_exp_neg(exp(alpha * (log(e1) - logS)));
      yv = qnorm_exp_neg(exp(alpha * (log(e2) - logS)));
    }
    x[i] = (OT)xv;
    y[i] = (OT)yv;
  }
}

}  // namespace

hipError_t launch_sample(int fam, double theta, uint64_t seed, int64_t row0, int64_t n, int f32, void* x, void* y,
                         hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t want = (n + 255) / 256;
  const unsigned grid = (unsigned)(want < 8192 ? want : 8192);
  if (f32)
    hipLaunchKernelGGL(k_sample<float>, dim3(grid), dim3(256), 0, s, fam, theta, seed, row0, n, (float*)x, (float*)y);
  else
    hipLaunchKernelGGL(k_sample<double>, dim3(grid), dim3(256), 0, s, fam, theta, seed, row0, n, (double*)x,
                       (double*)y);
  return hipGetLastError();
}

}  // namespace cpc
