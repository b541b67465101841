// k_study.hip — the evaluation side of the simulation study of
// arXiv:1609.05530 (Sec. 2.5-2.6):
//   - replicate summaries: eq. (17) and (18) (means over the S replicates of
//     the combined and the full-data estimates), the estimated bias and MSE
//     of Sec. 2.6 items 1-2;
//   - distances between the copula densities at two parameter values,
//     eq. (19) (relative L1) and eq. (20) (relative L2), by a tensor-product
//     quadrature in normal-score coordinates u = Phi(s), v = Phi(t):
//       int int f(c(u, v)) du dv = int int f(c(Phi(s), Phi(t))) phi(s) phi(t) ds dt,
//     which moves the corners of the unit square (where the Gaussian and
//     Gumbel densities are unbounded) to infinity, where the integrands
//     decay; the box |s|, |t| <= L is covered by `panels` equal panels per
//     axis with the 8-point Gauss-Legendre rule on each, and the inner
//     integral of |c_a - c_b| is split where the two densities cross.
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace cpc {

namespace {

constexpr int QT = 256;  // threads per workgroup

// 8-point Gauss-Legendre rule on [-1, 1] (nodes +-x_k, weights w_k).
__constant__ double kGLx[4] = {0.1834346424956498049, 0.5255324099163289858, 0.7966664774136267396,
                               0.9602898564975362317};
__constant__ double kGLw[4] = {0.3626837833783619830, 0.3137066458778872873, 0.2223810344533744706,
                               0.1012285362903762592};

// node k (0..7) of a panel: abscissa on [-1, 1] and weight
__device__ __forceinline__ void gl_node(int k, double& x, double& w) {
  const int j = k < 4 ? 3 - k : k - 4;
  x = k < 4 ? -kGLx[j] : kGLx[j];
  w = kGLw[j];
}

__device__ __forceinline__ double std_normal_pdf(double s) { return 0.3989422804014326779 * exp(-0.5 * s * s); }

// Node j of the axis: normal score s, quadrature weight times phi(s), and
// u = Phi(s), 1 - u = Phi(-s) (each from erfc, so both tails keep their
// relative accuracy).
struct Node {
  double s, w, u, omu;
};
__device__ __forceinline__ Node axis_node(int64_t j, double L, int panels) {
  const double h = 2.0 * L / panels;
  double x, wk;
  gl_node((int)(j & 7), x, wk);
  Node nd;
  nd.s = -L + h * ((double)(j >> 3) + 0.5 * (x + 1.0));
  nd.w = 0.5 * h * wk * std_normal_pdf(nd.s);
  nd.u = 0.5 * erfc(-nd.s * 0.7071067811865475244);
  nd.omu = 0.5 * erfc(nd.s * 0.7071067811865475244);
  return nd;
}

// log c at the node pair (eq. 5 applied to eq. 8, 10, 11, FP64).
template <int FAM>
__device__ __forceinline__ double log_density(double theta, const Node& a, const Node& b) {
  if constexpr (FAM == FAM_GAUSSIAN) {
    // the normal scores are the node abscissae themselves
    const GaussConst<double> k = gauss_const<double>(theta);
    const double sp = a.s + b.s, sm = a.s - b.s;
    return k.lA * sp * sp - k.lD * sm * sm - k.half_log_omr2;
  } else if constexpr (FAM == FAM_FRANK) {
    double l, s, h, g1, g2;
    frank_row_d(theta, a.u, a.omu, b.u, b.omu, l, s, h, g1, g2);
    return l;
  } else {
    const GumbelConst<double> k = gumbel_const<double>(theta);
    const double lx = gumbel_lx(a.u, a.omu), ly = gumbel_lx(b.u, b.omu);
    double l, s, g1, g2;
    gumbel_full(k, lx, ly, a.u, b.u, l, s, g1, g2);
    return l;
  }
}

// The point t of the t axis (u = Phi(t), 1 - u = Phi(-t)), weight unset.
__device__ __forceinline__ Node point(double t) {
  Node nd;
  nd.s = t;
  nd.w = 0.0;
  nd.u = 0.5 * erfc(-t * 0.7071067811865475244);
  nd.omu = 0.5 * erfc(t * 0.7071067811865475244);
  return nd;
}

template <int FAM>
__device__ __forceinline__ double diff_at(double ta, double tb, const Node& a, const Node& b) {
  return exp(log_density<FAM>(ta, a, b)) - exp(log_density<FAM>(tb, a, b));
}

// int_lo^hi |c_a - c_b| phi(t) dt on the line of node a (8-point rule).
template <int FAM>
__device__ double abs_piece(double ta, double tb, const Node& a, double lo, double hi) {
  double acc = 0.0;
#pragma unroll 1
  for (int k = 0; k < 8; ++k) {
    double x, wk;
    gl_node(k, x, wk);
    const double t = 0.5 * (lo + hi) + 0.5 * (hi - lo) * x;
    acc += 0.5 * (hi - lo) * wk * fabs(diff_at<FAM>(ta, tb, a, point(t))) * std_normal_pdf(t);
  }
  return acc;
}

__device__ __forceinline__ bool crosses(double d0, double d1) { return (d0 < 0.0 && d1 > 0.0) || (d0 > 0.0 && d1 < 0.0); }

// Workgroup (panel i of the s axis, pair p): for each of the panel's 8
// s-nodes, thread j takes t-panels j, j + QT, ...: the densities at the
// panel's 8 nodes give int c_a, int (c_a - c_b)^2 and int c_a^2; for
// int |c_a - c_b| the difference is also taken at the panel's two ends, and
// where it changes sign between two of these samples the panel is split at
// the crossing (bisection in t) and each piece integrated by the same rule
// (the kink of |c_a - c_b| would otherwise limit the rule to second order).
// Four compensated sums per thread, reduced in a fixed order into
// part[(p * panels + i) * 4 + 0..3].
template <int FAM>
__global__ void __launch_bounds__(QT) k_density_partial(const double* theta_a, const double* theta_b, double L,
                                                         int panels, double* part) {
  __shared__ double red[(QT / WAVE) * 4];
  const int i = blockIdx.x, p = blockIdx.y;
  const double ta = theta_a[p], tb = theta_b[p];
  const bool same = ta == tb;
  const double h = 2.0 * L / panels;
  KSum<double> k0, k1, k2, k3;
#pragma unroll 1
  for (int k = 0; k < 8; ++k) {
    const Node a = axis_node((int64_t)i * 8 + k, L, panels);
#pragma unroll 1
    for (int j = threadIdx.x; j < panels; j += QT) {
      const double lo = -L + h * j, hi = lo + h;
      double t[10], d[10];
      t[0] = lo;
      d[0] = same ? 0.0 : diff_at<FAM>(ta, tb, a, point(lo));
      double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
#pragma unroll 1
      for (int q = 0; q < 8; ++q) {
        const Node b = axis_node((int64_t)j * 8 + q, L, panels);
        const double ca = exp(log_density<FAM>(ta, a, b));
        const double cb = same ? ca : exp(log_density<FAM>(tb, a, b));
        const double dd = ca - cb;
        s0 += fabs(dd) * b.w;
        s1 += ca * b.w;
        s2 += dd * dd * b.w;
        s3 += ca * ca * b.w;
        t[q + 1] = b.s;
        d[q + 1] = dd;
      }
      t[9] = hi;
      d[9] = same ? 0.0 : diff_at<FAM>(ta, tb, a, point(hi));
      bool split = false;
#pragma unroll
      for (int q = 1; q < 10; ++q) split |= crosses(d[q - 1], d[q]);
      if (split) {
        s0 = 0.0;
        double from = lo;
#pragma unroll 1
        for (int q = 1; q < 10; ++q) {
          if (!crosses(d[q - 1], d[q])) continue;
          double x0 = t[q - 1], x1 = t[q];
          const bool neg0 = d[q - 1] < 0.0;
#pragma unroll 1
          for (int it = 0; it < 64 && x1 - x0 > 1e-15 * (1.0 + fabs(x0)); ++it) {
            const double xm = 0.5 * (x0 + x1);
            if ((diff_at<FAM>(ta, tb, a, point(xm)) < 0.0) == neg0) x0 = xm; else x1 = xm;
          }
          const double root = 0.5 * (x0 + x1);
          s0 += abs_piece<FAM>(ta, tb, a, from, root);
          from = root;
        }
        s0 += abs_piece<FAM>(ta, tb, a, from, hi);
      }
      k0.add(s0 * a.w);
      k1.add(s1 * a.w);
      k2.add(s2 * a.w);
      k3.add(s3 * a.w);
    }
  }
  double v[4] = {k0.value(), k1.value(), k2.value(), k3.value()};
  block_sum<QT / WAVE, 4, false>(v, red);
  if (threadIdx.x == 0) {
    double* o = part + ((int64_t)p * panels + i) * 4;
    o[0] = v[0]; o[1] = v[1]; o[2] = v[2]; o[3] = v[3];
  }
}

// One wave per pair: the panels' partial sums in panel order.
__global__ void __launch_bounds__(WAVE) k_density_finish(int panels, const double* part, double* out) {
  const int p = blockIdx.x, lane = threadIdx.x;
  KSum<double> s[4];
  for (int i = lane; i < panels; i += WAVE)
#pragma unroll
    for (int c = 0; c < 4; ++c) s[c].add(part[((int64_t)p * panels + i) * 4 + c]);
  __shared__ double red[4];
  double v[4] = {s[0].value(), s[1].value(), s[2].value(), s[3].value()};
  block_sum<1, 4, false>(v, red);
  if (lane == 0)
#pragma unroll
    for (int c = 0; c < 4; ++c) out[p * 4 + c] = v[c];
}

// Sec. 2.6 over S replicates (one workgroup): the combined estimates of
// eq. (16) and the full-data estimates, a replicate counting when both of
// its fits have status 0. out: [0] eq. (17), [1] eq. (18), [2] bias =
// [0] - [1], [3] MSE = mean of squared differences, [4] replicates used.
__global__ void __launch_bounds__(QT) k_replicate_summary(int64_t S, const CombinedOut* comb, const CombinedOut* full,
                                                          double* out) {
  __shared__ double red[(QT / WAVE) * 4];
  KSum<double> sc, sf, sq, cnt;
  for (int64_t s = threadIdx.x; s < S; s += QT) {
    const CombinedOut a = comb[s], b = full[s];
    if (a.status != 0 || b.status != 0) continue;
    const double d = a.theta - b.theta;
    sc.add(a.theta);
    sf.add(b.theta);
    sq.add(d * d);
    cnt.add(1.0);
  }
  double v[4] = {sc.value(), sf.value(), sq.value(), cnt.value()};
  block_sum<QT / WAVE, 4, false>(v, red);
  if (threadIdx.x == 0) {
    const double m = v[3];
    const double mc = v[0] / m, mf = v[1] / m;
    out[0] = mc;
    out[1] = mf;
    out[2] = mc - mf;
    out[3] = v[2] / m;
    out[4] = m;
  }
}

}  // namespace

hipError_t launch_density_distance(int fam, int64_t P, const double* theta_a, const double* theta_b, double L,
                                   int panels, double* part, double* out, hipStream_t s) {
  if (P <= 0) return hipSuccess;
  const dim3 grid((unsigned)panels, (unsigned)P);
  switch (fam) {
    case FAM_GAUSSIAN: hipLaunchKernelGGL(k_density_partial<FAM_GAUSSIAN>, grid, dim3(QT), 0, s, theta_a, theta_b, L, panels, part); break;
    case FAM_FRANK: hipLaunchKernelGGL(k_density_partial<FAM_FRANK>, grid, dim3(QT), 0, s, theta_a, theta_b, L, panels, part); break;
    default: hipLaunchKernelGGL(k_density_partial<FAM_GUMBEL>, grid, dim3(QT), 0, s, theta_a, theta_b, L, panels, part); break;
  }
  hipLaunchKernelGGL(k_density_finish, dim3((unsigned)P), dim3(WAVE), 0, s, panels, part, out);
  return hipGetLastError();
}

hipError_t launch_replicate_summary(int64_t S, const CombinedOut* comb, const CombinedOut* full, double* out,
                                    hipStream_t s) {
  hipLaunchKernelGGL(k_replicate_summary, dim3(1), dim3(QT), 0, s, S, comb, full, out);
  return hipGetLastError();
}

}  // namespace cpc
