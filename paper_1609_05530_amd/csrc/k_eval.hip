// k_eval.hip — the adjoint of the pseudo log-likelihood eq. (13) of
// arXiv:1609.05530: for each subset m at a given theta_m, the sums over the
// subset's rows of l, dl/dtheta and d2l/dtheta2 (eq. 5 applied to eq. 8, 10
// or 11), from doubled ranks. One workgroup per subset, its size chosen from
// the largest subset of the call; the family is a template argument and the
// FP32 / FP64 row decision (the precision bands of row_eval.h) is taken once
// per subset, with the family constants formed once. Rows are streamed with
// coalesced loads; per-thread compensated sums meet in a fixed-order
// workgroup reduction (bitwise reproducible). Frank and Gumbel rows evaluate
// l, s and h from one set of intermediate terms; the Gaussian sums the
// sufficient statistics S+ = sum (z1 + z2)^2 and S- = sum (z1 - z2)^2 and
// forms l, s, h from them in FP64, as the maximisation does.
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace cpc {

namespace {

// this thread's partial sums over the rows of one subset (v[0..2]: l, s, h;
// the Gaussian: S+, S-, unused)
template <int T, typename CT, int FAM, int FORM>
__device__ __forceinline__ void eval_rows(const uint32_t* R1, const uint32_t* R2, int n, const Consts<CT>& c,
                                          double (&v)[3]) {
  const uint32_t twon1 = 2u * (uint32_t)(n + 1);
  const CT inv = (CT)1 / (CT)twon1;
  RowSum<CT> k0, k1, k2;
  for (int i = threadIdx.x; i < n; i += T) {
    const uint32_t r1 = R1[i], r2 = R2[i];
    if constexpr (FAM == FAM_GAUSSIAN) {
      CT z1, z2;
      gauss_z<CT>(r1, r2, twon1, z1, z2);
      const CT a = z1 + z2, d = z1 - z2;
      k0.add(a * a);
      k1.add(d * d);
    } else if constexpr (FAM == FAM_FRANK) {
      CT l, s, h;
      if constexpr (sizeof(CT) == 8) {
        const PObs<CT> p = pobs<CT>(r1, twon1, inv), q = pobs<CT>(r2, twon1, inv);
        double g1, g2;
        frank_row_d(c.theta, p.u, p.omu, q.u, q.omu, l, s, h, g1, g2);
      } else {
        const PObs<CT> p = pobs<CT>(r1, twon1, inv), q = pobs<CT>(r2, twon1, inv);
        const CT vv = c.neg ? q.omu : q.u, omv = c.neg ? q.u : q.omu;
        frank_lsh<CT, FORM>(c.fk, p.u, vv, omv, l, s, h);
        l += (CT)c.fk.logthE;
        if (c.neg) s = -s;
      }
      k0.add(l);
      k1.add(s);
      k2.add(h);
    } else {
      CT lx, ly, l, s, h;
      gumbel_lxy<CT>(r1, r2, twon1, inv, lx, ly);
      gumbel_lsh(c.gk, lx, ly, l, s, h);
      k0.add(l);
      k1.add(s);
      k2.add(h);
    }
  }
  v[0] = k0.value();
  v[1] = k1.value();
  v[2] = k2.value();
}

template <int T, typename CT, int FAM>
__global__ void __launch_bounds__(T) k_eval_wg(const uint32_t* R1, const uint32_t* R2, const SubDesc* subs,
                                               const double* theta, double* out) {
  constexpr int W = T / WAVE;
  __shared__ double red[W * 3];
  const int m = blockIdx.x;
  const SubDesc sd = subs[m];
  const int n = sd.n;
  const double th = theta[m];
  const bool inside = (FAM == FAM_GAUSSIAN) ? (th > -1.0 && th < 1.0) : (FAM == FAM_GUMBEL ? th >= 1.0 : isfinite(th));
  if (!inside || n < 1) {
    if (threadIdx.x == 0) {
      const double v = (n < 1) ? 0.0 : NAN;
      out[3 * m] = v; out[3 * m + 1] = v; out[3 * m + 2] = v;
    }
    return;
  }
  const uint32_t* r1 = R1 + sd.begin;
  const uint32_t* r2 = R2 + sd.begin;
  double v[3];
  if (sizeof(CT) == 4 && rows_in_fp64(FAM, th)) {  // workgroup-uniform
    const Consts<double> c = make_consts<double>(FAM, th);
    eval_rows<T, double, FAM, -1>(r1, r2, n, c, v);
  } else {
    const Consts<CT> c = make_consts<CT>(FAM, th);
    if constexpr (FAM == FAM_FRANK && sizeof(CT) == 4) {
      if (c.fk.th < (CT)FRANK_SCALED_BELOW)
        eval_rows<T, CT, FAM, 1>(r1, r2, n, c, v);
      else
        eval_rows<T, CT, FAM, 0>(r1, r2, n, c, v);
    } else {
      eval_rows<T, CT, FAM, -1>(r1, r2, n, c, v);
    }
  }
  block_sum<W, 3>(v, red);
  if (threadIdx.x == 0) {
    if constexpr (FAM == FAM_GAUSSIAN) {
      double S, H;
      gauss_score_hess(th, (double)n, v[0], v[1], S, H);
      out[3 * m] = gauss_loglik(th, (double)n, v[0], v[1]);
      out[3 * m + 1] = S;
      out[3 * m + 2] = H;
    } else {
      out[3 * m] = v[0];
      out[3 * m + 1] = v[1];
      out[3 * m + 2] = v[2];
    }
  }
}

template <int T>
hipError_t launch_eval_t(const uint32_t* R1, const uint32_t* R2, const SubDesc* subs, int64_t K, int fam, int fp64,
                         const double* theta, double* out, hipStream_t s) {
  const dim3 grid((unsigned)K), block(T);
  if (fp64) {
    if (fam == FAM_GAUSSIAN) hipLaunchKernelGGL((k_eval_wg<T, double, FAM_GAUSSIAN>), grid, block, 0, s, R1, R2, subs, theta, out);
    else if (fam == FAM_FRANK) hipLaunchKernelGGL((k_eval_wg<T, double, FAM_FRANK>), grid, block, 0, s, R1, R2, subs, theta, out);
    else hipLaunchKernelGGL((k_eval_wg<T, double, FAM_GUMBEL>), grid, block, 0, s, R1, R2, subs, theta, out);
  } else {
    if (fam == FAM_GAUSSIAN) hipLaunchKernelGGL((k_eval_wg<T, float, FAM_GAUSSIAN>), grid, block, 0, s, R1, R2, subs, theta, out);
    else if (fam == FAM_FRANK) hipLaunchKernelGGL((k_eval_wg<T, float, FAM_FRANK>), grid, block, 0, s, R1, R2, subs, theta, out);
    else hipLaunchKernelGGL((k_eval_wg<T, float, FAM_GUMBEL>), grid, block, 0, s, R1, R2, subs, theta, out);
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_eval_wg(const uint32_t* R1, const uint32_t* R2, const SubDesc* subs, int64_t K, int fam,
                          int fp64, int64_t n_max, const double* theta, double* out, hipStream_t s) {
  if (K <= 0) return hipSuccess;
  // workgroup size from the largest subset: about 8 or more rows per thread
  if (n_max <= 512) return launch_eval_t<64>(R1, R2, subs, K, fam, fp64, theta, out, s);
  if (n_max <= 2048) return launch_eval_t<128>(R1, R2, subs, K, fam, fp64, theta, out, s);
  return launch_eval_t<256>(R1, R2, subs, K, fam, fp64, theta, out, s);
}

}  // namespace cpc
