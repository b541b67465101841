// k_eval.hip — the adjoint of the pseudo log-likelihood eq. (13) of
// arXiv:1609.05530: for each subset m at a given theta_m, the sums over the
// subset's rows of l, dl/dtheta and d2l/dtheta2 (eq. 5 applied to eq. 8, 10
// or 11), from doubled ranks. One workgroup per subset; rows are streamed
// with coalesced loads; per-thread compensated sums meet in a fixed-order
// workgroup reduction (bitwise reproducible).
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace cpc {

template <int T, typename CT>
__global__ void __launch_bounds__(T) k_eval_wg(const uint32_t* R1, const uint32_t* R2, const SubDesc* subs,
                                               int fam, const double* theta, double* out) {
  constexpr int W = T / WAVE;
  __shared__ double red[W * 3];
  const int m = blockIdx.x;
  const SubDesc sd = subs[m];
  const int n = sd.n;
  const double th = theta[m];
  const bool inside = (fam == FAM_GAUSSIAN) ? (th > -1.0 && th < 1.0) : (fam == FAM_GUMBEL ? th >= 1.0 : isfinite(th));
  if (!inside || n < 1) {
    if (threadIdx.x == 0) {
      const double v = (n < 1) ? 0.0 : NAN;
      out[3 * m] = v; out[3 * m + 1] = v; out[3 * m + 2] = v;
    }
    return;
  }
  const Consts<CT> c = make_consts<CT>(fam, th);
  const uint32_t twon1 = 2u * (uint32_t)(n + 1);
  RowSum<CT> kl, ks, kh;
  for (int i = threadIdx.x; i < n; i += T) {
    CT l, s, h, g1, g2;
    row_lshf<CT>(c, R1[sd.begin + i], R2[sd.begin + i], twon1, l, s, h, g1, g2);
    kl.add(l);
    ks.add(s);
    kh.add(h);
  }
  double v[3] = {kl.value(), ks.value(), kh.value()};
  block_sum<W, 3>(v, red);
  if (threadIdx.x == 0) {
    out[3 * m] = v[0];
    out[3 * m + 1] = v[1];
    out[3 * m + 2] = v[2];
  }
}

hipError_t launch_eval_wg(const uint32_t* R1, const uint32_t* R2, const SubDesc* subs, int64_t K, int fam,
                          int fp64, const double* theta, double* out, hipStream_t s) {
  if (K <= 0) return hipSuccess;
  if (fp64)
    hipLaunchKernelGGL((k_eval_wg<256, double>), dim3((unsigned)K), dim3(256), 0, s, R1, R2, subs, fam, theta, out);
  else
    hipLaunchKernelGGL((k_eval_wg<256, float>), dim3((unsigned)K), dim3(256), 0, s, R1, R2, subs, fam, theta, out);
  return hipGetLastError();
}

}  // namespace cpc
