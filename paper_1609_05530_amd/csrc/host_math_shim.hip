// host_math_shim.hip — host-only build of the kernels' per-row arithmetic
// (family_math.h, row_eval.h) for unit tests on machines without a GPU.
// Exposes C functions that evaluate, on host arrays, exactly the branch logic
// the kernels run per row. Not part of libcpc; never loaded by the product.
#include <stdint.h>

#include "row_eval.h"

extern "C" {

// z = Phi^{-1}(R / twon1) by AS 241 in the given precision (0 = double, 1 = float).
void cpcm_qnorm(int32_t prec, const int64_t* R, int64_t twon1, int64_t n, double* z) {
  for (int64_t i = 0; i < n; ++i)
    z[i] = prec ? (double)cpc::qnorm_rank<float>(R[i], twon1) : cpc::qnorm_rank<double>(R[i], twon1);
}

// Per row: out[5i + 0..4] = l, dl/dtheta, d2l/dtheta2, d2l/dtheta du, d2l/dtheta dv
// computed from doubled ranks with the kernels' code paths.
void cpcm_rows(int32_t family, int32_t prec, double theta, const uint32_t* R1, const uint32_t* R2,
               int64_t n, double* out) {
  const uint32_t twon1 = (uint32_t)(2 * (n + 1));
  if (prec) {
    const cpc::Consts<float> c = cpc::make_consts<float>(family, theta);
    for (int64_t i = 0; i < n; ++i) {
      float l, s, h, g1, g2;
      cpc::row_lshf(c, R1[i], R2[i], twon1, l, s, h, g1, g2);
      out[5 * i + 0] = l; out[5 * i + 1] = s; out[5 * i + 2] = h; out[5 * i + 3] = g1; out[5 * i + 4] = g2;
    }
  } else {
    const cpc::Consts<double> c = cpc::make_consts<double>(family, theta);
    for (int64_t i = 0; i < n; ++i) {
      double l, s, h, g1, g2;
      cpc::row_lshf(c, R1[i], R2[i], twon1, l, s, h, g1, g2);
      out[5 * i + 0] = l; out[5 * i + 1] = s; out[5 * i + 2] = h; out[5 * i + 3] = g1; out[5 * i + 4] = g2;
    }
  }
}

// Gaussian sufficient-statistic score / Hessian / log-likelihood (FP64).
void cpcm_gauss_suff(double r, double n, double Sp, double Sm, double* out) {
  cpc::gauss_score_hess(r, n, Sp, Sm, out[0], out[1]);
  out[2] = cpc::gauss_loglik(r, n, Sp, Sm);
}

}  // extern "C"
