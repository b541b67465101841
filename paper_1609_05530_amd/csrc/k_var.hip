// k_var.hip — asymptotic variance of each subset's estimate (arXiv:1609.05530,
// Sec. 2.3, "according to Genest et al. (1995)"), with the subset's pseudo
// log-likelihood and score at the estimate; one workgroup per subset of up
// to 16384 rows. Plug-in Genest-Ghoudi-Rivest sandwich:
//   s_i = dl/dtheta, g1_i = d2l/dtheta du, g2_i = d2l/dtheta dv at (u_i, v_i)
//   W1_i = (1/n) sum_{l : u_l >= u_i} g1_l   (suffix sum in u order; a tie
//          group takes the sum from its first member), W2_i likewise in v
//   psi_i = s_i + W1_i + W2_i
//   sigma^2 = [mean(psi^2) - mean(psi)^2] / (n mean(s^2)^2)
// (or 1 / (n mean(s^2)) for the inverse-information option). The g values
// are scattered to sorted position in LDS and suffix-summed there.
#include <hip/hip_runtime.h>

#include "kernels.h"
#include "solver.h"

namespace cpc {

// In-place inclusive suffix sums of A[0..n): A[i] <- sum_{q >= i} A[q];
// per-thread chunks of E consecutive entries, chunk sums and the workgroup
// scan in double.
template <int T, int E, typename CT>
__device__ __forceinline__ void lds_suffix_sum(CT* A, int n, double* scratch) {
  constexpr int W = T / WAVE;
  const int c0 = threadIdx.x * E;
  double cs = 0.0;
#pragma unroll
  for (int i = 0; i < E; ++i)
    if (c0 + i < n) cs += (double)A[c0 + i];
  double run = block_excl_suffix<W>(cs, scratch);
#pragma unroll
  for (int i = E - 1; i >= 0; --i) {
    if (c0 + i < n) {
      run += (double)A[c0 + i];
      A[c0 + i] = (CT)run;
    }
  }
  __syncthreads();
}

template <int T, int CAP, typename CT, int FAM>
__global__ void __launch_bounds__(T) k_var_wg(VarParams P) {
  constexpr int W = T / WAVE;
  constexpr int E = CAP / T;
  constexpr bool TWO = 2 * sizeof(CT) * CAP <= 144 * 1024;
  __shared__ CT A1[CAP];
  __shared__ CT A2[TWO ? CAP : 1];
  __shared__ double red[W * 5];
  const int tid = threadIdx.x;
  const int sid = P.order[blockIdx.x];
  const SubDesc sd = P.subs[sid];
  const int n = sd.n;
  const SubState st = P.state[sid];
  int status = st.status;
  double theta;
  if (P.mode == MODE_VARIANCE) {
    if (status != ST_OK) {
      if (tid == 0) P.var_out[sid] = NAN;
      return;
    }
    theta = P.theta_in[sid];
  } else {
    if (status == ST_DEGENERATE || status == ST_NONFINITE) {
      if (tid == 0) {
        ResultOut r;
        r.theta = NAN; r.var = NAN; r.loglik = NAN; r.score = NAN;
        r.n = n; r.iters = st.iters; r.status = status;
        P.out[sid] = r;
      }
      return;
    }
    theta = st.theta;
  }
  const int64_t o = sd.begin;
  const uint16_t *R1 = P.rows.R1 + o, *R2 = P.rows.R2 + o;
  const uint16_t *E1 = P.rows.E1 + o, *E2 = P.rows.E2 + o;
  const uint16_t *L1 = P.rows.L1 + o, *L2 = P.rows.L2 + o;
  CT* S = (CT*)P.rows.S + o;
  const uint32_t twon1 = 2u * (uint32_t)(n + 1);
  const CT inv = (CT)1 / (CT)twon1;
  const double dn = (double)n;
  const Consts<CT> c = make_consts<CT>(FAM, theta);
  const bool rd = sizeof(CT) == 4 && c.use_d;  // FP64 rows near the family boundaries
  const Consts<double> cd = make_consts<double>(FAM, theta);

  auto row_eval = [&](int i, CT& l, CT& s, CT& g1, CT& g2) {
    const uint32_t a = R1[i], b = R2[i];
    if (rd) {
      const double invd = 1.0 / (double)twon1;
      double ld, sdd, g1d, g2d;
      if constexpr (FAM == FAM_FRANK) {
        frank_rfull<double>(cd, a, b, twon1, invd, ld, sdd, g1d, g2d);
      } else if constexpr (FAM == FAM_GUMBEL) {
        double lx, ly;
        gumbel_lxy<double>(a, b, twon1, invd, lx, ly);
        gumbel_rfull<double>(cd, a, b, twon1, invd, lx, ly, ld, sdd, g1d, g2d);
      } else {
        double z1, z2;
        gauss_z<double>(a, b, twon1, z1, z2);
        gauss_rfull<double>(cd, z1, z2, ld, sdd, g1d, g2d);
      }
      l = (CT)ld; s = (CT)sdd; g1 = (CT)g1d; g2 = (CT)g2d;
    } else {
      if constexpr (FAM == FAM_FRANK) {
        frank_rfull<CT>(c, a, b, twon1, inv, l, s, g1, g2);
      } else if constexpr (FAM == FAM_GUMBEL) {
        CT lx, ly;
        gumbel_lxy<CT>(a, b, twon1, inv, lx, ly);
        gumbel_rfull<CT>(c, a, b, twon1, inv, lx, ly, l, s, g1, g2);
      } else {
        CT z1, z2;
        gauss_z<CT>(a, b, twon1, z1, z2);
        gauss_rfull<CT>(c, z1, z2, l, s, g1, g2);
      }
    }
  };

  KSum<CT> kl, ksc, ks2;
  double psum = 0.0, psq = 0.0;
  if constexpr (TWO) {
    for (int i = tid; i < n; i += T) {
      CT l, s, g1, g2;
      row_eval(i, l, s, g1, g2);
      kl.add(l); ksc.add(s); ks2.add(s * s);
      A1[E1[i]] = g1;
      A2[E2[i]] = g2;
      S[i] = s;
    }
    __syncthreads();
    lds_suffix_sum<T, E, CT>(A1, n, red);
    lds_suffix_sum<T, E, CT>(A2, n, red);
    for (int i = tid; i < n; i += T) {
      const double psi = (double)S[i] + ((double)A1[L1[i]] + (double)A2[L2[i]]) / dn;
      psum += psi;
      psq += psi * psi;
    }
  } else {
    for (int i = tid; i < n; i += T) {
      CT l, s, g1, g2;
      row_eval(i, l, s, g1, g2);
      kl.add(l); ksc.add(s); ks2.add(s * s);
      A1[E1[i]] = g1;
      S[i] = s;
    }
    __syncthreads();
    lds_suffix_sum<T, E, CT>(A1, n, red);
    for (int i = tid; i < n; i += T) S[i] = (CT)((double)S[i] + (double)A1[L1[i]] / dn);
    __syncthreads();
    for (int i = tid; i < n; i += T) {
      CT l, s, g1, g2;
      row_eval(i, l, s, g1, g2);
      A1[E2[i]] = g2;
    }
    __syncthreads();
    lds_suffix_sum<T, E, CT>(A1, n, red);
    for (int i = tid; i < n; i += T) {
      const double psi = (double)S[i] + (double)A1[L2[i]] / dn;
      psum += psi;
      psq += psi * psi;
    }
  }
  double v[5] = {kl.value(), ksc.value(), ks2.value(), psum, psq};
  block_sum<W, 5>(v, red);
  if (tid == 0) {
    const double mpsi = v[3] / dn;
    const double nu = v[4] / dn - mpsi * mpsi;
    const double beta = v[2] / dn;
    const double var = (P.var_method == 1) ? 1.0 / (dn * beta) : nu / (dn * beta * beta);
    if (P.mode == MODE_VARIANCE) {
      P.var_out[sid] = var;
    } else {
      double loglik = v[0], score = v[1];
      if (FAM == FAM_GAUSSIAN) {  // from the FP64 sufficient statistics
        double H;
        loglik = gauss_loglik(theta, dn, st.Sp, st.Sm);
        gauss_score_hess(theta, dn, st.Sp, st.Sm, score, H);
      }
      const bool usable = (status == ST_OK || status == ST_BOUNDARY_NATURAL);
      if (usable && !(var > 0.0 && isfinite(var))) status = ST_BADVAR;
      ResultOut r;
      r.theta = theta;
      r.var = usable ? var : NAN;
      r.loglik = loglik;
      r.score = score;
      r.n = n;
      r.iters = st.iters;
      r.status = status;
      P.out[sid] = r;
    }
  }
}

template <int T, int CAP, typename CT>
static hipError_t launch_t(int fam, const VarParams& p, int grid, hipStream_t s) {
  if (grid <= 0) return hipSuccess;
  switch (fam) {
    case FAM_GAUSSIAN: hipLaunchKernelGGL((k_var_wg<T, CAP, CT, FAM_GAUSSIAN>), dim3(grid), dim3(T), 0, s, p); break;
    case FAM_FRANK: hipLaunchKernelGGL((k_var_wg<T, CAP, CT, FAM_FRANK>), dim3(grid), dim3(T), 0, s, p); break;
    default: hipLaunchKernelGGL((k_var_wg<T, CAP, CT, FAM_GUMBEL>), dim3(grid), dim3(T), 0, s, p); break;
  }
  return hipGetLastError();
}

hipError_t launch_var_wg(int cls, int fam, int fp64, const VarParams& p, int grid, hipStream_t s) {
  switch (cls) {
    case 0: return fp64 ? launch_t<64, 512, double>(fam, p, grid, s) : launch_t<64, 512, float>(fam, p, grid, s);
    case 1: return fp64 ? launch_t<256, 2048, double>(fam, p, grid, s) : launch_t<256, 2048, float>(fam, p, grid, s);
    case 2: return fp64 ? launch_t<512, 8192, double>(fam, p, grid, s) : launch_t<512, 8192, float>(fam, p, grid, s);
    case 3: return fp64 ? launch_t<1024, 16384, double>(fam, p, grid, s) : launch_t<1024, 16384, float>(fam, p, grid, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace cpc
