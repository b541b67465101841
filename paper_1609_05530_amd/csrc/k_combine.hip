// k_combine.hip — inverse-variance combination of the subset estimates,
// eq. (15) of arXiv:1609.05530 (eq. 16 per simulation replicate): for each
// group g, theta = sum w_m theta_m / sum w_m with w_m = 1 / sigma_m^2 over the
// group's usable subsets (status OK or BOUNDARY_NATURAL). One wave per group;
// lanes stride the group's subsets and the partial sums meet in a fixed
// butterfly, so the result does not depend on scheduling.
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace cpc {

__global__ void __launch_bounds__(256) k_combine(const ResultOut* sub, const int64_t* gofs, int64_t G,
                                                 CombinedOut* comb) {
  const int lane = threadIdx.x & (WAVE - 1);
  const int64_t g = (int64_t)blockIdx.x * (blockDim.x / WAVE) + threadIdx.x / WAVE;
  if (g >= G) return;
  const int64_t m0 = gofs[g], m1 = gofs[g + 1];
  double sw = 0.0, swt = 0.0;
  long long used = 0;
  for (int64_t m = m0 + lane; m < m1; m += WAVE) {
    const int32_t st = sub[m].status;
    if (st != ST_OK && st != ST_BOUNDARY_NATURAL) continue;
    const double w = 1.0 / sub[m].var;
    sw += w;
    swt += w * sub[m].theta;
    used += 1;
  }
  sw = wave_sum(sw);
  swt = wave_sum(swt);
  used = wave_sum_ll(used);
  if (lane == 0) {
    CombinedOut c;
    c.n_used = used;
    c.n_excluded = (m1 - m0) - used;
    c.pad = 0;
    if (used > 0) {
      c.theta = swt / sw;
      c.var_combined = 1.0 / sw;
      c.status = 0;
    } else {
      c.theta = NAN;
      c.var_combined = NAN;
      c.status = 1;
    }
    comb[g] = c;
  }
}

hipError_t launch_combine(const ResultOut* sub, const int64_t* group_offsets, int64_t G,
                          CombinedOut* comb, hipStream_t s) {
  if (G <= 0) return hipSuccess;
  const int per_block = 4;  // waves (groups) per workgroup
  const int64_t blocks = (G + per_block - 1) / per_block;
  hipLaunchKernelGGL(k_combine, dim3((unsigned)blocks), dim3(per_block * WAVE), 0, s, sub, group_offsets, G, comb);
  return hipGetLastError();
}

}  // namespace cpc
