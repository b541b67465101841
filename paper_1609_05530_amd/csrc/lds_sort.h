// lds_sort.h — one stable 8-bit counting pass of a workgroup's elements in
// LDS (a ballot multisplit), the tile step of the streaming path's global
// radix sort behind the ranks of eq. (12) of arXiv:1609.05530.
#pragma once

#include <hip/hip_runtime.h>

#include "block_rank.h"
#include "cpc_device.h"

namespace cpc {

// One stable counting pass over the digits d[j] of the elements held in
// wave-striped order (element e = (w*E + j)*64 + lane; only e < n take
// part): each wave ranks its elements among its own earlier elements with the
// same digit by a ballot multisplit, then per-wave digit counts are combined
// in a digit-major exclusive scan. On return dst[j] is the element's position
// in the stably sorted order of the workgroup's n elements, dtot[0..255] the
// first position of each digit, and dtot[256 + (pass & 1)] is nonzero when
// one digit holds all n elements (the pass is the identity). cnt: W*256 u16.
template <int T, int E>
__device__ __forceinline__ void lds_multisplit(const uint32_t (&d)[E], int n, int pass, uint16_t* cnt,
                                               uint32_t* dtot, uint32_t (&dst)[E]) {
  constexpr int W = T / WAVE;
  constexpr int NT = (T < 256) ? T : 256;  // threads that scan digits
  constexpr int DPT = 256 / NT;            // digits per scanning thread
  const int tid = threadIdx.x, lane = tid & (WAVE - 1), w = tid / WAVE;
  const uint64_t lt = lanemask_lt();
  for (int i = lane; i < 256; i += WAVE) cnt[w * 256 + i] = 0;
  // the identity flag alternates between two slots so that resetting it for
  // this pass cannot race with reads of the previous pass's flag
  if (tid == 0) dtot[256 + (pass & 1)] = 0u;
#pragma unroll
  for (int j = 0; j < E; ++j) {
    const int e = (w * E + j) * WAVE + lane;
    const bool valid = e < n;
    uint64_t m = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const bool bit = (d[j] >> b) & 1u;
      const uint64_t bb = __ballot(bit);
      m &= bit ? bb : ~bb;
    }
    const uint32_t lower = (uint32_t)__popcll(m & lt);
    const uint32_t old = cnt[w * 256 + d[j]];
    dst[j] = old + lower;
    if (valid && lower == 0u) cnt[w * 256 + d[j]] = (uint16_t)(old + (uint32_t)__popcll(m));
    // keep the slots' ballot chains from being interleaved (register pressure)
    __builtin_amdgcn_sched_barrier(0);
  }
  __syncthreads();
  uint32_t colsum[DPT];
  uint32_t local = 0;
  if (tid < NT) {
#pragma unroll
    for (int q = 0; q < DPT; ++q) {
      const int dg = tid * DPT + q;
      uint32_t run = 0;
      for (int k = 0; k < W; ++k) {
        const uint32_t c = cnt[k * 256 + dg];
        cnt[k * 256 + dg] = (uint16_t)run;
        run += c;
      }
      colsum[q] = run;
      local += run;
      if (run == (uint32_t)n) dtot[256 + (pass & 1)] = 1u;
    }
  }
  const uint32_t incl = wave_incl_sum_u32(local);
  if (tid < NT && lane == WAVE - 1) dtot[258 + w] = incl;
  __syncthreads();
  if (tid < NT) {
    uint32_t base = incl - local;
    for (int k = 0; k < w; ++k) base += dtot[258 + k];
#pragma unroll
    for (int q = 0; q < DPT; ++q) {
      dtot[tid * DPT + q] = base;
      base += colsum[q];
    }
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < E; ++j) dst[j] += dtot[d[j]] + cnt[w * 256 + d[j]];
}

}  // namespace cpc
