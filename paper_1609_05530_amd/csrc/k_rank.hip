// k_rank.hip — launch shapes of the workgroup-per-subset rank kernel
// (rank_wg.h) per size class.
#include <hip/hip_runtime.h>

#include "rank_wg.h"

namespace cpc {

// Launch shapes per size class: (threads, items per thread, digit bits,
// counters sharing LDS with the exchange buffer, 32-bit payloads). The class
// capacity threads * items must match kClassThreads * kClassItems. Every
// launch uses the bank-conflict-free padded exchange layout.
template <int T, int E, int B, bool ALIAS, bool P32>
static hipError_t launch_t(int kw, const RankParams& p, int grid, hipStream_t s) {
  if (grid <= 0) return hipSuccess;
  if (kw == 2)
    hipLaunchKernelGGL((k_rank_wg<T, E, B, 2, ALIAS, P32, false, true>), dim3(grid), dim3(T), 0, s, p);
  else
    hipLaunchKernelGGL((k_rank_wg<T, E, B, 1, ALIAS, P32, false, true>), dim3(grid), dim3(T), 0, s, p);
  return hipGetLastError();
}

static_assert(kClassThreads[0] * kClassItems[0] == 64 * 8, "class 0 capacity");
static_assert(kClassThreads[1] * kClassItems[1] == 256 * 8, "class 1 capacity");
static_assert(kClassThreads[2] * kClassItems[2] == 512 * 16, "class 2 capacity");
static_assert(kClassThreads[3] * kClassItems[3] == 1024 * 16, "class 3 capacity");

template <int T, int E, bool PACK>
static hipError_t launch_shape1(const RankParams& p, int grid, hipStream_t s) {
  if (grid <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_rank_wg<T, E, 4, 1, false, false, PACK, true>), dim3(grid), dim3(T), 0, s, p);
  return hipGetLastError();
}

template <int T, int E>
static hipError_t launch_shape_merge(const RankParams& p, int grid, hipStream_t s) {
  if (grid <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_rank_wg<T, E, 4, 1, false, false, false, true, true>), dim3(grid), dim3(T), 0, s, p);
  return hipGetLastError();
}

template <int T, int E>
static hipError_t launch_shape_trunc(const RankParams& p, int grid, hipStream_t s) {
  if (grid <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_rank_wg<T, E, 4, 1, false, false, false, true, false, 24>), dim3(grid), dim3(T), 0, s, p);
  return hipGetLastError();
}

hipError_t launch_rank_shape(int shape, int kw, const RankParams& p, int grid, hipStream_t s) {
  if (shape < 0 || shape >= kNumRankShapes) return hipErrorInvalidValue;
  if (kw == 2) {  // 64-bit keys: the unpacked default of the class the shape serves
    for (int c = 0; c < kNumClasses; ++c)
      if (kRankShapes[shape].cap == kClassThreads[c] * kClassItems[c]) return launch_rank_wg(c, kw, p, grid, s);
    return hipErrorInvalidValue;
  }
  switch (shape) {
    case 0: return launch_shape1<64, 8, false>(p, grid, s);
    case 1: return launch_shape1<256, 8, false>(p, grid, s);
    case 2: return launch_shape1<128, 16, false>(p, grid, s);
    case 3: return launch_shape1<512, 16, false>(p, grid, s);
    case 4: return launch_shape1<256, 32, false>(p, grid, s);
    case 5: return launch_shape1<1024, 16, false>(p, grid, s);
    case 6: return launch_shape1<512, 32, false>(p, grid, s);
    case 7: return launch_shape1<64, 8, true>(p, grid, s);
    case 8: return launch_shape1<256, 8, true>(p, grid, s);
    case 9: return launch_shape1<128, 16, true>(p, grid, s);
    case 10: return launch_shape1<512, 16, true>(p, grid, s);
    case 11: return launch_shape1<256, 32, true>(p, grid, s);
    case 12: return launch_shape1<1024, 16, true>(p, grid, s);
    case 13: return launch_shape1<512, 32, true>(p, grid, s);
    case 14: return launch_shape_merge<64, 8>(p, grid, s);
    case 15: return launch_shape_trunc<64, 8>(p, grid, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_rank_wg(int cls, int kw, const RankParams& p, int grid, hipStream_t s) {
  switch (cls) {
    case 0: return launch_t<64, 8, 4, false, false>(kw, p, grid, s);
    case 1: return launch_t<256, 8, 4, false, false>(kw, p, grid, s);
    case 2: return launch_t<512, 16, 4, false, false>(kw, p, grid, s);
    case 3: return launch_t<1024, 16, 4, false, false>(kw, p, grid, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace cpc
