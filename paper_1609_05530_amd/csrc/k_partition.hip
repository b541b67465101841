// k_partition.hip — the rows of each replicate split into M subsets by a
// partitioning scheme (the row partition of eq. 14 of arXiv:1609.05530; the
// schemes serve the study of partitioning methods that its Sec. 4 leaves as
// future work). Row i of replicate r (rows b .. b + N - 1) sits at position
// p = R1[i] / 2 - 1 of the replicate's x-order: R1 holds the doubled ranks of
// eq. (12) with ties broken by row order, so p runs over a permutation of
// 0 .. N - 1. The row moves to
//   blocks     : b + p                          (M slices of the x-order)
//   strided    : b + m a + min(m, c) + q,       with p = q M + m, N = a M + c
//                (subset m holds ceil((N - m) / M) rows, so its first row
//                 follows the m a + min(m, c) rows of subsets 0 .. m - 1)
//   contiguous : i                              (the rows stay in place)
// One thread per row, a grid-stride loop over at most 16384 workgroups (a
// thread has few rows, so many loads are in flight); x, y and R1 are read
// coalesced and each replicate's writes are a permutation of its own rows.
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace cpc {

template <typename T>
__global__ void __launch_bounds__(256) k_partition(const T* __restrict__ x, const T* __restrict__ y,
                                                   const uint32_t* __restrict__ R1, const int64_t* __restrict__ rep,
                                                   int64_t R, int64_t n, uint32_t M, int scheme, T* __restrict__ xo,
                                                   T* __restrict__ yo) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    int64_t dest = i;
    if (scheme != PART_CONTIGUOUS) {
      // the replicate holding row i: rep[lo] <= i < rep[hi] throughout
      int64_t lo = 0, hi = R;
      while (hi - lo > 1) {
        const int64_t mid = (lo + hi) >> 1;
        if (rep[mid] <= i)
          lo = mid;
        else
          hi = mid;
      }
      const int64_t b = rep[lo];
      const uint32_t N = (uint32_t)(rep[lo + 1] - b);
      const uint32_t p = (R1[i] >> 1) - 1u;
      if (p >= N) continue;  // not a position of this replicate: nothing is written
      if (scheme == PART_BLOCKS) {
        dest = b + p;
      } else {
        const uint32_t q = p / M, m = p - q * M;
        const uint32_t a = N / M, c = N - a * M;
        dest = b + (int64_t)m * a + (m < c ? m : c) + q;
      }
    }
    xo[dest] = x[i];
    yo[dest] = y[i];
  }
}

hipError_t launch_partition(int f32, const void* x, const void* y, const uint32_t* R1, const int64_t* rep,
                            int64_t R, int64_t n, int64_t M, int scheme, void* xo, void* yo, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int threads = 256;
  int64_t blocks = (n + threads - 1) / threads;
  if (blocks > 16384) blocks = 16384;
  if (f32)
    hipLaunchKernelGGL(k_partition<float>, dim3((unsigned)blocks), dim3(threads), 0, s, (const float*)x,
                       (const float*)y, R1, rep, R, n, (uint32_t)M, scheme, (float*)xo, (float*)yo);
  else
    hipLaunchKernelGGL(k_partition<double>, dim3((unsigned)blocks), dim3(threads), 0, s, (const double*)x,
                       (const double*)y, R1, rep, R, n, (uint32_t)M, scheme, (double*)xo, (double*)yo);
  return hipGetLastError();
}

}  // namespace cpc
