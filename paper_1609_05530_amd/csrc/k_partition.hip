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
// Replicates of more than kResidentMaxRows rows take the gather below
// instead: their x is sorted on the streaming path, whose payloads give the
// row at each sorted position, so output row o (subset m, its q-th row)
// takes the row at position p = o (blocks) or p = q M + m (strided). Each
// 8-byte read from a random place in the replicate brings in a whole line,
// which bounds the gather; for blocks, x is the inverse of the position's
// order-preserving key instead (read in order; a key of 0 is read from x,
// which keeps the sign of -0), so that only y is read at random. The
// writes are coalesced.
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace cpc {

template <typename T>
__global__ void __launch_bounds__(256) k_partition(const T* __restrict__ x, const T* __restrict__ y,
                                                   const uint32_t* __restrict__ R1, const int64_t* __restrict__ rep,
                                                   int64_t R, int64_t n, uint32_t M, int scheme, int skip_big,
                                                   T* __restrict__ xo, T* __restrict__ yo) {
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
      if (skip_big && N > (uint32_t)kResidentMaxRows) continue;  // the gather's rows
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

// The value whose order-preserving key is k (the key turns a non-negative
// value's bits b into b with the top bit set, a negative one's into ~b);
// false for the key of +-0, whose sign the key does not keep.
__device__ __forceinline__ bool value_of_key(uint32_t k, float& v) {
  const uint32_t b = (k & 0x80000000u) ? (k & 0x7FFFFFFFu) : ~k;
  v = __uint_as_float(b);
  return b != 0u;
}
__device__ __forceinline__ bool value_of_key(uint64_t k, double& v) {
  const uint64_t b = (k >> 63) ? (k & 0x7FFFFFFFFFFFFFFFull) : ~k;
  v = __longlong_as_double((long long)b);
  return b != 0ull;
}

template <typename T>
__global__ void __launch_bounds__(256) k_partition_gather(BigParams P, BigSorted so, const T* __restrict__ x,
                                                          const T* __restrict__ y, uint32_t M, int scheme,
                                                          T* __restrict__ xo, T* __restrict__ yo) {
  const int64_t ti = P.xorder[blockIdx.x];
  if (ti < 0) return;  // idle slot (uniform)
  const BigTile t = P.tiles[ti];
  const BigSeg sg = P.segs[t.seg];
  const uint32_t N = (uint32_t)sg.n;
  const uint32_t a = N / M, c = N - a * M;
  const uint32_t big = (a + 1u) * c;  // rows of the subsets that hold a + 1 rows
  // the tile's index range is output rows, so that the writes are coalesced
  // (walking sorted positions instead, the strided writes scatter: 1.5x slower)
  for (int k = threadIdx.x; k < t.count; k += blockDim.x) {
    const uint32_t o = (uint32_t)(t.start + k);  // output row within the replicate
    uint32_t p = o;
    if (scheme == PART_STRIDED) {  // o is row q of subset m: position q M + m
      uint32_t m, q;
      if (o < big) {
        m = o / (a + 1u);
        q = o - m * (a + 1u);
      } else {  // (a >= 1 here, since o < N = a M + c)
        const uint32_t r = o - big;
        q = r % a;
        m = c + r / a;
      }
      p = q * M + m;
    }
    const int64_t c = sg.roff + p;
    const uint32_t row = so.rows[c];
    if (row >= N) continue;  // not a row of this replicate: nothing is written
    T xv;
    bool from_key = false;
    if (scheme == PART_BLOCKS) {  // keys in order (strided: a stride of M, dearer than x itself)
      if constexpr (sizeof(T) == 8)
        from_key = value_of_key(((uint64_t)so.khi[c] << 32) | so.klo[c], xv);
      else
        from_key = value_of_key(so.klo[c], xv);
    }
    if (!from_key) xv = x[sg.begin + row];
    xo[sg.begin + o] = xv;
    yo[sg.begin + o] = y[sg.begin + row];
  }
}

hipError_t launch_partition_gather(int f32, const BigParams& P, const BigSorted& so, const void* x, const void* y,
                                   int64_t M, int scheme, void* xo, void* yo, hipStream_t s) {
  if (P.nsegs == 0 || P.nslots == 0) return hipSuccess;
  const unsigned nt = (unsigned)P.nslots;
  if (f32)
    hipLaunchKernelGGL(k_partition_gather<float>, dim3(nt), dim3(256), 0, s, P, so, (const float*)x,
                       (const float*)y, (uint32_t)M, scheme, (float*)xo, (float*)yo);
  else
    hipLaunchKernelGGL(k_partition_gather<double>, dim3(nt), dim3(256), 0, s, P, so, (const double*)x,
                       (const double*)y, (uint32_t)M, scheme, (double*)xo, (double*)yo);
  return hipGetLastError();
}

// Strided rows from blocks-order rows, one 32 x 32 tile of (q, m) per
// workgroup: read along m (consecutive positions q M + m), written along q
// (consecutive rows of subset m) through LDS; blocks run over the
// replicates' tiles, replicate by replicate.
template <typename T>
__global__ void __launch_bounds__(256) k_partition_transpose(BigParams P, const T* __restrict__ tx,
                                                             const T* __restrict__ ty, uint32_t M, int64_t max_tiles,
                                                             T* __restrict__ xo, T* __restrict__ yo) {
  __shared__ T sx[32][33];
  __shared__ T sy[32][33];
  const int64_t seg = (int64_t)blockIdx.x / max_tiles;
  const uint32_t tile = (uint32_t)((int64_t)blockIdx.x - seg * max_tiles);
  const BigSeg sg = P.segs[seg];
  const uint32_t N = (uint32_t)sg.n;
  const uint32_t a = N / M, c = N - a * M, Q = a + (c ? 1u : 0u);
  const uint32_t Mc = M < N ? M : N;  // (columns m >= N are empty)
  const uint32_t tiles_m = (Mc + 31u) / 32u;
  if ((uint64_t)tile >= (uint64_t)((Q + 31u) / 32u) * tiles_m) return;  // (uniform)
  const uint32_t tq = tile / tiles_m, tm = tile - tq * tiles_m;
  const int lx = threadIdx.x & 31, ly = threadIdx.x >> 5;
  for (int i = ly; i < 32; i += 8) {
    const uint32_t q = tq * 32u + (uint32_t)i, m = tm * 32u + (uint32_t)lx;
    const uint64_t p = (uint64_t)q * M + m;
    if (m < M && p < N) {
      sx[i][lx] = tx[sg.begin + (int64_t)p];
      sy[i][lx] = ty[sg.begin + (int64_t)p];
    }
  }
  __syncthreads();
  for (int j = ly; j < 32; j += 8) {
    const uint32_t m = tm * 32u + (uint32_t)j, q = tq * 32u + (uint32_t)lx;
    const uint64_t p = (uint64_t)q * M + m;
    if (m < M && p < N) {
      const int64_t o = sg.begin + (int64_t)(m * a + (m < c ? m : c) + q);
      xo[o] = sx[lx][j];
      yo[o] = sy[lx][j];
    }
  }
}

hipError_t launch_partition_transpose(int f32, const BigParams& P, const void* tx, const void* ty, int64_t M,
                                      int64_t max_tiles, void* xo, void* yo, hipStream_t s) {
  if (P.nsegs == 0 || max_tiles <= 0) return hipSuccess;
  const unsigned blocks = (unsigned)((int64_t)P.nsegs * max_tiles);
  if (f32)
    hipLaunchKernelGGL(k_partition_transpose<float>, dim3(blocks), dim3(256), 0, s, P, (const float*)tx,
                       (const float*)ty, (uint32_t)M, max_tiles, (float*)xo, (float*)yo);
  else
    hipLaunchKernelGGL(k_partition_transpose<double>, dim3(blocks), dim3(256), 0, s, P, (const double*)tx,
                       (const double*)ty, (uint32_t)M, max_tiles, (double*)xo, (double*)yo);
  return hipGetLastError();
}

hipError_t launch_partition(int f32, const void* x, const void* y, const uint32_t* R1, const int64_t* rep,
                            int64_t R, int64_t n, int64_t M, int scheme, int skip_big, void* xo, void* yo,
                            hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int threads = 256;
  int64_t blocks = (n + threads - 1) / threads;
  if (blocks > 16384) blocks = 16384;
  if (f32)
    hipLaunchKernelGGL(k_partition<float>, dim3((unsigned)blocks), dim3(threads), 0, s, (const float*)x,
                       (const float*)y, R1, rep, R, n, (uint32_t)M, scheme, skip_big, (float*)xo, (float*)yo);
  else
    hipLaunchKernelGGL(k_partition<double>, dim3((unsigned)blocks), dim3(threads), 0, s, (const double*)x,
                       (const double*)y, R1, rep, R, n, (uint32_t)M, scheme, skip_big, (double*)xo,
                       (double*)yo);
  return hipGetLastError();
}

}  // namespace cpc
