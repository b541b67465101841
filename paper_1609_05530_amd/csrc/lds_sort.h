// lds_sort.h — workgroup-local stable LSD radix sort in LDS and the tie-group
// bookkeeping used to turn sorted order into the doubled ranks of eq. (12)
// of arXiv:1609.05530 (average ranks for ties, or ties broken by row order).
#pragma once

#include <hip/hip_runtime.h>

#include "cpc_device.h"

namespace cpc {

// Group start (first sorted position with the same key) and group end (one
// past the last) of sorted position e, from a bitmask with a bit per sorted
// position that marks the first element of each group (and every position
// >= n). Position 0 is always a group start.
__device__ __forceinline__ int group_lb(const uint32_t* heads, int e) {
  int wi = e >> 5;
  const int b = e & 31;
  uint32_t m = heads[wi] & (0xFFFFFFFFu >> (31 - b));
  while (m == 0u) m = heads[--wi];
  return wi * 32 + 31 - __clz((int)m);
}
__device__ __forceinline__ int group_ub(const uint32_t* heads, int e, int n, int nwords) {
  int wi = e >> 5;
  const int b = e & 31;
  uint32_t m = (b == 31) ? 0u : (heads[wi] & (0xFFFFFFFFu << (b + 1)));
  while (m == 0u) {
    if (++wi >= nwords) return n;
    m = heads[wi];
  }
  const int ub = wi * 32 + __ffs((int)m) - 1;
  return ub < n ? ub : n;
}

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
  uint32_t incl = local;
#pragma unroll
  for (int off = 1; off < WAVE; off <<= 1) {
    const uint32_t t = __shfl_up(incl, off, WAVE);
    if (lane >= off) incl += t;
  }
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

// Stable LSD radix sort of up to CAP = T*E keys held in registers in
// wave-striped order. Only e < n take part. The payload (the element's
// original index) does not occupy registers: it moves between two LDS
// buffers, starting as the identity in vb0. Returns which of the two buffers
// holds the final payload (vb[k][e] = original index of sorted position e).
// 8-bit digits, least significant first; a pass in which every element has
// the same digit moves nothing and is skipped (uniformly).
template <int T, int E, int KW>
__device__ __forceinline__ int lds_radix_sort(uint32_t (&klo)[E], uint32_t (&khi)[E], int n,
                                              uint32_t* buf, uint16_t* vb0, uint16_t* vb1,
                                              uint16_t* cnt, uint32_t* dtot) {
  const int tid = threadIdx.x, lane = tid & (WAVE - 1), w = tid / WAVE;
  for (int e = tid; e < n; e += T) vb0[e] = (uint16_t)e;
  int cur = 0;
  uint32_t dst[E];
#pragma unroll 1
  for (int pass = 0; pass < 4 * KW; ++pass) {
    const int word = pass >> 2;
    const int shift = (pass & 3) * 8;
    uint32_t d[E];
#pragma unroll
    for (int j = 0; j < E; ++j) d[j] = (((KW == 2 && word) ? khi[j] : klo[j]) >> shift) & 0xFFu;
    lds_multisplit<T, E>(d, n, pass, cnt, dtot, dst);
    if (dtot[256 + (pass & 1)] != 0u) continue;  // identity permutation: nothing moves
    const uint16_t* vs = cur ? vb1 : vb0;
    uint16_t* vd = cur ? vb0 : vb1;
#pragma unroll
    for (int j = 0; j < E; ++j) {
      const int e = (w * E + j) * WAVE + lane;
      if (e < n) {
        buf[dst[j]] = klo[j];
        vd[dst[j]] = vs[e];
      }
    }
    cur ^= 1;
    __syncthreads();
#pragma unroll
    for (int j = 0; j < E; ++j) {
      const int e = (w * E + j) * WAVE + lane;
      if (e < n) klo[j] = buf[e];
    }
    __syncthreads();
    if (KW == 2) {
#pragma unroll
      for (int j = 0; j < E; ++j) {
        const int e = (w * E + j) * WAVE + lane;
        if (e < n) buf[dst[j]] = khi[j];
      }
      __syncthreads();
#pragma unroll
      for (int j = 0; j < E; ++j) {
        const int e = (w * E + j) * WAVE + lane;
        if (e < n) khi[j] = buf[e];
      }
      __syncthreads();
    }
  }
  return cur;
}

}  // namespace cpc
