// block_rank.h — workgroup-local stable radix ranking, the sorting step
// behind the ranks of eq. (12) of arXiv:1609.05530.
//
// Elements live in registers in blocked arrangement: thread t holds the
// elements at positions t*E .. t*E+E-1 of the current order. One counting
// pass over a B-bit digit gives every thread a private 16-bit counter per
// digit value in LDS, two digit values per 32-bit word: digit d of thread t
// lives in word (d mod C)*T + t, half d / C, with C = 2^(B-1). The lanes of a
// wave therefore always touch 64 consecutive words (no bank conflicts).
//   1. each thread counts its own elements in order with LDS atomic adds; the
//      returned old value is the element's offset among the thread's earlier
//      elements with the same digit;
//   2. the counter words are exclusive-scanned in (d mod C, t) order, packed:
//      each half accumulates separately because no half can exceed the
//      element count (< 2^16), and the upper halves then take the total of
//      the lower ones, which gives the digit-major, thread-minor prefix;
//   3. an element's position in the stable order is its counter's prefix
//      plus its offset: the 16-bit half of (prefix word + returned word)
//      that holds its digit (neither half of that sum can carry into the
//      other: each is at most the element count).
// No cross-lane matching is needed: a pass costs a few LDS operations and
// about ten VALU instructions per element (32-bit keys).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "cpc_device.h"

namespace cpc {

// Lane i's value of src from lane i - n of its 16-lane row, 0 for the first
// n lanes of the row (DPP row shift; dpp_ctrl 0x110 + n).
template <int N>
__device__ __forceinline__ uint32_t row_shr(uint32_t src) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)src, 0x110 + N, 0xF, 0xF, false);
}

// Inclusive prefix sum within each 16-lane row.
__device__ __forceinline__ uint32_t row_incl_sum_u32(uint32_t v) {
  v += row_shr<1>(v);
  v += row_shr<2>(v);
  v += row_shr<4>(v);
  v += row_shr<8>(v);
  return v;
}

// Inclusive prefix sum over the lanes of a wave: row scans, then the last
// lane of row 0 is added into row 1 and of row 2 into row 3 (row_bcast:15,
// dpp_ctrl 0x142, rows 1 and 3), then the last lane of row 1 into rows 2 and
// 3 (row_bcast:31, dpp_ctrl 0x143).
__device__ __forceinline__ uint32_t wave_incl_sum_u32(uint32_t v) {
  v = row_incl_sum_u32(v);
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xA, 0xF, false);
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xC, 0xF, false);
  return v;
}

// Inclusive max-scan within each 16-lane row (identity INT_MIN), and over the
// whole wave (the row ends carried forward as in wave_incl_sum_u32).
__device__ __forceinline__ int row_incl_max_i32(int v) {
  v = max(v, __builtin_amdgcn_update_dpp(INT_MIN, v, 0x111, 0xF, 0xF, false));
  v = max(v, __builtin_amdgcn_update_dpp(INT_MIN, v, 0x112, 0xF, 0xF, false));
  v = max(v, __builtin_amdgcn_update_dpp(INT_MIN, v, 0x114, 0xF, 0xF, false));
  v = max(v, __builtin_amdgcn_update_dpp(INT_MIN, v, 0x118, 0xF, 0xF, false));
  return v;
}
__device__ __forceinline__ int wave_incl_max_i32(int v) {
  v = row_incl_max_i32(v);
  v = max(v, __builtin_amdgcn_update_dpp(INT_MIN, v, 0x142, 0xA, 0xF, false));
  v = max(v, __builtin_amdgcn_update_dpp(INT_MIN, v, 0x143, 0xC, 0xF, false));
  return v;
}
// Inclusive min-scan from the right (lane i: minimum over lanes >= i) within
// each 16-lane row (DPP row shift left; identity INT_MAX), and over the wave:
// the first lane of a row then holds the row's minimum, read into scalars
// and folded into the rows before it.
__device__ __forceinline__ int row_incl_suffix_min_i32(int v) {
  v = min(v, __builtin_amdgcn_update_dpp(INT_MAX, v, 0x101, 0xF, 0xF, false));
  v = min(v, __builtin_amdgcn_update_dpp(INT_MAX, v, 0x102, 0xF, 0xF, false));
  v = min(v, __builtin_amdgcn_update_dpp(INT_MAX, v, 0x104, 0xF, 0xF, false));
  v = min(v, __builtin_amdgcn_update_dpp(INT_MAX, v, 0x108, 0xF, 0xF, false));
  return v;
}
__device__ __forceinline__ int wave_incl_suffix_min_i32(int v) {
  v = row_incl_suffix_min_i32(v);
  const int r1 = __builtin_amdgcn_readlane(v, 16), r2 = __builtin_amdgcn_readlane(v, 32),
            r3 = __builtin_amdgcn_readlane(v, 48);
  const int lane = threadIdx.x & (WAVE - 1);
  const int m23 = min(r2, r3);
  const int after = lane < 16 ? min(r1, m23) : (lane < 32 ? m23 : (lane < 48 ? r3 : INT_MAX));
  return min(v, after);
}

// AND and OR over the lanes of a wave (DPP scans with identity ~0 / 0; the
// last lane's value read into a scalar).
__device__ __forceinline__ uint32_t wave_and_u32(uint32_t v) {
  v &= (uint32_t)__builtin_amdgcn_update_dpp(-1, (int)v, 0x111, 0xF, 0xF, false);
  v &= (uint32_t)__builtin_amdgcn_update_dpp(-1, (int)v, 0x112, 0xF, 0xF, false);
  v &= (uint32_t)__builtin_amdgcn_update_dpp(-1, (int)v, 0x114, 0xF, 0xF, false);
  v &= (uint32_t)__builtin_amdgcn_update_dpp(-1, (int)v, 0x118, 0xF, 0xF, false);
  v &= (uint32_t)__builtin_amdgcn_update_dpp(-1, (int)v, 0x142, 0xA, 0xF, false);
  v &= (uint32_t)__builtin_amdgcn_update_dpp(-1, (int)v, 0x143, 0xC, 0xF, false);
  return (uint32_t)__builtin_amdgcn_readlane((int)v, WAVE - 1);
}
__device__ __forceinline__ uint32_t wave_or_u32(uint32_t v) {
  v |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xF, 0xF, false);
  v |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xF, 0xF, false);
  v |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xF, 0xF, false);
  v |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xF, 0xF, false);
  v |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xA, 0xF, false);
  v |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xC, 0xF, false);
  return (uint32_t)__builtin_amdgcn_readlane((int)v, WAVE - 1);
}

template <int T, int E, int B>
struct BlockDigitRank {
  static_assert(T % WAVE == 0, "whole waves");
  static_assert(B >= 2 && B <= 8, "digit width");
  static_assert(T * E <= 65535, "16-bit counters");
  static constexpr int W = T / WAVE;
  static constexpr int C = 1 << (B - 1);  // counter words per thread
  static constexpr int kCounterWords = C * T;
  static constexpr int kScratchWords = W;
  static constexpr uint32_t kMask = (1u << B) - 1u;

  // The digit of item j is bits [off, off + B) of its key (klo[j], and
  // khi[j] above bit 31 when KW == 2); it is computed twice rather than kept
  // live across the barriers. All items of a wave take part when `active`
  // (wave-uniform) is set, none otherwise; on return pos[j] is the item's
  // position in the stable digit order (undefined for an inactive wave).
  // cnt: kCounterWords u32 of LDS, red: kScratchWords u32 of LDS. Contains
  // three workgroup barriers; between calls a thread touches no counter word
  // but its own.
  template <int KW>
  __device__ static __forceinline__ uint32_t digit_of(uint32_t lo, uint32_t hi, int off) {
    if constexpr (KW == 2) return (uint32_t)((((uint64_t)hi << 32) | lo) >> off) & kMask;
    return (lo >> off) & kMask;
  }
  // counter word (d mod C) and half (d / C) of an item's digit. INSIDE: the
  // whole digit lies in the 32-bit key (off + B <= 32), so that each part is
  // one field extract; otherwise the digit is extracted once (bits past 31
  // read as zero) and split.
  template <int KW, bool INSIDE>
  __device__ static __forceinline__ void digit_parts(uint32_t lo, uint32_t hi, int off, uint32_t& col,
                                                     uint32_t& half) {
    if constexpr (KW == 1 && INSIDE) {
      col = __builtin_amdgcn_ubfe(lo, (uint32_t)off, (uint32_t)(B - 1));
      half = __builtin_amdgcn_ubfe(lo, (uint32_t)(off + B - 1), 1u);
    } else if constexpr (KW == 1) {
      const uint32_t d = __builtin_amdgcn_ubfe(lo, (uint32_t)off, (uint32_t)B);
      col = d & (C - 1);
      half = d >> (B - 1);
    } else {
      const uint32_t d = digit_of<KW>(lo, hi, off);
      col = d & (C - 1);
      half = d >> (B - 1);
    }
  }
  template <int KW>
  __device__ static __forceinline__ void rank(const uint32_t (&klo)[E], const uint32_t (&khi)[E], int off, bool active,
                                              uint32_t* cnt, uint32_t* red, uint32_t (&pos)[E]) {
    if (KW == 1 && off + B <= 32)  // workgroup-uniform
      rank_t<KW, true>(klo, khi, off, active, cnt, red, pos);
    else
      rank_t<KW, false>(klo, khi, off, active, cnt, red, pos);
  }
  template <int KW, bool INSIDE>
  __device__ static __forceinline__ void rank_t(const uint32_t (&klo)[E], const uint32_t (&khi)[E], int off,
                                                bool active, uint32_t* cnt, uint32_t* red, uint32_t (&pos)[E]) {
    const int t = threadIdx.x, lane = t & (WAVE - 1), w = t / WAVE;
    // 1. private counters: clear, then count in order (pos[j] holds the
    //    counter word before the item's increment)
#pragma unroll
    for (int c = 0; c < C; ++c) cnt[c * T + t] = 0u;
    if (active) {
#pragma unroll
      for (int j = 0; j < E; ++j) {
        uint32_t col, half;
        digit_parts<KW, INSIDE>(klo[j], khi[j], off, col, half);
        pos[j] = atomicAdd(&cnt[col * T + t], half * 0xFFFFu + 1u);  // 1 or 1 << 16
      }
    }
    __syncthreads();
    // 2. exclusive scan of the words in linear order; thread t owns words
    //    [t*C, t*C + C)
    uint32_t v[C];
    if constexpr (C % 4 == 0) {
      const uint4* src = reinterpret_cast<const uint4*>(cnt + t * C);
#pragma unroll
      for (int q = 0; q < C / 4; ++q) {
        const uint4 x = src[q];
        v[4 * q] = x.x; v[4 * q + 1] = x.y; v[4 * q + 2] = x.z; v[4 * q + 3] = x.w;
      }
    } else {
#pragma unroll
      for (int c = 0; c < C; ++c) v[c] = cnt[t * C + c];
    }
    uint32_t run = 0u;
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const uint32_t x = v[c];
      v[c] = run;
      run += x;
    }
    const uint32_t incl = wave_incl_sum_u32(run);
    if (lane == WAVE - 1) red[w] = incl;
    __syncthreads();
    // the waves' totals, scanned across the first W lanes of every wave
    static_assert(W <= 16, "wave totals fit one DPP row");
    const uint32_t wsum = row_incl_sum_u32(lane < W ? red[lane] : 0u);
    const int wu = __builtin_amdgcn_readfirstlane(w);
    const uint32_t before = wu ? (uint32_t)__builtin_amdgcn_readlane((int)wsum, wu - 1) : 0u;
    const uint32_t grand = (uint32_t)__builtin_amdgcn_readlane((int)wsum, W - 1);
    uint32_t base = incl - run + before;
    base += (grand & 0xFFFFu) << 16;  // upper halves follow every lower-half digit
    if constexpr (C % 4 == 0) {
      uint4* dst = reinterpret_cast<uint4*>(cnt + t * C);
#pragma unroll
      for (int q = 0; q < C / 4; ++q)
        dst[q] = make_uint4(v[4 * q] + base, v[4 * q + 1] + base, v[4 * q + 2] + base, v[4 * q + 3] + base);
    } else {
#pragma unroll
      for (int c = 0; c < C; ++c) cnt[t * C + c] = v[c] + base;
    }
    __syncthreads();
    // 3. positions (the shift and column index are laundered so that the
    //    counting phase's digits and addresses are recomputed, not kept live
    //    across the scan)
    int tl = t, offl = __builtin_amdgcn_readfirstlane(off);
    asm volatile("" : "+v"(tl));
    asm volatile("" : "+s"(offl));
    if (active) {
#pragma unroll
      for (int j = 0; j < E; ++j) {
        uint32_t col, half;
        digit_parts<KW, INSIDE>(klo[j], khi[j], offl, col, half);
        const uint32_t word = cnt[col * T + tl];
        pos[j] = __builtin_amdgcn_ubfe(word + pos[j], half << 4, 16u);
      }
    }
  }
};

}  // namespace cpc
