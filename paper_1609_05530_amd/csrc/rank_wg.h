// rank_wg.h — the workgroup-per-subset rank kernel: ranks of eq. (12) of
// arXiv:1609.05530 within each subset of the partition (eq. 14), for subsets
// of up to T*E rows. Each margin is read once from HBM into registers
// (blocked arrangement), stably radix-sorted by its order-preserving key
// with the row index as payload (block_rank.h) or, in the one-wave merge
// shape, merge-sorted as (key, row) words, and tie groups are found in
// sorted order by two workgroup scans. Outputs per row: the doubled rank
// R = 2 r (average ranks for ties: R = 2 #{less} + #{equal} + 1, or ties
// broken by row order), the sorted position and the start of the row's tie
// group (the last two feed the variance kernel's suffix sums).
//
// Only the key bits that vary within the subset are sorted on: the AND and
// OR of all keys give the varying range, and B-bit digit passes cover it
// from its lowest bit; a digit that is constant over the subset is skipped.
#pragma once

#include <hip/hip_runtime.h>

#include <climits>
#include <type_traits>

#include "block_rank.h"
#include "kernels.h"

namespace cpc {

// LDS of the rank kernel: digit counters (CNT words), the exchange buffer
// (CAP u32 keys, then CAP payloads of 16 or 32 bits) and a few small arrays.
// ALIAS: counters share memory with the exchange buffer (less LDS, two more
// barriers per pass). P32: 32-bit payloads (a scatter lane writes a whole
// word instead of half of one). Without ALIAS the small arrays live in memory
// that is idle while they are in use: the counter-scan scratch `red` in the
// exchange keys (between a pass's gather and its next scatter), the AND / OR
// of the keys in the payload area (load phase), the tie-phase arrays in the
// counters (after the last pass).
// PAD: each thread's block of E keys (and of E payloads) is followed by 16
// unused bytes where needed, so that the per-lane stride is an odd multiple
// of 16 bytes and the lanes' 16-byte reads of their own blocks fall in
// distinct banks.
template <int T, int E, int B, int KW, bool ALIAS, bool P32, bool PAD = false>
struct RankLds {
  static constexpr int W = T / WAVE;
  static constexpr int CAP = T * E;
  static constexpr int CNT = BlockDigitRank<T, E, B>::kCounterWords;
  static constexpr int KPAD = PAD ? 4 : 0;                     // u32 words after each key block
  static constexpr int VPAD = !PAD ? 0 : P32 ? 4 : (E == 8 ? 0 : 8);  // payload elements after each block
  static constexpr int CAPK = CAP + (CAP / E) * KPAD;          // key words
  static constexpr int CAPV = CAP + (CAP / E) * VPAD;          // payload elements
  static constexpr int XW = CAPK + (P32 ? CAPV : (CAPV + 1) / 2);
  static_assert(E % 8 == 0 || !PAD, "padded blocks stay 16-byte aligned");
  // exchange index of position p (keys; payloads)
  __device__ static __forceinline__ int kx(int p) { return PAD ? p + (p / E) * KPAD : p; }
  __device__ static __forceinline__ int vx(int p) { return PAD ? p + (p / E) * VPAD : p; }
  static constexpr int SMALL = 3 * W + W * KW + 8;  // red, wmax, wmin, wl, andor (+ non-finite flag)
  static constexpr int MAIN = ALIAS ? (CNT > XW ? CNT : XW) + SMALL : CNT + XW;
  // tie phase (not aliased): wmax, wmin, wl and the per-wave tie flags in the counters
  static_assert(ALIAS || CNT >= 4 * W + W * KW, "tie-phase arrays fit in the counters");
  alignas(16) uint32_t main[MAIN];  // 16-byte vector reads of keys, payloads, counters
  __device__ __forceinline__ uint32_t* cnt() { return main; }
  __device__ __forceinline__ uint32_t* xk() { return ALIAS ? main : main + CNT; }
  __device__ __forceinline__ uint32_t* xv32() { return xk() + CAPK; }
  __device__ __forceinline__ uint16_t* xv16() { return reinterpret_cast<uint16_t*>(xk() + CAPK); }
  __device__ __forceinline__ uint32_t* small() { return main + (MAIN - SMALL); }
  __device__ __forceinline__ uint32_t* red() { return ALIAS ? small() : xk(); }
  __device__ __forceinline__ int32_t* wmax() { return (int32_t*)(ALIAS ? small() + W : cnt()); }
  __device__ __forceinline__ int32_t* wmin() { return wmax() + W; }
  __device__ __forceinline__ uint32_t* wl() { return (uint32_t*)(wmax() + 2 * W); }
  // per-wave "has a tie" votes (counter region, free after the passes;
  // unaliased layout only)
  __device__ __forceinline__ int32_t* wflag() { return wmax() + 2 * W + W * KW; }
  // per-wave longest run of equal leading key bits (truncated sorts)
  __device__ __forceinline__ int32_t* wrun() { return wflag() + W; }
  __device__ __forceinline__ uint32_t* andor() { return ALIAS ? small() + 3 * W + W * KW : xv32(); }
};
static_assert(sizeof(RankLds<1024, 16, 4, 2, false, false, true>) <= 160 * 1024, "largest rank LDS layout fits");


// Merge-sort alternative to the radix passes (32-bit keys): each element is
// the 64-bit word (key << 32 | row), so that the sorted order of the words
// is the stable order of the keys. Each thread sorts its E words in
// registers (bitonic network), then runs of E, 2E, ... are merged by merge
// path in LDS: a thread's E outputs start where the diagonal through its
// first output crosses the two runs (one binary search), and the words are
// merged with two pointers into registers; after a barrier they are written
// back in place. Levels stop once one run holds every valid element (the
// words past n are the largest and already in order).
template <int E>
__device__ __forceinline__ void sort_regs_u64(uint64_t (&w)[E]) {
#pragma unroll
  for (int k = 2; k <= E; k <<= 1)
#pragma unroll
    for (int j = k >> 1; j > 0; j >>= 1)
#pragma unroll
      for (int i = 0; i < E; ++i) {
        const int l = i ^ j;
        if (l > i) {
          const bool up = (i & k) == 0;
          const uint64_t a = w[i], b = w[l];
          const bool swap = up ? (a > b) : (a < b);
          w[i] = swap ? b : a;
          w[l] = swap ? a : b;
        }
      }
}

template <int T, int E>
__device__ __forceinline__ void merge_sort_words(uint64_t (&w)[E], uint64_t* buf, int n) {
  const int p0 = threadIdx.x * E;
  sort_regs_u64<E>(w);
#pragma unroll 1
  for (int L = E; L < n; L <<= 1) {
#pragma unroll
    for (int j = 0; j < E; ++j) buf[p0 + j] = w[j];
    __syncthreads();
    const int base = p0 & ~(2 * L - 1);
    const uint64_t* A = buf + base;
    const uint64_t* Bv = buf + base + L;
    const int d0 = p0 - base;
    int lo = max(0, d0 - L), hi = min(d0, L);
    while (lo < hi) {
      const int i = (lo + hi) >> 1;
      if (A[i] < Bv[d0 - i - 1]) lo = i + 1; else hi = i;
    }
    int ia = lo, ib = d0 - lo;
    uint64_t a = ia < L ? A[ia] : ~0ull, b = ib < L ? Bv[ib] : ~0ull;
#pragma unroll
    for (int j = 0; j < E; ++j) {
      const bool ta = a < b;  // (an exhausted run reads as ~0, above every word)
      w[j] = ta ? a : b;
      ia += ta ? 1 : 0;
      ib += ta ? 0 : 1;
      const int idx = ta ? ia : ib;
      const uint64_t v = idx < L ? (ta ? A : Bv)[idx] : ~0ull;
      a = ta ? v : a;
      b = ta ? b : v;
    }
    __syncthreads();
  }
}

// Ranks one margin and writes, per row of the subset, the sorted position e
// and, if the margin has ties, the doubled rank R and the tie-group start lb
// (without ties R = 2e + 2 and lb = e, and e_is_l is set in every thread;
// MODE_RANK writes R alone, as 32-bit values). Returns true (in every thread)
// if the margin holds a non-finite value; sets all_tied (in thread 0) if
// every value is equal.
template <int T, int E, int B, int KW, bool ALIAS, bool P32, bool PACK, bool PAD, bool MERGE, int TRUNC, typename DT>
__device__ __forceinline__ bool rank_one_margin(const DT* data, int n, int ties, bool int_keys,
                                                RankLds<T, E, B, KW, ALIAS, P32, PAD>& sm, uint16_t* Rg, uint16_t* Eg,
                                                uint16_t* Lg, uint32_t* R32, bool& all_tied, bool& e_is_l,
                                                bool& redo) {
  using Rank = BlockDigitRank<T, E, B>;
  using Lds = RankLds<T, E, B, KW, ALIAS, P32, PAD>;
  constexpr int W = T / WAVE;
  constexpr uint32_t MASK = Rank::kMask;
  const int t = threadIdx.x, lane = t & (WAVE - 1), w = t / WAVE;
  const int p0 = t * E;
  const int nv = min(max(n - p0, 0), E);
  uint32_t* cnt = sm.cnt();
  uint32_t* xk = sm.xk();
  uint32_t* andor = sm.andor();
  all_tied = false;
  e_is_l = false;
  redo = false;
  if (n <= 0) return false;

  // Truncated sorts (TRUNC > 0, 32-bit keys) first sort on the TRUNC leading
  // varying key bits only and put the elements of each run of equal leading
  // bits in order by counting, in the run, the keys below theirs; a run
  // longer than RUN_MAX returns with `redo` set, nothing written: the caller
  // then sorts the margin again over every varying bit.
  static_assert(TRUNC == 0 || (KW == 1 && !ALIAS && !PACK && !MERGE), "truncated sorts: 32-bit keys, unpacked");
  constexpr int RUN_MAX = 32;
  // load, keys, non-finite flag, AND / OR of the keys. 32-bit keys are read
  // coalesced and transposed to the blocked arrangement through LDS; 64-bit
  // keys are read blocked. An item past the end takes the largest key: the
  // stable sort keeps it behind every valid element, at a position >= n.
  uint32_t klo[E], khi[E], pay[E];
  uint64_t kand = ~0ull, kor = 0ull;
  bool bad = false;
  if (t == 0) {
    andor[0] = andor[1] = ~0u;
    andor[2] = andor[3] = andor[4] = 0u;
  }
#pragma unroll
  for (int j = 0; j < E; ++j) pay[j] = (uint32_t)(p0 + j);
  if constexpr (KW == 1) {
    auto load = [&](auto ik) {
      constexpr bool IK = decltype(ik)::value;
#pragma unroll
      for (int j = 0; j < E; ++j) {
        const int e = j * T + t;
        const bool valid = e < n;
        uint32_t k;
        if constexpr (IK) {
          k = ((const uint32_t*)data)[min(e, n - 1)];
        } else {
          const DT v = data[min(e, n - 1)];
          bad |= valid && !isfinite(v);
          k = key_of((float)v);
        }
        kand &= valid ? (uint64_t)k : ~0ull;
        kor |= valid ? (uint64_t)k : 0ull;
        xk[Lds::kx(e)] = valid ? k : ~0u;
      }
    };
    if (int_keys)
      load(std::true_type{});
    else
      load(std::false_type{});
  } else {
#pragma unroll
    for (int j = 0; j < E; ++j) {
      const bool valid = j < nv;
      const DT v = data[min(p0 + j, n - 1)];
      bad |= valid && !isfinite(v);
      uint64_t k = key_of((double)v);
      kand &= valid ? k : ~0ull;
      kor |= valid ? k : 0ull;
      k = valid ? k : ~0ull;
      klo[j] = (uint32_t)k;
      khi[j] = (uint32_t)(k >> 32);
    }
  }
  kand = ((uint64_t)wave_and_u32((uint32_t)(kand >> 32)) << 32) | wave_and_u32((uint32_t)kand);
  kor = ((uint64_t)wave_or_u32((uint32_t)(kor >> 32)) << 32) | wave_or_u32((uint32_t)kor);
  __syncthreads();  // andor initialised; previous margin's LDS use finished
  if (lane == 0) {
    atomicAnd(&andor[0], (uint32_t)kand);
    atomicAnd(&andor[1], (uint32_t)(kand >> 32));
    atomicOr(&andor[2], (uint32_t)kor);
    atomicOr(&andor[3], (uint32_t)(kor >> 32));
  }
  const uint64_t badw = __ballot(bad);
  if (lane == 0 && badw != 0ull) atomicOr(&andor[4], 1u);
  __syncthreads();
  if constexpr (KW == 1) {
    const uint4* sk = reinterpret_cast<const uint4*>(xk + Lds::kx(p0));
#pragma unroll
    for (int q = 0; q < E / 4; ++q) {
      const uint4 a = sk[q];
      klo[4 * q] = a.x; klo[4 * q + 1] = a.y; klo[4 * q + 2] = a.z; klo[4 * q + 3] = a.w;
      khi[4 * q] = khi[4 * q + 1] = khi[4 * q + 2] = khi[4 * q + 3] = 0u;
    }
    if (ALIAS) __syncthreads();  // the first pass clears counters over these keys
  }
  // workgroup-uniform from here on (read into scalar registers)
  const uint32_t a0 = __builtin_amdgcn_readfirstlane(andor[0]), a1 = __builtin_amdgcn_readfirstlane(andor[1]);
  const uint32_t o0 = __builtin_amdgcn_readfirstlane(andor[2]), o1 = __builtin_amdgcn_readfirstlane(andor[3]);
  const uint64_t var = ((((uint64_t)a1) << 32) | a0) ^ ((((uint64_t)o1) << 32) | o0);
  bad = __builtin_amdgcn_readfirstlane(andor[4]) != 0u;

  // radix passes over the varying bits; waves wholly past the end sit out
  // (their items keep their own positions >= n and their payloads).
  // Packed exchange (PACK, 32-bit keys): once the key bits that later passes
  // still need fit beside the payload in one word, key and payload move
  // together (one scatter per element instead of two); the word then holds
  // key bits from `kbase` up at bit PB, and the payload in the low PB bits.
  // The tie groups then need the full keys, read back from the margin by row.
  constexpr int CAP = T * E;
  constexpr bool CAN_PACK = PACK && (KW == 1) && !P32;
  constexpr int PB = (CAP <= 512) ? 9 : (CAP <= 2048) ? 11 : (CAP <= 4096) ? 12 : (CAP <= 8192) ? 13 : 14;
  static_assert(CAP <= (1 << PB), "payload field holds every position");
  constexpr uint32_t PMASK = (1u << PB) - 1u;
  bool packed = false;
  int kbase = 0;
  int tsh = 0;  // truncated sort: the lowest key bit sorted on (0: every varying bit)
  const bool active = w * WAVE * E < n;
  if constexpr (MERGE) {
    static_assert(KW == 1 && !ALIAS && !PACK, "merge sort: 32-bit keys, own buffer");
    static_assert(Lds::MAIN >= 2 * CAP, "the 64-bit merge buffer fits the LDS layout");
    if (var != 0ull && n > 1) {
      uint64_t wd[E];
#pragma unroll
      for (int j = 0; j < E; ++j) wd[j] = ((uint64_t)klo[j] << 32) | pay[j];
      __syncthreads();  // the keys' transposition buffer is read
      merge_sort_words<T, E>(wd, reinterpret_cast<uint64_t*>(sm.main), n);
#pragma unroll
      for (int j = 0; j < E; ++j) {
        klo[j] = (uint32_t)(wd[j] >> 32);
        pay[j] = (uint32_t)wd[j];
      }
    }
  } else if (var != 0ull && n > 1) {
    const int hi = 63 - __builtin_clzll(var);
    int lo = __builtin_ctzll(var);
    if (TRUNC > 0 && hi + 1 - TRUNC > lo) {
      lo = hi + 1 - TRUNC;
      tsh = lo;
    }
    const int npass = (hi - lo) / B + 1;
    int ps = 0;
    // passes with separate key and payload (the last of them may already
    // write packed words)
#pragma unroll 1
    for (; ps < npass; ++ps) {
      const int off = lo + ps * B;
      if (((var >> off) & MASK) == 0ull) continue;  // constant digit: identity pass
      uint32_t pos[E];
      Rank::template rank<KW>(klo, khi, off, active, cnt, sm.red(), pos);
      if (ALIAS) __syncthreads();  // counters are read until here
      bool pack_now = false;
      if constexpr (CAN_PACK) {
        const int rem = hi - (off + B) + 1;  // key bits that later passes need
        pack_now = rem <= 0 || rem + PB <= 32;
      }
      if (active) {
        if (pack_now) {
          const int sh = off + B;
#pragma unroll
          for (int j = 0; j < E; ++j) xk[Lds::kx(pos[j])] = ((sh >= 32) ? 0u : (klo[j] >> sh) << PB) | pay[j];
        } else {
#pragma unroll
          for (int j = 0; j < E; ++j) {
            xk[Lds::kx(pos[j])] = klo[j];
            if constexpr (P32)
              sm.xv32()[Lds::vx(pos[j])] = pay[j];
            else
              sm.xv16()[Lds::vx(pos[j])] = (uint16_t)pay[j];
          }
        }
      }
      __syncthreads();
      if (active) {
        const uint4* sk = reinterpret_cast<const uint4*>(xk + Lds::kx(p0));
#pragma unroll
        for (int q = 0; q < E / 4; ++q) {
          const uint4 a = sk[q];
          klo[4 * q] = a.x; klo[4 * q + 1] = a.y; klo[4 * q + 2] = a.z; klo[4 * q + 3] = a.w;
        }
        if (!pack_now) {
          if constexpr (P32) {
            const uint4* sv = reinterpret_cast<const uint4*>(sm.xv32() + Lds::vx(p0));
#pragma unroll
            for (int q = 0; q < E / 4; ++q) {
              const uint4 a = sv[q];
              pay[4 * q] = a.x; pay[4 * q + 1] = a.y; pay[4 * q + 2] = a.z; pay[4 * q + 3] = a.w;
            }
          } else {
            const uint4* sv = reinterpret_cast<const uint4*>(sm.xv16() + Lds::vx(p0));
#pragma unroll
            for (int q = 0; q < E / 8; ++q) {
              const uint4 a = sv[q];
              pay[8 * q] = a.x & 0xFFFFu; pay[8 * q + 1] = a.x >> 16;
              pay[8 * q + 2] = a.y & 0xFFFFu; pay[8 * q + 3] = a.y >> 16;
              pay[8 * q + 4] = a.z & 0xFFFFu; pay[8 * q + 5] = a.z >> 16;
              pay[8 * q + 6] = a.w & 0xFFFFu; pay[8 * q + 7] = a.w >> 16;
            }
          }
        }
      }
      if constexpr (KW == 2) {
        __syncthreads();
        if (active) {
#pragma unroll
          for (int j = 0; j < E; ++j) xk[Lds::kx(pos[j])] = khi[j];
        }
        __syncthreads();
        if (active) {
          const uint4* sk = reinterpret_cast<const uint4*>(xk + Lds::kx(p0));
#pragma unroll
          for (int q = 0; q < E / 4; ++q) {
            const uint4 a = sk[q];
            khi[4 * q] = a.x; khi[4 * q + 1] = a.y; khi[4 * q + 2] = a.z; khi[4 * q + 3] = a.w;
          }
        }
      }
      if (ALIAS) __syncthreads();  // exchange buffer is read until here
      if (pack_now) {
        packed = true;
        kbase = off + B;
        ++ps;
        break;
      }
    }
    // passes over packed words
    if constexpr (CAN_PACK) {
      if (packed) {
#pragma unroll 1
        for (; ps < npass; ++ps) {
          const int off = lo + ps * B;
          if (((var >> off) & MASK) == 0ull) continue;
          uint32_t pos[E];
          Rank::template rank<KW>(klo, khi, PB + off - kbase, active, cnt, sm.red(), pos);
          if (ALIAS) __syncthreads();
          if (active) {
#pragma unroll
            for (int j = 0; j < E; ++j) xk[Lds::kx(pos[j])] = klo[j];
          }
          __syncthreads();
          if (active) {
            const uint4* sk = reinterpret_cast<const uint4*>(xk + Lds::kx(p0));
#pragma unroll
            for (int q = 0; q < E / 4; ++q) {
              const uint4 a = sk[q];
              klo[4 * q] = a.x; klo[4 * q + 1] = a.y; klo[4 * q + 2] = a.z; klo[4 * q + 3] = a.w;
            }
          }
          if (ALIAS) __syncthreads();
        }
      }
    }
  }
  if constexpr (CAN_PACK) {
    if (packed) {
      // payloads out of the packed words; the full keys (for the tie groups)
      // are read back from the margin by row (an item past the end re-reads
      // the last row: its key is not used)
#pragma unroll
      for (int j = 0; j < E; ++j) pay[j] = klo[j] & PMASK;
#pragma unroll
      for (int j = 0; j < E; ++j) {
        const int r = min((int)pay[j], n - 1);
        if (int_keys)
          klo[j] = ((const uint32_t*)data)[r];
        else
          klo[j] = key_of((float)data[r]);
      }
    }
  }

  // tie groups: a sorted position starts a group unless its key equals its
  // predecessor's (truncated sorts: runs of equal leading bits, put in order
  // and split into tie groups below)
  if (lane == WAVE - 1) {
    sm.wl()[w * KW] = klo[E - 1];
    if (KW == 2) sm.wl()[w * KW + KW - 1] = khi[E - 1];
  }
  uint32_t plo = __shfl_up(klo[E - 1], 1, WAVE);
  uint32_t phi = (KW == 2) ? __shfl_up(khi[E - 1], 1, WAVE) : 0u;
  __syncthreads();
  if (lane == 0 && w > 0) {
    plo = sm.wl()[(w - 1) * KW];
    if (KW == 2) phi = sm.wl()[(w - 1) * KW + KW - 1];
  }
  static_assert(E <= 32, "the group-start bits of a thread's items fit one word");
  uint32_t headm = 0u;  // bit j: item j starts a group
  int hmax = -1, hmin = INT_MAX;
#pragma unroll
  for (int j = 0; j < E; ++j) {
    const uint32_t ql = j ? klo[j - 1] : plo;
    const uint32_t qh = j ? khi[j - 1] : phi;
    const bool head = (j < nv) && ((p0 + j == 0) || (ql >> tsh) != (klo[j] >> tsh) || (KW == 2 && qh != khi[j]));
    headm |= head ? (1u << j) : 0u;
    hmax = head ? p0 + j : hmax;
    hmin = head ? min(hmin, p0 + j) : hmin;
  }
  // exclusive max-scan from the left and min-scan from the right
  const int imax = wave_incl_max_i32(hmax);
  const int imin = wave_incl_suffix_min_i32(hmin);
  if (lane == WAVE - 1) sm.wmax()[w] = imax;
  if (lane == 0) sm.wmin()[w] = imin;
  // does any valid item continue a tie group? (then the doubled ranks and
  // group starts are stored beside the sorted positions)
  const uint32_t vmask = nv >= 32 ? 0xFFFFFFFFu : ((1u << nv) - 1u);
  const bool tied_here = (headm & vmask) != vmask;
  if (!ALIAS && tsh == 0) {
    const bool wtie = __ballot(tied_here) != 0ull;
    if (lane == 0) sm.wflag()[w] = wtie ? 1 : 0;
  }
  int cl = __shfl_up(imax, 1, WAVE);
  int cr = __shfl_down(imin, 1, WAVE);
  if (lane == 0) cl = -1;
  if (lane == WAVE - 1) cr = INT_MAX;
  if (TRUNC > 0 && tsh > 0) {
    // truncated sort: the longest stretch of one run inside this wave (a run
    // over two waves is at most twice that; one over three fills a wave)
    int cur = max(cl, w * WAVE * E), rl = 0;
#pragma unroll
    for (int j = 0; j < E; ++j) {
      if ((headm >> j) & 1u) cur = p0 + j;
      rl = (j < nv) ? max(rl, p0 + j - cur + 1) : rl;
    }
    rl = __builtin_amdgcn_readlane(wave_incl_max_i32(rl), WAVE - 1);
    if (lane == 0) sm.wrun()[w] = rl;
  }
  __syncthreads();
  if (TRUNC > 0 && tsh > 0) {  // workgroup-uniform
    const int mr = __builtin_amdgcn_readlane(row_incl_max_i32(lane < W ? sm.wrun()[lane] : 0), W - 1);
    if (mr > RUN_MAX) {
      __syncthreads();  // every thread has read the run lengths
      redo = true;      // the caller sorts again over every varying bit
      return bad;
    }
  }
  {
    // the waves before (max) and after (min) this one: every lane of row 0
    // reads one wave's value, scanned across the row
    static_assert(W <= 16, "wave values fit one DPP row");
    const int a = row_incl_max_i32(lane < W ? sm.wmax()[lane] : INT_MIN);
    const int b = row_incl_suffix_min_i32(lane < W ? sm.wmin()[lane] : INT_MAX);
    const int wu = __builtin_amdgcn_readfirstlane(w);
    if (wu > 0) cl = max(cl, __builtin_amdgcn_readlane(a, wu - 1));
    if (wu + 1 < W) cr = min(cr, __builtin_amdgcn_readlane(b, wu + 1));
  }
  cr = min(cr, n);
  uint32_t lb[E], ub[E];
  {
    int cur = cl;
#pragma unroll
    for (int j = 0; j < E; ++j) {
      if ((headm >> j) & 1u) cur = p0 + j;
      lb[j] = (uint32_t)cur;
    }
    cur = cr;
#pragma unroll
    for (int j = E - 1; j >= 0; --j) {
      ub[j] = (uint32_t)cur;
      if ((headm >> j) & 1u) cur = p0 + j;
    }
  }
  // sorted positions; truncated sorts: the order inside each run of equal
  // leading bits, from the full keys of the run (in sorted order in the
  // exchange buffer since the last pass), and the exact tie groups
  uint32_t epos[E];
#pragma unroll
  for (int j = 0; j < E; ++j) epos[j] = (uint32_t)(p0 + j);
  const bool fixup = TRUNC > 0 && tsh > 0;  // workgroup-uniform
  if (fixup) {
    bool tie = false;
#pragma unroll
    for (int j = 0; j < E; ++j) {
      if (j < nv && ub[j] - lb[j] > 1u) {
        const uint32_t k = klo[j], p = (uint32_t)(p0 + j);
        uint32_t less = 0u, eqc = 0u, eqb = 0u;
#pragma unroll 1
        for (uint32_t q = lb[j]; q < ub[j]; ++q) {
          const uint32_t kq = xk[Lds::kx((int)q)];
          less += kq < k ? 1u : 0u;
          eqc += kq == k ? 1u : 0u;
          eqb += (kq == k && q < p) ? 1u : 0u;
        }
        epos[j] = lb[j] + less + eqb;
        lb[j] += less;
        ub[j] = lb[j] + eqc;
        tie |= eqc > 1u;
      }
    }
    const bool wtie = __ballot(tie) != 0ull;
    if (lane == 0) sm.wflag()[w] = wtie ? 1 : 0;  // read after the row-order scatter
    __syncthreads();  // the runs' keys are read before the scatter overwrites them
  }
  // workgroup-uniform: every row's group start equals its sorted position
  // (and its doubled rank is 2 x position + 2: neither is stored then); after
  // a fix-up the tie flags are read after the row-order scatter
  bool eq = false;
  auto read_eq = [&]() {
    if constexpr (!ALIAS) {
      const int f = lane < W ? sm.wflag()[lane] : 0;
      eq = (ties == 1) || (__ballot(f != 0) == 0ull);
    }
  };
  if (!fixup) read_eq();
  all_tied = (n >= 1) && (t == 0) && (ub[0] >= (uint32_t)n);
  // R, sorted position and group start, scattered to row order in LDS
  uint16_t* xl = sm.xv16();
  // (an item past the end carries a payload >= n)
#pragma unroll
  for (int j = 0; j < E; ++j) {
    const uint32_t e = epos[j];
    const uint32_t R = (ties == 1) ? 2u * (e + 1u) : lb[j] + ub[j] + 1u;
    const uint32_t l = (ties == 1) ? e : lb[j];
    xk[pay[j]] = R | (e << 16);
    if (!eq) xl[pay[j]] = (uint16_t)l;
  }
  __syncthreads();
  if (fixup) read_eq();
  e_is_l = eq;
  if (R32) {
    for (int i = t; i < n; i += T) R32[i] = xk[i] & 0xFFFFu;
  } else {
    // 32-bit stores of row pairs that start at an even row of the arrays (the
    // three arrays share that parity); a first or last row without its pair
    // is stored alone, so no store touches another subset's rows
    const int odd = (int)((reinterpret_cast<uintptr_t>(Rg) >> 1) & 1u);
    const int npair = (n - odd) >> 1;
    for (int q = t; q < npair; q += T) {
      const int i = odd + 2 * q;
      const uint32_t v0 = xk[i], v1 = xk[i + 1];
      if (!eq) *reinterpret_cast<uint32_t*>(Rg + i) = (v0 & 0xFFFFu) | (v1 << 16);
      *reinterpret_cast<uint32_t*>(Eg + i) = (v0 >> 16) | (v1 & 0xFFFF0000u);
      if (!eq) *reinterpret_cast<uint32_t*>(Lg + i) = (uint32_t)xl[i] | ((uint32_t)xl[i + 1] << 16);
    }
    const int single = (t == 0 && odd) ? 0 : ((t == T - 1 && odd + 2 * npair < n) ? n - 1 : -1);
    if (single >= 0) {
      const uint32_t v = xk[single];
      if (!eq) Rg[single] = (uint16_t)(v & 0xFFFFu);
      Eg[single] = (uint16_t)(v >> 16);
      if (!eq) Lg[single] = xl[single];
    }
  }
  __syncthreads();
  return bad;
}

template <int T, int E, int B, int KW, bool ALIAS, bool P32, bool PACK = false, bool PAD = false, bool MERGE = false,
          int TRUNC = 0>
__global__ void __launch_bounds__(T) k_rank_wg(RankParams P) {
  __shared__ RankLds<T, E, B, KW, ALIAS, P32, PAD> sm;
  const int sid = P.order[blockIdx.x];
  const SubDesc sd = P.subs[sid];
  const int n = sd.n;
  if (P.mode != MODE_RANK && (int64_t)n < P.n_min) {
    if (threadIdx.x == 0) {
      P.state[sid].status = ST_DEGENERATE;
      P.state[sid].iters = 0;
      P.state[sid].theta = NAN;
      P.state[sid].eqmask = 0;
    }
    return;
  }
  const bool rk = P.mode == MODE_RANK;
  bool t1, t2, b1, b2, q1, q2, redo;
  const int64_t o = sd.begin;
  if constexpr (KW == 2) {
    b1 = rank_one_margin<T, E, B, KW, ALIAS, P32, PACK, PAD, MERGE, TRUNC, double>(
        (const double*)P.x + o, n, P.ties, false, sm, P.rows.R1 + o, P.rows.E1 + o, P.rows.L1 + o,
        rk ? P.R1out + o : nullptr, t1, q1, redo);
    b2 = rank_one_margin<T, E, B, KW, ALIAS, P32, PACK, PAD, MERGE, TRUNC, double>(
        (const double*)P.y + o, n, P.ties, false, sm, P.rows.R2 + o, P.rows.E2 + o, P.rows.L2 + o,
        rk ? P.R2out + o : nullptr, t2, q2, redo);
  } else {
    const bool ik = P.int_keys != 0;
    const float* xp = ik ? (const float*)((const uint32_t*)P.x + o) : (const float*)P.x + o;
    const float* yp = ik ? (const float*)((const uint32_t*)P.y + o) : (const float*)P.y + o;
    // a truncated sort that met a long run of equal leading bits leaves the
    // margin to the full sort
    b1 = rank_one_margin<T, E, B, KW, ALIAS, P32, PACK, PAD, MERGE, TRUNC, float>(
        xp, n, P.ties, ik, sm, P.rows.R1 + o, P.rows.E1 + o, P.rows.L1 + o, rk ? P.R1out + o : nullptr, t1, q1, redo);
    if (TRUNC > 0 && redo)
      b1 = rank_one_margin<T, E, B, KW, ALIAS, P32, PACK, PAD, MERGE, 0, float>(
          xp, n, P.ties, ik, sm, P.rows.R1 + o, P.rows.E1 + o, P.rows.L1 + o, rk ? P.R1out + o : nullptr, t1, q1, redo);
    b2 = rank_one_margin<T, E, B, KW, ALIAS, P32, PACK, PAD, MERGE, TRUNC, float>(
        yp, n, P.ties, ik, sm, P.rows.R2 + o, P.rows.E2 + o, P.rows.L2 + o, rk ? P.R2out + o : nullptr, t2, q2, redo);
    if (TRUNC > 0 && redo)
      b2 = rank_one_margin<T, E, B, KW, ALIAS, P32, PACK, PAD, MERGE, 0, float>(
          yp, n, P.ties, ik, sm, P.rows.R2 + o, P.rows.E2 + o, P.rows.L2 + o, rk ? P.R2out + o : nullptr, t2, q2, redo);
  }
  if (rk) return;
  const bool bad = b1 || b2;
  // all_tied is known to thread 0 only
  if (threadIdx.x == 0) {
    P.state[sid].status = bad ? ST_NONFINITE : ((t1 || t2) ? ST_DEGENERATE : ST_OK);
    P.state[sid].iters = 0;
    P.state[sid].theta = NAN;
    P.state[sid].eqmask = (q1 ? 1 : 0) | (q2 ? 2 : 0);
  }
}

}  // namespace cpc
