// k_rank.hip — ranks of eq. (12) of arXiv:1609.05530 within each subset of
// the partition (eq. 14), one workgroup per subset, for subsets of up to
// 16384 rows. Both margins are read once from HBM (coalesced), sorted in LDS
// (stable LSD radix sort, 8-bit digits) with the row index as payload, and
// tie groups are found in sorted order. Outputs per row: the doubled rank
// R = 2 r (average ranks for ties: R = 2 #{less} + #{equal} + 1, or ties
// broken by row order), the sorted position and the start of the row's tie
// group (the last two feed the variance kernel's suffix sums).
#include <hip/hip_runtime.h>

#include "kernels.h"
#include "lds_sort.h"

namespace cpc {

template <int T, int E, int KW>
struct RankSmem {
  static constexpr int W = T / WAVE;
  static constexpr int CAP = T * E;
  uint32_t buf[CAP];
  uint16_t vb[2][CAP];
  uint16_t cnt[W * 256];
  uint32_t heads[CAP / 32];
  uint32_t dtot[256 + 2 + 4];
};

// Sorts one margin and writes, per row of the subset, R (and the sorted
// position e and tie-group start lb). Returns true if the margin holds a
// non-finite value; sets all_tied if every value is equal.
template <int T, int E, int KW, typename DT>
__device__ __forceinline__ bool rank_one_margin(const DT* data, int n, int ties, bool int_keys,
                                                RankSmem<T, E, KW>& sm, uint16_t* Rg, uint16_t* Eg,
                                                uint16_t* Lg, uint32_t* R32, bool& all_tied) {
  constexpr int HW = T * E / 32;
  const int tid = threadIdx.x, lane = tid & (WAVE - 1), w = tid / WAVE;
  uint32_t klo[E], khi[E];
  bool bad = false;
#pragma unroll
  for (int j = 0; j < E; ++j) {
    const int e = (w * E + j) * WAVE + lane;
    klo[j] = 0u;
    khi[j] = 0u;
    if (e < n) {
      if (int_keys) {
        klo[j] = ((const uint32_t*)data)[e];
      } else {
        const DT v = data[e];
        bad |= !isfinite(v);
        if constexpr (KW == 2) {
          const uint64_t k = key_of((double)v);
          klo[j] = (uint32_t)k;
          khi[j] = (uint32_t)(k >> 32);
        } else {
          klo[j] = key_of((float)v);
        }
      }
    }
  }
  const int cur = lds_radix_sort<T, E, KW>(klo, khi, n, sm.buf, sm.vb[0], sm.vb[1], sm.cnt, sm.dtot);
  const uint16_t* perm = sm.vb[cur];  // original index of each sorted position
  uint16_t* lbrow = sm.vb[cur ^ 1];
  // Tie groups: a sorted position starts a group unless its key equals its
  // predecessor's. `heads` first collects the equal-to-predecessor bits word
  // by word, then becomes the group-start mask (every position >= n counts
  // as a start).
#pragma unroll
  for (int word = 0; word < KW; ++word) {
#pragma unroll
    for (int j = 0; j < E; ++j) {
      const int e = (w * E + j) * WAVE + lane;
      if (e < n) sm.buf[e] = word ? khi[j] : klo[j];
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < E; ++j) {
      const int e = (w * E + j) * WAVE + lane;
      const uint32_t mine = word ? khi[j] : klo[j];
      const uint64_t eq = __ballot((e > 0) && (e < n) && (sm.buf[e - 1] == mine));
      if (lane == 0) {
        uint32_t* h = &sm.heads[(w * E + j) * 2];
        h[0] = word ? (h[0] & (uint32_t)eq) : (uint32_t)eq;
        h[1] = word ? (h[1] & (uint32_t)(eq >> 32)) : (uint32_t)(eq >> 32);
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int j = 0; j < E; ++j) {
    const int e = (w * E + j) * WAVE + lane;
    const uint64_t valid = __ballot(e < n);
    if (lane == 0) {
      uint32_t* h = &sm.heads[(w * E + j) * 2];
      h[0] = ~h[0] | ~(uint32_t)valid;
      h[1] = ~h[1] | ~(uint32_t)(valid >> 32);
    }
  }
  __syncthreads();
  // R and the tie-group start by sorted position, scattered to row order in LDS
  for (int e = tid; e < n; e += T) {
    uint32_t R, lb;
    if (ties == 1) {
      R = 2u * (uint32_t)(e + 1);
      lb = (uint32_t)e;
    } else {
      const int l = group_lb(sm.heads, e), ub = group_ub(sm.heads, e, n, HW);
      R = (uint32_t)(l + ub + 1);
      lb = (uint32_t)l;
    }
    const int row = perm[e];
    sm.buf[row] = R | ((uint32_t)e << 16);
    lbrow[row] = (uint16_t)lb;
  }
  all_tied = (n >= 1) && (group_ub(sm.heads, 0, n, HW) >= n);
  __syncthreads();
  for (int i = tid; i < n; i += T) {
    const uint32_t v = sm.buf[i];
    if (R32) {
      R32[i] = v & 0xFFFFu;
    } else {
      Rg[i] = (uint16_t)(v & 0xFFFFu);
      Eg[i] = (uint16_t)(v >> 16);
      Lg[i] = lbrow[i];
    }
  }
  __syncthreads();
  return bad;
}

template <int T, int E, int KW>
__global__ void __launch_bounds__(T) k_rank_wg(RankParams P) {
  __shared__ RankSmem<T, E, KW> sm;
  const int sid = P.order[blockIdx.x];
  const SubDesc sd = P.subs[sid];
  const int n = sd.n;
  if (P.mode != MODE_RANK && (int64_t)n < P.n_min) {
    if (threadIdx.x == 0) {
      P.state[sid].status = ST_DEGENERATE;
      P.state[sid].iters = 0;
      P.state[sid].theta = NAN;
    }
    return;
  }
  const bool rk = P.mode == MODE_RANK;
  bool t1, t2, b1, b2;
  const int64_t o = sd.begin;
  if constexpr (KW == 2) {
    b1 = rank_one_margin<T, E, KW, double>((const double*)P.x + o, n, P.ties, false, sm, P.rows.R1 + o,
                                           P.rows.E1 + o, P.rows.L1 + o, rk ? P.R1out + o : nullptr, t1);
    b2 = rank_one_margin<T, E, KW, double>((const double*)P.y + o, n, P.ties, false, sm, P.rows.R2 + o,
                                           P.rows.E2 + o, P.rows.L2 + o, rk ? P.R2out + o : nullptr, t2);
  } else {
    const bool ik = P.int_keys != 0;
    const float* xp = ik ? (const float*)((const uint32_t*)P.x + o) : (const float*)P.x + o;
    const float* yp = ik ? (const float*)((const uint32_t*)P.y + o) : (const float*)P.y + o;
    b1 = rank_one_margin<T, E, KW, float>(xp, n, P.ties, ik, sm, P.rows.R1 + o, P.rows.E1 + o,
                                          P.rows.L1 + o, rk ? P.R1out + o : nullptr, t1);
    b2 = rank_one_margin<T, E, KW, float>(yp, n, P.ties, ik, sm, P.rows.R2 + o, P.rows.E2 + o,
                                          P.rows.L2 + o, rk ? P.R2out + o : nullptr, t2);
  }
  if (rk) return;
  const bool bad = __syncthreads_or((int)(b1 || b2)) != 0;
  if (threadIdx.x == 0) {
    P.state[sid].status = bad ? ST_NONFINITE : ((t1 || t2) ? ST_DEGENERATE : ST_OK);
    P.state[sid].iters = 0;
    P.state[sid].theta = NAN;
  }
}

template <int T, int E, int KW>
static hipError_t launch_t(const RankParams& p, int grid, hipStream_t s) {
  if (grid <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_rank_wg<T, E, KW>), dim3(grid), dim3(T), 0, s, p);
  return hipGetLastError();
}

hipError_t launch_rank_wg(int cls, int kw, const RankParams& p, int grid, hipStream_t s) {
  switch (cls) {
    case 0: return kw == 2 ? launch_t<64, 8, 2>(p, grid, s) : launch_t<64, 8, 1>(p, grid, s);
    case 1: return kw == 2 ? launch_t<256, 8, 2>(p, grid, s) : launch_t<256, 8, 1>(p, grid, s);
    case 2: return kw == 2 ? launch_t<512, 16, 2>(p, grid, s) : launch_t<512, 16, 1>(p, grid, s);
    case 3: return kw == 2 ? launch_t<1024, 16, 2>(p, grid, s) : launch_t<1024, 16, 1>(p, grid, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace cpc
