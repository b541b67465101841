// cpc_device.h — device-side building blocks shared by the libcpc kernels:
// order-preserving sort keys, wave / workgroup reductions and scans with a
// fixed combination order (bitwise reproducible), compensated FP32 sums, and
// the descriptor types the host passes in.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "row_eval.h"

namespace cpc {

constexpr int WAVE = 64;

// One subset as the kernels see it.
struct SubDesc {
  int64_t begin;   // first row
  int32_t n;       // rows (the kernels handle n < 2^31 per subset)
  int16_t family;  // Family
  int16_t group;   // unused by kernels (kept for alignment / debugging)
};

struct ResultOut {  // identical layout to cpc_subset_result_t
  double theta, var, loglik, score;
  int64_t n;
  int32_t iters, status;
};

enum Status {
  ST_OK = 0,
  ST_BOUNDARY_NATURAL = 1,
  ST_BOUNDARY_BOX = 2,
  ST_DEGENERATE = 3,
  ST_NONFINITE = 4,
  ST_NOCONV = 5,
  ST_BADVAR = 6
};

// ---------------------------------------------------------------------------
// Order-preserving keys: unsigned comparison of the key equals numeric
// comparison of the value; -0 and +0 map to the same key.
__device__ __forceinline__ uint32_t key_of(float f) {
  uint32_t b = __float_as_uint(f);
  if (f == 0.0f) b = 0u;
  return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
__device__ __forceinline__ uint64_t key_of(double d) {
  uint64_t b = (uint64_t)__double_as_longlong(d);
  if (d == 0.0) b = 0ull;
  return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}

__device__ __forceinline__ uint64_t lanemask_lt() {
  const uint32_t lane = __lane_id();
  return (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
}

// ---------------------------------------------------------------------------
// Compensated (Kahan) summation. For double the compensation is kept too; it
// is cheap and keeps FP64 sums over long subsets at full accuracy.
template <typename T>
struct KSum {
  T s, c;
  __device__ __forceinline__ KSum() : s((T)0), c((T)0) {}
  __device__ __forceinline__ void add(T x) {
    const T y = x - c;
    const T t = s + y;
    c = (t - s) - y;
    s = t;
  }
  __device__ __forceinline__ double value() const { return (double)s - (double)c; }
};

// Per-thread sum of per-row terms, compensated in the row arithmetic type
// (Kahan); the workgroup then combines the per-thread values in FP64.
template <typename T>
using RowSum = KSum<T>;

// ---------------------------------------------------------------------------
// Reductions in a fixed order (results do not depend on timing): wave_sum is
// a butterfly; the workgroup reductions below scan each wave with DPP and
// combine the waves' partials with a DPP row scan.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, WAVE);
  return v;
}
// DPP move of a double (each 32-bit half; lanes without a source read 0.0).
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_f64(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROWS, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROWS, 0xF, false);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double readlane_f64(double v, int lane) {
  return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), lane),
                          __builtin_amdgcn_readlane(__double2loint(v), lane));
}
// Sum over the lanes of a wave, left in the last lane (inclusive scan: row
// shifts right, then each row's last lane carried into the rows after it).
__device__ __forceinline__ double wave_sum_last(double v) {
  v += dpp_f64<0x111, 0xF>(v);
  v += dpp_f64<0x112, 0xF>(v);
  v += dpp_f64<0x114, 0xF>(v);
  v += dpp_f64<0x118, 0xF>(v);
  v += dpp_f64<0x142, 0xA>(v);
  v += dpp_f64<0x143, 0xC>(v);
  return v;
}
// Inclusive sum and inclusive suffix sum within each 16-lane row.
__device__ __forceinline__ double row_incl_sum_f64(double v) {
  v += dpp_f64<0x111, 0xF>(v);
  v += dpp_f64<0x112, 0xF>(v);
  v += dpp_f64<0x114, 0xF>(v);
  v += dpp_f64<0x118, 0xF>(v);
  return v;
}
__device__ __forceinline__ double row_incl_suffix_sum_f64(double v) {
  v += dpp_f64<0x101, 0xF>(v);
  v += dpp_f64<0x102, 0xF>(v);
  v += dpp_f64<0x104, 0xF>(v);
  v += dpp_f64<0x108, 0xF>(v);
  return v;
}
// The waves' totals after wave w (scratch[k] holds wave k's), in every lane:
// lane k < W of each wave reads scratch[k], summed from the right in row 0.
template <int W>
__device__ __forceinline__ double waves_after(const double* scratch, int w) {
  static_assert(W <= 16, "wave totals fit one DPP row");
  const int lane = threadIdx.x & (WAVE - 1);
  const double s = row_incl_suffix_sum_f64(lane < W ? scratch[lane] : 0.0);
  const int wu = __builtin_amdgcn_readfirstlane(w);
  return wu + 1 < W ? readlane_f64(s, wu + 1) : 0.0;
}
// Inclusive suffix sum over the lanes of a wave (lane i: sum over lanes >= i):
// row shifts left within each row, then the totals of the later rows (the
// first lane of each) added in.
__device__ __forceinline__ double wave_incl_suffix_sum(double v) {
  v += dpp_f64<0x101, 0xF>(v);
  v += dpp_f64<0x102, 0xF>(v);
  v += dpp_f64<0x104, 0xF>(v);
  v += dpp_f64<0x108, 0xF>(v);
  const double r1 = readlane_f64(v, 16), r2 = readlane_f64(v, 32), r3 = readlane_f64(v, 48);
  const int lane = threadIdx.x & (WAVE - 1);
  const double r23 = r2 + r3;
  const double after = lane < 16 ? r1 + r23 : (lane < 32 ? r23 : (lane < 48 ? r3 : 0.0));
  return v + after;
}
// Sum of 64-bit integers over the lanes of a wave, left in the last lane
// (exact, so the same value as any other order).
template <int CTRL, int ROWS>
__device__ __forceinline__ long long dpp_i64(long long v) {
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(uint64_t)v, CTRL, ROWS, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)((uint64_t)v >> 32), CTRL, ROWS, 0xF, false);
  return (long long)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}
__device__ __forceinline__ long long wave_sum_ll_last(long long v) {
  v += dpp_i64<0x111, 0xF>(v);
  v += dpp_i64<0x112, 0xF>(v);
  v += dpp_i64<0x114, 0xF>(v);
  v += dpp_i64<0x118, 0xF>(v);
  v += dpp_i64<0x142, 0xA>(v);
  v += dpp_i64<0x143, 0xC>(v);
  return v;
}
__device__ __forceinline__ long long wave_sum_ll(long long v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, WAVE);
  return v;
}

// Sums NV doubles over the workgroup; result valid in thread 0.
// scratch: at least W * NV doubles of LDS. TAIL = false leaves out the
// closing barrier: the caller then synchronises the workgroup before
// scratch is written again.
template <int W, int NV, bool TAIL = true>
__device__ __forceinline__ void block_sum(double (&v)[NV], double* scratch) {
  const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE;
#pragma unroll
  for (int i = 0; i < NV; ++i) v[i] = wave_sum_last(v[i]);
  if (lane == WAVE - 1) {
#pragma unroll
    for (int i = 0; i < NV; ++i) scratch[w * NV + i] = v[i];
  }
  __syncthreads();
  static_assert(W <= 16, "wave partials fit one DPP row");
  if (w == 0) {  // wave 0 sums the W partials (lane k reads wave k's) in row 0
#pragma unroll
    for (int i = 0; i < NV; ++i)
      v[i] = readlane_f64(row_incl_sum_f64(lane < W ? scratch[lane * NV + i] : 0.0), W - 1);
  }
  if (TAIL) __syncthreads();
}

template <int W, bool TAIL = true>
__device__ __forceinline__ long long block_sum_ll(long long v, long long* scratch) {
  const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE;
  v = wave_sum_ll_last(v);
  if (lane == WAVE - 1) scratch[w] = v;
  __syncthreads();
  long long a = 0;
  if (threadIdx.x == 0)
    for (int k = 0; k < W; ++k) a += scratch[k];
  if (TAIL) __syncthreads();
  return a;
}

// Exclusive suffix sum over the workgroup: returns sum_{t' > t} v_t'.
// scratch: W doubles.
template <int W>
__device__ __forceinline__ double block_excl_suffix(double v, double* scratch) {
  const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE;
  const double incl = wave_incl_suffix_sum(v);
  if (lane == 0) scratch[w] = incl;
  __syncthreads();
  const double carry = waves_after<W>(scratch, w);
  __syncthreads();
  return incl + carry - v;
}

// Two exclusive suffix sums at once (the same arithmetic as block_excl_suffix
// on each value; one pair of workgroup barriers for both). scratch: 2W doubles.
template <int W>
__device__ __forceinline__ void block_excl_suffix2(double va, double vb, double* scratch, double& ea, double& eb) {
  const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE;
  const double ia = wave_incl_suffix_sum(va), ib = wave_incl_suffix_sum(vb);
  if (lane == 0) {
    scratch[w] = ia;
    scratch[W + w] = ib;
  }
  __syncthreads();
  const double ca = waves_after<W>(scratch, w), cb = waves_after<W>(scratch + W, w);
  __syncthreads();
  ea = ia + ca - va;
  eb = ib + cb - vb;
}

}  // namespace cpc
