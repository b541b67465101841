// probe_valu.hip — issue-rate probe of FP32 FMA and of the FP32
// transcendental instructions (include/cpc_probe.h). Every lane runs 8
// independent chains of the same instruction so that issue, not latency,
// bounds the loop; the chains' values are written out so that nothing is
// dropped by the compiler.
#include <hip/hip_runtime.h>

#include "cpc_probe.h"

namespace {

constexpr int PT = 256;     // threads per workgroup
constexpr int CHAINS = 8;   // independent chains per lane

template <int OP>
__global__ void __launch_bounds__(PT) k_probe(float* out, int iters, float seed) {
  float a[CHAINS];
#pragma unroll
  for (int k = 0; k < CHAINS; ++k) a[k] = seed + 1e-3f * (float)(threadIdx.x & 63) + 0.125f * (float)k;
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int k = 0; k < CHAINS; ++k) {
      if constexpr (OP == CPC_PROBE_FMA) a[k] = __builtin_fmaf(a[k], 0.99951171875f, 0.000244140625f);
      if constexpr (OP == CPC_PROBE_EXP2) a[k] = __builtin_amdgcn_exp2f(-a[k]);
      if constexpr (OP == CPC_PROBE_LOG2) a[k] = __builtin_amdgcn_logf(a[k]);
      if constexpr (OP == CPC_PROBE_RCP) a[k] = __builtin_amdgcn_rcpf(a[k]);
      if constexpr (OP == CPC_PROBE_SQRT) a[k] = __builtin_amdgcn_sqrtf(a[k]);
    }
  }
  float s = 0.0f;
#pragma unroll
  for (int k = 0; k < CHAINS; ++k) s += a[k];
  out[(size_t)blockIdx.x * PT + threadIdx.x] = s;
}

template <int OP>
hipError_t launch(float* out, int blocks, int iters, hipStream_t s) {
  hipLaunchKernelGGL((k_probe<OP>), dim3(blocks), dim3(PT), 0, s, out, iters, 0.75f);
  return hipGetLastError();
}

hipError_t launch_op(int op, float* out, int blocks, int iters, hipStream_t s) {
  switch (op) {
    case CPC_PROBE_FMA: return launch<CPC_PROBE_FMA>(out, blocks, iters, s);
    case CPC_PROBE_EXP2: return launch<CPC_PROBE_EXP2>(out, blocks, iters, s);
    case CPC_PROBE_LOG2: return launch<CPC_PROBE_LOG2>(out, blocks, iters, s);
    case CPC_PROBE_RCP: return launch<CPC_PROBE_RCP>(out, blocks, iters, s);
    default: return launch<CPC_PROBE_SQRT>(out, blocks, iters, s);
  }
}

}  // namespace

extern "C" int cpc_probe_valu(int device, int op, int iters, double* lane_ops_per_s, float* ms) {
  if (op < CPC_PROBE_FMA || op > CPC_PROBE_SQRT || iters < 1 || iters > (1 << 20) || !lane_ops_per_s || !ms)
    return -1;
  if (hipSetDevice(device) != hipSuccess) return -2;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) return -2;
  const int blocks = prop.multiProcessorCount * 32;  // several waves of workgroups: ramp-up and tail stay small
  float* out = nullptr;
  hipStream_t s = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int rc = -2;
  if (hipMalloc((void**)&out, sizeof(float) * (size_t)blocks * PT) != hipSuccess) return -2;
  if (hipStreamCreate(&s) == hipSuccess && hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess &&
      launch_op(op, out, blocks, iters, s) == hipSuccess && hipEventRecord(e0, s) == hipSuccess &&
      launch_op(op, out, blocks, iters, s) == hipSuccess && hipEventRecord(e1, s) == hipSuccess &&
      hipEventSynchronize(e1) == hipSuccess && hipEventElapsedTime(ms, e0, e1) == hipSuccess && *ms > 0.0f) {
    *lane_ops_per_s = (double)blocks * PT * CHAINS * (double)iters / (*ms * 1e-3);
    rc = 0;
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (s) {
    (void)hipStreamSynchronize(s);
    (void)hipStreamDestroy(s);
  }
  (void)hipFree(out);
  return rc;
}
