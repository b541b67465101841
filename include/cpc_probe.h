/* cpc_probe.h — issue-rate probe for the VALU instructions the per-row
 * arithmetic of the fit and variance kernels is built from. Not part of the
 * estimation API (include/cpc.h): it measures, on one device, how many lane
 * operations per second the hardware sustains for FP32 FMA and for the
 * FP32 transcendental instructions (exp2, log2, reciprocal, square root),
 * so that the VALU roofline of those kernels can use measured rates beside
 * the published peak. Library: libcpc_probe.so. */
#ifndef CPC_PROBE_H
#define CPC_PROBE_H

#ifdef __cplusplus
extern "C" {
#endif

enum cpc_probe_op {
  CPC_PROBE_FMA = 0,  /* v_fma_f32 */
  CPC_PROBE_EXP2 = 1, /* v_exp_f32 */
  CPC_PROBE_LOG2 = 2, /* v_log_f32 */
  CPC_PROBE_RCP = 3,  /* v_rcp_f32 */
  CPC_PROBE_SQRT = 4  /* v_sqrt_f32 */
};

/* Runs `iters` rounds of 8 independent dependent chains of operation `op`
 * in every lane of a grid of 32 workgroups of 256 lanes per compute unit,
 * timed with HIP events on a stream of its own after one untimed run. On success stores the kernel time (ms) and the lane
 * operations per second and returns 0. Returns -1 for an unknown op or
 * iters outside [1, 1 << 20], -2 for a HIP error (device selection,
 * allocation, launch). Allocates and frees its own device memory; makes the
 * device current on the calling thread. */
int cpc_probe_valu(int device, int op, int iters, double* lane_ops_per_s, float* ms);

#ifdef __cplusplus
}
#endif

#endif /* CPC_PROBE_H */
