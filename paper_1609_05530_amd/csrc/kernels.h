// kernels.h — parameter blocks and launchers of the libcpc kernels
// (implemented in k_*.hip), shared with the host code.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "cpc_device.h"

namespace cpc {

enum Mode { MODE_FIT = 0, MODE_RANK = 1, MODE_VARIANCE = 2 };

// Per-subset state handed from the rank kernel to the fit kernel to the
// variance kernel (workspace, one per subset).
struct SubState {
  double theta;
  double Sp, Sm;  // Gaussian sufficient statistics
  int32_t status, iters;
};

// Size classes of the workgroup-per-subset kernels: (threads, items per
// thread); a class holds subsets of up to threads * items rows.
constexpr int kNumClasses = 4;
constexpr int kClassThreads[kNumClasses] = {64, 256, 512, 1024};
constexpr int kClassItems[kNumClasses] = {8, 8, 16, 16};
constexpr int kResidentMaxRows = 1024 * 16;

// Per-row arrays of the workgroup path (u16: subsets hold < 32768 rows).
struct RowArrays {
  uint16_t *R1, *R2;  // doubled ranks
  uint16_t *E1, *E2;  // sorted positions
  uint16_t *L1, *L2;  // start of the row's tie group in sorted order
  void* S;            // per-row score scratch (row arithmetic type)
};

struct RankParams {
  const void* x;  // float (kw 1), double (kw 2), or uint32 ranks (int_keys)
  const void* y;
  const SubDesc* subs;
  const int32_t* order;
  int32_t mode, ties, int_keys, pad;
  int64_t n_min;
  RowArrays rows;
  uint32_t* R1out;  // MODE_RANK
  uint32_t* R2out;
  SubState* state;
};

struct FitParams {
  const SubDesc* subs;
  const int32_t* order;
  RowArrays rows;
  SubState* state;
  int32_t max_iter, pad;
  double tol;
};

struct VarParams {
  const SubDesc* subs;
  const int32_t* order;
  RowArrays rows;
  const SubState* state;
  int32_t mode, var_method;
  const double* theta_in;  // MODE_VARIANCE
  double* var_out;         // MODE_VARIANCE
  ResultOut* out;          // MODE_FIT
};

hipError_t launch_rank_wg(int cls, int kw, const RankParams& p, int grid, hipStream_t s);
hipError_t launch_fit_wg(int cls, int fam, int fp64, const FitParams& p, int grid, hipStream_t s);
hipError_t launch_var_wg(int cls, int fam, int fp64, const VarParams& p, int grid, hipStream_t s);

// Adjoint of eq. (13): per-subset sums of l, dl/dtheta, d2l/dtheta2.
hipError_t launch_eval_wg(const uint32_t* R1, const uint32_t* R2, const SubDesc* subs, int64_t K, int fam,
                          int fp64, const double* theta, double* out, hipStream_t s);

// eq. (15) / (16) per group.
struct CombinedOut {  // identical layout to cpc_combined_t
  double theta, var_combined;
  int64_t n_used, n_excluded;
  int32_t status, pad;
};
hipError_t launch_combine(const ResultOut* sub, const int64_t* group_offsets, int64_t G,
                          CombinedOut* comb, hipStream_t s);

}  // namespace cpc
