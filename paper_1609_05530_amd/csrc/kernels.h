// kernels.h — parameter blocks and launchers of the libcpc kernels
// (implemented in k_*.hip), shared with the host code.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "cpc_device.h"
#include "rank_shapes.h"
#include "solver.h"

namespace cpc {

enum Mode { MODE_FIT = 0, MODE_RANK = 1, MODE_VARIANCE = 2 };

// Per-subset state handed from the rank kernel to the fit kernel to the
// variance kernel (workspace, one per subset).
struct SubState {
  double theta;
  double Sp, Sm;  // Gaussian sufficient statistics
  int32_t status, iters;
  // bit m (margin x: 0, y: 1): every row's sorted position E equals its
  // tie-group start (no ties, or ties in row order), its doubled rank is
  // 2E + 2, and only the positions were stored (set by the rank kernel)
  int32_t eqmask, pad;
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
  void* G;            // per-row d2l/dtheta dv scratch (row arithmetic type)
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

static_assert(kNumClasses == kRankClasses, "one row of rank shape choices per size class");
hipError_t launch_rank_shape(int shape, int kw, const RankParams& p, int grid, hipStream_t s);
hipError_t launch_fit_wg(int cls, int fam, int fp64, const FitParams& p, int grid, hipStream_t s);
hipError_t launch_var_wg(int cls, int fam, int fp64, const VarParams& p, int grid, hipStream_t s);

// Streaming path for subsets of more than kResidentMaxRows rows: tiles of
// 4096 rows over all such subsets; per-row arrays at compact indices
// (roff + row within the subset).
struct BigSeg {
  int64_t begin;   // first row in x / y
  int64_t n;       // rows
  int64_t roff;    // first compact index
  int64_t tile0;   // first tile
  int32_t ntiles;
  int32_t sid;     // subset id (result index)
  int32_t family;
  int32_t pad;
};
struct BigTile {
  int32_t seg;
  int32_t count;
  int64_t start;  // first row of the tile within its subset
};
struct BigParams {
  const BigSeg* segs;
  const BigTile* tiles;
  int32_t nsegs;
  int32_t pad;
  int64_t ntiles;
  int64_t n_min;
  int32_t* flags;  // per subset: bit 0 non-finite data, bit 1 a margin with one value
  double* gsum;    // per subset: Gaussian S+, S-
  // tile launch slots: block b runs tile xorder[b] (-1: idle). Blocks go to
  // the 8 XCDs in turn, so slot order puts a subset's tiles on one XCD (its
  // L2 then holds the subset's arrays); a subset larger than an XCD's share
  // is spread over all eight.
  const int64_t* xorder;
  int64_t nslots;
};
struct BigBuffers {
  uint32_t *ka, *kb, *kc, *kd, *va, *vb;  // sort keys / payloads (ping-pong)
  uint32_t *R1, *R2, *E1, *E2, *L1, *L2;  // doubled ranks, sorted positions, tie-group starts
  void *LX, *LY, *A1, *A2, *S;            // Gumbel logs, suffix-sum arrays, scores (row arithmetic type)
  uint32_t* hist;                         // 256 per tile
  double* part;                           // 5 per tile
  double* tsum;                           // 2 per tile
  NewtonState* st;                        // per subset
  int* pending;                           // subsets still iterating
};
// The sorted order of x on the streaming path: entry roff + p of a subset
// holds the row (within the subset) at its sorted position p and that row's
// order-preserving key (low and high words; the high words only for FP64).
struct BigSorted {
  const uint32_t* rows;
  const uint32_t* klo;
  const uint32_t* khi;
};
// margins = 1 ranks x alone (R2out and the staged y arrays are left as they
// are). sorted != nullptr: x is only sorted (stably, so ties keep row
// order), no ranks are formed, and *sorted receives the sorted order.
hipError_t big_rank(const BigParams& P, const BigBuffers& B, const void* x, const void* y, int dtype_kw,
                    int int_keys, int ties, uint32_t* R1out, uint32_t* R2out, hipStream_t s, int margins = 2,
                    BigSorted* sorted = nullptr);
hipError_t big_solve(const BigParams& P, const BigBuffers& B, double tol, int max_iter, int fp64, int* pending_host,
                     hipStream_t s);
hipError_t big_variance(const BigParams& P, const BigBuffers& B, int fp64, const double* theta_in, int var_method,
                        int mode, double* var_out, ResultOut* out, hipStream_t s);
constexpr int kBigTile = 4096;
// Largest subset whose sorted-to-row permutation is staged through LDS tile
// by tile: each tile reads its whole subset's sorted row indices, so the work
// grows as rows^2 / kBigTile; larger subsets scatter to row order directly.
constexpr int64_t kBigChunkMaxRows = 1 << 17;

// Adjoint of eq. (13): per-subset sums of l, dl/dtheta, d2l/dtheta2.
hipError_t launch_eval_wg(const uint32_t* R1, const uint32_t* R2, const SubDesc* subs, int64_t K, int fam,
                          int fp64, int64_t n_max, const double* theta, double* out, hipStream_t s);

// eq. (15) / (16) per group.
struct CombinedOut {  // identical layout to cpc_combined_t
  double theta, var_combined;
  int64_t n_used, n_excluded;
  int32_t status, pad;
};
hipError_t launch_combine(const ResultOut* sub, const int64_t* group_offsets, int64_t G,
                          CombinedOut* comb, hipStream_t s);

// Simulation inputs (Sec. 2.5): rows row0 .. row0 + n - 1 of the family's
// copula with N(0, 1) margins, counter-based (k_sample.hip).
hipError_t launch_sample(int fam, double theta, uint64_t seed, int64_t row0, int64_t n, int f32, void* x, void* y,
                         hipStream_t s);

// Evaluation metrics of Sec. 2.6 (k_study.hip): density distances of
// eq. (19)-(20) for P parameter pairs (part: 4 * P * panels doubles), and
// the replicate summary of eq. (17), (18), bias and MSE.
hipError_t launch_density_distance(int fam, int64_t P, const double* theta_a, const double* theta_b, double L,
                                   int panels, double* part, double* out, hipStream_t s);
hipError_t launch_replicate_summary(int64_t S, const CombinedOut* comb, const CombinedOut* full, double* out,
                                    hipStream_t s);

// Partitioning schemes of each replicate into M subsets (k_partition.hip):
// rows of replicate r (rep[r] .. rep[r + 1] - 1) move to xo, yo by their
// x-order position R1 / 2 - 1 (doubled ranks, ties by row order).
enum { PART_CONTIGUOUS = 0, PART_BLOCKS = 1, PART_STRIDED = 2 };
// skip_big: rows of replicates above kResidentMaxRows are left to
// launch_partition_gather.
hipError_t launch_partition(int f32, const void* x, const void* y, const uint32_t* R1, const int64_t* rep,
                            int64_t R, int64_t n, int64_t M, int scheme, int skip_big, void* xo, void* yo,
                            hipStream_t s);
// The x-order schemes for the replicates of the streaming path, from their
// sorted order (big_rank with sorted): output row o of a replicate takes
// the row at the sorted position its scheme assigns to o.
hipError_t launch_partition_gather(int f32, const BigParams& P, const BigSorted& so, const void* x, const void* y,
                                   int64_t M, int scheme, void* xo, void* yo, hipStream_t s);
// Strided from blocks order for the replicates of the streaming path: row q
// of subset m, at position q M + m of the blocks-order rows tx, ty, goes to
// m a + min(m, c) + q of xo, yo (N = a M + c); max_tiles: the most 32 x 32
// tiles of (q, m) any of those replicates has.
hipError_t launch_partition_transpose(int f32, const BigParams& P, const void* tx, const void* ty, int64_t M,
                                      int64_t max_tiles, void* xo, void* yo, hipStream_t s);

// Spearman-inversion estimates per subset from doubled ranks (k_moment.hip);
// H1, H2: 2 (n + K) int64 each.
// subsets base .. base + K - 1 of `subs`, results to out[base ..].
hipError_t launch_spearman(int fam, const uint32_t* R1, const uint32_t* R2, const SubDesc* subs, int64_t base,
                           int64_t K, int64_t n_min, int64_t n_max, long long* H1, long long* H2, ResultOut* out,
                           hipStream_t s);
// The k-dimensional Gaussian copula of eq. (7) per subset (k_gaussk.hip),
// 2 <= k <= 8: R holds k columns of n_total doubled ranks; Z (8 k B per
// row), X (8 gaussk_ldx(k) B per row) and B ((2 n + 2) k doubles per subset
// from 2 (begin + m) k) are scratch; out is parameter-major (q K + m).
int gaussk_ldx(int k);
hipError_t launch_gaussk(const uint32_t* R, int64_t n_total, int k, const SubDesc* subs, int64_t K, int64_t n_min,
                         double* Z, double* X, double* B, ResultOut* out, hipStream_t s);
// The inversion of Kendall's tau per subset (k_moment.hip): subsets of at
// most 2^20 rows, whose rows own W0, W1 (8 B) and C (4 B) at their begin.
hipError_t launch_kendall(int fam, const uint32_t* R1, const uint32_t* R2, const SubDesc* subs, int64_t base,
                          int64_t K, int64_t n_min, unsigned long long* W0, unsigned long long* W1, int* C,
                          int* flag,
                          ResultOut* out, hipStream_t s);

}  // namespace cpc
