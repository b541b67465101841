/*
 * cpc.h — C ABI of libcpc: partition-and-combine maximum-pseudo-likelihood
 * (MPL) copula estimation on AMD Instinct MI355X (gfx950).
 *
 * Method: Wei, Kim & Conlon, "Parallel Computing for Copula Parameter
 * Estimation with Big Data: A Simulation Study" (arXiv:1609.05530).
 *   - eq. (14), Sec. 2.4: the N x 2 sample is split by rows into M disjoint
 *     subsets. Here subset m is rows [offsets[m], offsets[m+1]).
 *   - Sec. 2.3, eq. (12): within each subset each margin is replaced by its
 *     normalised ranks u = r / (n_m + 1) (n_m = subset size).
 *   - eq. (13): the pseudo log-likelihood sum_i log c(u_i1, u_i2; theta) is
 *     maximised numerically for the Gaussian (eq. 8), Frank (eq. 10) or
 *     Gumbel (eq. 11) copula, with c from eq. (5).
 *   - Sec. 2.3: the asymptotic variance of each subset estimate after
 *     Genest, Ghoudi & Rivest (1995).
 *   - eq. (15) / (16): subset estimates are combined with weights
 *     w_m = 1 / sigma_m^2, per group of subsets (one group per simulation
 *     replicate in a batch).
 *
 * Conventions for every entry point:
 *   - Data x, y are device pointers to n values each (structure of arrays),
 *     FP64 or FP32 as given by cpc_dtype_t. The library only reads them.
 *   - offsets / group_offsets / family tables are HOST arrays; they are
 *     copied into the workspace during the call and may be reused on return.
 *   - workspace is a caller-owned DEVICE buffer of at least the size reported
 *     by cpc_workspace_bytes_for() for the call's partition (or the upper
 *     bound cpc_workspace_bytes()); the library allocates no device memory
 *     in any call except cpc_create().
 *   - All outputs are DEVICE buffers owned by the caller. Work is enqueued on
 *     `stream` (a hipStream_t passed as void*; NULL = default stream) and is
 *     complete once the stream is synchronised.
 *   - Return value 0 = success; a negative CPC_E_* code on misuse detected on
 *     the host (nothing is enqueued then). cpc_last_error() gives a
 *     thread-local description of the last failure.
 *   - Data-dependent trouble is never an error: it is reported per subset in
 *     cpc_subset_result_t.status (CPC_ST_*).
 *   - A handle serves one call at a time (not re-entrant).
 */
#ifndef CPC_H
#define CPC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CPC_VERSION_MAJOR 0
#define CPC_VERSION_MINOR 1

/* Copula families (Sec. 2.2): eq. (8), eq. (10), eq. (11). */
typedef enum { CPC_GAUSSIAN = 0, CPC_FRANK = 1, CPC_GUMBEL = 2 } cpc_family_t;

/* Storage type of x and y. */
typedef enum { CPC_F64 = 0, CPC_F32 = 1 } cpc_dtype_t;

/* Per-row arithmetic: plain FP64, or FP32 rows with compensated FP32 sums
 * (per-subset totals, the Newton update and the combine stay FP64; rows near
 * the family boundaries switch to FP64). */
typedef enum { CPC_PREC_FP64 = 0, CPC_PREC_FP32C = 1 } cpc_prec_t;

/* Tie rule for eq. (12) (the paper assumes continuous data). AVERAGE gives
 * tied values their mean rank; FIRST breaks ties by row order. */
typedef enum { CPC_TIES_AVERAGE = 0, CPC_TIES_FIRST = 1 } cpc_ties_t;

/* Variance of a subset estimate: GGR sandwich (Sec. 2.3) or the inverse of
 * the observed score variance (ignores the rank effect; for comparison). */
typedef enum { CPC_VAR_GGR = 0, CPC_VAR_INVINFO = 1 } cpc_var_t;

/* Per-subset status. Only OK and BOUNDARY_NATURAL enter the combination. */
enum {
  CPC_ST_OK = 0,
  CPC_ST_BOUNDARY_NATURAL = 1, /* Gumbel estimate at theta = 1 (independence) */
  CPC_ST_BOUNDARY_BOX = 2,     /* estimate at an edge of the search box */
  CPC_ST_DEGENERATE = 3,       /* n_m < n_min, or a margin with a single value */
  CPC_ST_NONFINITE = 4,        /* NaN or +-Inf in the subset's x or y */
  CPC_ST_NOCONV = 5,           /* max_iter Newton passes without convergence */
  CPC_ST_BADVAR = 6            /* variance not positive and finite */
};

/* Error codes (host-side misuse). */
enum {
  CPC_SUCCESS = 0,
  CPC_E_NULL = -1,        /* a required pointer is NULL */
  CPC_E_SIZE = -2,        /* n < 0, K < 1, G < 1, or a count out of range */
  CPC_E_OFFSETS = -3,     /* offsets not non-decreasing from 0 to n, or groups not spanning 0..K */
  CPC_E_ENUM = -4,        /* unknown family / dtype / precision / ties / variance value */
  CPC_E_WORKSPACE = -5,   /* workspace NULL or smaller than required */
  CPC_E_HIP = -6,         /* a HIP runtime call failed */
  CPC_E_HANDLE = -7,      /* invalid handle */
  CPC_E_OPTIONS = -8,     /* an option out of range (max_iter < 1, tol <= 0, ...) */
  CPC_E_UNSUPPORTED = -9  /* a size this build cannot handle (e.g. n >= 2^31 rows in one subset) */
};

typedef struct {
  int32_t prec;      /* cpc_prec_t, default CPC_PREC_FP64 */
  int32_t ties;      /* cpc_ties_t, default CPC_TIES_AVERAGE */
  int32_t var;       /* cpc_var_t, default CPC_VAR_GGR */
  int32_t max_iter;  /* Newton passes per subset, default 60 */
  double tol;        /* stop when |dtheta| <= tol (1 + |theta|); 0 = default (1e-12 FP64, 1e-9 FP32C) */
  int64_t n_min;     /* subsets with fewer rows are DEGENERATE; default (and minimum) 2 */
  int32_t schedule;  /* -1 = rank-kernel launch shapes chosen by the autotuner (default); 0 = built-in shapes;
                        1 + s (0 <= s < 16) forces rank-kernel shape s on FP32 data for the size class of its
                        capacity (0..13: radix-sort variants; 14: the one-wave merge sort and 15 the
                        one-wave sort truncated to 24 leading key bits, for up to 512 rows), the built-in
                        shapes elsewhere */
  int32_t flags;     /* bit 0: capture/replay the launch sequence as a hipGraph */
} cpc_options_t;

#define CPC_FLAG_GRAPH 1
#define CPC_FLAG_PHASE_TIMES 2 /* record hipEvents between the phases of a fit */

/* 48 bytes, natural alignment. */
typedef struct {
  double theta;   /* MPL estimate theta_m (NaN if DEGENERATE / NONFINITE) */
  double var;     /* sigma_m^2, the estimated variance of theta_m (NaN unless OK / BOUNDARY_NATURAL / BADVAR) */
  double loglik;  /* eq. (13) at theta_m */
  double score;   /* d/dtheta of eq. (13) at theta_m */
  int64_t n;      /* subset size n_m */
  int32_t iters;  /* Newton passes over the rows */
  int32_t status; /* CPC_ST_* */
} cpc_subset_result_t;

/* 40 bytes. One per group. */
typedef struct {
  double theta;        /* eq. (15): sum w_m theta_m / sum w_m over usable subsets (NaN if none) */
  double var_combined; /* 1 / sum w_m */
  int64_t n_used;      /* subsets that entered the combination */
  int64_t n_excluded;  /* subsets left out (status other than OK / BOUNDARY_NATURAL) */
  int32_t status;      /* 0 = ok, 1 = no usable subset in the group */
  int32_t pad;
} cpc_combined_t;

typedef struct cpc_context* cpc_handle_t;

/* Create a handle bound to HIP device `device` (makes it current). */
int cpc_create(int device, cpc_handle_t* out);
int cpc_destroy(cpc_handle_t h);

/* Fill `opt` with the defaults listed above. */
void cpc_default_options(cpc_options_t* opt);

/* Workspace bytes that suffice for any call with at most n rows, K subsets
 * and G groups of the given storage type and options (an upper bound: it
 * assumes every row may belong to a subset of more than 16384 rows). */
size_t cpc_workspace_bytes(int64_t n, int64_t K, int64_t G, int32_t dtype, const cpc_options_t* opt);

/* Workspace bytes a call needs for exactly this partition (eq. 14): offsets
 * is the host array of K+1 subset bounds (offsets[K] = n), G the number of
 * groups (1 for cpc_fit / cpc_rank / cpc_eval / cpc_variance). Per row
 * about 28 bytes, plus 88 bytes per row of the subsets of more than 16384
 * rows (the streaming path's sort and scan arrays). Returns 0 if offsets is
 * NULL or not a partition. */
size_t cpc_workspace_bytes_for(const int64_t* offsets, int64_t K, int64_t G, int32_t dtype,
                               const cpc_options_t* opt);

/* Fit every subset of one family and combine them (eq. 12-15).
 *   x, y     : device, n values each, type `dtype`
 *   offsets  : host, K+1 values, offsets[0] = 0, non-decreasing, offsets[K] = n
 *   out      : device, K results;  comb : device, 1 combined result
 */
int cpc_fit(cpc_handle_t h, const void* x, const void* y, int32_t dtype, int64_t n,
            const int64_t* offsets, int64_t K, int32_t family, const cpc_options_t* opt,
            void* workspace, size_t ws_bytes, cpc_subset_result_t* out, cpc_combined_t* comb,
            void* stream);

/* Batched form (eq. 16): G groups of consecutive subsets, group g being
 * subsets [group_offsets[g], group_offsets[g+1]) fitted with family
 * family_per_group[g] and combined on their own.
 *   group_offsets    : host, G+1 values, 0 .. K non-decreasing
 *   family_per_group : host, G values (cpc_family_t)
 *   comb             : device, G combined results
 */
int cpc_fit_batched(cpc_handle_t h, const void* x, const void* y, int32_t dtype, int64_t n,
                    const int64_t* offsets, int64_t K, const int64_t* group_offsets, int64_t G,
                    const int32_t* family_per_group, const cpc_options_t* opt, void* workspace,
                    size_t ws_bytes, cpc_subset_result_t* out, cpc_combined_t* comb, void* stream);

/* Allocation-free form of cpc_fit_batched, for callers that cannot allocate
 * device memory (code under stream capture, tight serving loops, harnesses
 * that forbid hipMalloc): the same arguments without the workspace, which is
 * a static device array of the library (64 MiB per device, held from the
 * library's first use of that device until the process ends). The call
 * allocates nothing, never synchronises (no autotuning trials: a launch
 * shape not yet chosen by an earlier cpc_fit / cpc_fit_batched on the handle
 * takes the built-in one; the streaming path enqueues its whole Newton pass
 * budget) and rejects CPC_FLAG_GRAPH (CPC_E_OPTIONS).
 *   - A partition that needs more than 64 MiB of workspace
 *     (cpc_workspace_bytes_for: about 28 bytes per row, + 88 per row of
 *     subsets above 16384 rows, so ~2.3 M rows without such subsets) is
 *     rejected with CPC_E_WORKSPACE before anything is enqueued.
 *   - Every call on a device shares that device's array, which keeps the last
 *     call's contents (nothing in it needs to start at zero). Calls that
 *     overlap on one device (other streams, other threads, other handles)
 *     race on it: serialise them.
 *   - CPC_E_HIP if the array's device address could not be looked up.
 */
int cpc_fit_batched_noalloc(cpc_handle_t h, const void* x, const void* y, int32_t dtype, int64_t n,
                            const int64_t* offsets, int64_t K, const int64_t* group_offsets, int64_t G,
                            const int32_t* family_per_group, const cpc_options_t* opt,
                            cpc_subset_result_t* out, cpc_combined_t* comb, void* stream);

/* Ranks of eq. (12) within each subset, as doubled integers R = 2 r (so
 * average ties stay integral): u = R / (2 (n_m + 1)).
 *   R1, R2 : device, n values each, row order (same indexing as x, y).
 */
int cpc_rank(cpc_handle_t h, const void* x, const void* y, int32_t dtype, int64_t n,
             const int64_t* offsets, int64_t K, const cpc_options_t* opt, void* workspace,
             size_t ws_bytes, uint32_t* R1, uint32_t* R2, void* stream);

/* Adjoint of eq. (13): for each subset m at theta[m] (device, K doubles),
 * out[3m + 0..2] = sum_i l, sum_i dl/dtheta, sum_i d2l/dtheta2 (device, 3K
 * doubles), from doubled ranks R1, R2 (device, n each) as made by cpc_rank.
 * theta outside the family's domain gives NaN sums for that subset. */
int cpc_eval(cpc_handle_t h, const uint32_t* R1, const uint32_t* R2, int64_t n,
             const int64_t* offsets, int64_t K, int32_t family, const double* theta,
             const cpc_options_t* opt, void* workspace, size_t ws_bytes, double* out, void* stream);

/* Asymptotic variance of Sec. 2.3 for each subset at theta[m] (device, K):
 * var[m] (device, K doubles), from doubled ranks R1, R2 (device, n each). */
int cpc_variance(cpc_handle_t h, const uint32_t* R1, const uint32_t* R2, int64_t n,
                 const int64_t* offsets, int64_t K, int32_t family, const double* theta,
                 const cpc_options_t* opt, void* workspace, size_t ws_bytes, double* var,
                 void* stream);

/* Simulation input of Sec. 2.5 drawn on the device: rows row0 .. row0+n-1
 * of a stream of pairs (x, y) with N(0,1) margins whose copula is `family`
 * at theta (eq. 8, 10, 11), written to the device arrays x, y (n values of
 * type dtype: FP64, or the FP64 draw rounded to FP32).
 *   Generator: Philox4x32-10 (Salmon et al., SC 2011) at counter (row low
 *   word, row high word, block, 0) with key (seed low word, seed high word);
 *   each block gives two uniforms u = (k + 1/2) 2^-52 from 52 of its bits.
 *   Row r of a stream depends only on (family, theta, seed, r), so a
 *   replicate study draws replicate s as rows [s N, (s + 1) N).
 *   Gaussian: Cholesky factor of the correlation matrix applied to two
 *   N(0,1) draws; Frank: conditional inversion of dC/du in closed form;
 *   Gumbel: Marshall-Olkin with a positive stable frailty drawn by Kanter's
 *   representation. CPC_E_OPTIONS if theta is outside the family's range
 *   (Gaussian |rho| < 1, Frank finite, Gumbel theta >= 1). */
int cpc_sample(cpc_handle_t h, int32_t family, double theta, uint64_t seed, int64_t row0, int64_t n,
               int32_t dtype, void* x, void* y, void* stream);

/* Distances of Sec. 2.6 between the densities c_a = c(.; theta_a[p]) and
 * c_b = c(.; theta_b[p]) of one family, for p = 0 .. P-1 (device arrays):
 *   out[4p + 0] = int |c_a - c_b|,  out[4p + 1] = int c_a,
 *   out[4p + 2] = int (c_a - c_b)^2, out[4p + 3] = int c_a^2
 * over the unit square, so that eq. (19) is out[4p] / out[4p + 1] and
 * eq. (20) is sqrt(out[4p + 2] / out[4p + 3]). Integrated in normal-score
 * coordinates u = Phi(s), v = Phi(t) over |s|, |t| <= box with `panels`
 * equal panels per axis and the 8-point Gauss-Legendre rule on each, the
 * inner integral of |c_a - c_b| split where the densities cross. box = 20
 * holds the squared Gaussian density to 1e-9 up to |rho| = 0.9 (its L2 mass
 * reaches far along the diagonal). The Gumbel density is not square
 * integrable at (1, 1): its out[4p + 2], out[4p + 3] grow with box and
 * eq. (20) is the ratio over the box; box = 8.3 (u, v within 1e-16 of the
 * square's edges) keeps its band along the diagonal resolved by 256 panels
 * up to theta = 5. workspace: device, at least
 * 32 * P * panels bytes. out: device, 4P doubles. */
int cpc_density_distance(cpc_handle_t h, int32_t family, int64_t P, const double* theta_a,
                         const double* theta_b, double box, int32_t panels, void* workspace,
                         size_t ws_bytes, double* out, void* stream);

/* Sec. 2.5-2.6 over S replicates: combined[s] from the subsets of replicate
 * s (eq. 16, a cpc_fit_batched group) and full[s] from its full data (a
 * group of one subset), device arrays. Replicates whose two results both
 * have status 0 enter: out[0] = eq. (17), out[1] = eq. (18), out[2] = the
 * estimated bias out[0] - out[1], out[3] = the estimated MSE (mean squared
 * difference of the two estimates), out[4] = replicates used (device, 5
 * doubles). */
int cpc_replicate_summary(cpc_handle_t h, int64_t S, const cpc_combined_t* combined,
                          const cpc_combined_t* full, double* out, void* stream);

/* Partitioning schemes: how the rows of each replicate are split into its M
 * subsets (the row partition of eq. 14). Sec. 4 leaves the effect of the
 * partitioning method on the estimate to future work; these schemes are the
 * inputs of that study. p(i) is row i's position, from 0, in its
 * replicate's order of x with ties (-0 equal to +0) broken by row order. */
typedef enum {
  CPC_PART_CONTIGUOUS = 0, /* subset m = stored rows floor(m N/M) .. floor((m+1) N/M) - 1 (Sec. 2.5's split) */
  CPC_PART_BLOCKS = 1,     /* subset m = positions floor(m N/M) .. floor((m+1) N/M) - 1 of the x-order */
  CPC_PART_STRIDED = 2     /* subset m = positions p with p mod M = m (ceil((N - m) / M) rows) */
} cpc_partition_t;

/* Workspace bytes of cpc_partition for these replicates (rep_offsets: host,
 * R+1 values); 0 if rep_offsets is not a partition of 0 .. rep_offsets[R] or
 * an argument is out of range. About 36 bytes per row for the x-order
 * schemes (doubled ranks of both margins and the rank kernels' own
 * workspace, + 88 per row of replicates above 16384 rows), 2 values per
 * row more for CPC_PART_STRIDED (its rows in blocks order before their
 * transpose), plus the replicate table of 8 (R + 1) bytes (all that
 * CPC_PART_CONTIGUOUS needs). */
size_t cpc_partition_workspace_bytes(const int64_t* rep_offsets, int64_t R, int32_t dtype, int32_t scheme);

/* Splits every replicate r (rows rep_offsets[r] .. rep_offsets[r+1] - 1, N_r
 * rows; host array of R+1 values) into M subsets by `scheme` and writes the
 * rows, subset after subset, to x_out, y_out (device, n values each of type
 * dtype; buffers of their own, not overlapping x or y): subset (r, m) is
 * rows offsets_out[r M + m] .. offsets_out[r M + m + 1] - 1 (offsets_out:
 * host, R M + 1 values, written before the call returns), inside the
 * replicate's own row range. Inside a subset the rows keep their stored order
 * (CPC_PART_CONTIGUOUS) or follow the x-order (the other schemes); more
 * subsets than rows leave some empty. The x-order comes from a stable sort
 * of x (ties by row order): replicates of more than 16384 rows are sorted
 * on the streaming path and their rows gathered in order, smaller ones are
 * ranked by the workgroup rank kernels of eq. (12), which take y along. x must be finite: with a NaN or an infinity in a
 * replicate, its output is a permutation of its rows in an unspecified order.
 * The result is ready when the stream has run the call's work; offsets_out
 * and x_out / y_out can be passed to cpc_fit_batched (one group of M subsets
 * per replicate). workspace: device, at least
 * cpc_partition_workspace_bytes(rep_offsets, R, dtype, scheme).
 * CPC_E_SIZE for M < 1, M >= 2^31, R M + 1 beyond int64, or x_out / y_out
 * the same buffer as x, y or each other; CPC_E_ENUM for an
 * unknown scheme or dtype; CPC_E_OFFSETS / CPC_E_UNSUPPORTED as for the
 * offsets of cpc_fit. */
int cpc_partition(cpc_handle_t h, const void* x, const void* y, int32_t dtype, int64_t n,
                  const int64_t* rep_offsets, int64_t R, int64_t M, int32_t scheme, void* workspace,
                  size_t ws_bytes, void* x_out, void* y_out, int64_t* offsets_out, void* stream);

/* Workspace bytes of cpc_spearman_fit for n rows, K subsets and G groups. */
size_t cpc_spearman_workspace_bytes(int64_t n, int64_t K, int64_t G);

/* The inversion of Spearman's rho as the estimator of each subset (Sec. 2.3
 * names it beside the pseudo-likelihood), combined per group by eq. (15):
 *   rho_S hat = 12 / (n (n^2 - 1)) sum (r1 - (n+1)/2)(r2 - (n+1)/2) from the
 *   doubled ranks R1, R2 (device, n each, as made by cpc_rank; any subset
 *   size), theta with rho_S(theta) = rho_S hat (Gaussian 2 sin(pi rho_S / 6);
 *   Frank through its Debye-function form; Gumbel through its Pickands
 *   function, rho_S = 12 int_0^1 (1 + a(w))^-2 dw - 3), and the variance of
 *   the estimate by the plug-in sandwich of the moment equation
 *   12 (u - 1/2)(v - 1/2) = rho_S(theta): var(psi) / (n rho_S'(theta)^2) with
 *   psi_i = J_i + W1(u_i) + W2(v_i) (W as in the pseudo-likelihood's variance).
 * out (device, K): theta, var, loglik = rho_S hat, score = rho_S(theta) -
 * rho_S hat, n, iters (Newton steps), status (DEGENERATE for fewer than
 * n_min rows or a margin of one value; Gumbel with rho_S hat <= 0 gives
 * theta = 1, BOUNDARY_NATURAL; beyond the search box BOUNDARY_BOX).
 * comb (device, G): eq. (15) over the OK / BOUNDARY_NATURAL subsets of each
 * group. Of opt only n_min is used. workspace: device, at least
 * cpc_spearman_workspace_bytes(n, K, G). */
int cpc_spearman_fit(cpc_handle_t h, const uint32_t* R1, const uint32_t* R2, int64_t n,
                     const int64_t* offsets, int64_t K, const int64_t* group_offsets, int64_t G,
                     const int32_t* family_per_group, const cpc_options_t* opt, void* workspace,
                     size_t ws_bytes, cpc_subset_result_t* out, cpc_combined_t* comb, void* stream);

/* Workspace bytes of cpc_kendall_fit for n rows, K subsets and G groups. */
size_t cpc_kendall_workspace_bytes(int64_t n, int64_t K, int64_t G);

/* The inversion of Kendall's tau as the estimator of each subset (Sec. 2.3
 * names it beside Spearman's rho), combined per group by eq. (15):
 *   tau hat = (concordant - discordant pairs) / (n (n - 1) / 2) of the
 *   doubled ranks R1, R2 (device, n each, as made by cpc_rank; a pair tied in
 *   either margin counts as neither), theta with tau(theta) = tau hat
 *   (Gaussian sin(pi tau / 2), Gumbel 1 / (1 - tau), Frank through
 *   tau = 1 - 4 (1 - D1(theta)) / theta with the Debye function D1), and the
 *   variance of the estimate as that of a U-statistic of degree two:
 *   4 var(S_i / (n - 1)) / (n tau'(theta)^2) with
 *   S_i = sum_l sign(r1_i - r1_l) sign(r2_i - r2_l).
 * Subsets of at most 2^20 rows (CPC_E_UNSUPPORTED beyond). out, comb,
 * statuses and opt as for cpc_spearman_fit, with loglik = tau hat and
 * score = tau(theta) - tau hat. workspace: device, at least
 * cpc_kendall_workspace_bytes(n, K, G). */
int cpc_kendall_fit(cpc_handle_t h, const uint32_t* R1, const uint32_t* R2, int64_t n,
                    const int64_t* offsets, int64_t K, const int64_t* group_offsets, int64_t G,
                    const int32_t* family_per_group, const cpc_options_t* opt, void* workspace,
                    size_t ws_bytes, cpc_subset_result_t* out, cpc_combined_t* comb, void* stream);

/* Workspace bytes of cpc_gaussk_fit for n rows of k margins, K subsets and
 * G groups (0 for k outside 2..8). */
size_t cpc_gaussk_workspace_bytes(int64_t n, int32_t k, int64_t K, int64_t G);

/* The k-dimensional Gaussian copula of eq. (7), C(u; R) =
 * Phi_R(Phi^-1(u_1), ..., Phi^-1(u_k)), fitted by maximum pseudo-likelihood
 * on every subset (the multi-parameter extension Sec. 4 leaves as future
 * work), with 2 <= k <= 8 (CPC_E_UNSUPPORTED above):
 *   R: device, k columns of n doubled ranks (column j at R + j n, as made by
 *   cpc_rank for each margin); per subset the normal scores
 *   z = Phi^-1(R / (2 (n + 1))), the Gram matrix G = sum z z', and the
 *   p = k (k - 1) / 2 correlations r_jl (j < l, order (0,1), (0,2), ...,
 *   (k-2,k-1)) maximising -(n/2) log det R - (1/2) tr((R^-1 - I) G) (Newton
 *   from the normalised Gram matrix); each correlation's variance from the
 *   rank-based sandwich J^-1 Omega J^-1 / n (J the mean outer product of the
 *   per-row scores, Omega the covariance of the scores plus their rank
 *   corrections, as in the one-parameter variance).
 * out (device, p K entries, parameter-major: entry q K + m is parameter q of
 * subset m): theta = r_q, var, loglik (of the subset), score (dl/dr_q), n,
 * iters, status (DEGENERATE for fewer than max(n_min, k + 1) rows or a
 * margin of one value; BOUNDARY_BOX when the normalised Gram matrix is not
 * positive definite; NOCONV; BADVAR). comb (device, p G entries, entry
 * q G + g): eq. (15) per parameter over the OK subsets of group g. Of opt
 * only n_min is used. workspace: ordinary (coarse-grained) device memory as
 * hipMalloc returns it (its rank bins take hardware FP64 atomic adds), at
 * least cpc_gaussk_workspace_bytes(n, k, K, G). */
int cpc_gaussk_fit(cpc_handle_t h, const uint32_t* R, int64_t n, int32_t k, const int64_t* offsets, int64_t K,
                   const int64_t* group_offsets, int64_t G, const cpc_options_t* opt, void* workspace,
                   size_t ws_bytes, cpc_subset_result_t* out, cpc_combined_t* comb, void* stream);

/* Durations (milliseconds) of the phases of the handle's last cpc_fit /
 * cpc_fit_batched call made with CPC_FLAG_PHASE_TIMES: ms[0] ranks (eq. 12),
 * ms[1] maximisation of eq. (13), ms[2] variance (Sec. 2.3), ms[3] combine
 * (eq. 15). Measured with hipEvents on the call's stream. With
 * CPC_FLAG_GRAPH as well, the call captures one graph per phase and every
 * replay records the events between the four graph launches. Blocks until
 * the last phase has completed. CPC_E_OPTIONS if no such call was made. */
int cpc_phase_times(cpc_handle_t h, float* ms);

/* Message for an error code, and the thread-local detail of the last error. */
const char* cpc_strerror(int code);
const char* cpc_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* CPC_H */
