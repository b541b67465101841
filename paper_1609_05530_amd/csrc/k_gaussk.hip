// k_gaussk.hip — the k-dimensional Gaussian copula of eq. (7) of
// arXiv:1609.05530 (C(u; R) = Phi_R(Phi^-1(u_1), ..., Phi^-1(u_k))) fitted by
// maximum pseudo-likelihood on every subset: the multi-parameter extension
// the paper leaves as future work. Parameters: the p = k (k - 1) / 2
// correlations r_jl (j < l) in the order (0,1), (0,2), ..., (k-2,k-1).
//
// One workgroup of 256 threads per subset (k <= 8, any subset size):
//   1. normal scores z_ij = Phi^-1(R_ij / (2 (n + 1))) of the doubled ranks;
//   2. the Gram matrix G = sum_i z_i z_i' on the FP64 matrix cores
//      (16 x 16 x 4 MFMA, four rows per instruction, the k margins padded to
//      16; each wave takes every fourth block of rows);
//   3. l(R) = -(n/2) log det R - (1/2) tr((R^-1 - I) G) is maximised by
//      Newton on the p correlations (one wave, everything in LDS): with
//      P = R^-1, M = P G P, dl/dr_jl = -n P_jl + M_jl and
//      d2l/dr_jl dr_st = n (P_js P_tl + P_jt P_sl)
//                        - (P_js M_tl + P_jt M_sl + M_js P_tl + M_jt P_sl),
//      from the normalised Gram matrix, a step halved until R stays positive
//      definite, to max |step| <= 1e-12 (1 + max |r|);
//   4. the sandwich variance: per row the scores s_i,jl = -P_jl + y_ij y_il
//      (y_i = P z_i) and psi_i = s_i + sum_m W_m(u_im), W_m(u_im) the mean over
//      the rows with u_lm >= u_im of ds_l/du_m = (P_jm y_l + y_j P_lm) /
//      phi(z_m): in one pass over the rows the vectors y_l / phi(z_lm) are
//      added into margin m's bins, indexed by the doubled rank, for every m
//      (only tied rows share a bin: margins found tie-free through a bitmap
//      of the bins in LDS take plain stores, the others FP64 atomics), the
//      bins are suffix-summed
//      (a tie group takes the whole group), and one more pass forms each
//      row's psi from the bins at its ranks. J = (1/n) sum s s' and Omega = cov(psi) are p x p contractions
//      over the rows, again on the FP64 MFMA (p padded to 16 or 32: one or
//      three 16 x 16 tiles); V = J^-1 Omega J^-1 / n, each parameter's
//      variance V_qq.
// The results are parameter-major (entry q K + m) so that the combination of
// eq. (15) runs per parameter over each group (k_combine).
#include <hip/hip_runtime.h>

#include "family_math.h"
#include "kernels.h"

namespace cpc {

namespace {

constexpr int GT = 256;  // threads per workgroup
constexpr int GW = GT / WAVE;
constexpr int KMAX = 8;
constexpr int PMAX = KMAX * (KMAX - 1) / 2;  // 28
constexpr int PPAD = 32;
// Subsets of up to kSeenRows rows find out which margins have ties (rows
// sharing a rank bin) from a bitmap in LDS; their tie-free margins fill the
// bins with plain stores, every bin but bin 0 once. Larger subsets, and
// margins with ties, add into the bins atomically.
constexpr int kSeenWords = 6144;  // 24 KiB
constexpr int kSeenRows = kSeenWords * 32 / KMAX - 1;

typedef double d4 __attribute__((ext_vector_type(4)));

struct GkParams {
  const uint32_t* R;   // k columns of n_total doubled ranks
  int64_t n_total;
  int k, p, ldx, pad;
  const SubDesc* subs;
  int64_t n_min;
  double* Z;           // rows x k (row-major), a subset's rows at its begin
  double* X;           // rows x ldx: scores, then psi
  double* B;           // bins: subset m owns k (n + 1) k doubles from k k (begin + m) (k margins' bins)
  ResultOut* out;      // parameter-major: q K + m
  int64_t K;
};

// sum over rows r of A[r][i0 + i] A[r][j0 + j] (i, j < 16), A row-major with
// leading dimension lda and ncol valid columns (the rest read as 0); rows
// r0 = 4 (first + t step) .. of [0, n). Operands: lane l gives A[l % 16][l / 16]
// and B[l / 16][l % 16]; the lane's 4 results are D[l / 16 + 4 e][l % 16]
// (e = 0..3; the rows interleave across the four 16-lane groups, as measured
// on gfx950).
__device__ __forceinline__ d4 tile_gram(const double* A, int lda, int n, int i0, int j0, int ncol, int first,
                                         int step) {
  constexpr int U = 8;  // row blocks whose loads are in flight together
  const int lane = threadIdx.x & (WAVE - 1);
  const int c = lane & 15, rr = lane >> 4;
  const bool ci = i0 + c < ncol, cj = j0 + c < ncol;
  d4 acc = {0.0, 0.0, 0.0, 0.0};
  for (int r0 = 4 * first; r0 < n; r0 += 4 * step * U) {
    double a[U], b[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int r = r0 + 4 * step * u + rr;
      a[u] = (r < n && ci) ? A[(int64_t)r * lda + i0 + c] : 0.0;
      b[u] = (r < n && cj) ? A[(int64_t)r * lda + j0 + c] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u], b[u], acc, 0, 0, 0);
  }
  return acc;
}

struct GkShared {
  double tiles[GW][16][16];  // per-wave MFMA tiles, reduced into G / J / Omega
  double G[KMAX][KMAX];
  double P[KMAX][KMAX];
  double M[KMAX][KMAX];
  double Rm[KMAX][KMAX];
  double J[PPAD][PPAD];
  double Om[PPAD][PPAD];
  double Hm[PMAX][PMAX];
  double th[PMAX], g[PMAX], st[PMAX], mu[PPAD], cand[PMAX];
  double L[KMAX][KMAX], PG[KMAX][KMAX];
  double scal[4];  // loglik, status, iterations
  double tot[GT][KMAX];
  int pj[PMAX], pl[PMAX];
  unsigned int mm[2 * KMAX];
  unsigned int tied[KMAX];         // margin m has two rows in one rank bin
  unsigned int seen[kSeenWords];   // per margin, one bit per rank bin (subsets of up to kSeenRows rows)
};

// The small dense linear algebra below runs on wave 0 with its matrices in
// LDS; its lanes take the rows, entries or right-hand sides of each step.

// Orders one wave's LDS operations around a hand-off between its lanes (a
// wave's LDS operations are performed in program order; the fences keep the
// compiler from moving them across).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ double wave_max_d(double v) {
  for (int off = 32; off >= 1; off >>= 1) v = fmax(v, __shfl_xor(v, off, WAVE));
  return v;
}
__device__ __forceinline__ double wave_sum_d(double v) {
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, WAVE);
  return v;
}

// Cholesky factor (lower, in place) of the N x N matrix A (leading dimension
// LD), right-looking: per column the pivot, the column divided by its square
// root, then the lanes update the trailing lower triangle. Every entry sees
// the subtractions of the column-by-column form, in the same order. False
// (in every lane) if a pivot is not positive.
template <int N, int LD>
__device__ __noinline__ bool wave_chol(double* A) {
  const int lane = threadIdx.x & (WAVE - 1);
#pragma unroll 1
  for (int j = 0; j < N; ++j) {
    const double d = A[j * LD + j];
    if (!(d > 0.0)) return false;  // the same value in every lane
    const double sd = sqrt(d);
    for (int i = j + 1 + lane; i < N; i += WAVE) A[i * LD + j] /= sd;
    if (lane == 0) A[j * LD + j] = sd;
    wave_sync();
    const int m = N - j - 1;
    for (int idx = lane; idx < m * m; idx += WAVE) {
      const int i = j + 1 + idx / m, c = j + 1 + idx % m;
      if (c <= i) A[i * LD + c] -= A[i * LD + j] * A[c * LD + j];
    }
    wave_sync();
  }
  return true;
}

// Solve L L' x = b in place (b: N entries in LDS), by columns: each solved
// entry is subtracted from the later (then the earlier) ones by the lanes.
template <int N, int LD>
__device__ __noinline__ void wave_chol_solve(const double* L, double* b) {
  const int lane = threadIdx.x & (WAVE - 1);
#pragma unroll 1
  for (int i = 0; i < N; ++i) {
    const double xi = b[i] / L[i * LD + i];
    for (int r = i + 1 + lane; r < N; r += WAVE) b[r] -= L[r * LD + i] * xi;
    if (lane == 0) b[i] = xi;
    wave_sync();
  }
#pragma unroll 1
  for (int i = N - 1; i >= 0; --i) {
    const double xi = b[i] / L[i * LD + i];
    for (int r = lane; r < i; r += WAVE) b[r] -= L[i * LD + r] * xi;
    if (lane == 0) b[i] = xi;
    wave_sync();
  }
}

// Solve L L' x = e_c for the lane's column c (x in registers; L in LDS,
// read by every lane alike).
template <int N, int LD>
__device__ __forceinline__ void lane_chol_solve_unit(const double* L, int c, double (&x)[N]) {
#pragma unroll
  for (int i = 0; i < N; ++i) {
    double v = (i == c) ? 1.0 : 0.0;
#pragma unroll
    for (int s = 0; s < i; ++s) v -= L[i * LD + s] * x[s];
    x[i] = v / L[i * LD + i];
  }
#pragma unroll
  for (int i = N - 1; i >= 0; --i) {
    double v = x[i];
#pragma unroll
    for (int s = i + 1; s < N; ++s) v -= L[s * LD + i] * x[s];
    x[i] = v / L[i * LD + i];
  }
}

// The same, in place in column c of X (leading dimension LDX, in LDS): for
// right-hand sides too many for registers.
template <int N, int LD, int LDX>
__device__ __noinline__ void lane_chol_solve_unit_lds(const double* L, int c, double* X) {
#pragma unroll 1
  for (int i = 0; i < N; ++i) {
    double v = (i == c) ? 1.0 : 0.0;
    for (int s = 0; s < i; ++s) v -= L[i * LD + s] * X[s * LDX + c];
    X[i * LDX + c] = v / L[i * LD + i];
  }
#pragma unroll 1
  for (int i = N - 1; i >= 0; --i) {
    double v = X[i * LDX + c];
    for (int s = i + 1; s < N; ++s) v -= L[s * LD + i] * X[s * LDX + c];
    X[i * LDX + c] = v / L[i * LD + i];
  }
}

// index of parameter (j, l), j < l, in the order (0,1), (0,2), ..., (k-2,k-1)
template <int KD>
__device__ __forceinline__ int pidx_of(int j, int l) {
  return j * (2 * KD - j - 1) / 2 + (l - j - 1);
}

// R from theta into dst (k x k, leading dimension KMAX)
template <int KD>
__device__ void wave_corr_from(double (*dst)[KMAX], const double* th) {
  const int lane = threadIdx.x & (WAVE - 1);
  if (lane < KD * KD) {
    const int j = lane / KD, l = lane % KD;
    dst[j][l] = (j == l) ? 1.0 : th[j < l ? pidx_of<KD>(j, l) : pidx_of<KD>(l, j)];
  }
  wave_sync();
}

// Is the correlation matrix of th positive definite? (M as scratch)
template <int KD>
__device__ __noinline__ bool wave_corr_pd(GkShared& S, const double* th) {
  wave_corr_from<KD>(S.M, th);
  return wave_chol<KD, KMAX>(&S.M[0][0]);
}

// From R in S.Rm (positive definite): P = R^-1, M = P G P; returns log det R
// (in every lane)
template <int KD>
__device__ __noinline__ double wave_inverse_and_m(GkShared& S) {
  const int lane = threadIdx.x & (WAVE - 1);
  if (lane < KD * KD) S.L[lane / KD][lane % KD] = S.Rm[lane / KD][lane % KD];
  wave_sync();
  wave_chol<KD, KMAX>(&S.L[0][0]);
  double logdet = 0.0;
#pragma unroll
  for (int j = 0; j < KD; ++j) logdet += 2.0 * log(S.L[j][j]);
  if (lane < KD) {
    double x[KD];
    lane_chol_solve_unit<KD, KMAX>(&S.L[0][0], lane, x);
#pragma unroll
    for (int j = 0; j < KD; ++j) S.P[j][lane] = x[j];
  }
  wave_sync();
  if (lane < KD * KD) {
    const int j = lane / KD, l = lane % KD;
    double v = 0.0;
#pragma unroll
    for (int s = 0; s < KD; ++s) v += S.P[j][s] * S.G[s][l];
    S.PG[j][l] = v;
  }
  wave_sync();
  if (lane < KD * KD) {
    const int j = lane / KD, l = lane % KD;
    double v = 0.0;
#pragma unroll
    for (int s = 0; s < KD; ++s) v += S.PG[j][s] * S.P[s][l];
    S.M[j][l] = v;
  }
  wave_sync();
  return logdet;
}

// gradient of l into S.g and the negated Hessian into S.Hm (after
// wave_inverse_and_m)
template <int KD>
__device__ __noinline__ void wave_grad_neg_hess(GkShared& S, double dn) {
  constexpr int p = KD * (KD - 1) / 2;
  const int lane = threadIdx.x & (WAVE - 1);
  for (int a = lane; a < p; a += WAVE) S.g[a] = -dn * S.P[S.pj[a]][S.pl[a]] + S.M[S.pj[a]][S.pl[a]];
  for (int idx = lane; idx < p * p; idx += WAVE) {
    const int a = idx / p, b = idx % p;
    const int j = S.pj[a], l = S.pl[a], s = S.pj[b], t = S.pl[b];
    const double h = dn * (S.P[j][s] * S.P[t][l] + S.P[j][t] * S.P[s][l]) -
                     (S.P[j][s] * S.M[t][l] + S.P[j][t] * S.M[s][l] + S.M[j][s] * S.P[t][l] + S.M[j][t] * S.P[s][l]);
    S.Hm[a][b] = -h;
  }
  wave_sync();
}

// the workgroup's four wave tiles summed into dst[i0 + i][j0 + j] (i, j < 16)
// and, off the diagonal, its transpose
__device__ __forceinline__ void store_tile(GkShared& S, d4 acc, double (*dst)[PPAD], int i0, int j0, bool sum_waves) {
  const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE;
  const int c = lane & 15, r0 = lane >> 4;  // result e is row r0 + 4 e, column c
  if (sum_waves) {
#pragma unroll
    for (int e = 0; e < 4; ++e) S.tiles[w][r0 + 4 * e][c] = acc[e];
    __syncthreads();
    const int t = threadIdx.x;  // 256 threads, 256 entries
    const int i = t >> 4, j = t & 15;
    double v = 0.0;
    for (int u = 0; u < GW; ++u) v += S.tiles[u][i][j];
    dst[i0 + i][j0 + j] = v;
    if (i0 != j0) dst[j0 + j][i0 + i] = v;
    __syncthreads();
  } else {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      dst[i0 + r0 + 4 * e][j0 + c] = acc[e];
      if (i0 != j0) dst[j0 + c][i0 + r0 + 4 * e] = acc[e];
    }
  }
}

// p x p contraction X' X over the subset's rows into dst: each 16 x 16 tile
// ((0,0); with p > 16 also (0,1) and (1,1)) by all four waves, each taking
// every fourth block of rows, summed through LDS
__device__ void contract(GkShared& S, const double* X, int ldx, int n, int p, double (*dst)[PPAD]) {
  const int w = threadIdx.x / WAVE;
  const int ntiles = p <= 16 ? 1 : 3;
  for (int tile = 0; tile < ntiles; ++tile) {
    const int i0 = (tile == 2) ? 16 : 0, j0 = (tile == 0) ? 0 : 16;
    const d4 acc = tile_gram(X, ldx, n, i0, j0, p, w, GW);
    store_tile(S, acc, dst, i0, j0, true);
  }
}

template <int KD>
__global__ void __launch_bounds__(GT, 2) k_gaussk(GkParams P) {
  constexpr int k = KD, p = KD * (KD - 1) / 2, ldx = p <= 16 ? 16 : 32;
  __shared__ GkShared S;
  const int sid = blockIdx.x, t = threadIdx.x;
  const SubDesc sd = P.subs[sid];
  const int n = sd.n;
  const int64_t o = sd.begin;
  const double dn = (double)n;
  if (t < PMAX) {
    int q = 0, jj = 0, ll = 1;
    for (int j = 0; j < k; ++j)
      for (int l = j + 1; l < k; ++l, ++q)
        if (q == t) { jj = j; ll = l; }
    S.pj[t] = jj;
    S.pl[t] = ll;
  }
  if (t < 2 * KMAX) S.mm[t] = (t & 1) ? 0u : ~0u;
  __syncthreads();

  // 1. normal scores and each margin's range
  const int64_t twon1 = 2 * (int64_t)n + 2;
  double* Z = P.Z + o * k;
  for (int64_t e = t; e < (int64_t)n * k; e += GT) {
    const int i = (int)(e / k), j = (int)(e - (int64_t)i * k);
    const uint32_t r = P.R[(int64_t)j * P.n_total + o + i];
    Z[e] = qnorm_ppnd16((int64_t)r, twon1);
    atomicMin(&S.mm[2 * j], r);
    atomicMax(&S.mm[2 * j + 1], r);
  }
  __syncthreads();
  bool degenerate = n < P.n_min || n < 2 || n <= k;
  for (int j = 0; j < k; ++j) degenerate = degenerate || S.mm[2 * j] == S.mm[2 * j + 1];
  if (degenerate) {  // workgroup-uniform
    if (t < p) {
      ResultOut r;
      r.theta = NAN; r.var = NAN; r.loglik = NAN; r.score = NAN;
      r.n = n; r.iters = 0; r.status = ST_DEGENERATE;
      P.out[(int64_t)t * P.K + sid] = r;
    }
    return;
  }

  // 2. G on the matrix cores
  {
    const int w = t / WAVE;
    const d4 acc = tile_gram(Z, k, n, 0, 0, k, w, GW);
    store_tile(S, acc, S.Om, 0, 0, true);  // (Om as scratch)
    if (t < KMAX * KMAX) {
      const int j = t / KMAX, l = t % KMAX;
      if (j < k && l < k) S.G[j][l] = S.Om[j][l];
    }
    __syncthreads();
  }

  // 3. Newton (wave 0; the other waves wait at the barrier after it)
  if (t < WAVE) {
    const int lane = t;
    int status = ST_OK, it = 0;
    for (int q = lane; q < p; q += WAVE) {
      const int j = S.pj[q], l = S.pl[q];
      S.th[q] = S.G[j][l] / (sqrt(S.G[j][j]) * sqrt(S.G[l][l]));
    }
    wave_sync();
    if (!wave_corr_pd<KD>(S, S.th)) {
      status = ST_BOUNDARY_BOX;
    } else {
      status = ST_NOCONV;
      for (it = 1; it <= 100; ++it) {
        wave_corr_from<KD>(S.Rm, S.th);
        wave_inverse_and_m<KD>(S);
        wave_grad_neg_hess<KD>(S, dn);
        if (!wave_chol<p, PMAX>(&S.Hm[0][0])) break;  // NOCONV
        for (int a = lane; a < p; a += WAVE) S.st[a] = S.g[a];
        wave_sync();
        wave_chol_solve<p, PMAX>(&S.Hm[0][0], S.st);
        double lam = 1.0;
        for (int h = 0; h < 30; ++h) {
          for (int a = lane; a < p; a += WAVE) S.cand[a] = S.th[a] + lam * S.st[a];
          wave_sync();
          if (wave_corr_pd<KD>(S, S.cand)) break;
          lam *= 0.5;
        }
        double mstep = 0.0, mth = 0.0;
        for (int a = lane; a < p; a += WAVE) {
          mstep = fmax(mstep, fabs(lam * S.st[a]));
          mth = fmax(mth, fabs(S.th[a]));
          S.th[a] += lam * S.st[a];
        }
        mstep = wave_max_d(mstep);
        mth = wave_max_d(mth);
        wave_sync();
        if (mstep <= 1e-12 * (1.0 + mth)) {
          status = ST_OK;
          break;
        }
      }
      if (it > 100) it = 100;
    }
    double ll = NAN;
    if (status == ST_OK) {
      wave_corr_from<KD>(S.Rm, S.th);
      const double logdet = wave_inverse_and_m<KD>(S);
      wave_grad_neg_hess<KD>(S, dn);
      double tr = 0.0;
      if (lane < KD * KD) {
        const int j = lane / KD, l = lane % KD;
        tr = (S.P[j][l] - (j == l ? 1.0 : 0.0)) * S.G[l][j];
      }
      tr = wave_sum_d(tr);
      ll = -0.5 * dn * logdet - 0.5 * tr;
    }
    if (lane == 0) {
      S.scal[0] = ll;
      S.scal[1] = (double)status;
      S.scal[2] = (double)it;
    }
  }
  __syncthreads();
  const int status = (int)S.scal[1];
  if (status != ST_OK) {
    if (t < p) {
      ResultOut r;
      r.theta = S.th[t]; r.var = NAN; r.loglik = NAN; r.score = NAN;
      r.n = n; r.iters = (int)S.scal[2]; r.status = status;
      P.out[(int64_t)t * P.K + sid] = r;
    }
    return;
  }

  // 4. scores into X, then J = X'X / n
  double* X = P.X + o * ldx;
  for (int i = t; i < n; i += GT) {
    double z[KMAX], y[KMAX];
    for (int j = 0; j < k; ++j) z[j] = Z[(int64_t)i * k + j];
    for (int j = 0; j < k; ++j) {
      double v = 0.0;
      for (int l = 0; l < k; ++l) v += S.P[j][l] * z[l];
      y[j] = v;
    }
    double* xi = X + (int64_t)i * ldx;
    int q = 0;
#pragma unroll
    for (int j = 0; j < k; ++j)
#pragma unroll
      for (int l = j + 1; l < k; ++l, ++q) xi[q] = -S.P[j][l] + y[j] * y[l];
#pragma unroll
    for (int c = p; c < ldx; ++c) xi[c] = 0.0;
  }
  __syncthreads();
  contract(S, X, ldx, n, p, S.J);

  // 5. psi = s + sum_m W_m. One pass over the rows adds each row's
  //    y / phi(z_m) into margin m's bins at its doubled rank, for every
  //    margin; each margin's bins are then suffix-summed; a last pass forms
  //    psi from s and the bins at the row's ranks, writing each row once.
  // bins floor(R / 2), 0 .. n: distinct tie groups differ by at least 2 in
  // doubled rank, so no bin holds two groups
  const int64_t NB = (int64_t)n + 1;
  double* Bn = P.B + (o + (int64_t)sid) * k * k;  // margin m's bins at Bn + m NB k
  const double inv_n = 1.0 / dn, inv_s2pi = 0.39894228040143267794;
  const bool small = n <= kSeenRows;  // workgroup-uniform
  const int wpm = (int)((NB + 31) / 32);  // bitmap words per margin
  if (t < KMAX) S.tied[t] = small ? 0u : 1u;
  if (small) {
    for (int e = t; e < wpm * KD; e += GT) S.seen[e] = 0u;
    __syncthreads();
    for (int i = t; i < n; i += GT) {
#pragma unroll
      for (int m = 0; m < KD; ++m) {
        const uint32_t r = P.R[(int64_t)m * P.n_total + o + i] >> 1;
        const uint32_t bit = 1u << (r & 31u);
        const uint32_t old = atomicOr(&S.seen[m * wpm + (int)(r >> 5)], bit);
        if (old & bit) S.tied[m] = 1u;
      }
    }
  }
  __syncthreads();
  // clear the bins that stores will not cover: all of a margin with ties (or
  // of a large subset), bin 0 of the others
  for (int m = 0; m < KD; ++m) {
    double* Bm = Bn + (int64_t)m * NB * KD;
    const int64_t len = S.tied[m] ? NB * KD : KD;
    for (int64_t e = t; e < len; e += GT) Bm[e] = 0.0;
  }
  __syncthreads();
  for (int i = t; i < n; i += GT) {
    double z[KD], y[KD];
#pragma unroll
    for (int j = 0; j < KD; ++j) z[j] = Z[(int64_t)i * KD + j];
#pragma unroll
    for (int j = 0; j < KD; ++j) {
      double v = 0.0;
#pragma unroll
      for (int l = 0; l < KD; ++l) v += S.P[j][l] * z[l];
      y[j] = v;
    }
#pragma unroll
    for (int m = 0; m < KD; ++m) {
      const double iphi = 1.0 / (inv_s2pi * exp(-0.5 * z[m] * z[m]));
      const uint32_t r = P.R[(int64_t)m * P.n_total + o + i] >> 1;
      double* bm = Bn + ((int64_t)m * NB + r) * KD;
      if (S.tied[m]) {  // workgroup-uniform
#pragma unroll
        for (int j = 0; j < KD; ++j) unsafeAtomicAdd(&bm[j], y[j] * iphi);  // the hardware FP64 add (device memory)
      } else {
#pragma unroll
        for (int j = 0; j < KD; ++j) bm[j] = y[j] * iphi;
      }
    }
  }
  __syncthreads();
  for (int m = 0; m < KD; ++m) {
    double* Bm = Bn + (int64_t)m * NB * KD;
    // suffix sums over the bins: thread t takes bins [t C, (t + 1) C)
    const int64_t C = (NB + GT - 1) / GT;
    const int64_t b0 = t * C, b1 = min(b0 + C, NB);
    // (the chunk total first, from independent loads; then the carries; then
    // one walk down the chunk writing the suffix sums)
    double run[KMAX];
    for (int j = 0; j < k; ++j) run[j] = 0.0;
#pragma unroll 4
    for (int64_t b = b0; b < b1; ++b)
      for (int j = 0; j < k; ++j) run[j] += Bm[b * k + j];
    // the totals of the later threads: suffix sums within the wave
    // (shuffles), then the later waves' totals through LDS
    double acc[KMAX];
    {
      const int lane = t & (WAVE - 1), w = t / WAVE;
      for (int j = 0; j < k; ++j) {
        double v = run[j];
        for (int d = 1; d < WAVE; d <<= 1) {
          const double o2 = __shfl_down(v, d, WAVE);
          if (lane + d < WAVE) v += o2;
        }
        const double nxt = __shfl_down(v, 1, WAVE);
        acc[j] = (lane + 1 < WAVE) ? nxt : 0.0;
        if (lane == 0) S.tot[w][j] = v;
      }
      __syncthreads();
      for (int j = 0; j < k; ++j)
        for (int u = w + 1; u < GW; ++u) acc[j] += S.tot[u][j];
    }
#pragma unroll 4
    for (int64_t b = b1 - 1; b >= b0; --b)
      for (int j = 0; j < k; ++j) {
        acc[j] += Bm[b * k + j];
        Bm[b * k + j] = acc[j];
      }
    __syncthreads();
  }
  for (int i = t; i < n; i += GT) {
    double* xi = X + (int64_t)i * ldx;
    double psi[p];
#pragma unroll
    for (int q = 0; q < p; ++q) psi[q] = xi[q];
#pragma unroll 1
    for (int m = 0; m < KD; ++m) {
      const uint32_t r = P.R[(int64_t)m * P.n_total + o + i] >> 1;
      const double* bm = Bn + ((int64_t)m * NB + r) * KD;
      double A[KD], Pm[KD];
#pragma unroll
      for (int j = 0; j < KD; ++j) {
        A[j] = bm[j] * inv_n;
        Pm[j] = S.P[j][m];
      }
      int q = 0;
#pragma unroll
      for (int j = 0; j < KD; ++j)
#pragma unroll
        for (int l = j + 1; l < KD; ++l, ++q) psi[q] += Pm[j] * A[l] + A[j] * Pm[l];
    }
#pragma unroll
    for (int q = 0; q < p; ++q) xi[q] = psi[q];
  }
  __syncthreads();

  // 6. Omega = X'X / n - mean mean'
  contract(S, X, ldx, n, p, S.Om);
  {
    // column sums of psi: per thread, per wave (shuffles), across waves (LDS)
    for (int q = 0; q < p; ++q) {
      double s = 0.0;
      for (int i = t; i < n; i += GT) s += X[(int64_t)i * ldx + q];
      for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off, WAVE);
      if ((t & (WAVE - 1)) == 0) S.tiles[t / WAVE][q >> 4][q & 15] = s;
    }
    __syncthreads();
    if (t < p) {
      double s = 0.0;
      for (int u = 0; u < GW; ++u) s += S.tiles[u][t >> 4][t & 15];
      S.mu[t] = s * inv_n;
    }
    __syncthreads();
  }

  // 7. V = J^-1 Omega J^-1 / n (wave 0 factors J, lane c solves column c of
  //    its inverse; thread q forms V_qq)
  for (int idx = t; idx < p * p; idx += GT) {
    const int a = idx / p, b = idx % p;
    S.J[a][b] *= inv_n;
    S.Om[a][b] = S.Om[a][b] * inv_n - S.mu[a] * S.mu[b];
    S.Hm[a][b] = S.J[a][b];
  }
  __syncthreads();
  if (t < WAVE) {
    const bool ok = wave_chol<p, PMAX>(&S.Hm[0][0]);
    if (t < p) {
      if (ok) {
        lane_chol_solve_unit_lds<p, PMAX, PPAD>(&S.Hm[0][0], t, &S.J[0][0]);
      } else {
        for (int a = 0; a < p; ++a) S.J[a][t] = NAN;
      }
    }
  }
  __syncthreads();
  if (t < p) {
    const int q = t;
    double v = 0.0;
    for (int a = 0; a < p; ++a) {
      double w = 0.0;
      for (int b = 0; b < p; ++b) w += S.Om[a][b] * S.J[b][q];
      v += S.J[a][q] * w;
    }
    v *= inv_n;
    ResultOut r;
    r.theta = S.th[q];
    r.var = v;
    r.loglik = S.scal[0];
    r.score = S.g[q];
    r.n = n;
    r.iters = (int)S.scal[2];
    r.status = (v > 0.0 && isfinite(v)) ? ST_OK : ST_BADVAR;
    P.out[(int64_t)q * P.K + sid] = r;
  }
}

}  // namespace

int gaussk_ldx(int k) { return k * (k - 1) / 2 <= 16 ? 16 : 32; }

hipError_t launch_gaussk(const uint32_t* R, int64_t n_total, int k, const SubDesc* subs, int64_t K, int64_t n_min,
                         double* Z, double* X, double* B, ResultOut* out, hipStream_t s) {
  GkParams p = {};
  p.R = R; p.n_total = n_total; p.k = k; p.p = k * (k - 1) / 2; p.ldx = gaussk_ldx(k);
  p.subs = subs; p.n_min = n_min; p.Z = Z; p.X = X; p.B = B; p.out = out; p.K = K;
  if (K <= 0) return hipSuccess;
  const dim3 grid((unsigned)K), block(GT);
  switch (k) {
    case 2: hipLaunchKernelGGL(k_gaussk<2>, grid, block, 0, s, p); break;
    case 3: hipLaunchKernelGGL(k_gaussk<3>, grid, block, 0, s, p); break;
    case 4: hipLaunchKernelGGL(k_gaussk<4>, grid, block, 0, s, p); break;
    case 5: hipLaunchKernelGGL(k_gaussk<5>, grid, block, 0, s, p); break;
    case 6: hipLaunchKernelGGL(k_gaussk<6>, grid, block, 0, s, p); break;
    case 7: hipLaunchKernelGGL(k_gaussk<7>, grid, block, 0, s, p); break;
    case 8: hipLaunchKernelGGL(k_gaussk<8>, grid, block, 0, s, p); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace cpc
