// k_moment.hip — the inversion of Spearman's rho as an estimator of the
// copula parameter (Sec. 2.3 of arXiv:1609.05530 names it beside the
// pseudo-likelihood), per subset from its doubled ranks (eq. 12), combined
// by eq. (15) like the pseudo-likelihood estimates.
//
// One workgroup per subset, any size:
//   - rho_S hat = 12 / (n (n^2 - 1)) sum (r1 - (n+1)/2)(r2 - (n+1)/2), the sum
//     in exact 64-bit integers;
//   - theta hat solves rho_S(theta) = rho_S hat: Gaussian in closed form
//     (rho = 2 sin(pi rho_S / 6)); Frank rho_S = 1 - 12 (D1 - D2) / theta with
//     Debye functions D_k; Gumbel, an extreme-value copula with Pickands
//     function a(w) = (w^theta + (1 - w)^theta)^(1/theta), has
//     int int C = int_0^1 (1 + a(w))^-2 dw, so rho_S = 12 int_0^1
//     (1 + a(w))^-2 dw - 3. The integrals are taken by the workgroup (one
//     Gauss-Legendre node per thread) inside a safeguarded Newton iteration;
//   - the asymptotic variance by the plug-in sandwich of the moment
//     equation J(u, v) = 12 (u - 1/2)(v - 1/2) = rho_S(theta):
//     psi_i = J_i + W1(u_i) + W2(v_i) with W1(u_i) = (1/n) sum over
//     u_l >= u_i of dJ/du (u_l, v_l) (a tie group takes the whole group),
//     sigma^2 = var(psi) / (n rho_S'(theta)^2). dJ/du = 12 (v - 1/2) is a
//     multiple of the integer r2 - (n+1)/2, so the suffix sums are exact
//     64-bit integer sums over a histogram indexed by the doubled rank.
//
// The inversion of Kendall's tau, one workgroup per subset of up to 2^20
// rows (subsets of up to 16384 rows count in LDS: k_kendall_lds below):
// tau hat = sum_i S_i / (n (n - 1)) with
// S_i = sum_l sign(a_i - a_l) sign(b_i - b_l) (a, b the doubled ranks), and
// var(tau hat) = 4 var(S_i / (n - 1)) / n (a U-statistic of degree two).
// The S_i come from two merge sorts through the workspace: the rows sorted by
// (a, b) give the sequence B_p of b values; a second merge sort of B counts,
// for every position p, sum_{q<p} sign(B_p - B_q) (at each level a right-run
// element adds (#left < B_p) - (#left > B_p), two binary searches in the left
// run). Then with the runs of equal a and of equal (a, b) around p (binary
// searches in the first sorted order), S = 2 (count - #{same a, b < b_p}) +
// (#{same a, b < b_p} - #{same a, b > b_p}) - (R2 - n - 1), where
// R2 - n - 1 = #{b_l < b_i} - #{b_l > b_i}. All counts are exact integers.
// theta: Gaussian sin(pi tau / 2), Gumbel 1 / (1 - tau) in closed form;
// Frank tau = 1 - 4 (1 - D1(theta)) / theta by the workgroup Newton.
#include <hip/hip_runtime.h>

#include "block_rank.h"
#include "kernels.h"

namespace cpc {

namespace {

constexpr int MT = 256;  // threads per workgroup = quadrature nodes per evaluation
constexpr int64_t kSpearmanLdsRows = 16384;  // rank bins in LDS up to this subset size

// 8-point Gauss-Legendre rule on [-1, 1]
__constant__ double kMx[4] = {0.1834346424956498049, 0.5255324099163289858, 0.7966664774136267396,
                              0.9602898564975362317};
__constant__ double kMw[4] = {0.3626837833783619830, 0.3137066458778872873, 0.2223810344533744706,
                              0.1012285362903762592};

// Node `j` (0 .. MT-1) of 32 equal panels of [a, b] with 8 nodes each.
__device__ __forceinline__ void quad_node(int j, double a, double b, double& x, double& w) {
  const int panel = j >> 3, k = j & 7;
  const int m = k < 4 ? 3 - k : k - 4;
  const double xi = k < 4 ? -kMx[m] : kMx[m];
  const double h = (b - a) / 32.0;
  x = a + h * (panel + 0.5 * (xi + 1.0));
  w = 0.5 * h * kMw[m];
}

// This thread's share of rho_S(theta) + 3 (Gumbel) or of the Debye
// integrals (Frank), and of their theta-derivatives.
template <int FAM>
__device__ __forceinline__ void rho_terms(double th, double& f0, double& f1, double& f2, double& f3) {
  f0 = f1 = f2 = f3 = 0.0;
  if constexpr (FAM == FAM_GUMBEL) {
    // 12 int_0^1 (1 + a)^-2 dw = 24 int_0^{1/2} (1 + a)^-2 dw (a(w) = a(1 - w))
    double w, wt;
    quad_node(threadIdx.x, 0.0, 0.5, w, wt);
    const double lw = log(w), lv = log1p(-w);  // lw <= lv on (0, 1/2]
    const double q = exp(th * (lw - lv));
    const double l1q = log1p(q);
    const double la = lv + l1q / th;  // log a
    const double a = exp(la);
    const double dla = -l1q / (th * th) + (q * (lw - lv)) / (th * (1.0 + q));  // d log a / d theta
    const double ia = 1.0 / (1.0 + a);
    f0 = 24.0 * wt * ia * ia;
    f1 = -48.0 * wt * ia * ia * ia * a * dla;
  } else if constexpr (FAM == FAM_FRANK) {
    // int_0^A t^k / (e^t - 1) dt, k = 1, 2, over [0, min(A, 60)] (the rest is
    // below e^-60 of it)
    const double A = fabs(th);
    double t, wt;
    quad_node(threadIdx.x, 0.0, fmin(A, 60.0), t, wt);
    const double g = t / expm1(t);
    f2 = wt * g;
    f3 = wt * g * t;
  }
}

struct MomParams {
  const uint32_t* R1;
  const uint32_t* R2;
  const SubDesc* subs;
  int64_t n_min;
  long long* H1;  // subset m (m = base + block) owns 2n + 2 entries from 2 (begin + m)
  long long* H2;
  int64_t base;   // index of the launch's first subset
  ResultOut* out;
  // Kendall: per row of the subset (at its begin), two 64-bit sort buffers
  // and the 32-bit sign counts
  unsigned long long* W0;
  unsigned long long* W1;
  int* C;
  int* flag;  // per subset of the launch (Kendall): 0 done, 1 left to the workspace kernel, 2 sums in W0
};

enum { KIND_SPEARMAN = 0, KIND_KENDALL = 1 };

// rho_S (KIND_SPEARMAN) or tau (KIND_KENDALL) at th and its theta-derivative
// from the workgroup sums v of rho_terms (valid in thread 0).
template <int FAM, int KIND>
__device__ __forceinline__ void moment_value(double th, const double (&v)[4], double& val, double& der) {
  if constexpr (FAM == FAM_GUMBEL) {  // (Spearman only: Kendall's Gumbel is closed form)
    val = v[0] - 3.0;
    der = v[1];
  } else {
    const double A = fabs(th);
    if (A < 1e-2) {
      const double t2 = th * th;
      if constexpr (KIND == KIND_SPEARMAN) {
        val = th * (1.0 / 6.0 - t2 / 450.0 + t2 * t2 / 23520.0);
        der = 1.0 / 6.0 - t2 / 150.0 + t2 * t2 / 4704.0;
      } else {
        val = th * (1.0 / 9.0 - t2 / 900.0 + t2 * t2 / 52920.0);
        der = 1.0 / 9.0 - t2 / 300.0 + t2 * t2 / 10584.0;
      }
    } else {
      const double D1 = v[2] / A, e = 1.0 / expm1(A);
      const double dD1 = -D1 / A + e;
      double ra;
      if constexpr (KIND == KIND_SPEARMAN) {
        const double D2 = 2.0 * v[3] / (A * A), dD2 = -2.0 * D2 / A + 2.0 * e;
        ra = 1.0 - 12.0 * (D1 - D2) / A;
        der = 12.0 * (D1 - D2) / (A * A) - 12.0 * (dD1 - dD2) / A;  // even in theta
      } else {
        ra = 1.0 - 4.0 * (1.0 - D1) / A;
        der = 4.0 * (1.0 - D1) / (A * A) + 4.0 * dD1 / A;  // even in theta
      }
      val = th < 0.0 ? -ra : ra;  // odd in theta
    }
  }
}

// theta in [BLO, BHI] with m(theta) = target (m = rho_S or tau, increasing)
// by safeguarded Newton from th: the workgroup evaluates m and its slope at
// each iterate, thread 0 takes the step and broadcasts it with the stopping
// decision through bc[0..3] (so every thread leaves the loop together). On
// return (every thread): th, slope at the last evaluated iterate, status
// (OK or BOUNDARY_*), it (passes; > 100 means no convergence); fit = m at the
// last iterate (thread 0).
template <int FAM, int KIND, int W>
__device__ void newton_invert(double target, double& th, double& slope, double& fit, int& it, int& status,
                              double* red, double* bc) {
  constexpr double BLO = FAM == FAM_FRANK ? -200.0 : 1.0, BHI = FAM == FAM_FRANK ? 200.0 : 100.0;
  const int t = threadIdx.x;
  double lo = BLO, hi = BHI;  // the bracket (thread 0's copy is the one used)
  if (!(th > BLO && th < BHI)) th = 0.5 * (BLO + BHI);
  for (it = 1; it <= 100; ++it) {
    double f0, f1, f2, f3;
    rho_terms<FAM>(th, f0, f1, f2, f3);
    double v[4] = {f0, f1, f2, f3};
    block_sum<W, 4>(v, red);
    if (t == 0) {
      double val, der;
      moment_value<FAM, KIND>(th, v, val, der);
      const double g = val - target;  // increasing in theta
      int st = ST_OK;
      double done = 0.0, tn = th;
      if (g != 0.0) {  // (an exact root stops at th itself)
        if (g < 0.0) lo = th; else hi = th;
        tn = (der > 0.0) ? th - g / der : NAN;
        if (!(tn > lo && tn < hi)) tn = 0.5 * (lo + hi);
      }
      if (g == 0.0 || fabs(tn - th) <= 1e-12 * (1.0 + fabs(th))) {
        done = 1.0;
      } else if (tn - BLO <= 1e-9 * (1.0 + fabs(BLO))) {
        done = 1.0;
        tn = BLO;
        st = FAM == FAM_GUMBEL ? ST_BOUNDARY_NATURAL : ST_BOUNDARY_BOX;
      } else if (BHI - tn <= 1e-9 * (1.0 + fabs(BHI))) {
        done = 1.0;
        tn = BHI;
        st = ST_BOUNDARY_BOX;
      }
      bc[1] = tn;
      bc[2] = done;
      bc[3] = der;
      bc[0] = (double)st;
      fit = val;
    }
    __syncthreads();
    th = bc[1];
    const bool done = bc[2] != 0.0;
    slope = bc[3];
    status = (int)bc[0];
    __syncthreads();  // bc is written again in the next iteration
    if (done) break;
  }
  if (it > 100) status = ST_NOCONV;
}

// LDSB: the rank bins in LDS (every subset of the launch has at most
// kSpearmanLdsRows rows; dynamic LDS of 8 (n_max + 1) bytes), else in the
// workspace.
template <int FAM, bool LDSB>
__global__ void __launch_bounds__(MT) k_spearman(MomParams P) {
  constexpr int W = MT / WAVE;
  __shared__ double red[W * 4];
  __shared__ long long redl[W];
  __shared__ unsigned int mm[4];
  __shared__ double bc[4];  // broadcast: status, iterate, stop flag, slope
  const int sid = blockIdx.x, t = threadIdx.x;
  const SubDesc sd = P.subs[sid];
  const int64_t n = sd.n, o = sd.begin;
  ResultOut r;
  r.theta = NAN; r.var = NAN; r.loglik = NAN; r.score = NAN;
  r.n = n; r.iters = 0; r.status = ST_OK;
  if (n < P.n_min || n < 2) {
    if (t == 0) { r.status = ST_DEGENERATE; P.out[sid] = r; }
    return;
  }
  const uint32_t* R1 = P.R1 + o;
  const uint32_t* R2 = P.R2 + o;
  const long long n1 = n + 1;

  // rho_S hat (exact integer sum) and whether a margin has a single value
  if (t == 0) { mm[0] = ~0u; mm[1] = 0u; mm[2] = ~0u; mm[3] = 0u; }
  __syncthreads();
  long long s = 0;
  uint32_t a0 = ~0u, a1 = 0u, b0 = ~0u, b1 = 0u;
  for (int64_t i = t; i < n; i += MT) {
    const uint32_t x = R1[i], y = R2[i];
    s += ((long long)x - n1) * ((long long)y - n1);
    a0 = min(a0, x); a1 = max(a1, x); b0 = min(b0, y); b1 = max(b1, y);
  }
  atomicMin(&mm[0], a0); atomicMax(&mm[1], a1); atomicMin(&mm[2], b0); atomicMax(&mm[3], b1);
  const long long S = block_sum_ll<W>(s, redl);
  if (mm[0] == mm[1] || mm[2] == mm[3]) {  // uniform (after the barrier in block_sum_ll)
    if (t == 0) { r.status = ST_DEGENERATE; P.out[sid] = r; }
    return;
  }
  const double dn = (double)n;
  double rho = 0.0;
  if (t == 0) {
    rho = 3.0 * (double)S / (dn * (dn * dn - 1.0));
    bc[0] = rho;
  }
  __syncthreads();
  rho = bc[0];

  // theta with rho_S(theta) = rho
  double th = 0.0, slope = 0.0, fit = 0.0;
  int it = 0, status = ST_OK;
  if constexpr (FAM == FAM_GAUSSIAN) {
    th = 2.0 * sin(3.14159265358979323846 * rho / 6.0);
    const double edge = 1.0 - 1e-9;
    if (fabs(th) >= edge) { status = ST_BOUNDARY_BOX; th = th > 0.0 ? edge : -edge; }
    slope = 3.0 / (3.14159265358979323846 * sqrt(1.0 - 0.25 * th * th));
    fit = 6.0 / 3.14159265358979323846 * asin(0.5 * th);
  } else {
    if (FAM == FAM_GUMBEL && rho <= 0.0) {
      status = ST_BOUNDARY_NATURAL;
      th = 1.0;
    } else {
      th = FAM == FAM_FRANK ? fmin(fmax(6.0 * rho / sqrt(fmax(1.0 - rho * rho, 1e-12)), -150.0), 150.0)
                            : fmin(1.0 / (1.0 - 2.0 / 3.14159265358979323846 *
                                                   asin(fmin(2.0 * sin(3.14159265358979323846 * rho / 6.0), 1.0))),
                                   80.0);
      newton_invert<FAM, KIND_SPEARMAN, W>(rho, th, slope, fit, it, status, red, bc);
    }
    if (status == ST_BOUNDARY_NATURAL) {  // the variance needs the slope at theta = 1
      double f0, f1, f2, f3;
      rho_terms<FAM>(1.0, f0, f1, f2, f3);
      double v[4] = {f0, f1, f2, f3};
      block_sum<W, 4>(v, red);
      if (t == 0) {
        bc[3] = v[1];
        fit = v[0] - 3.0;
      }
      __syncthreads();
      slope = bc[3];
    }
  }

  // variance (OK and at the natural boundary)
  double var = NAN;
  if (status == ST_OK || status == ST_BOUNDARY_NATURAL) {
    // the suffix sums as bins indexed by the doubled rank; distinct tie
    // groups differ by at least 2 in doubled rank, so the bins floor(R / 2)
    // (n + 1 of them) never merge two groups
    const int64_t NH = n + 1;
    const int64_t C = (NH + MT - 1) / MT;
    const int64_t k0 = t * C, k1 = min(k0 + C, NH);
    __shared__ long long tot[2][MT];
    if constexpr (LDSB) {
      // exact int32 sums in LDS (|sum| <= n^2 < 2^31 for n <= 16384), one
      // margin's bins at a time (n + 1 words, so that two workgroups share a
      // CU); each row's u-order term waits in the workspace between the two
      // (the slots of the global-bin path; a thread reads back only its own
      // rows, the second bins stay in LDS for the psi pass below)
      extern __shared__ int hb[];
      double* WU = (double*)(P.H1 + 2 * (o + P.base + sid));
      for (int mg = 0; mg < 2; ++mg) {
        for (int64_t k = t; k < NH; k += MT) hb[k] = 0;
        __syncthreads();
        for (int64_t i = t; i < n; i += MT) {
          const uint32_t x = R1[i], y = R2[i];
          if (mg == 0)
            atomicAdd(&hb[x >> 1], (int)((long long)y - n1));
          else
            atomicAdd(&hb[y >> 1], (int)((long long)x - n1));
        }
        __syncthreads();
        int t1 = 0;
        for (int64_t k = k1 - 1; k >= k0; --k) {
          t1 += hb[k]; hb[k] = t1;
        }
        tot[0][t] = t1;
        __syncthreads();
        int c1 = 0;
        for (int u = t + 1; u < MT; ++u) c1 += (int)tot[0][u];
        for (int64_t k = k0; k < k1; ++k) hb[k] += c1;
        __syncthreads();
        if (mg == 0) {
          for (int64_t i = t; i < n; i += MT) WU[i] = (double)hb[R1[i] >> 1];
          __syncthreads();
        }
      }
    } else {
      long long* H1 = P.H1 + 2 * (o + P.base + sid);
      long long* H2 = P.H2 + 2 * (o + P.base + sid);
      for (int64_t k = t; k < NH; k += MT) { H1[k] = 0; H2[k] = 0; }
      __syncthreads();
      for (int64_t i = t; i < n; i += MT) {
        const uint32_t x = R1[i], y = R2[i];
        atomicAdd((unsigned long long*)&H1[x >> 1], (unsigned long long)((long long)y - n1));
        atomicAdd((unsigned long long*)&H2[y >> 1], (unsigned long long)((long long)x - n1));
      }
      __syncthreads();
      // thread t takes the block of consecutive bins [t*C, (t+1)*C), then
      // adds the totals of the blocks above it
      long long t1 = 0, t2 = 0;
      for (int64_t k = k1 - 1; k >= k0; --k) {
        t1 += H1[k]; H1[k] = t1;
        t2 += H2[k]; H2[k] = t2;
      }
      tot[0][t] = t1;
      tot[1][t] = t2;
      __syncthreads();
      long long c1 = 0, c2 = 0;
      for (int u = t + 1; u < MT; ++u) { c1 += tot[0][u]; c2 += tot[1][u]; }
      for (int64_t k = k0; k < k1; ++k) { H1[k] += c1; H2[k] += c2; }
      __syncthreads();
    }
    const double inv1 = 1.0 / (double)n1;
    const double wsc = 6.0 / (dn * (double)n1);
    KSum<double> sp, sq;
    for (int64_t i = t; i < n; i += MT) {
      const uint32_t x = R1[i], y = R2[i];
      const double J = 3.0 * (double)((long long)x - n1) * (double)((long long)y - n1) * inv1 * inv1;
      double w;
      if constexpr (LDSB) {
        extern __shared__ int hb[];
        w = ((const double*)(P.H1 + 2 * (o + P.base + sid)))[i] + (double)hb[y >> 1];
      } else {
        w = (double)P.H1[2 * (o + P.base + sid) + (x >> 1)] + (double)P.H2[2 * (o + P.base + sid) + (y >> 1)];
      }
      const double psi = J + wsc * w;
      sp.add(psi);
      sq.add(psi * psi);
    }
    double v[2] = {sp.value(), sq.value()};
    block_sum<W, 2>(v, red);
    if (t == 0) {
      const double m = v[0] / dn;
      const double nu = v[1] / dn - m * m;
      var = nu / (dn * slope * slope);
    }
  }
  if (t == 0) {
    r.theta = th;
    r.var = var;
    r.loglik = rho;
    r.score = fit - rho;
    r.iters = it;
    r.status = status;
    if ((status == ST_OK || status == ST_BOUNDARY_NATURAL) && !(var > 0.0 && isfinite(var))) r.status = ST_BADVAR;
    P.out[sid] = r;
  }
}

// V binary searches stepped together (so that their loads overlap):
// cnt[v] = number of entries of a[v][0 .. len[v]) below x[v] (each sorted
// ascending).
template <int V>
__device__ __forceinline__ void lower_counts(const unsigned long long* const (&a)[V], const int (&len)[V],
                                             const unsigned long long (&x)[V], int (&cnt)[V]) {
  int lo[V], hi[V];
#pragma unroll
  for (int v = 0; v < V; ++v) { lo[v] = 0; hi[v] = len[v]; }
  while (true) {
    bool more = false;
    int mid[V];
    unsigned long long val[V];
#pragma unroll
    for (int v = 0; v < V; ++v) {
      mid[v] = (lo[v] + hi[v]) >> 1;
      val[v] = lo[v] < hi[v] ? a[v][mid[v]] : 0ull;
    }
#pragma unroll
    for (int v = 0; v < V; ++v) {
      if (lo[v] < hi[v]) {
        if (val[v] < x[v]) lo[v] = mid[v] + 1; else hi[v] = mid[v];
        more = true;
      }
    }
    if (!more) break;
  }
#pragma unroll
  for (int v = 0; v < V; ++v) cnt[v] = lo[v];
}

// One bottom-up merge level (runs of L entries, L a power of two) of distinct
// 64-bit words from src into dst, KV words per thread at a time. COUNT: the
// words are (value << 32 | position) and every right-run word adds
// 2 ((#left < value) - (#left > value)) to C[position] (the left run holds
// exactly the positions before the right run's).
constexpr int KV = 4;
template <bool COUNT>
__device__ __forceinline__ void merge_level(const unsigned long long* src, unsigned long long* dst, int n, int L,
                                            int lg, int* C) {
  for (int base = threadIdx.x; base < n; base += MT * KV) {
    const unsigned long long* arr[KV];
    int len[KV], cnt[KV], pos[KV];
    unsigned long long w[KV];
    bool right[KV];
#pragma unroll
    for (int v = 0; v < KV; ++v) {
      const int p = base + v * MT;
      pos[v] = p;
      right[v] = false;
      arr[v] = src;
      len[v] = 0;
      w[v] = 0ull;
      if (p < n) {
        const int r = p >> lg, start = r << lg;
        w[v] = src[p];
        if (r & 1) {
          right[v] = true;
          arr[v] = src + (start - L);
          len[v] = L;
        } else {
          const int rs = start + L;
          if (rs < n) {
            arr[v] = src + rs;
            len[v] = min(L, n - rs);
          }
        }
      }
    }
    lower_counts<KV>(arr, len, w, cnt);
#pragma unroll
    for (int v = 0; v < KV; ++v) {
      const int p = pos[v];
      if (p < n) {
        if (right[v]) {
          const int start = (p >> lg) << lg;
          dst[start - L + (p - start) + cnt[v]] = w[v];  // cnt: left words below w, values <= this one's
        } else {
          dst[p + cnt[v]] = w[v];
        }
      }
    }
    if constexpr (COUNT) {
      unsigned long long x[KV];
      int len2[KV], lt[KV];
#pragma unroll
      for (int v = 0; v < KV; ++v) {
        x[v] = (w[v] >> 32) << 32;
        len2[v] = (pos[v] < n && right[v]) ? cnt[v] : 0;
      }
      lower_counts<KV>(arr, len2, x, lt);  // values below this one's
#pragma unroll
      for (int v = 0; v < KV; ++v)
        if (pos[v] < n && right[v]) C[(uint32_t)w[v]] += 2 * (lt[v] - (L - cnt[v]));
    }
  }
}

// tau and theta from the exact sums S1 = sum_i S_i and S2 = sum_i S_i^2, the
// U-statistic variance, and the subset's result (thread 0 writes it)
template <int FAM, int W>
__device__ void kendall_finish(long long S1, long long S2, int n, double* red, double* bc, ResultOut r,
                               ResultOut* out) {
  const int t = threadIdx.x;
  const double dn = (double)n, dn1 = (double)(n - 1);
  double tau = 0.0, zeta = 0.0;
  if (t == 0) {
    tau = (double)S1 / (dn * dn1);
    zeta = (double)S2 / (dn * dn1 * dn1) - tau * tau;
    bc[0] = tau;
  }
  __syncthreads();
  tau = bc[0];
  __syncthreads();

  // theta with tau(theta) = tau
  double th = 0.0, slope = 0.0, fit = 0.0;
  int it = 0, status = ST_OK;
  constexpr double PI = 3.14159265358979323846;
  if constexpr (FAM == FAM_GAUSSIAN) {
    th = sin(0.5 * PI * tau);
    const double edge = 1.0 - 1e-9;
    if (th <= -edge) { status = ST_BOUNDARY_BOX; th = -edge; }
    if (th >= edge) { status = ST_BOUNDARY_BOX; th = edge; }
    slope = 2.0 / (PI * sqrt(1.0 - th * th));
    fit = 2.0 / PI * asin(th);
  } else if constexpr (FAM == FAM_GUMBEL) {
    if (tau <= 0.0) {
      status = ST_BOUNDARY_NATURAL;
      th = 1.0;
    } else if (tau >= 1.0 - 1.0 / 100.0) {
      status = ST_BOUNDARY_BOX;
      th = 100.0;
    } else {
      th = 1.0 / (1.0 - tau);
    }
    slope = 1.0 / (th * th);
    fit = 1.0 - 1.0 / th;
  } else {
    th = fmin(fmax(4.0 * tau / (1.0 - fabs(tau)) + 5.0 * tau, -150.0), 150.0);
    newton_invert<FAM, KIND_KENDALL, W>(tau, th, slope, fit, it, status, red, bc);
  }
  if (t == 0) {
    r.theta = th;
    r.loglik = tau;
    r.score = fit - tau;
    r.iters = it;
    r.status = status;
    if (status == ST_OK || status == ST_BOUNDARY_NATURAL) {
      const double var = 4.0 * zeta / (dn * slope * slope);
      r.var = var;
      if (!(var > 0.0 && isfinite(var))) r.status = ST_BADVAR;
    }
    *out = r;
  }
}

template <int FAM>
__global__ void __launch_bounds__(MT) k_kendall(MomParams P) {
  constexpr int W = MT / WAVE;
  __shared__ double red[W * 4];
  __shared__ long long redl[W];
  __shared__ unsigned int mm[4];
  __shared__ double bc[4];
  const int sid = blockIdx.x, t = threadIdx.x;
  const int flag = P.flag[sid];
  if (flag == 0) return;  // done in LDS (a degenerate subset)
  const SubDesc sd = P.subs[sid];
  const int n = sd.n;
  const int64_t o = sd.begin;
  ResultOut r;
  r.theta = NAN; r.var = NAN; r.loglik = NAN; r.score = NAN;
  r.n = n; r.iters = 0; r.status = ST_OK;
  if (flag == 2) {  // the sums from the LDS kernel
    kendall_finish<FAM, W>((long long)P.W0[o], (long long)P.W0[o + 1], n, red, bc, r, P.out + sid);
    return;
  }
  if (n < P.n_min || n < 2) {
    if (t == 0) { r.status = ST_DEGENERATE; P.out[sid] = r; }
    return;
  }
  const uint32_t* R1 = P.R1 + o;
  const uint32_t* R2 = P.R2 + o;
  unsigned long long* w0 = P.W0 + o;
  unsigned long long* w1 = P.W1 + o;
  int* C = P.C + o;
  // index bits, and the multiplier of a in the (a, b) key (b <= 2n < M)
  const int IB = 32 - __clz(n - 1);
  const unsigned long long M = 2ull * (unsigned long long)n + 2ull;

  // words (a M + b) << IB | row, and whether a margin has a single value
  if (t == 0) { mm[0] = ~0u; mm[1] = 0u; mm[2] = ~0u; mm[3] = 0u; }
  __syncthreads();
  uint32_t a0 = ~0u, a1 = 0u, b0 = ~0u, b1 = 0u;
  for (int i = t; i < n; i += MT) {
    const uint32_t a = R1[i], b = R2[i];
    w0[i] = (((unsigned long long)a * M + b) << IB) | (unsigned long long)i;
    a0 = min(a0, a); a1 = max(a1, a); b0 = min(b0, b); b1 = max(b1, b);
  }
  atomicMin(&mm[0], a0); atomicMax(&mm[1], a1); atomicMin(&mm[2], b0); atomicMax(&mm[3], b1);
  __syncthreads();
  if (mm[0] == mm[1] || mm[2] == mm[3]) {  // workgroup-uniform
    if (t == 0) { r.status = ST_DEGENERATE; P.out[sid] = r; }
    return;
  }

  // 1. the rows in (a, b, row) order
  unsigned long long* src = w0;
  unsigned long long* dst = w1;
  int lg = 0;
  for (int L = 1; L < n; L <<= 1, ++lg) {
    merge_level<false>(src, dst, n, L, lg, nullptr);
    __syncthreads();
    unsigned long long* x = src; src = dst; dst = x;
  }
  // 2. per position p: the runs of equal a and of equal (a, b) around it give
  //    #{same a, b < b_p} and #{same a, b > b_p}; C[p] starts at the terms of
  //    S that do not need the second sort; dst gets (b << 32 | p)
  const unsigned long long imask = (1ull << IB) - 1ull;
  constexpr int PV = 2;  // positions per thread at a time (4 searches each)
  for (int base = t; base < n; base += MT * PV) {
    const unsigned long long* arr[4 * PV];
    int len[4 * PV], cnt[4 * PV];
    unsigned long long x[4 * PV], bv[PV];
#pragma unroll
    for (int v = 0; v < PV; ++v) {
      const int p = base + v * MT;
      unsigned long long a = 0, b = 0, key = 0;
      if (p < n) {
        const unsigned long long w = src[p];
        const int i = (int)(w & imask);
        a = R1[i];
        b = R2[i];
        key = w >> IB;
      }
      bv[v] = b;
      x[4 * v] = (a * M) << IB;             // first of the run of equal a
      x[4 * v + 1] = ((a + 1ull) * M) << IB;  // past it
      x[4 * v + 2] = key << IB;             // first of the run of equal (a, b)
      x[4 * v + 3] = (key + 1ull) << IB;    // past it
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        arr[4 * v + e] = src;
        len[4 * v + e] = p < n ? n : 0;
      }
    }
    lower_counts<4 * PV>(arr, len, x, cnt);
#pragma unroll
    for (int v = 0; v < PV; ++v) {
      const int p = base + v * MT;
      if (p < n) {
        const int A0 = cnt[4 * v], A1 = cnt[4 * v + 1], J0 = cnt[4 * v + 2], J1 = cnt[4 * v + 3];
        C[p] = (n + 1) - (int)bv[v] - (J0 - A0) - (A1 - J1);
        dst[p] = (bv[v] << 32) | (unsigned long long)p;
      }
    }
  }
  __syncthreads();
  // 3. the sign counts: merge sort of (b << 32 | p)
  src = dst;
  dst = (src == w0) ? w1 : w0;
  lg = 0;
  for (int L = 1; L < n; L <<= 1, ++lg) {
    merge_level<true>(src, dst, n, L, lg, C);
    __syncthreads();
    unsigned long long* x = src; src = dst; dst = x;
  }
  // 4. sum S and S^2 (exact)
  long long s1 = 0, s2 = 0;
  for (int p = t; p < n; p += MT) {
    const long long v = C[p];
    s1 += v;
    s2 += v * v;
  }
  const long long S1 = block_sum_ll<W>(s1, redl);
  const long long S2 = block_sum_ll<W>(s2, redl);
  kendall_finish<FAM, W>(S1, S2, n, red, bc, r, P.out + sid);
}

// The Kendall estimator in LDS, for subsets of up to KL rows (1024 threads,
// KE rows each); the others, and subsets with a tie group of more than
// kKendallTieMax rows in the first margin, are flagged for the workspace
// kernel above, which runs after it on the same subsets and takes the
// inversion of the others from their sums S and S^2 (left in the subset's
// first two words of the workspace). Same counts, in 32-bit words:
//   1. the rows in (a, b, row) order without a sort: a histogram of a's bins
//      floor(a / 2) (distinct tie groups never share one) gives each group
//      its first position; the rows of a group (mostly one) are put in
//      (b, row) order by counting, within the group, the (b, row) keys below
//      theirs, which also gives the runs of equal a and of equal (a, b);
//   2. the sign counts by a merge sort of (b << 14 | p) in place: at each
//      level every thread reads its words, finds their destinations and,
//      for right-run words, the left words of smaller value by binary
//      searches stepped together, then after a barrier writes them back and
//      adds 2 (#left < b - #left > b) to C[p].
constexpr int KT = 1024;
constexpr int KL = 16384;
constexpr int KE = KL / KT;
constexpr int kKendallTieMax = 32;

// cnt[v] = number of entries of A[base[v] .. base[v] + len[v]) below x[v]
// (sorted ascending), the V searches stepped together
template <int V>
__device__ __forceinline__ void lds_lower_counts(const uint32_t* A, const int (&base)[V], const int (&len)[V],
                                                 const uint32_t (&x)[V], int (&cnt)[V]) {
  int lo[V], hi[V];
#pragma unroll
  for (int v = 0; v < V; ++v) { lo[v] = base[v]; hi[v] = base[v] + len[v]; }
  while (true) {
    bool more = false;
#pragma unroll
    for (int v = 0; v < V; ++v) {
      if (lo[v] < hi[v]) {
        const int mid = (lo[v] + hi[v]) >> 1;
        if (A[mid] < x[v]) lo[v] = mid + 1; else hi[v] = mid;
        more = true;
      }
    }
    if (!more) break;
  }
#pragma unroll
  for (int v = 0; v < V; ++v) cnt[v] = lo[v] - base[v];
}

template <int FAM>
__global__ void __launch_bounds__(KT) k_kendall_lds(MomParams P) {
  constexpr int W = KT / WAVE;
  static_assert(KL <= (1 << 14) && KE * KT == KL, "positions fit 14 bits");
  __shared__ uint32_t buf[KL];   // group members, then the (b << 14 | p) words
  __shared__ int cv[KL + 1];     // bins (first position << 16 | size), then C
  __shared__ double red[W * 4];
  __shared__ long long redl[W];
  __shared__ unsigned int mm[5];
  __shared__ double bc[4];
  const int sid = blockIdx.x, t = threadIdx.x;
  const SubDesc sd = P.subs[sid];
  const int n = sd.n;
  const int64_t o = sd.begin;
  if (n > KL) {
    if (t == 0) P.flag[sid] = 1;
    return;
  }
  ResultOut r;
  r.theta = NAN; r.var = NAN; r.loglik = NAN; r.score = NAN;
  r.n = n; r.iters = 0; r.status = ST_OK;
  if (n < P.n_min || n < 2) {
    if (t == 0) { r.status = ST_DEGENERATE; P.out[sid] = r; P.flag[sid] = 0; }
    return;
  }
  uint32_t a[KE], b[KE];
  if (t == 0) { mm[0] = ~0u; mm[1] = 0u; mm[2] = ~0u; mm[3] = 0u; mm[4] = 0u; }
  for (int e = t; e <= n; e += KT) cv[e] = 0;
  __syncthreads();
  uint32_t a0 = ~0u, a1 = 0u, b0 = ~0u, b1 = 0u;
#pragma unroll
  for (int k = 0; k < KE; ++k) {
    const int i = t + k * KT;
    a[k] = i < n ? P.R1[o + i] : 0u;
    b[k] = i < n ? P.R2[o + i] : 0u;
    if (i < n) {
      a0 = min(a0, a[k]); a1 = max(a1, a[k]); b0 = min(b0, b[k]); b1 = max(b1, b[k]);
      atomicAdd(&cv[a[k] >> 1], 1);
    }
  }
  atomicMin(&mm[0], a0); atomicMax(&mm[1], a1); atomicMin(&mm[2], b0); atomicMax(&mm[3], b1);
  __syncthreads();
  if (mm[0] == mm[1] || mm[2] == mm[3]) {  // workgroup-uniform
    if (t == 0) { r.status = ST_DEGENERATE; P.out[sid] = r; P.flag[sid] = 0; }
    return;
  }
  // 1. first position of every bin (exclusive scan of the counts, thread t
  //    taking bins [t CB, (t + 1) CB)), packed with the bin's size
  {
    constexpr int CB = (KL + 1 + KT - 1) / KT;
    const int c0 = t * CB;
    int cnt[CB], run = 0, big = 0;
#pragma unroll
    for (int j = 0; j < CB; ++j) {
      cnt[j] = (c0 + j <= n) ? cv[c0 + j] : 0;
      run += cnt[j];
      big = max(big, cnt[j]);
    }
    const int lane = t & (WAVE - 1), w = t / WAVE;
    const uint32_t incl = wave_incl_sum_u32((uint32_t)run);
    if (lane == WAVE - 1) redl[w] = (long long)incl;
    if (big > kKendallTieMax) mm[4] = 1u;
    __syncthreads();
    long long before = 0;
    for (int u = 0; u < w; ++u) before += redl[u];
    int pos = (int)before + (int)(incl - (uint32_t)run);
#pragma unroll
    for (int j = 0; j < CB; ++j) {
      if (c0 + j <= n) cv[c0 + j] = (pos << 16) | cnt[j];
      pos += cnt[j];
    }
  }
  __syncthreads();
  if (mm[4] != 0u) {  // a long tie group: the workspace kernel
    if (t == 0) P.flag[sid] = 1;
    return;
  }
  // the group members, (b << 14 | row), in arrival order
#pragma unroll
  for (int k = 0; k < KE; ++k) {
    const int i = t + k * KT;
    if (i < n) {
      const int slot = atomicAdd(&cv[a[k] >> 1], 1 << 16) >> 16;
      buf[slot] = (b[k] << 14) | (uint32_t)i;
    }
  }
  __syncthreads();
  // each row's position in (a, b, row) order and the first terms of C
  int pos[KE], c[KE];
#pragma unroll
  for (int k = 0; k < KE; ++k) {
    const int i = t + k * KT;
    pos[k] = 0;
    c[k] = 0;
    if (i < n) {
      const int v = cv[a[k] >> 1];
      const int g = v & 0xFFFF, s0 = (v >> 16) - g;
      int less = 0, blt = 0, ble = g;
      if (g > 1) {
        const uint32_t key = (b[k] << 14) | (uint32_t)i;
        ble = 0;
        for (int q = s0; q < s0 + g; ++q) {
          const uint32_t kq = buf[q];
          less += kq < key ? 1 : 0;
          blt += (kq >> 14) < b[k] ? 1 : 0;
          ble += (kq >> 14) <= b[k] ? 1 : 0;
        }
      }
      pos[k] = s0 + less;
      // (n + 1) - b - #{same a, b < b_p} - #{same a, b > b_p}
      c[k] = (n + 1) - (int)b[k] - blt - (g - ble);
    }
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < KE; ++k) {
    const int i = t + k * KT;
    if (i < n) {
      buf[pos[k]] = (b[k] << 14) | (uint32_t)pos[k];
      cv[pos[k]] = c[k];
    }
  }
  __syncthreads();
  // 2. the sign counts: merge sort of (b << 14 | p), in place
  int lg = 0;
  for (int L = 1; L < n; L <<= 1, ++lg) {
    uint32_t wd[KE];
    int base[KE], len[KE], cnt[KE], dst[KE];
    bool right[KE];
#pragma unroll
    for (int k = 0; k < KE; ++k) {
      const int p = t + k * KT;
      wd[k] = 0u;
      base[k] = 0;
      len[k] = 0;
      right[k] = false;
      if (p < n) {
        wd[k] = buf[p];
        const int rr = p >> lg, start = rr << lg;
        if (rr & 1) {
          right[k] = true;
          base[k] = start - L;
          len[k] = L;
        } else if (start + L < n) {
          base[k] = start + L;
          len[k] = min(L, n - start - L);
        }
      }
    }
    lds_lower_counts<KE>(buf, base, len, wd, cnt);
    uint32_t xb[KE];
    int len2[KE], lt[KE];
#pragma unroll
    for (int k = 0; k < KE; ++k) {
      const int p = t + k * KT;
      dst[k] = p + cnt[k];
      if (right[k]) {
        const int start = (p >> lg) << lg;
        dst[k] = start - L + (p - start) + cnt[k];  // cnt: left words below, values <= this one's
      }
      xb[k] = (wd[k] >> 14) << 14;
      len2[k] = (p < n && right[k]) ? cnt[k] : 0;
    }
    lds_lower_counts<KE>(buf, base, len2, xb, lt);  // left values below this one's
    __syncthreads();
#pragma unroll
    for (int k = 0; k < KE; ++k) {
      const int p = t + k * KT;
      if (p < n) {
        buf[dst[k]] = wd[k];
        if (right[k]) cv[wd[k] & 0x3FFFu] += 2 * (lt[k] - (L - cnt[k]));
      }
    }
    __syncthreads();
  }
  // 3. sum S and S^2 (exact)
  long long s1 = 0, s2 = 0;
  for (int p = t; p < n; p += KT) {
    const long long v = cv[p];
    s1 += v;
    s2 += v * v;
  }
  const long long S1 = block_sum_ll<W>(s1, redl);
  const long long S2 = block_sum_ll<W>(s2, redl);
  // the inversion (a Newton iteration with workgroup quadrature for Frank)
  // runs in the workspace kernel, whose small workgroups share a CU
  if (t == 0) {
    P.W0[o] = (unsigned long long)S1;
    P.W0[o + 1] = (unsigned long long)S2;
    P.flag[sid] = 2;
  }
}

}  // namespace

hipError_t launch_kendall(int fam, const uint32_t* R1, const uint32_t* R2, const SubDesc* subs, int64_t base,
                          int64_t K, int64_t n_min, unsigned long long* W0, unsigned long long* W1, int* C,
                          int* flag, ResultOut* out, hipStream_t s) {
  MomParams p = {};
  p.R1 = R1; p.R2 = R2; p.subs = subs + base; p.n_min = n_min; p.base = base;
  p.out = out + base;
  p.W0 = W0; p.W1 = W1; p.C = C; p.flag = flag + base;
  if (K <= 0) return hipSuccess;
  // subsets of up to KL rows in LDS; the rest (flagged) in the workspace
  switch (fam) {
    case FAM_GAUSSIAN: hipLaunchKernelGGL(k_kendall_lds<FAM_GAUSSIAN>, dim3((unsigned)K), dim3(KT), 0, s, p); break;
    case FAM_FRANK: hipLaunchKernelGGL(k_kendall_lds<FAM_FRANK>, dim3((unsigned)K), dim3(KT), 0, s, p); break;
    default: hipLaunchKernelGGL(k_kendall_lds<FAM_GUMBEL>, dim3((unsigned)K), dim3(KT), 0, s, p); break;
  }
  if (hipError_t e = hipGetLastError(); e != hipSuccess) return e;
  switch (fam) {
    case FAM_GAUSSIAN: hipLaunchKernelGGL(k_kendall<FAM_GAUSSIAN>, dim3((unsigned)K), dim3(MT), 0, s, p); break;
    case FAM_FRANK: hipLaunchKernelGGL(k_kendall<FAM_FRANK>, dim3((unsigned)K), dim3(MT), 0, s, p); break;
    default: hipLaunchKernelGGL(k_kendall<FAM_GUMBEL>, dim3((unsigned)K), dim3(MT), 0, s, p); break;
  }
  return hipGetLastError();
}

hipError_t launch_spearman(int fam, const uint32_t* R1, const uint32_t* R2, const SubDesc* subs, int64_t base,
                           int64_t K, int64_t n_min, int64_t n_max, long long* H1, long long* H2, ResultOut* out,
                           hipStream_t s) {
  MomParams p = {};
  p.R1 = R1; p.R2 = R2; p.subs = subs + base; p.n_min = n_min; p.H1 = H1; p.H2 = H2; p.base = base;
  p.out = out + base;
  if (K <= 0) return hipSuccess;
  const dim3 grid((unsigned)K), block(MT);
  if (n_max <= kSpearmanLdsRows) {
    const size_t lds = sizeof(int) * (size_t)(n_max + 1);
    static bool attr = false;  // allow the largest dynamic LDS once per process
    if (!attr) {
      const int most = (int)(sizeof(int) * (kSpearmanLdsRows + 1));
      hipError_t e = hipFuncSetAttribute((const void*)k_spearman<FAM_GAUSSIAN, true>,
                                         hipFuncAttributeMaxDynamicSharedMemorySize, most);
      if (e == hipSuccess)
        e = hipFuncSetAttribute((const void*)k_spearman<FAM_FRANK, true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                most);
      if (e == hipSuccess)
        e = hipFuncSetAttribute((const void*)k_spearman<FAM_GUMBEL, true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                most);
      if (e != hipSuccess) return e;
      attr = true;
    }
    switch (fam) {
      case FAM_GAUSSIAN: hipLaunchKernelGGL((k_spearman<FAM_GAUSSIAN, true>), grid, block, lds, s, p); break;
      case FAM_FRANK: hipLaunchKernelGGL((k_spearman<FAM_FRANK, true>), grid, block, lds, s, p); break;
      default: hipLaunchKernelGGL((k_spearman<FAM_GUMBEL, true>), grid, block, lds, s, p); break;
    }
  } else {
    switch (fam) {
      case FAM_GAUSSIAN: hipLaunchKernelGGL((k_spearman<FAM_GAUSSIAN, false>), grid, block, 0, s, p); break;
      case FAM_FRANK: hipLaunchKernelGGL((k_spearman<FAM_FRANK, false>), grid, block, 0, s, p); break;
      default: hipLaunchKernelGGL((k_spearman<FAM_GUMBEL, false>), grid, block, 0, s, p); break;
    }
  }
  return hipGetLastError();
}

}  // namespace cpc
