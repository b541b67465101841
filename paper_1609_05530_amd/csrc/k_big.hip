// k_big.hip — the streaming path for subsets too large for one workgroup's
// LDS (more than 16384 rows), for the same method (arXiv:1609.05530, Sec. 2.3
// per subset of the partition eq. 14). Every kernel works on fixed tiles of
// 4096 rows drawn from all large subsets at once; per-subset totals are
// formed from per-tile partial sums in tile order (bitwise reproducible).
//
//   ranks (eq. 12):   segmented LSD radix sort in global memory (8-bit
//                     digits: tile histograms, per-subset scan, stable tile
//                     scatter), then tie groups by binary search in sorted order
//   start:            Spearman's rho (+ Gaussian sufficient statistics)
//   solve (eq. 13):   per Newton pass a tile kernel (score, Hessian partials)
//                     and a per-subset FP64 update
//   variance:         per-row score and mixed partials scattered to sorted
//                     position, segmented suffix sums, then the GGR moments
#include <hip/hip_runtime.h>

#include <utility>

#include "kernels.h"
#include "lds_sort.h"
#include "solver.h"

namespace cpc {

constexpr int BT = 256;          // threads per tile workgroup
constexpr int BE = 16;           // elements per thread
constexpr int BTILE = BT * BE;   // rows per tile
static_assert(BT == 256, "one thread per digit value in the scatter pass");

// ---------------------------------------------------------------------------
// Sort

__global__ void __launch_bounds__(256) k_big_zero_flags(BigParams P) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g < P.nsegs) P.flags[g] = 0;
}

// keys (order-preserving) and the row's index within its subset as payload.
template <typename DT>
__global__ void __launch_bounds__(BT) k_big_init(const DT* data, int int_keys, BigParams P, uint32_t* klo,
                                                 uint32_t* khi, uint32_t* val) {
  const int64_t ti = P.xorder[blockIdx.x];
  if (ti < 0) return;  // idle slot (uniform)
  const BigTile t = P.tiles[ti];
  const BigSeg s = P.segs[t.seg];
  int bad = 0;
  for (int i = threadIdx.x; i < t.count; i += BT) {
    const int64_t loc = t.start + i;
    const int64_t c = s.roff + loc;
    val[c] = (uint32_t)loc;
    if (int_keys) {
      klo[c] = ((const uint32_t*)data)[s.begin + loc];
    } else {
      const DT v = data[s.begin + loc];
      bad |= !isfinite(v);
      if constexpr (sizeof(DT) == 8) {
        const uint64_t k = key_of((double)v);
        klo[c] = (uint32_t)k;
        khi[c] = (uint32_t)(k >> 32);
      } else {
        klo[c] = key_of((float)v);
      }
    }
  }
  if (__syncthreads_or(bad) && threadIdx.x == 0) atomicOr(&P.flags[t.seg], 1);
}

__global__ void __launch_bounds__(BT) k_big_hist(const uint32_t* kw, int shift, BigParams P, uint32_t* hist) {
  __shared__ uint32_t h[256];
  const int64_t ti = P.xorder[blockIdx.x];
  if (ti < 0) return;  // idle slot (uniform)
  const BigTile t = P.tiles[ti];
  const BigSeg s = P.segs[t.seg];
  h[threadIdx.x] = 0u;
  __syncthreads();
  for (int i = threadIdx.x; i < t.count; i += BT) atomicAdd(&h[(kw[s.roff + t.start + i] >> shift) & 0xFFu], 1u);
  __syncthreads();
  hist[ti * 256 + threadIdx.x] = h[threadIdx.x];
}

// Per subset: hist[tile][d] <- first destination (subset-local) of the tile's
// elements with digit d (digit-major over the subset, tiles in order).
__global__ void __launch_bounds__(256) k_big_scan(BigParams P, uint32_t* hist) {
  __shared__ uint32_t wt[4];
  const BigSeg s = P.segs[blockIdx.x];
  const int d = threadIdx.x, lane = d & (WAVE - 1), w = d / WAVE;
  uint32_t run = 0;
  for (int k = 0; k < s.ntiles; ++k) {
    uint32_t* hp = hist + (s.tile0 + k) * 256 + d;
    const uint32_t c = *hp;
    *hp = run;
    run += c;
  }
  const uint32_t incl = wave_incl_sum_u32(run);
  if (lane == WAVE - 1) wt[w] = incl;
  __syncthreads();
  uint32_t base = incl - run;
  for (int k = 0; k < w; ++k) base += wt[k];
  for (int k = 0; k < s.ntiles; ++k) hist[(s.tile0 + k) * 256 + d] += base;
}

// Stable scatter of one digit pass: tile-local stable rank by the LDS
// multisplit, global destination from the scanned histograms. The tile is
// first reordered by digit in LDS, so that consecutive lanes write
// consecutive destinations (one contiguous run per digit and tile).
template <int KW>
__global__ void __launch_bounds__(BT) k_big_scatter(const uint32_t* klo, const uint32_t* khi, const uint32_t* val,
                                                    uint32_t* klo_o, uint32_t* khi_o, uint32_t* val_o, int word,
                                                    int shift, int pass, BigParams P, const uint32_t* hist) {
  __shared__ uint16_t cnt[(BT / WAVE) * 256];
  __shared__ uint32_t dtot[256 + 2 + 4];
  __shared__ uint32_t gofs[256];  // global destination minus tile-local position, per digit
  __shared__ uint32_t xk[BTILE], xv[BTILE];
  __shared__ uint32_t xh[KW == 2 ? BTILE : 1];
  const int64_t ti = P.xorder[blockIdx.x];
  if (ti < 0) return;  // idle slot (uniform)
  const BigTile t = P.tiles[ti];
  const BigSeg s = P.segs[t.seg];
  const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE;
  const int n = t.count;
  const int64_t c0 = s.roff + t.start;
  uint32_t d[BE], dst[BE], lo[BE], hi[BE], v[BE];
#pragma unroll
  for (int j = 0; j < BE; ++j) {
    const int e = (w * BE + j) * WAVE + lane;
    lo[j] = 0u; hi[j] = 0u; v[j] = 0u;
    if (e < n) {
      lo[j] = klo[c0 + e];
      if (KW == 2) hi[j] = khi[c0 + e];
      v[j] = val[c0 + e];
    }
    d[j] = (((KW == 2 && word) ? hi[j] : lo[j]) >> shift) & 0xFFu;
  }
  lds_multisplit<BT, BE>(d, n, pass, cnt, dtot, dst);
  gofs[threadIdx.x] = hist[ti * 256 + threadIdx.x] - dtot[threadIdx.x];  // BT == 256 digits
#pragma unroll
  for (int j = 0; j < BE; ++j) {
    const int e = (w * BE + j) * WAVE + lane;
    if (e < n) {
      xk[dst[j]] = lo[j];
      if (KW == 2) xh[dst[j]] = hi[j];
      xv[dst[j]] = v[j];
    }
  }
  __syncthreads();
#pragma unroll 4
  for (int i = threadIdx.x; i < n; i += BT) {
    const uint32_t kl = xk[i];
    const uint32_t kh = (KW == 2) ? xh[i] : 0u;
    const uint32_t dg = (((KW == 2 && word) ? kh : kl) >> shift) & 0xFFu;
    const int64_t g = s.roff + (int64_t)(gofs[dg] + (uint32_t)i);
    klo_o[g] = kl;
    if (KW == 2) khi_o[g] = kh;
    val_o[g] = xv[i];
  }
}

// Tie groups in sorted order -> doubled ranks, sorted positions, group starts
// (all subset-local). A subset of at most kBigChunkMaxRows rows keeps R and the
// group start in sorted order (RS, LS: coalesced) for k_big_unpermute; a
// larger one writes R, E, L at the row's compact index directly; the rank
// entry point writes R at the row's input index.
template <int KW>
__global__ void __launch_bounds__(BT) k_big_ranks(const uint32_t* klo, const uint32_t* khi, const uint32_t* val,
                                                  int ties, BigParams P, uint32_t* R, uint32_t* Eo, uint32_t* Lo,
                                                  uint32_t* R32, uint32_t* RS, uint32_t* LS) {
  const int64_t ti = P.xorder[blockIdx.x];
  if (ti < 0) return;  // idle slot (uniform)
  const BigTile t = P.tiles[ti];
  const BigSeg s = P.segs[t.seg];
  const bool staged = !R32 && s.n <= kBigChunkMaxRows;  // uniform per tile
  const uint32_t* K0 = klo + s.roff;
  const uint32_t* K1 = khi + s.roff;
  auto key = [&](int64_t p) -> uint64_t { return KW == 2 ? (((uint64_t)K1[p] << 32) | K0[p]) : (uint64_t)K0[p]; };
  for (int i = threadIdx.x; i < t.count; i += BT) {
    const int64_t p = t.start + i;
    const uint64_t k = key(p);
    int64_t lb = p, ub = p + 1;
    if (p > 0 && key(p - 1) == k) {  // first position with this key
      int64_t lo = 0, hi = p;
      while (lo < hi) {
        const int64_t m = (lo + hi) >> 1;
        if (key(m) < k) lo = m + 1; else hi = m;
      }
      lb = lo;
    }
    if (p + 1 < s.n && key(p + 1) == k) {  // one past the last
      int64_t lo = p + 1, hi = s.n;
      while (lo < hi) {
        const int64_t m = (lo + hi) >> 1;
        if (key(m) <= k) lo = m + 1; else hi = m;
      }
      ub = lo;
    }
    const uint32_t r = (ties == 1) ? (uint32_t)(2 * (p + 1)) : (uint32_t)(lb + ub + 1);
    if (staged) {
      RS[s.roff + p] = r;
      LS[s.roff + p] = (uint32_t)((ties == 1) ? p : lb);
      if (p == 0 && ub >= s.n) atomicOr(&P.flags[t.seg], 2);
      continue;
    }
    const int64_t row = val[s.roff + p];
    if (R32) {
      R32[s.begin + row] = r;
    } else {
      R[s.roff + row] = r;
      Eo[s.roff + row] = (uint32_t)p;
      Lo[s.roff + row] = (uint32_t)((ties == 1) ? p : lb);
    }
    if (p == 0 && ub >= s.n) atomicOr(&P.flags[t.seg], 2);  // a single value
  }
}

// Sorted order -> row order for one tile of rows of a subset of at most
// kBigChunkMaxRows rows: the workgroup reads the subset's sorted row indices
// (coalesced) and keeps, in LDS, the sorted position of every row of its
// tile; it then writes R, E (that position) and L for its rows contiguously,
// R and L gathered from the sorted-order arrays. The tiles of a subset run on
// one XCD at about the same time (slot order), so these reads are served by
// its L2; this replaces three scattered 4-byte writes per row.
constexpr int UT = 1024;
__global__ void __launch_bounds__(UT) k_big_unpermute(BigParams P, const uint32_t* val, const uint32_t* RS,
                                                      const uint32_t* LS, uint32_t* R, uint32_t* Eo, uint32_t* Lo) {
  __shared__ uint32_t le[kBigTile];
  const int64_t ti = P.xorder[blockIdx.x];
  if (ti < 0) return;  // idle slot (uniform)
  const BigTile t = P.tiles[ti];
  const BigSeg s = P.segs[t.seg];
  if (s.n > kBigChunkMaxRows) return;  // scattered directly by k_big_ranks
  const uint32_t* V = val + s.roff;
  const uint32_t r0 = (uint32_t)t.start, cnt = (uint32_t)t.count;
  const uint32_t n = (uint32_t)s.n;
  constexpr int U = 8;  // loads in flight per thread
  for (uint32_t base = 0; base < n; base += UT * U) {
    uint32_t rows[U];
#pragma unroll
    for (int k = 0; k < U; ++k) {
      const uint32_t p = base + k * UT + threadIdx.x;
      rows[k] = p < n ? V[p] : 0xFFFFFFFFu;
    }
#pragma unroll
    for (int k = 0; k < U; ++k) {
      const uint32_t p = base + k * UT + threadIdx.x;
      const uint32_t d = rows[k] - r0;  // rows below the tile wrap to large values
      if (p < n && d < cnt) le[d] = p;
    }
  }
  __syncthreads();
  const int64_t o = s.roff + (int64_t)r0;
  const uint32_t* RSs = RS + s.roff;
  const uint32_t* LSs = LS + s.roff;
  for (uint32_t i = threadIdx.x; i < cnt; i += UT) {
    const uint32_t p = min(le[i], n - 1u);  // every entry is set (val is a permutation); the clamp keeps reads in bounds regardless
    R[o + i] = RSs[p];
    Eo[o + i] = p;
    Lo[o + i] = LSs[p];
  }
}

// ---------------------------------------------------------------------------
// Per-tile partial sums; per-subset reductions in tile order.

template <int NV, int T = BT>
__device__ __forceinline__ void tile_partials(double (&v)[NV], double* red, double* out) {
  block_sum<T / WAVE, NV>(v, red);
  if (threadIdx.x == 0)
    for (int k = 0; k < NV; ++k) out[k] = v[k];
}

// Spearman numerator (exact integers per tile, summed in double), Gaussian
// S+, S-, and Gumbel's log(-log u), log(-log v) per row.
template <typename CT>
__global__ void __launch_bounds__(BT) k_big_start(BigParams P, const uint32_t* R1, const uint32_t* R2, CT* LX,
                                                  CT* LY, double* part) {
  __shared__ double red[(BT / WAVE) * 3];
  const int64_t ti = P.xorder[blockIdx.x];
  if (ti < 0) return;  // idle slot (uniform)
  const BigTile t = P.tiles[ti];
  const BigSeg s = P.segs[t.seg];
  const uint32_t twon1 = (uint32_t)(2 * (s.n + 1));
  const CT inv = (CT)1 / (CT)twon1;
  long long sp = 0;
  KSum<double> kp, km;
  for (int i = threadIdx.x; i < t.count; i += BT) {
    const int64_t c = s.roff + t.start + i;
    const uint32_t a = R1[c], b = R2[c];
    sp += ((long long)a - (s.n + 1)) * ((long long)b - (s.n + 1));
    if (s.family == FAM_GAUSSIAN) {
      CT z1, z2;
      gauss_z<CT>(a, b, twon1, z1, z2);
      kp.add((double)(z1 + z2) * (double)(z1 + z2));
      km.add((double)(z1 - z2) * (double)(z1 - z2));
    } else if (s.family == FAM_GUMBEL) {
      gumbel_lxy<CT>(a, b, twon1, inv, LX[c], LY[c]);
    }
  }
  double v[3] = {(double)sp, kp.value(), km.value()};
  tile_partials<3>(v, red, part + ti * 5);
}

__global__ void __launch_bounds__(256) k_big_start_update(BigParams P, const double* part, NewtonState* st,
                                                          double tol, int* pending) {
  __shared__ int cnt;
  if (threadIdx.x == 0) cnt = 0;
  __syncthreads();
  int mine = 0;
  for (int g = threadIdx.x; g < P.nsegs; g += blockDim.x) {
    const BigSeg s = P.segs[g];
    NewtonState& S = st[g];
    double sp = 0.0, a = 0.0, b = 0.0;
    for (int k = 0; k < s.ntiles; ++k) {
      const double* q = part + (s.tile0 + k) * 5;
      sp += q[0]; a += q[1]; b += q[2];
    }
    const double dn = (double)s.n;
    const double rho_s = 3.0 * sp / (dn * (dn * dn - 1.0));
    newton_init(S, s.family, start_theta(s.family, rho_s));
    if (P.flags[g] != 0) {
      S.done = 1;
      S.status = (P.flags[g] & 1) ? ST_NONFINITE : ST_DEGENERATE;
      S.theta = NAN;
    } else if (s.n < P.n_min) {
      S.done = 1;
      S.status = ST_DEGENERATE;
      S.theta = NAN;
    } else if (s.family == FAM_GAUSSIAN) {
      gauss_solve(S, dn, a, b, 1e-14);
      P.gsum[2 * g] = a;
      P.gsum[2 * g + 1] = b;
    }
    mine += S.done ? 0 : 1;
  }
  (void)tol;
  atomicAdd(&cnt, mine);
  __syncthreads();
  if (threadIdx.x == 0) *pending = cnt;
}

// One Newton pass: per-tile sums of the score, Hessian and squared score.
template <typename CT>
__global__ void __launch_bounds__(BT) k_big_eval(BigParams P, const uint32_t* R1, const uint32_t* R2, const CT* LX,
                                                 const CT* LY, const NewtonState* st, double* part,
                                                 const int* pending) {
  __shared__ double red[(BT / WAVE) * 3];
  if (*pending == 0) return;  // every subset has converged
  const int64_t ti = P.xorder[blockIdx.x];
  if (ti < 0) return;  // idle slot (uniform)
  const BigTile t = P.tiles[ti];
  const BigSeg s = P.segs[t.seg];
  if (st[t.seg].done) return;  // uniform per tile
  const double th = st[t.seg].theta;
  const uint32_t twon1 = (uint32_t)(2 * (s.n + 1));
  const CT inv = (CT)1 / (CT)twon1;
  const Consts<CT> c = make_consts<CT>(s.family, th);
  double v[3];
  if (sizeof(CT) == 4 && c.use_d) {
    // FP64 rows (Frank near independence or far out, Gumbel next to theta = 1)
    const Consts<double> cd = make_consts<double>(s.family, th);
    const double invd = 1.0 / (double)twon1;
    KSum<double> ks, kh;
    double s2 = 0.0;
    for (int i = threadIdx.x; i < t.count; i += BT) {
      const int64_t q = s.roff + t.start + i;
      double sv, hv;
      if (s.family == FAM_FRANK) {
        frank_rsh<double>(cd, R1[q], R2[q], twon1, invd, sv, hv);
      } else {
        double lx, ly;
        gumbel_lxy<double>(R1[q], R2[q], twon1, invd, lx, ly);
        gumbel_sh(cd.gk, lx, ly, sv, hv);
      }
      ks.add(sv); kh.add(hv); s2 += sv * sv;
    }
    v[0] = ks.value(); v[1] = kh.value(); v[2] = s2;
  } else {
    RowSum<CT> ks, kh;
    CT s2 = (CT)0;
    for (int i = threadIdx.x; i < t.count; i += BT) {
      const int64_t q = s.roff + t.start + i;
      CT sv, hv;
      if (s.family == FAM_FRANK) frank_rsh<CT>(c, R1[q], R2[q], twon1, inv, sv, hv);
      else gumbel_sh(c.gk, LX[q], LY[q], sv, hv);
      ks.add(sv); kh.add(hv); s2 += sv * sv;
    }
    v[0] = ks.value(); v[1] = kh.value(); v[2] = (double)s2;
  }
  tile_partials<3>(v, red, part + ti * 5);
}

__global__ void __launch_bounds__(256) k_big_update(BigParams P, const double* part, NewtonState* st, double tol,
                                                    int max_iter, int fp64, int* pending) {
  __shared__ int cnt;
  if (*pending == 0) return;  // every subset has converged (the count stays 0)
  if (threadIdx.x == 0) cnt = 0;
  __syncthreads();
  int mine = 0;
  for (int g = threadIdx.x; g < P.nsegs; g += blockDim.x) {
    const BigSeg s = P.segs[g];
    NewtonState& S = st[g];
    if (!S.done) {
      double a = 0.0, b = 0.0, c2 = 0.0;
      for (int k = 0; k < s.ntiles; ++k) {
        const double* q = part + (s.tile0 + k) * 5;
        a += q[0]; b += q[1]; c2 += q[2];
      }
      const bool d_rows = fp64 || rows_in_fp64(s.family, S.theta);
      const double noise = 16.0 * (d_rows ? 1.1102230246251565e-16 : 5.9604644775390625e-08);
      newton_update(S, s.family, a, b, c2, tol, noise, max_iter);
    }
    mine += S.done ? 0 : 1;
  }
  atomicAdd(&cnt, mine);
  __syncthreads();
  if (threadIdx.x == 0) *pending = cnt;
}

// ---------------------------------------------------------------------------
// Variance at theta (Sec. 2.3): rows -> score, g1, g2 scattered by sorted
// position; segmented suffix sums; moments of psi; finalisation.

template <typename CT>
__global__ void __launch_bounds__(BT) k_big_var_rows(BigParams P, const uint32_t* R1, const uint32_t* R2,
                                                     const uint32_t* E1, const uint32_t* E2, const NewtonState* st,
                                                     const double* theta_in, CT* A1, CT* A2, CT* S, double* part) {
  __shared__ double red[(BT / WAVE) * 3];
  const int64_t ti = P.xorder[blockIdx.x];
  if (ti < 0) return;  // idle slot (uniform)
  const BigTile t = P.tiles[ti];
  const BigSeg s = P.segs[t.seg];
  const int fam = s.family;
  const double th = theta_in ? theta_in[s.sid] : st[t.seg].theta;
  const bool skip = P.flags[t.seg] != 0 || !isfinite(th);
  const uint32_t twon1 = (uint32_t)(2 * (s.n + 1));
  const CT inv = (CT)1 / (CT)twon1;
  const Consts<CT> c = make_consts<CT>(fam, th);
  const Consts<double> cd = make_consts<double>(fam, th);
  const bool rd = sizeof(CT) == 4 && c.use_d;
  RowSum<CT> kl, ks, k2;
  for (int i = threadIdx.x; i < t.count && !skip; i += BT) {
    const int64_t q = s.roff + t.start + i;
    const uint32_t a = R1[q], b = R2[q];
    CT l, sv, g1, g2;
    if (rd) {
      const double invd = 1.0 / (double)twon1;
      double ld, sd, g1d, g2d;
      if (fam == FAM_FRANK) {
        frank_rfull<double>(cd, a, b, twon1, invd, ld, sd, g1d, g2d);
      } else if (fam == FAM_GUMBEL) {
        double lx, ly;
        gumbel_lxy<double>(a, b, twon1, invd, lx, ly);
        gumbel_rfull<double>(cd, a, b, twon1, invd, lx, ly, ld, sd, g1d, g2d);
      } else {
        double z1, z2;
        gauss_z<double>(a, b, twon1, z1, z2);
        gauss_rfull<double>(cd, z1, z2, ld, sd, g1d, g2d);
      }
      l = (CT)ld; sv = (CT)sd; g1 = (CT)g1d; g2 = (CT)g2d;
    } else if (fam == FAM_FRANK) {
      frank_rfull<CT>(c, a, b, twon1, inv, l, sv, g1, g2);
    } else if (fam == FAM_GUMBEL) {
      CT lx, ly;
      gumbel_lxy<CT>(a, b, twon1, inv, lx, ly);
      gumbel_rfull<CT>(c, a, b, twon1, inv, lx, ly, l, sv, g1, g2);
    } else {
      CT z1, z2;
      gauss_z<CT>(a, b, twon1, z1, z2);
      gauss_rfull<CT>(c, z1, z2, l, sv, g1, g2);
    }
    kl.add(l); ks.add(sv); k2.add(sv * sv);
    A1[s.roff + E1[q]] = g1;
    A2[s.roff + E2[q]] = g2;
    S[q] = sv;
  }
  double v[3] = {kl.value(), ks.value(), k2.value()};
  tile_partials<3>(v, red, part + ti * 5);
}

// Segmented suffix sums of A (by tiles of positions): tile sums, then per
// subset a suffix over tiles, then in-tile suffixes plus the carry. Both tile
// kernels read their tile coalesced.
template <typename CT>
__global__ void __launch_bounds__(BT) k_big_tilesum(BigParams P, const CT* A1, const CT* A2, double* tsum) {
  __shared__ double red[(BT / WAVE) * 2];
  const int64_t ti = P.xorder[blockIdx.x];
  if (ti < 0) return;  // idle slot (uniform)
  const BigTile t = P.tiles[ti];
  const BigSeg s = P.segs[t.seg];
  double a = 0.0, b = 0.0;
  const int64_t c0 = s.roff + t.start;
#pragma unroll 4
  for (int q = threadIdx.x; q < t.count; q += BT) {
    a += (double)A1[c0 + q];
    b += (double)A2[c0 + q];
  }
  double v[2] = {a, b};
  block_sum<BT / WAVE, 2>(v, red);
  if (threadIdx.x == 0) { tsum[2 * ti] = v[0]; tsum[2 * ti + 1] = v[1]; }
}

__global__ void __launch_bounds__(256) k_big_segsuffix(BigParams P, double* tsum) {
  for (int g = blockIdx.x * blockDim.x + threadIdx.x; g < P.nsegs; g += gridDim.x * blockDim.x) {
    const BigSeg s = P.segs[g];
    double ra = 0.0, rb = 0.0;
    for (int k = s.ntiles - 1; k >= 0; --k) {
      double* q = tsum + 2 * (s.tile0 + k);
      const double a = q[0], b = q[1];
      q[0] = ra;  // exclusive: sum of later tiles
      q[1] = rb;
      ra += a;
      rb += b;
    }
  }
}

// In-tile suffix sums: the tile is staged through LDS (coalesced load and
// store; one pad entry per 16 so that each thread's run of BE entries is
// conflict-free), each thread sums its own run in double.
template <typename CT>
__global__ void __launch_bounds__(BT) k_big_tilesuffix(BigParams P, CT* A1, CT* A2, const double* tsum) {
  __shared__ double sc[BT / WAVE];
  __shared__ CT lt[BTILE + BTILE / 16];
  const int64_t ti = P.xorder[blockIdx.x];
  if (ti < 0) return;  // idle slot (uniform)
  const BigTile t = P.tiles[ti];
  const BigSeg s = P.segs[t.seg];
  const int64_t c0 = s.roff + t.start;
  const int q0 = threadIdx.x * BE;
  auto pad = [](int q) { return q + (q >> 4); };
  for (int arr = 0; arr < 2; ++arr) {
    CT* A = arr ? A2 : A1;
#pragma unroll
    for (int k = 0; k < BE; ++k) {
      const int q = k * BT + threadIdx.x;
      if (q < t.count) lt[pad(q)] = A[c0 + q];
    }
    __syncthreads();
    double cs = 0.0;
    for (int i = 0; i < BE; ++i)
      if (q0 + i < t.count) cs += (double)lt[pad(q0 + i)];
    double run = block_excl_suffix<BT / WAVE>(cs, sc) + tsum[2 * ti + arr];
    for (int i = BE - 1; i >= 0; --i) {
      if (q0 + i < t.count) {
        run += (double)lt[pad(q0 + i)];
        lt[pad(q0 + i)] = (CT)run;
      }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < BE; ++k) {
      const int q = k * BT + threadIdx.x;
      if (q < t.count) A[c0 + q] = lt[pad(q)];
    }
    __syncthreads();  // lt is refilled for the second array
  }
}

// Wide workgroups (VT threads per tile): fewer tiles in flight per XCD, so
// that the suffix arrays of the subsets being read stay in its L2.
constexpr int VT = 1024;
template <typename CT>
__global__ void __launch_bounds__(VT) k_big_psi(BigParams P, const CT* A1, const CT* A2, const CT* S,
                                                const uint32_t* L1, const uint32_t* L2, double* part) {
  __shared__ double red[(VT / WAVE) * 2];
  const int64_t ti = P.xorder[blockIdx.x];
  if (ti < 0) return;  // idle slot (uniform)
  const BigTile t = P.tiles[ti];
  const BigSeg s = P.segs[t.seg];
  const double dn = (double)s.n;
  double a = 0.0, b = 0.0;
  if (P.flags[t.seg] == 0) {
    for (int i = threadIdx.x; i < t.count; i += VT) {
      const int64_t q = s.roff + t.start + i;
      const double psi = (double)S[q] + ((double)A1[s.roff + L1[q]] + (double)A2[s.roff + L2[q]]) / dn;
      a += psi;
      b += psi * psi;
    }
  }
  double v[2] = {a, b};
  block_sum<VT / WAVE, 2>(v, red);
  if (threadIdx.x == 0) { part[ti * 5 + 3] = v[0]; part[ti * 5 + 4] = v[1]; }
}

__global__ void __launch_bounds__(256) k_big_finalize(BigParams P, const double* part, const NewtonState* st,
                                                      int var_method, int mode, double* var_out, ResultOut* out) {
  for (int g = blockIdx.x * blockDim.x + threadIdx.x; g < P.nsegs; g += gridDim.x * blockDim.x) {
    const BigSeg s = P.segs[g];
    double v[5] = {0, 0, 0, 0, 0};
    for (int k = 0; k < s.ntiles; ++k)
      for (int j = 0; j < 5; ++j) v[j] += part[(s.tile0 + k) * 5 + j];
    const double dn = (double)s.n;
    const double mpsi = v[3] / dn;
    const double nu = v[4] / dn - mpsi * mpsi;
    const double beta = v[2] / dn;
    double var = (var_method == 1) ? 1.0 / (dn * beta) : nu / (dn * beta * beta);
    if (mode == MODE_VARIANCE) {
      var_out[s.sid] = (P.flags[g] != 0) ? NAN : var;
      continue;
    }
    const NewtonState& S = st[g];
    ResultOut r;
    r.n = s.n;
    r.iters = S.it;
    r.status = S.status;
    if (P.flags[g] != 0) {
      r.theta = NAN; r.var = NAN; r.loglik = NAN; r.score = NAN;
      r.iters = 0;
    } else {
      r.theta = S.theta;
      r.loglik = v[0];
      r.score = v[1];
      if (s.family == FAM_GAUSSIAN) {
        double H;
        r.loglik = gauss_loglik(S.theta, dn, P.gsum[2 * g], P.gsum[2 * g + 1]);
        gauss_score_hess(S.theta, dn, P.gsum[2 * g], P.gsum[2 * g + 1], r.score, H);
      }
      const bool usable = (S.status == ST_OK || S.status == ST_BOUNDARY_NATURAL);
      if (usable && !(var > 0.0 && isfinite(var))) r.status = ST_BADVAR;
      r.var = usable ? var : NAN;
    }
    out[s.sid] = r;
  }
}

// ---------------------------------------------------------------------------
// Host-side drivers (launch sequences); all buffers come from BigBuffers.

static inline unsigned nblk(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

hipError_t big_rank(const BigParams& P, const BigBuffers& B, const void* x, const void* y, int dtype_kw,
                    int int_keys, int ties, uint32_t* R1out, uint32_t* R2out, hipStream_t s, int margins,
                    BigSorted* sorted) {
  if (P.nsegs == 0) return hipSuccess;
  const unsigned nt = (unsigned)P.nslots;  // tile slots in XCD order
  hipLaunchKernelGGL(k_big_zero_flags, dim3(nblk(P.nsegs, 256)), dim3(256), 0, s, P);
  for (int margin = 0; margin < margins; ++margin) {
    const void* data = margin ? y : x;
    uint32_t *klo = B.ka, *khi = B.kb, *val = B.va;
    uint32_t *klo2 = B.kc, *khi2 = B.kd, *val2 = B.vb;
    if (dtype_kw == 2)
      hipLaunchKernelGGL((k_big_init<double>), dim3(nt), dim3(BT), 0, s, (const double*)data, 0, P, klo, khi, val);
    else
      hipLaunchKernelGGL((k_big_init<float>), dim3(nt), dim3(BT), 0, s, (const float*)data, int_keys, P, klo, khi,
                         val);
    const int passes = 4 * dtype_kw;
    for (int pass = 0; pass < passes; ++pass) {
      const int word = pass >> 2, shift = (pass & 3) * 8;
      hipLaunchKernelGGL(k_big_hist, dim3(nt), dim3(BT), 0, s, word ? khi : klo, shift, P, B.hist);
      hipLaunchKernelGGL(k_big_scan, dim3((unsigned)P.nsegs), dim3(256), 0, s, P, B.hist);
      if (dtype_kw == 2)
        hipLaunchKernelGGL((k_big_scatter<2>), dim3(nt), dim3(BT), 0, s, klo, khi, val, klo2, khi2, val2, word, shift,
                           pass, P, B.hist);
      else
        hipLaunchKernelGGL((k_big_scatter<1>), dim3(nt), dim3(BT), 0, s, klo, khi, val, klo2, khi2, val2, word, shift,
                           pass, P, B.hist);
      std::swap(klo, klo2);
      std::swap(khi, khi2);
      std::swap(val, val2);
    }
    if (sorted) {
      sorted->rows = val;
      sorted->klo = klo;
      sorted->khi = khi;
      return hipGetLastError();
    }
    uint32_t* Rm = margin ? B.R2 : B.R1;
    uint32_t* Em = margin ? B.E2 : B.E1;
    uint32_t* Lm = margin ? B.L2 : B.L1;
    uint32_t* R32 = margin ? R2out : R1out;
    // the other ping-pong buffers are free after the last pass: R and group
    // starts in sorted order for the staged subsets
    uint32_t *RS = klo2, *LS = khi2;
    if (dtype_kw == 2)
      hipLaunchKernelGGL((k_big_ranks<2>), dim3(nt), dim3(BT), 0, s, klo, khi, val, ties, P, Rm, Em, Lm, R32, RS,
                         LS);
    else
      hipLaunchKernelGGL((k_big_ranks<1>), dim3(nt), dim3(BT), 0, s, klo, khi, val, ties, P, Rm, Em, Lm, R32, RS,
                         LS);
    if (!R32) hipLaunchKernelGGL(k_big_unpermute, dim3(nt), dim3(UT), 0, s, P, val, RS, LS, Rm, Em, Lm);
  }
  return hipGetLastError();
}

template <typename CT>
static hipError_t big_solve_t(const BigParams& P, const BigBuffers& B, double tol, int max_iter, int fp64,
                              int* pending_host, hipStream_t s) {
  const unsigned nt = (unsigned)P.nslots;  // tile slots in XCD order
  hipLaunchKernelGGL((k_big_start<CT>), dim3(nt), dim3(BT), 0, s, P, B.R1, B.R2, (CT*)B.LX, (CT*)B.LY, B.part);
  hipLaunchKernelGGL(k_big_start_update, dim3(1), dim3(256), 0, s, P, B.part, B.st, tol, B.pending);
  // Newton passes in blocks of 4; the host stops once every subset is done.
  // Without a host flag (graph capture) every pass of the budget is enqueued
  // and the passes after convergence return at once on the device counter.
  for (int it = 0; it < max_iter; it += 4) {
    for (int k = 0; k < 4 && it + k < max_iter; ++k) {
      hipLaunchKernelGGL((k_big_eval<CT>), dim3(nt), dim3(BT), 0, s, P, B.R1, B.R2, (const CT*)B.LX, (const CT*)B.LY,
                         B.st, B.part, B.pending);
      hipLaunchKernelGGL(k_big_update, dim3(1), dim3(256), 0, s, P, B.part, B.st, tol, max_iter, fp64, B.pending);
    }
    if (!pending_host) continue;
    hipError_t e = hipMemcpyAsync(pending_host, B.pending, sizeof(int), hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return e;
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return e;
    if (*pending_host == 0) break;
  }
  return hipGetLastError();
}

template <typename CT>
static hipError_t big_variance_t(const BigParams& P, const BigBuffers& B, const double* theta_in, int var_method,
                                 int mode, double* var_out, ResultOut* out, hipStream_t s) {
  const unsigned nt = (unsigned)P.nslots;  // tile slots in XCD order
  hipLaunchKernelGGL((k_big_var_rows<CT>), dim3(nt), dim3(BT), 0, s, P, B.R1, B.R2, B.E1, B.E2, B.st, theta_in,
                     (CT*)B.A1, (CT*)B.A2, (CT*)B.S, B.part);
  hipLaunchKernelGGL((k_big_tilesum<CT>), dim3(nt), dim3(BT), 0, s, P, (const CT*)B.A1, (const CT*)B.A2, B.tsum);
  hipLaunchKernelGGL(k_big_segsuffix, dim3(nblk(P.nsegs, 256)), dim3(256), 0, s, P, B.tsum);
  hipLaunchKernelGGL((k_big_tilesuffix<CT>), dim3(nt), dim3(BT), 0, s, P, (CT*)B.A1, (CT*)B.A2, B.tsum);
  hipLaunchKernelGGL((k_big_psi<CT>), dim3(nt), dim3(VT), 0, s, P, (const CT*)B.A1, (const CT*)B.A2, (const CT*)B.S,
                     B.L1, B.L2, B.part);
  hipLaunchKernelGGL(k_big_finalize, dim3(nblk(P.nsegs, 256)), dim3(256), 0, s, P, B.part, B.st, var_method, mode,
                     var_out, out);
  return hipGetLastError();
}

hipError_t big_solve(const BigParams& P, const BigBuffers& B, double tol, int max_iter, int fp64, int* pending_host,
                     hipStream_t s) {
  if (P.nsegs == 0) return hipSuccess;
  return fp64 ? big_solve_t<double>(P, B, tol, max_iter, 1, pending_host, s)
              : big_solve_t<float>(P, B, tol, max_iter, 0, pending_host, s);
}

hipError_t big_variance(const BigParams& P, const BigBuffers& B, int fp64, const double* theta_in, int var_method,
                        int mode, double* var_out, ResultOut* out, hipStream_t s) {
  if (P.nsegs == 0) return hipSuccess;
  return fp64 ? big_variance_t<double>(P, B, theta_in, var_method, mode, var_out, out, s)
              : big_variance_t<float>(P, B, theta_in, var_method, mode, var_out, out, s);
}

}  // namespace cpc
