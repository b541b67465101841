// k_var.hip — asymptotic variance of each subset's estimate (arXiv:1609.05530,
// Sec. 2.3, "according to Genest et al. (1995)"), with the subset's pseudo
// log-likelihood and score at the estimate; one workgroup per subset of up
// to 16384 rows. Plug-in Genest-Ghoudi-Rivest sandwich:
//   s_i = dl/dtheta, g1_i = d2l/dtheta du, g2_i = d2l/dtheta dv at (u_i, v_i)
//   W1_i = (1/n) sum_{l : u_l >= u_i} g1_l   (suffix sum in u order; a tie
//          group takes the sum from its first member), W2_i likewise in v
//   psi_i = s_i + W1_i + W2_i
//   sigma^2 = [mean(psi^2) - mean(psi)^2] / (n mean(s^2)^2)
// (or 1 / (n mean(s^2)) for the inverse-information option). The g values
// are scattered to sorted position in LDS and suffix-summed there.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "kernels.h"
#include "solver.h"

namespace cpc {

// LDS index of sorted position q: one pad word after every 16 entries, so
// that threads walking their own 16 consecutive entries hit distinct banks.
__device__ __forceinline__ int pidx(int q) { return q + (q >> 4); }
constexpr int padded(int cap) { return cap + cap / 16; }

// In-place inclusive suffix sums over sorted positions [0, n) of the padded
// array A: A[q] <- sum_{q' >= q} A[q']. Per-thread chunks of E consecutive
// positions, chunk sums and the workgroup scan in double.
template <int T, int E, typename CT>
__device__ __forceinline__ void lds_suffix_sum(CT* A, int n, double* scratch) {
  constexpr int W = T / WAVE;
  const int c0 = threadIdx.x * E;
  double cs = 0.0;
#pragma unroll
  for (int i = 0; i < E; ++i)
    if (c0 + i < n) cs += (double)A[pidx(c0 + i)];
  double run = block_excl_suffix<W>(cs, scratch);
#pragma unroll
  for (int i = E - 1; i >= 0; --i) {
    if (c0 + i < n) {
      run += (double)A[pidx(c0 + i)];
      A[pidx(c0 + i)] = (CT)run;
    }
  }
  __syncthreads();
}

// The same for two arrays at once (the u-order and v-order sums share the
// workgroup scan of their chunk totals).
template <int T, int E, typename CT>
__device__ __forceinline__ void lds_suffix_sum2(CT* A, CT* B, int n, double* scratch) {
  constexpr int W = T / WAVE;
  const int c0 = threadIdx.x * E;
  double ca = 0.0, cb = 0.0;
#pragma unroll
  for (int i = 0; i < E; ++i) {
    if (c0 + i < n) {
      ca += (double)A[pidx(c0 + i)];
      cb += (double)B[pidx(c0 + i)];
    }
  }
  double ra, rb;
  block_excl_suffix2<W>(ca, cb, scratch, ra, rb);
#pragma unroll
  for (int i = E - 1; i >= 0; --i) {
    if (c0 + i < n) {
      ra += (double)A[pidx(c0 + i)];
      A[pidx(c0 + i)] = (CT)ra;
      rb += (double)B[pidx(c0 + i)];
      B[pidx(c0 + i)] = (CT)rb;
    }
  }
  __syncthreads();
}

template <int T, int CAP, typename CT, int FAM, bool ONE = false, int MINW = 1>
__global__ void __launch_bounds__(T, MINW) k_var_wg(VarParams P) {
  constexpr int W = T / WAVE;
  constexpr int E = CAP / T;
  constexpr bool TWO = !ONE && 2 * sizeof(CT) * padded(CAP) <= 144 * 1024;
  __shared__ CT A1[padded(CAP)];
  __shared__ CT A2[TWO ? padded(CAP) : 1];
  __shared__ double red[W * 5];
  const int tid = threadIdx.x;
  const int sid = P.order[blockIdx.x];
  const SubDesc sd = P.subs[sid];
  const int n = sd.n;
  // (thread 0 reads the subset's state again at the end: kept live through
  // the row passes, its fields would be spilled by every thread)
  const int status = P.state[sid].status;
  double theta;
  if (P.mode == MODE_VARIANCE) {
    if (status != ST_OK) {
      if (tid == 0) P.var_out[sid] = NAN;
      return;
    }
    theta = P.theta_in[sid];
  } else {
    if (status == ST_DEGENERATE || status == ST_NONFINITE) {
      if (tid == 0) {
        ResultOut r;
        r.theta = NAN; r.var = NAN; r.loglik = NAN; r.score = NAN;
        r.n = n; r.iters = P.state[sid].iters; r.status = status;
        P.out[sid] = r;
      }
      return;
    }
    theta = P.state[sid].theta;
  }
  const int64_t o = sd.begin;
  // a margin without ties stored only the sorted positions E: they are also
  // the group starts, and the doubled rank is 2E + 2
  const int eqm = P.state[sid].eqmask;
  const bool q1 = (eqm & 1) != 0, q2 = (eqm & 2) != 0;
  const uint16_t* R1base = q1 ? P.rows.E1 : P.rows.R1;
  const uint16_t* R2base = q2 ? P.rows.E2 : P.rows.R2;
  const uint16_t* L1base = q1 ? P.rows.E1 : P.rows.L1;
  const uint16_t* L2base = q2 ? P.rows.E2 : P.rows.L2;
  const uint16_t *R1 = R1base + o, *R2 = R2base + o;
  const uint16_t *E1 = P.rows.E1 + o, *E2 = P.rows.E2 + o;
  const uint16_t *L1 = L1base + o, *L2 = L2base + o;
  auto rank_of = [](uint32_t v, bool from_e) { return from_e ? 2u * v + 2u : v; };
  const uint32_t twon1 = 2u * (uint32_t)(n + 1);
  const CT inv = (CT)1 / (CT)twon1;
  const double dn = (double)n;
  const double idn = 1.0 / dn;  // W1, W2 are means over the subset
  const Consts<CT> c = make_consts<CT>(FAM, theta);
  // Frank near independence (FRANK_SERIES_BELOW <= |theta| < FRANK_F32_MIN_ABS)
  // takes FP32 rows here: the rank of the variance needs no more (the
  // estimate itself came from FP64 rows), and l keeps its relative accuracy
  // in the log1p form, its per-subset constant added in FP64 below
  const bool fsmall = FAM == FAM_FRANK && sizeof(CT) == 4 && fabs(theta) >= FRANK_SERIES_BELOW &&
                      fabs(theta) < FRANK_F32_MIN_ABS;
  const bool rd = sizeof(CT) == 4 && c.use_d && !fsmall;  // FP64 rows near the family boundaries

  // Row arithmetic in RT (CT, or double near the family boundaries), results
  // in CT. The choice is uniform over the workgroup and made once, outside
  // the row loops.
  auto row_eval_ab = [&](auto rt_tag, const Consts<decltype(rt_tag)>& cc, auto form_tag, uint32_t a, uint32_t b,
                         CT& l, CT& s, CT& g1, CT& g2) {
    using RT = decltype(rt_tag);
    constexpr int FORM = decltype(form_tag)::value;
    const RT invr = (RT)1 / (RT)twon1;
    a = rank_of(a, q1);
    b = rank_of(b, q2);
    RT lr, sr, g1r, g2r;
    if constexpr (FAM == FAM_FRANK) {
      frank_rfull<RT, FORM>(cc, a, b, twon1, invr, lr, sr, g1r, g2r);
    } else if constexpr (FAM == FAM_GUMBEL) {
      RT lx, ly;
      gumbel_lxy<RT>(a, b, twon1, invr, lx, ly);
      gumbel_rfull<RT>(cc, a, b, twon1, invr, lx, ly, lr, sr, g1r, g2r);
    } else {
      RT z1, z2;
      gauss_z<RT>(a, b, twon1, z1, z2);
      gauss_rfull<RT>(cc, z1, z2, lr, sr, g1r, g2r);
    }
    l = (CT)lr; s = (CT)sr; g1 = (CT)g1r; g2 = (CT)g2r;
  };

  RowSum<CT> kl, ksc, ks2;
  double psum = 0.0, psq = 0.0;
  CT* S = (CT*)P.rows.S + o;  // per-row score (workspace), then s + W1 (one-array variant)
  auto rows = [&](auto rt_tag, auto form_tag) {
    using RT = decltype(rt_tag);
    using FT = decltype(form_tag);
    // the constants in the row type (the FP64 ones of an FP32 kernel are
    // formed only when its rows are evaluated in double)
    // (theta passes through an empty asm statement so that the FP64
    // constants share no intermediate with the FP32 ones: shared, those
    // stay live through the FP32 row passes and are spilled)
    const Consts<RT> cc = [&]() {
      if constexpr (std::is_same<RT, CT>::value) {
        return c;
      } else {
        double th = theta;
        asm volatile("" : "+v"(th));
        return make_consts<RT>(FAM, th);
      }
    }();
    // FP32 rows after the fit: the theta-free per-row terms the fit kernel
    // left in the workspace (Gaussian normal scores; Gumbel log(-log u),
    // log(-log v)), computed there by the same FP32 code
    constexpr bool ZFAM = FAM != FAM_FRANK && std::is_same<RT, float>::value && sizeof(CT) == 4;
    [[maybe_unused]] const bool zcache = ZFAM && P.mode == MODE_FIT;
    if constexpr (TWO && sizeof(CT) == 4) {
      // FP32 results (rows evaluated in FP32, or in FP64 near the family
      // boundaries): a thread's rows live in registers. The 16-bit row arrays
      // are read as aligned 32-bit words, two rows each (word j of the
      // subset's span, rows 2j - odd and 2j + 1 - odd; the span is at most
      // CAP/2 + 1 words, and the arrays start 256-byte aligned and are padded
      // to a multiple of 256 bytes, so every word read lies inside them);
      // thread t takes words t, t + T, ... Their loads are issued H words at a
      // time, the next H in flight while the current ones are evaluated (H
      // sized so that the rows in flight fit 128 VGPRs); the score s stays in
      // a register until the psi pass, and the tie-group starts for that pass
      // are loaded before the suffix sums.
      constexpr int EW = (CAP / 2 + T) / T;
      constexpr int HF = (std::is_same<RT, double>::value || FAM == FAM_FRANK) ? 1 : 2;
      constexpr int H = EW < HF ? EW : HF;
      const int64_t wlo = o >> 1;
      const int nw = (int)(((o + n + 1) >> 1) - wlo);
      const int odd = (int)(o & 1);
      auto words = [&](const uint16_t* base) { return reinterpret_cast<const uint32_t*>(base) + wlo; };
      const uint32_t *WE1 = words(P.rows.E1), *WE2 = words(P.rows.E2);
      const uint32_t *WR1 = words(R1base), *WR2 = words(R2base);
      const uint32_t *WL1 = words(L1base), *WL2 = words(L2base);
      const float4* ZC4 = reinterpret_cast<const float4*>(P.rows.G);
      const bool need_r = !zcache || FAM == FAM_GUMBEL;
      float sk[2 * EW];
      uint32_t qa[EW], qb[EW], ra[EW], rb[EW];
      float2 zk[ZFAM ? 2 * EW : 1];
      // words h .. h+H-1 (h a constant after unrolling)
      auto load_words = [&](int h) {
#pragma unroll
        for (int j = 0; j < H; ++j) {
          const int k = h + j;
          const int wj = min(tid + k * T, nw - 1);
          qa[k] = WE1[wj];
          qb[k] = WE2[wj];
          ra[k] = need_r ? WR1[wj] : 0u;
          rb[k] = need_r ? WR2[wj] : 0u;
          if constexpr (ZFAM) {
            // the word's two rows are rows 2(wlo + wj) and 2(wlo + wj) + 1 of
            // the 8-byte-per-row cache: one aligned 16-byte load
            const float4 z = zcache ? ZC4[wlo + wj] : make_float4(0.f, 0.f, 0.f, 0.f);
            zk[2 * k] = make_float2(z.x, z.y);
            zk[2 * k + 1] = make_float2(z.z, z.w);
          }
        }
      };
      load_words(0);
#pragma unroll
      for (int h = 0; h < EW; h += H) {
      if (h + H < EW) load_words(h + H);  // the next words are in flight while these are evaluated
#pragma unroll
      for (int j = 0; j < H; ++j) {
        const int k = h + j;
#pragma unroll
        for (int hh = 0; hh < 2; ++hh) {
        const int m = 2 * k + hh;
        const int i = 2 * (tid + k * T) + hh - odd;  // row within the subset
        sk[m] = 0.f;
        if (i >= 0 && i < n) {
          const uint32_t a = (ra[k] >> (16 * hh)) & 0xFFFFu, b = (rb[k] >> (16 * hh)) & 0xFFFFu;
          CT l, s, g1, g2;
          if constexpr (ZFAM) {
            if (zcache) {
              if constexpr (FAM == FAM_GUMBEL)
                gumbel_rfull<CT>(c, rank_of(a, q1), rank_of(b, q2), twon1, inv, zk[m].x, zk[m].y, l, s, g1, g2);
              else
                gauss_rfull<CT>(c, zk[m].x, zk[m].y, l, s, g1, g2);
            } else {
              row_eval_ab(RT{}, cc, FT{}, a, b, l, s, g1, g2);
            }
          } else {
            row_eval_ab(RT{}, cc, FT{}, a, b, l, s, g1, g2);
          }
          if constexpr (FAM != FAM_GAUSSIAN) {  // (the Gaussian's come from Sp, Sm)
            kl.add(l);
            ksc.add(s);
          }
          ks2.add(s * s);
          A1[pidx((int)((qa[k] >> (16 * hh)) & 0xFFFFu))] = g1;
          A2[pidx((int)((qb[k] >> (16 * hh)) & 0xFFFFu))] = g2;
          sk[m] = s;
        }
        }
      }
      }
      uint32_t la[EW], lb[EW];
#pragma unroll
      for (int k = 0; k < EW; ++k) {
        const int wj = min(tid + k * T, nw - 1);
        la[k] = WL1[wj];
        lb[k] = WL2[wj];
      }
      __syncthreads();
      lds_suffix_sum2<T, E, CT>(A1, A2, n, red);
#pragma unroll
      for (int k = 0; k < EW; ++k) {
#pragma unroll
        for (int hh = 0; hh < 2; ++hh) {
          const int i = 2 * (tid + k * T) + hh - odd;
          if (i >= 0 && i < n) {
            const int q1 = (int)((la[k] >> (16 * hh)) & 0xFFFFu), q2 = (int)((lb[k] >> (16 * hh)) & 0xFFFFu);
            const double psi = (double)sk[2 * k + hh] + ((double)A1[pidx(q1)] + (double)A2[pidx(q2)]) * idn;
            psum += psi;
            psq += psi * psi;
          }
        }
      }
    } else if constexpr (TWO) {
      // Rows i = tid, tid + T, ...; the loads of the next two rows are in
      // flight while a row is evaluated (their latency dominates otherwise).
      {
        const int last = n - 1;
        int i1 = min(tid + T, last), i2 = min(tid + 2 * T, last);
        const int i0 = min(tid, last);
        uint32_t r0 = (uint32_t)R1[i0] | ((uint32_t)R2[i0] << 16), q0 = (uint32_t)E1[i0] | ((uint32_t)E2[i0] << 16);
        uint32_t r1 = (uint32_t)R1[i1] | ((uint32_t)R2[i1] << 16), q1 = (uint32_t)E1[i1] | ((uint32_t)E2[i1] << 16);
#pragma unroll 1
        for (int i = tid; i < n; i += T) {
          i2 = min(i + 2 * T, last);
          const uint32_t r2 = (uint32_t)R1[i2] | ((uint32_t)R2[i2] << 16);
          const uint32_t q2 = (uint32_t)E1[i2] | ((uint32_t)E2[i2] << 16);
          CT l, s, g1, g2;
          row_eval_ab(RT{}, cc, FT{}, r0 & 0xFFFFu, r0 >> 16, l, s, g1, g2);
          if constexpr (FAM != FAM_GAUSSIAN) {  // (the Gaussian's come from Sp, Sm)
            kl.add(l);
            ksc.add(s);
          }
          ks2.add(s * s);
          A1[pidx((int)(q0 & 0xFFFFu))] = g1;
          A2[pidx((int)(q0 >> 16))] = g2;
          S[i] = s;
          r0 = r1; q0 = q1; r1 = r2; q1 = q2;
        }
      }
      __syncthreads();
      lds_suffix_sum2<T, E, CT>(A1, A2, n, red);
      {
        const int last = n - 1;
        const int i0 = min(tid, last), i1 = min(tid + T, last);
        CT s0 = S[i0], s1 = S[i1];
        uint32_t l0 = (uint32_t)L1[i0] | ((uint32_t)L2[i0] << 16), l1 = (uint32_t)L1[i1] | ((uint32_t)L2[i1] << 16);
#pragma unroll 1
        for (int i = tid; i < n; i += T) {
          const int i2 = min(i + 2 * T, last);
          const CT s2 = S[i2];
          const uint32_t l2 = (uint32_t)L1[i2] | ((uint32_t)L2[i2] << 16);
          const double psi =
              (double)s0 + ((double)A1[pidx((int)(l0 & 0xFFFFu))] + (double)A2[pidx((int)(l0 >> 16))]) * idn;
          psum += psi;
          psq += psi * psi;
          s0 = s1; l0 = l1; s1 = s2; l1 = l2;
        }
      }
    } else {
      // One suffix array in LDS: g2 waits in the workspace (row order) while
      // the u-order suffix sums are formed and read.
      CT* G2 = (CT*)P.rows.G + o;
      {
        const int last = n - 1;
        int i1 = min(tid + T, last);
        const int i0 = min(tid, last);
        uint32_t r0 = (uint32_t)R1[i0] | ((uint32_t)R2[i0] << 16), e0 = E1[i0];
        uint32_t r1 = (uint32_t)R1[i1] | ((uint32_t)R2[i1] << 16), e1 = E1[i1];
#pragma unroll 1
        for (int i = tid; i < n; i += T) {
          const int i2 = min(i + 2 * T, last);
          const uint32_t r2 = (uint32_t)R1[i2] | ((uint32_t)R2[i2] << 16), e2 = E1[i2];
          CT l, s, g1, g2;
          row_eval_ab(RT{}, cc, FT{}, r0 & 0xFFFFu, r0 >> 16, l, s, g1, g2);
          if constexpr (FAM != FAM_GAUSSIAN) {  // (the Gaussian's come from Sp, Sm)
            kl.add(l);
            ksc.add(s);
          }
          ks2.add(s * s);
          A1[pidx((int)e0)] = g1;
          S[i] = s;
          G2[i] = g2;
          r0 = r1; e0 = e1; r1 = r2; e1 = e2;
        }
      }
      __syncthreads();
      lds_suffix_sum<T, E, CT>(A1, n, red);
      for (int i = tid; i < n; i += T) S[i] = (CT)((double)S[i] + (double)A1[pidx(L1[i])] * idn);
      __syncthreads();
      for (int i = tid; i < n; i += T) A1[pidx(E2[i])] = G2[i];
      __syncthreads();
      lds_suffix_sum<T, E, CT>(A1, n, red);
      for (int i = tid; i < n; i += T) {
        const double psi = (double)S[i] + (double)A1[pidx(L2[i])] * idn;
        psum += psi;
        psq += psi * psi;
      }
    }
  };
  // the Frank form (FP32: scaled below FRANK_SCALED_BELOW, else direct) is
  // fixed per subset, outside the row loops
  using Auto = std::integral_constant<int, -1>;
  if (rd || sizeof(CT) == 8 || FAM != FAM_FRANK)
    rd ? rows(double{}, Auto{}) : rows(CT{}, Auto{});
  else if (fsmall)
    rows(CT{}, std::integral_constant<int, 2>{});
  else if (c.fk.th < (CT)FRANK_SCALED_BELOW)
    rows(CT{}, std::integral_constant<int, 1>{});
  else
    rows(CT{}, std::integral_constant<int, 0>{});
  double v[5] = {kl.value(), ksc.value(), ks2.value(), psum, psq};
  // (the closing barrier is kept: without it the register allocator spills
  // in the row passes of the largest class)
  block_sum<W, 5>(v, red);
  if (tid == 0) {
    const double mpsi = v[3] / dn;
    const double nu = v[4] / dn - mpsi * mpsi;
    const double beta = v[2] / dn;
    const double var = (P.var_method == 1) ? 1.0 / (dn * beta) : nu / (dn * beta * beta);
    if (P.mode == MODE_VARIANCE) {
      P.var_out[sid] = var;
    } else {
      const SubState st = P.state[sid];
      double loglik = v[0], score = v[1];
      if (fsmall) {  // n log(|theta| / E), E = 1 - e^{-|theta|}
        const double a = fabs(st.theta);
        loglik += dn * log(a / -expm1(-a));
      }
      if (FAM == FAM_GAUSSIAN) {  // from the FP64 sufficient statistics
        double H;
        loglik = gauss_loglik(st.theta, dn, st.Sp, st.Sm);
        gauss_score_hess(st.theta, dn, st.Sp, st.Sm, score, H);
      }
      const bool usable = (st.status == ST_OK || st.status == ST_BOUNDARY_NATURAL);
      const int status_out = (usable && !(var > 0.0 && isfinite(var))) ? (int)ST_BADVAR : st.status;
      ResultOut r;
      r.theta = st.theta;
      r.var = usable ? var : NAN;
      r.loglik = loglik;
      r.score = score;
      r.n = n;
      r.iters = st.iters;
      r.status = status_out;
      P.out[sid] = r;
    }
  }
}

// Waves per SIMD asked of the register allocator for FP32 Frank and Gumbel
// results: as many as the workgroup's LDS lets share a CU, up to 4 (128
// VGPRs), so that the rows a thread keeps in registers do not cost
// occupancy. FP64 results and the Gaussian (whose FP64 normal-quantile rows
// near |rho| = 1 need about 200 VGPRs) keep the allocator's default.
template <int T, int CAP, typename CT, int FAM>
constexpr int var_waves_per_simd() {
  if (sizeof(CT) == 8 || FAM == FAM_GAUSSIAN) return 1;
  constexpr int lds = 2 * (int)sizeof(CT) * padded(CAP) + 1024;
  constexpr int wgs = (160 * 1024) / lds;
  constexpr int w = wgs * (T / WAVE) / 4;
  return w < 1 ? 1 : (w > 4 ? 4 : w);
}

template <int T, int CAP, typename CT>
static hipError_t launch_t(int fam, const VarParams& p, int grid, hipStream_t s) {
  if (grid <= 0) return hipSuccess;
  constexpr int MG = var_waves_per_simd<T, CAP, CT, FAM_GAUSSIAN>();
  constexpr int MF = var_waves_per_simd<T, CAP, CT, FAM_FRANK>();
  constexpr int MU = var_waves_per_simd<T, CAP, CT, FAM_GUMBEL>();
  switch (fam) {
    case FAM_GAUSSIAN:
      hipLaunchKernelGGL((k_var_wg<T, CAP, CT, FAM_GAUSSIAN, false, MG>), dim3(grid), dim3(T), 0, s, p);
      break;
    case FAM_FRANK: hipLaunchKernelGGL((k_var_wg<T, CAP, CT, FAM_FRANK, false, MF>), dim3(grid), dim3(T), 0, s, p); break;
    default: hipLaunchKernelGGL((k_var_wg<T, CAP, CT, FAM_GUMBEL, false, MU>), dim3(grid), dim3(T), 0, s, p); break;
  }
  return hipGetLastError();
}

hipError_t launch_var_wg(int cls, int fam, int fp64, const VarParams& p, int grid, hipStream_t s) {
  switch (cls) {
    case 0: return fp64 ? launch_t<64, 512, double>(fam, p, grid, s) : launch_t<64, 512, float>(fam, p, grid, s);
    case 1: return fp64 ? launch_t<256, 2048, double>(fam, p, grid, s) : launch_t<256, 2048, float>(fam, p, grid, s);
    case 2: return fp64 ? launch_t<512, 8192, double>(fam, p, grid, s) : launch_t<512, 8192, float>(fam, p, grid, s);
    case 3: return fp64 ? launch_t<1024, 16384, double>(fam, p, grid, s) : launch_t<1024, 16384, float>(fam, p, grid, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace cpc
