// k_fit.hip — maximisation of the pseudo log-likelihood eq. (13) of
// arXiv:1609.05530 for every subset (Sec. 2.3, "numerically"), one
// workgroup per subset of up to 16384 rows. The subset's rows stay in LDS
// for the whole solve (packed doubled ranks; for Gumbel the theta-free
// log(-log u), log(-log v) instead):
//   - Spearman's rho of the ranks (exact integer sums) seeds the solve;
//   - Gaussian: one pass for S+ = sum (z1 + z2)^2 and S- = sum (z1 - z2)^2,
//     then the FP64 scalar solve on those sufficient statistics;
//   - Frank / Gumbel: safeguarded Newton passes; each pass sums the per-row
//     score and Hessian (FP32 rows with Kahan sums in the FP32-compensated
//     mode, FP64 rows near the family boundaries or in the FP64 mode), the
//     workgroup reduces them in a fixed order and thread 0 takes the FP64
//     Newton step.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "kernels.h"
#include "solver.h"

namespace cpc {

template <int CAP, typename CT, int FAM>
struct FitSmem {
  // Gumbel keeps (log(-log u), log(-log v)) per row when they fit
  static constexpr bool GC = FAM == FAM_GUMBEL && 2 * sizeof(CT) * CAP <= 144 * 1024;
  uint32_t rr[GC ? 1 : CAP];
  CT lx[GC ? CAP : 1];
  CT ly[GC ? CAP : 1];
};

// Waves per SIMD asked of the register allocator: up to 4 (128 VGPRs) where
// the workgroup's LDS lets that many waves share a CU, so that two or more
// subsets run side by side: while one workgroup sits in its reduction and
// serial FP64 Newton update, the other's rows keep the VALU busy.
template <int T, int CAP, typename CT, int FAM>
constexpr int fit_waves_per_simd() {
  constexpr int lds = (int)sizeof(FitSmem<CAP, CT, FAM>) + 1024;  // rows + reduction scratch and solver state
  constexpr int wgs = (160 * 1024) / lds;
  constexpr int w = wgs * (T / WAVE) / 4;
  return w < 1 ? 1 : (w > 4 ? 4 : w);
}

template <int T, int CAP, typename CT, int FAM>
__global__ void __launch_bounds__(T, (fit_waves_per_simd<T, CAP, CT, FAM>())) k_fit_wg(FitParams P) {
  constexpr int W = T / WAVE;
  using SM = FitSmem<CAP, CT, FAM>;
  __shared__ SM sm;
  __shared__ double red[W * 3];
  __shared__ NewtonState nst;
  __shared__ double bc[4];
  const int tid = threadIdx.x;
  const int sid = P.order[blockIdx.x];
  if (P.state[sid].status != ST_OK) return;  // uniform: set by the rank kernel
  const SubDesc sd = P.subs[sid];
  const int n = sd.n;
  const uint32_t twon1 = 2u * (uint32_t)(n + 1);
  const CT inv = (CT)1 / (CT)twon1;
  const double dn = (double)n;

  // The ranks are read as aligned 32-bit words (two rows each: the subset
  // spans at most CAP/2 + 1 words; a row of a word outside the subset is
  // skipped), all of a thread's words issued before any is used (the loop
  // body is too short to hide HBM latency otherwise). The rank arrays start
  // 256-byte aligned and are padded to a multiple of 256 bytes, so every word
  // read lies inside them.
  constexpr int EW = (CAP / 2 + T) / T;
  const int64_t wlo = sd.begin >> 1;
  const int nw = (int)(((sd.begin + n + 1) >> 1) - wlo);
  const int odd = (int)(sd.begin & 1);
  // a margin without ties stored only the sorted positions E (its doubled
  // rank is 2E + 2)
  const int eqm = P.state[sid].eqmask;
  const bool q1 = (eqm & 1) != 0, q2 = (eqm & 2) != 0;
  const uint32_t* W1 = reinterpret_cast<const uint32_t*>(q1 ? P.rows.E1 : P.rows.R1) + wlo;
  const uint32_t* W2 = reinterpret_cast<const uint32_t*>(q2 ? P.rows.E2 : P.rows.R2) + wlo;
  uint32_t wa[EW], wb[EW];
#pragma unroll
  for (int k = 0; k < EW; ++k) {
    const int j = min(tid + k * T, nw - 1);
    wa[k] = W1[j];
    wb[k] = W2[j];
  }
  long long sacc = 0;
#pragma unroll
  for (int k = 0; k < EW; ++k) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int i = 2 * (tid + k * T) + h - odd;  // row within the subset
      if (i >= 0 && i < n) {
        uint32_t a = (wa[k] >> (16 * h)) & 0xFFFFu, b = (wb[k] >> (16 * h)) & 0xFFFFu;
        a = q1 ? 2u * a + 2u : a;
        b = q2 ? 2u * b + 2u : b;
        sacc += ((long long)a - (n + 1)) * ((long long)b - (n + 1));
        if constexpr (SM::GC) {
          CT lx, ly;
          gumbel_lxy<CT>(a, b, twon1, inv, lx, ly);
          sm.lx[i] = lx;
          sm.ly[i] = ly;
          // FP32 rows: also left in the workspace for the variance kernel
          if constexpr (sizeof(CT) == 4) ((float2*)P.rows.G + sd.begin)[i] = make_float2(lx, ly);
        } else {
          sm.rr[i] = a | (b << 16);
        }
      }
    }
  }
  // only thread 0 reads the sums; the barrier after its update closes each
  // reduction before the scratch is written again
  const long long S = block_sum_ll<W, false>(sacc, (long long*)red);
  if (tid == 0) {
    const double rho_s = 3.0 * (double)S / (dn * (dn * dn - 1.0));
    newton_init(nst, FAM, start_theta(FAM, rho_s));
    bc[0] = rho_s;
  }
  __syncthreads();

  if constexpr (FAM == FAM_GAUSSIAN) {
    // z in double for near-perfect dependence (S- then needs the digits).
    // FP32 rows leave their normal scores in the workspace for the variance
    // kernel (which otherwise evaluates the same two quantiles per row again).
    const bool zd = sizeof(CT) == 4 && fabs(bc[0]) > 0.98;
    float2* ZC = (float2*)P.rows.G + sd.begin;
    double v[2];
    if (zd) {
      KSum<double> kp, km;
      for (int i = tid; i < n; i += T) {
        const uint32_t r = sm.rr[i];
        double z1, z2;
        gauss_z<double>(r & 0xFFFFu, r >> 16, twon1, z1, z2);
        kp.add((z1 + z2) * (z1 + z2));
        km.add((z1 - z2) * (z1 - z2));
        float f1, f2;
        gauss_z<float>(r & 0xFFFFu, r >> 16, twon1, f1, f2);
        ZC[i] = make_float2(f1, f2);
      }
      v[0] = kp.value();
      v[1] = km.value();
    } else {
      RowSum<CT> kp, km;
      for (int i = tid; i < n; i += T) {
        const uint32_t r = sm.rr[i];
        CT z1, z2;
        gauss_z<CT>(r & 0xFFFFu, r >> 16, twon1, z1, z2);
        kp.add((z1 + z2) * (z1 + z2));
        km.add((z1 - z2) * (z1 - z2));
        if constexpr (sizeof(CT) == 4) ZC[i] = make_float2(z1, z2);
      }
      v[0] = kp.value();
      v[1] = km.value();
    }
    block_sum<W, 2, false>(v, red);
    if (tid == 0) {
      gauss_solve(nst, dn, v[0], v[1], 1e-14);
      SubState& st = P.state[sid];
      st.theta = nst.theta;
      st.iters = nst.it;
      st.status = nst.status;
      st.Sp = v[0];
      st.Sm = v[1];
    }
    return;
  } else {
    for (;;) {
      const double th = nst.theta;
      const Consts<CT> c = make_consts<CT>(FAM, th);
      double v[3];
      double noise;
      if (sizeof(CT) == 4 && c.use_d) {
        // FP64 rows (Frank near independence or far out, Gumbel next to
        // theta = 1)
        const Consts<double> cd = make_consts<double>(FAM, th);
        const double invd = 1.0 / (double)twon1;
        KSum<double> ks, kh;
        double s2 = 0.0;
        if constexpr (FAM == FAM_GUMBEL) {
          // log(-log u), log(-log v) in FP64 from the ranks in the workspace
          // (the LDS holds the FP32 ones), read as the aligned words above
          for (int j = tid; j < nw; j += T) {
            const uint32_t w1 = W1[j], w2 = W2[j];
#pragma unroll 1
            for (int hh = 0; hh < 2; ++hh) {
              const int i = 2 * j + hh - odd;
              if (i >= 0 && i < n) {
                uint32_t a = (w1 >> (16 * hh)) & 0xFFFFu, b = (w2 >> (16 * hh)) & 0xFFFFu;
                a = q1 ? 2u * a + 2u : a;
                b = q2 ? 2u * b + 2u : b;
                double lx, ly, s, h;
                gumbel_lxy<double>(a, b, twon1, invd, lx, ly);
                gumbel_sh(cd.gk, lx, ly, s, h);
                s2 += s * s;
                ks.add(s);
                kh.add(h);
              }
            }
          }
        } else {
        // rows i and i + T added in pairs before the compensated sums
        for (int i = tid; i < n; i += 2 * T) {
          uint32_t r = sm.rr[i];
          double s, h;
          frank_rsh<double>(cd, r & 0xFFFFu, r >> 16, twon1, invd, s, h);
          s2 += s * s;
          if (i + T < n) {
            r = sm.rr[i + T];
            double sb, hb;
            frank_rsh<double>(cd, r & 0xFFFFu, r >> 16, twon1, invd, sb, hb);
            s2 += sb * sb;
            s += sb;
            h += hb;
          }
          ks.add(s);
          kh.add(h);
        }
        }
        v[0] = ks.value();
        v[1] = kh.value();
        v[2] = s2;
        noise = 16.0 * 1.1102230246251565e-16;
      } else {
        // the Frank form (scaled / direct) is fixed per pass, outside the row loop
        auto pass = [&](auto form_tag) {
          constexpr int FORM = decltype(form_tag)::value;
          RowSum<CT> ks, kh;
          CT s2 = (CT)0;
          auto row = [&](int i, CT& s, CT& h) {
            if constexpr (FAM == FAM_FRANK) {
              const uint32_t r = sm.rr[i];
              frank_rsh<CT, FORM>(c, r & 0xFFFFu, r >> 16, twon1, inv, s, h);
            } else if constexpr (SM::GC) {
              gumbel_sh(c.gk, sm.lx[i], sm.ly[i], s, h);
            } else {
              const uint32_t r = sm.rr[i];
              CT lx, ly;
              gumbel_lxy<CT>(r & 0xFFFFu, r >> 16, twon1, inv, lx, ly);
              gumbel_sh(c.gk, lx, ly, s, h);
            }
          };
          // rows i and i + T: their terms are added in pairs, each pair
          // entering the compensated sums once
          for (int i = tid; i < n; i += 2 * T) {
            CT s, h;
            row(i, s, h);
            s2 += s * s;
            if (i + T < n) {
              CT sb, hb;
              row(i + T, sb, hb);
              s2 += sb * sb;
              s += sb;
              h += hb;
            }
            ks.add(s);
            kh.add(h);
          }
          v[0] = ks.value();
          v[1] = kh.value();
          v[2] = (double)s2;
        };
        const bool scaled = FAM == FAM_FRANK && sizeof(CT) == 4 && c.fk.th < (CT)FRANK_SCALED_BELOW;
        if (FAM != FAM_FRANK || sizeof(CT) == 8)
          pass(std::integral_constant<int, -1>{});
        else if (scaled)
          pass(std::integral_constant<int, 1>{});
        else
          pass(std::integral_constant<int, 0>{});
        noise = 16.0 * (sizeof(CT) == 4 ? 5.9604644775390625e-08 : 1.1102230246251565e-16);
      }
      block_sum<W, 3, false>(v, red);
      if (tid == 0) newton_update(nst, FAM, v[0], v[1], v[2], P.tol, noise, P.max_iter);
      __syncthreads();
      if (nst.done) break;
    }
    if (tid == 0) {
      SubState& st = P.state[sid];
      st.theta = nst.theta;
      st.iters = nst.it;
      st.status = nst.status;
      st.Sp = 0.0;
      st.Sm = 0.0;
    }
  }
}

template <int T, int CAP, typename CT>
static hipError_t launch_t(int fam, const FitParams& p, int grid, hipStream_t s) {
  if (grid <= 0) return hipSuccess;
  switch (fam) {
    case FAM_GAUSSIAN: hipLaunchKernelGGL((k_fit_wg<T, CAP, CT, FAM_GAUSSIAN>), dim3(grid), dim3(T), 0, s, p); break;
    case FAM_FRANK: hipLaunchKernelGGL((k_fit_wg<T, CAP, CT, FAM_FRANK>), dim3(grid), dim3(T), 0, s, p); break;
    default: hipLaunchKernelGGL((k_fit_wg<T, CAP, CT, FAM_GUMBEL>), dim3(grid), dim3(T), 0, s, p); break;
  }
  return hipGetLastError();
}

// Threads per subset by size class: the LDS rows of a class-3 subset (64 KiB)
// allow two workgroups per CU, of a class-2 subset four; 512 and 256 threads
// then fill a CU with 16 waves. (The rank kernel's class shapes are separate.)
hipError_t launch_fit_wg(int cls, int fam, int fp64, const FitParams& p, int grid, hipStream_t s) {
  switch (cls) {
    case 0: return fp64 ? launch_t<64, 512, double>(fam, p, grid, s) : launch_t<64, 512, float>(fam, p, grid, s);
    case 1: return fp64 ? launch_t<256, 2048, double>(fam, p, grid, s) : launch_t<256, 2048, float>(fam, p, grid, s);
    case 2: return fp64 ? launch_t<256, 8192, double>(fam, p, grid, s) : launch_t<256, 8192, float>(fam, p, grid, s);
    case 3: return fp64 ? launch_t<512, 16384, double>(fam, p, grid, s) : launch_t<512, 16384, float>(fam, p, grid, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace cpc
