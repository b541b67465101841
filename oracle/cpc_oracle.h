/*
 * cpc_oracle.h — plain FP64 CPU oracle for the partition-and-combine
 * maximum-pseudo-likelihood (MPL) copula estimator of Wei, Kim & Conlon,
 * "Parallel Computing for Copula Parameter Estimation with Big Data:
 * A Simulation Study" (arXiv:1609.05530).
 *
 * TEST INFRASTRUCTURE. Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library. It shares no code,
 * header or table with the GPU library; the numeric codes below are an
 * interface agreement, written out separately on each side.
 */
#ifndef CPC_ORACLE_H
#define CPC_ORACLE_H
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

enum { OR_GAUSSIAN = 0, OR_FRANK = 1, OR_GUMBEL = 2 };
enum { OR_TIES_AVERAGE = 0, OR_TIES_FIRST = 1 };
enum { OR_VAR_GGR = 0, OR_VAR_INVINFO = 1 };
enum {
  OR_OK = 0,
  OR_BOUNDARY_NATURAL = 1, /* Gumbel estimate at theta = 1 */
  OR_BOUNDARY_BOX = 2,     /* estimate at an edge of the search box */
  OR_DEGENERATE = 3,       /* n < n_min or a margin with a single value */
  OR_NONFINITE = 4,        /* NaN or Inf in the subset's data */
  OR_NOCONV = 5,           /* iteration cap reached */
  OR_BADVAR = 6            /* variance not positive and finite */
};

typedef struct {
  int32_t ties;     /* OR_TIES_* */
  int32_t var;      /* OR_VAR_* */
  int32_t max_iter; /* Newton cap after the grid stage */
  int32_t pad;
  double tol;       /* |dtheta| <= tol * (1 + |theta|) */
  int64_t n_min;    /* subsets smaller than this are DEGENERATE (>= 2) */
} or_options;

typedef struct {
  double theta, var, loglik, score;
  int64_t n;
  int32_t iters, status;
} or_subset;

typedef struct {
  double theta, var_combined;
  int64_t n_used, n_excluded;
  int32_t status, pad;
} or_combined;

void or_default_options(or_options* o);

/* Doubled ranks of x[0..n) (eq. 12): R = 2 * rank, so average ties stay integer. */
void or_ranks(const double* x, int64_t n, int32_t ties, int64_t* R);

/* Standard normal quantile z with Phi(z) = p; omp = 1 - p given exactly. */
double or_qnorm(double p, double omp);

/* Per-row log copula density and its derivatives at theta:
 * out[5*i + 0..4] = l, dl/dtheta, d2l/dtheta2, d2l/dtheta du, d2l/dtheta dv. */
void or_logc_derivs(int32_t family, double theta, const double* u, const double* omu,
                    const double* v, const double* omv, int64_t n, double* out);

/* Kendall tau and Spearman rho of the one-parameter families. */
double or_tau(int32_t family, double theta);
double or_rho_s(int32_t family, double theta);
double or_debye(int32_t k, double x);

/* Fit one subset: ranks, MPL maximisation and asymptotic variance. */
void or_fit_subset(const double* x, const double* y, int64_t n, int32_t family,
                   const or_options* opt, or_subset* out);

/* GGR influence terms for one subset at theta, for tests:
 * psi_out[4*i + 0..3] = s_i, W1_i, W2_i, psi_i. Returns the variance. */
double or_ggr(const int64_t* R1, const int64_t* R2, int64_t n, int32_t family, double theta,
              int32_t var_method, double* psi_out);

/* Combine (eq. 15/16) subset results over groups of consecutive subsets. */
void or_combine(const or_subset* sub, const int64_t* group_offsets, int64_t G, or_combined* comb);

/* Whole path: subsets [offsets[m], offsets[m+1]), groups of subsets
 * [group_offsets[g], group_offsets[g+1]) with family_per_group[g]. */
void or_fit(const double* x, const double* y, const int64_t* offsets, int64_t K,
            const int64_t* group_offsets, int64_t G, const int32_t* family_per_group,
            const or_options* opt, int32_t nthreads, or_subset* out, or_combined* comb);

int32_t or_num_threads(int32_t requested);

/* Simulation inputs (Sec. 2.5) and evaluation metrics (Sec. 2.6). */
/* Philox4x32-10 block of a counter and a key (Salmon et al., SC 2011). */
void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
/* Rows row0 .. row0+n-1 of the seeded stream of pairs with N(0,1) margins
 * whose copula is the family's at theta. */
void or_sample(int32_t family, double theta, uint64_t seed, int64_t row0, int64_t n, double* x, double* y);
/* int |c_a - c_b|, int c_a, int (c_a - c_b)^2, int c_a^2 over the unit square
 * (normal-score coordinates, |s|, |t| <= Lbox, composite Gauss-Legendre). */
void or_density_distance(int32_t family, double theta_a, double theta_b, double Lbox, int32_t panels, int32_t m,
                         double out[4]);

/* The inversion of Spearman's rho as an estimator (Sec. 2.3). */
/* rho_S hat of doubled ranks */
double or_spearman(const int64_t* R1, const int64_t* R2, int64_t n);
/* theta with rho_S(theta) = r; status OK, BOUNDARY_NATURAL or BOUNDARY_BOX */
double or_spearman_theta(int32_t family, double r, int32_t* status);
/* variance of the estimate at theta (plug-in sandwich); var(psi) in *nu */
double or_spearman_var(const int64_t* R1, const int64_t* R2, int64_t n, int32_t family, double theta, double* nu);
/* one subset from its doubled ranks (loglik = rho_S hat, score = rho_S(theta) - rho_S hat) */
void or_spearman_fit_ranks(const int64_t* R1, const int64_t* R2, int64_t n, int32_t family, int64_t n_min,
                           or_subset* out);

/* The inversion of Kendall's tau as an estimator (Sec. 2.3). */
/* S_i = sum over l != i of sign(r1_i - r1_l) sign(r2_i - r2_l), all pairs */
void or_kendall_rows(const int64_t* R1, const int64_t* R2, int64_t n, int64_t* S);
/* tau hat of doubled ranks (ties count as neither concordant nor discordant) */
double or_kendall(const int64_t* R1, const int64_t* R2, int64_t n);
/* d tau / d theta */
double or_tau_slope(int32_t family, double theta);
/* theta with tau(theta) = t; status OK, BOUNDARY_NATURAL or BOUNDARY_BOX */
double or_kendall_theta(int32_t family, double t, int32_t* status);
/* variance of the estimate at theta (4 var(k1) / (n tau'^2)); var(k1) in
 * *zeta, tau hat in *tau_hat */
double or_kendall_var(const int64_t* R1, const int64_t* R2, int64_t n, int32_t family, double theta, double* zeta,
                      double* tau_hat);
/* one subset from its doubled ranks (loglik = tau hat, score = tau(theta) - tau hat) */
void or_kendall_fit_ranks(const int64_t* R1, const int64_t* R2, int64_t n, int32_t family, int64_t n_min,
                          or_subset* out);

#ifdef __cplusplus
}
#endif
#endif
