"""The k-dimensional Gaussian copula of eq. (7) of arXiv:1609.05530 fitted by
maximum pseudo-likelihood on every subset, with the rank-based sandwich
variance and the combination of eq. (15) applied to each parameter: the
multi-parameter extension that Sec. 4 leaves as future work.

TEST INFRASTRUCTURE, like ``oracle.py``: only the test suite,
``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` may import
it. Plain numpy in FP64; the normal quantiles come from the C oracle.

Parameters: the p = k (k - 1) / 2 correlations r_jl (j < l) of R, in the
order (0,1), (0,2), ..., (0,k-1), (1,2), ..., (k-2,k-1).

Per subset of n rows (doubled ranks R_ij, eq. (12): u = R / (2 (n + 1))):
  z_ij = Phi^-1(u_ij); G = sum_i z_i z_i' (k x k);
  l(R) = sum_i log c(u_i; R) = -(n/2) log det R - (1/2) tr((R^-1 - I) G)
      (eq. (7): c(u; R) = det(R)^(-1/2) exp(-(1/2) z' (R^-1 - I) z));
  with P = R^-1 and M = P G P: dl/dr_jl = -n P_jl + M_jl and
  d2l/dr_jl dr_st = n (P_js P_tl + P_jt P_sl)
                    - (P_js M_tl + P_jt M_sl + M_js P_tl + M_jt P_sl);
  Newton from the normalised Gram matrix, halving a step until R stays
  positive definite, to max |step| <= 1e-12 (1 + max |r|);
  variance (Sec. 2.3's plug-in sandwich for a parameter vector): per row
  psi_i = s_i + sum_m W_m(u_im), s_i,jl = -P_jl + y_ij y_il (y_i = P z_i),
  W_m(u_im) = (1/n) sum over rows l with u_lm >= u_im (a tie group takes the
  whole group) of ds_l / du_m, where ds_jl/du_m = (P_jm y_l + y_j P_lm) / phi(z_m);
  Omega = cov(psi), J = (1/n) sum_i s_i s_i' (the information as the mean
  outer product of the scores, the reading the one-parameter variance takes:
  beta = mean(s^2)), V = J^-1 Omega J^-1 / n; each parameter's variance is
  V_qq.
"""
from __future__ import annotations

import numpy as np

from . import oracle as O

OK, BOUNDARY_BOX, DEGENERATE, NOCONV, BADVAR = 0, 2, 3, 5, 6


def pairs(k: int):
    return [(j, l) for j in range(k) for l in range(j + 1, k)]


def corr_matrix(theta: np.ndarray, k: int) -> np.ndarray:
    Rm = np.eye(k)
    for q, (j, l) in enumerate(pairs(k)):
        Rm[j, l] = Rm[l, j] = theta[q]
    return Rm


def normal_scores(R: np.ndarray) -> np.ndarray:
    """z = Phi^-1(R / (2 (n + 1))) of the doubled ranks R (n x k)."""
    n = R.shape[0]
    den = 2.0 * (n + 1)
    R = np.asarray(R, dtype=np.float64)
    return O.qnorm((R / den).ravel(), ((den - R) / den).ravel()).reshape(R.shape)


def loglik(Rm: np.ndarray, G: np.ndarray, n: int) -> float:
    """Sum over rows of log c(u_i; R) (eq. (7))."""
    _, logdet = np.linalg.slogdet(Rm)
    P = np.linalg.inv(Rm)
    return -0.5 * n * logdet - 0.5 * float(np.trace((P - np.eye(len(Rm))) @ G))


def grad_hess(Rm: np.ndarray, G: np.ndarray, n: int):
    k = len(Rm)
    P = np.linalg.inv(Rm)
    M = P @ G @ P
    prs = pairs(k)
    g = np.array([-n * P[j, l] + M[j, l] for j, l in prs])
    H = np.empty((len(prs), len(prs)))
    for a, (j, l) in enumerate(prs):
        for b, (s, t) in enumerate(prs):
            H[a, b] = (n * (P[j, s] * P[t, l] + P[j, t] * P[s, l])
                       - (P[j, s] * M[t, l] + P[j, t] * M[s, l] + M[j, s] * P[t, l] + M[j, t] * P[s, l]))
    return g, H


def _is_pd(A: np.ndarray) -> bool:
    try:
        np.linalg.cholesky(A)
        return True
    except np.linalg.LinAlgError:
        return False


def mpl(G: np.ndarray, n: int, max_iter: int = 100):
    """(theta, iterations, status) maximising l(R) from the normalised Gram matrix."""
    k = len(G)
    d = np.sqrt(np.diag(G))
    R0 = G / np.outer(d, d)
    theta = np.array([R0[j, l] for j, l in pairs(k)])
    if not _is_pd(corr_matrix(theta, k)):
        return theta, 0, BOUNDARY_BOX
    for it in range(1, max_iter + 1):
        g, H = grad_hess(corr_matrix(theta, k), G, n)
        if not _is_pd(-H):
            return theta, it, NOCONV
        step = np.linalg.solve(-H, g)
        lam = 1.0
        for _ in range(30):
            if _is_pd(corr_matrix(theta + lam * step, k)):
                break
            lam *= 0.5
        new = theta + lam * step
        done = np.max(np.abs(lam * step)) <= 1e-12 * (1.0 + np.max(np.abs(theta)))
        theta = new
        if done:
            return theta, it, OK
    return theta, max_iter, NOCONV


def _suffix_by_rank(r: np.ndarray, V: np.ndarray) -> np.ndarray:
    """Row i: the sum of V over the rows l with r_l >= r_i."""
    vals, inv = np.unique(r, return_inverse=True)
    per = np.zeros((len(vals), V.shape[1]))
    np.add.at(per, inv, V)
    suf = np.cumsum(per[::-1], axis=0)[::-1]
    return suf[inv]


def variance(R: np.ndarray, Z: np.ndarray, theta: np.ndarray):
    """(V (p x p), Omega) of the estimate theta."""
    n, k = Z.shape
    Rm = corr_matrix(theta, k)
    P = np.linalg.inv(Rm)
    prs = pairs(k)
    Y = Z @ P
    S = np.stack([-P[j, l] + Y[:, j] * Y[:, l] for j, l in prs], axis=1)
    Psi = S.copy()
    phi = np.exp(-0.5 * Z * Z) / np.sqrt(2.0 * np.pi)
    for m in range(k):
        A = _suffix_by_rank(R[:, m], Y / phi[:, m:m + 1]) / n
        for q, (j, l) in enumerate(prs):
            Psi[:, q] += P[j, m] * A[:, l] + A[:, j] * P[l, m]
    mu = Psi.mean(axis=0)
    Omega = Psi.T @ Psi / n - np.outer(mu, mu)
    Jinv = np.linalg.inv(S.T @ S / n)
    return Jinv @ Omega @ Jinv / n, Omega


def fit_subset(R: np.ndarray, n_min: int = 2):
    """One subset (R: n x k doubled ranks): (theta (p), var (p), loglik, score (p), iters, status)."""
    n, k = R.shape
    p = k * (k - 1) // 2
    nan = np.full(p, np.nan)
    if n < max(n_min, k + 1, 2) or any(np.all(R[:, j] == R[0, j]) for j in range(k)):
        return nan, nan, np.nan, nan, 0, DEGENERATE
    Z = normal_scores(R)
    G = Z.T @ Z
    theta, it, st = mpl(G, n)
    if st != OK:
        return theta, nan, np.nan, nan, it, st
    Rm = corr_matrix(theta, k)
    g, _ = grad_hess(Rm, G, n)
    V, _ = variance(R, Z, theta)
    var = np.diag(V).copy()
    if not np.all(np.isfinite(var)) or np.any(var <= 0.0):
        st = BADVAR
    return theta, var, loglik(Rm, G, n), g, it, st


def fit_ranks(R: np.ndarray, offsets, group_offsets=None, n_min: int = 2):
    """Every subset of the doubled ranks R (n x k), and eq. (15) per group and
    parameter. Returns (sub, comb): sub a (p, K) SUBSET_DTYPE array (entry
    [q, m]: parameter q of subset m), comb a (p, G) COMBINED_DTYPE array."""
    R = np.asarray(R)
    k = R.shape[1]
    p = k * (k - 1) // 2
    offsets = np.asarray(offsets, dtype=np.int64)
    K = len(offsets) - 1
    if group_offsets is None:
        group_offsets = np.array([0, K], dtype=np.int64)
    group_offsets = np.asarray(group_offsets, dtype=np.int64)
    sub = np.zeros((p, K), dtype=O.SUBSET_DTYPE)
    for m in range(K):
        a, b = offsets[m], offsets[m + 1]
        theta, var, ll, score, it, st = fit_subset(R[a:b], n_min)
        for q in range(p):
            sub[q, m] = (theta[q], var[q], ll, score[q], b - a, it, st)
    comb = np.stack([O.combine(sub[q], group_offsets) for q in range(p)])
    return sub, comb
