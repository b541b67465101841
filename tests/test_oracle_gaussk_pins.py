"""Pins of the oracle's k-dimensional Gaussian copula (eq. (7)) fitted by
maximum pseudo-likelihood: the log-likelihood against scipy's multivariate
normal density, its gradient and Hessian against central differences of
that scipy form, the maximiser against scipy's optimiser, the reduction to
the (separately pinned) bivariate Gaussian fit and its GGR variance at
k = 2, the sandwich variance against the spread of estimates over
replicates, and the statuses."""
import numpy as np
import pytest
from scipy import optimize, stats

import oracle.oracle as O
from oracle import gaussk as GK

R3 = np.array([[1.0, 0.5, 0.3], [0.5, 1.0, -0.2], [0.3, -0.2, 1.0]])
R4 = np.array([[1.0, 0.6, 0.2, -0.3], [0.6, 1.0, 0.1, 0.0], [0.2, 0.1, 1.0, 0.4], [-0.3, 0.0, 0.4, 1.0]])


def draw(Rm, n, seed):
    rng = np.random.default_rng(seed)
    X = rng.multivariate_normal(np.zeros(len(Rm)), Rm, size=n)
    return np.stack([O.ranks(X[:, j]) for j in range(len(Rm))], axis=1), X


def scipy_loglik(Rm, Z):
    return float(np.sum(stats.multivariate_normal(np.zeros(len(Rm)), Rm).logpdf(Z))
                 - np.sum(stats.norm.logpdf(Z)))


def test_loglik_against_scipy():
    R, _ = draw(R4, 300, 1)
    Z = GK.normal_scores(R)
    for Rm in (R4, np.eye(4), 0.7 * R4 + 0.3 * np.eye(4)):
        assert GK.loglik(Rm, Z.T @ Z, len(Z)) == pytest.approx(scipy_loglik(Rm, Z), rel=1e-11, abs=1e-9)


def test_gradient_and_hessian_against_differences():
    R, _ = draw(R4, 400, 2)
    Z = GK.normal_scores(R)
    G, n, k = Z.T @ Z, len(Z), 4
    theta = np.array([R4[j, l] for j, l in GK.pairs(k)]) * 0.9
    g, H = GK.grad_hess(GK.corr_matrix(theta, k), G, n)
    h = 1e-5
    for q in range(len(theta)):
        e = np.zeros_like(theta); e[q] = h
        f = lambda t: scipy_loglik(GK.corr_matrix(t, k), Z)
        assert g[q] == pytest.approx((f(theta + e) - f(theta - e)) / (2 * h), rel=1e-6, abs=1e-6)
        gp, _ = GK.grad_hess(GK.corr_matrix(theta + e, k), G, n)
        gm, _ = GK.grad_hess(GK.corr_matrix(theta - e, k), G, n)
        assert np.allclose(H[:, q], (gp - gm) / (2 * h), rtol=1e-6, atol=1e-4)


def test_maximiser_against_scipy_optimiser():
    R, _ = draw(R3, 2000, 3)
    Z = GK.normal_scores(R)
    theta, it, st = GK.mpl(Z.T @ Z, len(Z))
    assert st == GK.OK and it <= 10
    def cost(t):
        Rm = GK.corr_matrix(t, 3)
        return -scipy_loglik(Rm, Z) if np.all(np.linalg.eigvalsh(Rm) > 1e-9) else np.inf
    res = optimize.minimize(cost, theta * 0.95, method="Nelder-Mead",
                            options={"xatol": 1e-10, "fatol": 1e-12, "maxiter": 20000, "maxfev": 40000})
    assert np.allclose(theta, res.x, atol=1e-6)
    assert cost(theta) <= res.fun + 1e-9


def test_two_margins_reduce_to_the_bivariate_fit():
    """At k = 2 the likelihood is eq. (8)'s: the estimate and its GGR
    variance equal the bivariate Gaussian fit of the C oracle."""
    rng = np.random.default_rng(4)
    x = rng.standard_normal(3000)
    y = 0.6 * x + rng.standard_normal(3000)
    x[:200] = np.round(x[:200])  # ties
    off = np.array([0, 1000, 3000])
    sub2, _ = O.fit(x, y, off, "gaussian")
    R = np.stack([np.concatenate([O.ranks(v[off[m]:off[m + 1]]) for m in range(2)]) for v in (x, y)], axis=1)
    subk, _ = GK.fit_ranks(R, off)
    assert np.allclose(subk["theta"][0], sub2["theta"], rtol=1e-9, atol=1e-12)
    assert np.allclose(subk["var"][0], sub2["var"], rtol=1e-8)


def test_variance_against_replicate_spread():
    n, S = 1500, 120
    est, var = [], []
    for s in range(S):
        R, _ = draw(R3, n, 100 + s)
        theta, v, _, _, _, st = GK.fit_subset(R)
        assert st == GK.OK
        est.append(theta); var.append(v)
    ratio = np.var(np.array(est), axis=0, ddof=1) / np.mean(np.array(var), axis=0)
    assert np.all((ratio > 0.68) & (ratio < 1.4)), ratio


def test_statuses():
    R, _ = draw(R3, 50, 5)
    Rc = R.copy(); Rc[:, 1] = 51           # a constant margin
    Rs = R.copy(); Rs[:, 2] = Rs[:, 0]     # two margins with equal ranks: R singular at the start
    Rall = np.concatenate([R, Rc, Rs, R[:3]])
    sub, comb = GK.fit_ranks(Rall, [0, 50, 100, 150, 153])
    assert list(sub["status"][0]) == [GK.OK, GK.DEGENERATE, GK.BOUNDARY_BOX, GK.DEGENERATE]
    assert np.all(comb["n_used"] == 1)
    assert np.allclose(comb["theta"][:, 0], sub["theta"][:, 0])
