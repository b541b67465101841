"""Pins of the oracle's Spearman-inversion estimator (Sec. 2.3): rho_S hat
against scipy, the inversion against the Gaussian closed form and round
trips through the (pinned) rho_S functions, the Pickands-function form of
Gumbel's rho_S (the form the GPU integrates) against the oracle's double
integral of C, and the sandwich variance against its closed form under
independence, brute force on tiny inputs and the spread of estimates over
replicates."""
import math

import numpy as np
import pytest
from scipy import integrate, stats

import oracle.oracle as O
import synth


def test_spearman_against_scipy():
    x, y = synth.copula_pairs("frank", 4.0, 3000, 3)
    R1, R2 = O.ranks(x), O.ranks(y)
    assert O.spearman(R1, R2) == pytest.approx(stats.spearmanr(x, y).statistic, abs=1e-13)


@pytest.mark.parametrize("fam,th", [("gaussian", 0.3), ("gaussian", -0.9), ("frank", 5.0), ("frank", -8.0),
                                    ("frank", 0.3), ("gumbel", 1.2), ("gumbel", 5.0), ("gumbel", 30.0)])
def test_inversion_round_trip(fam, th):
    r = O.rho_s(fam, th)
    got, st = O.spearman_theta(fam, r)
    assert st == 0
    assert got == pytest.approx(th, rel=1e-8, abs=1e-10)
    if fam == "gaussian":
        assert got == pytest.approx(2.0 * math.sin(math.pi * r / 6.0), rel=1e-14)


def test_inversion_boundaries():
    assert O.spearman_theta("gumbel", -0.1) == (1.0, 1)
    assert O.spearman_theta("frank", 0.99999)[1] == 2
    assert O.spearman_theta("gaussian", 0.9999999999)[1] == 2


@pytest.mark.parametrize("th", [1.0, 1.5, 2.0, 5.0, 20.0])
def test_gumbel_rho_s_by_pickands_function(th):
    def a(w):
        return (w ** th + (1.0 - w) ** th) ** (1.0 / th)
    I = integrate.quad(lambda w: (1.0 + a(w)) ** -2, 0.0, 1.0, epsabs=1e-14, epsrel=1e-13, limit=200)[0]
    assert 12.0 * I - 3.0 == pytest.approx(O.rho_s("gumbel", th), abs=2e-9)


def test_variance_under_independence():
    rng = np.random.default_rng(8)
    n = 20000
    R1 = O.ranks(rng.standard_normal(n)); R2 = O.ranks(rng.standard_normal(n))
    v, nu = O.spearman_var(R1, R2, "gaussian", 0.0)
    assert nu == pytest.approx(1.0, abs=0.05)          # var(12 (U - 1/2)(V - 1/2)) = 1
    assert n * v == pytest.approx((math.pi / 3.0) ** 2 * nu, rel=1e-12)  # (d theta / d rho_S)^2 at 0


@pytest.mark.parametrize("fam,th,slope", [
    # Gumbel at theta = 1: a(w) = 1 and d a / d theta = w log w + (1 - w) log(1 - w), so
    # d rho_S / d theta = -24/8 int_0^1 (w log w + (1 - w) log(1 - w)) dw = 3/2 (one-sided)
    ("gumbel", 1.0, 1.5),
    # Frank near independence: rho_S = theta/6 - theta^3/450 + ...
    ("frank", 0.0, 1.0 / 6.0),
    ("frank", 0.5, 1.0 / 6.0 - 0.25 / 150.0 + 0.0625 / 4704.0),
])
def test_variance_slope_closed_forms(fam, th, slope):
    """The variance divides var(psi) by n rho_S'(theta)^2; at these points
    rho_S' has a closed form. The oracle differences rho_S, itself integrated
    to ~1e-11, over steps of 1e-4: 2e-6 relative (a first-order difference at
    Gumbel's edge is off by 4e-4)."""
    rng = np.random.default_rng(12)
    n = 500
    R1 = O.ranks(rng.standard_normal(n)); R2 = O.ranks(rng.standard_normal(n))
    v, nu = O.spearman_var(R1, R2, fam, th)
    assert math.sqrt(nu / (n * v)) == pytest.approx(slope, rel=2e-6)


def test_variance_brute_force_with_ties():
    rng = np.random.default_rng(9)
    n = 40
    x = np.round(rng.standard_normal(n) * 2) / 2
    y = x + rng.standard_normal(n)
    R1, R2 = O.ranks(x), O.ranks(y)
    den = 2.0 * (n + 1)
    u, v = R1 / den, R2 / den
    J = 12 * (u - 0.5) * (v - 0.5)
    W1 = np.array([np.sum(12 * (v - 0.5) * (u >= u[i])) / n for i in range(n)])
    W2 = np.array([np.sum(12 * (u - 0.5) * (v >= v[i])) / n for i in range(n)])
    psi = J + W1 + W2
    _, nu = O.spearman_var(R1, R2, "frank", 2.0)
    assert nu == pytest.approx(np.mean(psi ** 2) - np.mean(psi) ** 2, rel=1e-12)


@pytest.mark.parametrize("fam,th,S,lo,hi", [("frank", 5.0, 160, 0.7, 1.35), ("gumbel", 2.0, 90, 0.6, 1.5)])
def test_variance_against_replicate_spread(fam, th, S, lo, hi):
    """The spread of S estimates against the mean estimated variance; the
    bounds are about three standard errors of a variance ratio with S - 1
    degrees of freedom (fewer Gumbel replicates: its rho_S is a double
    integral in the oracle)."""
    n = 1500
    est, var = [], []
    for s in range(S):
        x, y = synth.copula_pairs(fam, th, n, 60000 + s)
        R1, R2 = O.ranks(x), O.ranks(y)
        t, st = O.spearman_theta(fam, O.spearman(R1, R2))
        assert st == 0
        est.append(t)
        var.append(O.spearman_var(R1, R2, fam, t)[0])
    ratio = np.var(est, ddof=1) / np.mean(var)
    assert lo <= ratio <= hi, ratio


def test_statuses_from_ranks():
    R = np.array([5, 5, 5, 5], dtype=np.int64)      # a margin of one value (doubled ranks of 4 ties)
    S2 = np.array([2, 4, 6, 8], dtype=np.int64)
    sub, comb = O.spearman_fit_ranks(np.concatenate([R, S2]), np.concatenate([S2, S2[::-1]]),
                                     [0, 4, 8], "gumbel")
    assert sub["status"][0] == 3          # DEGENERATE
    assert sub["status"][1] == 1 and sub["theta"][1] == 1.0  # negative dependence: Gumbel at theta = 1
