"""Pins of the oracle's Kendall-inversion estimator (Sec. 2.3): tau hat
against scipy (tau-b, converted to the pair count with ties), the per-row
kernel sums S_i against the empirical-copula identity
S_i = 4 #{l: x_l < x_i, y_l < y_i} - 2 r1_i - 2 r2_i + n + 3 (no ties), the
inversion against the closed forms and round trips through the pinned tau
functions, the slope of tau against differences of tau and its values at
independence, and the U-statistic variance against its closed form under
independence and the spread of estimates over replicates."""
import math

import numpy as np
import pytest
from scipy import stats

import oracle.oracle as O
import synth


def test_tau_hat_against_scipy_without_ties():
    x, y = synth.copula_pairs("frank", 4.0, 3000, 3)
    R1, R2 = O.ranks(x), O.ranks(y)
    assert O.kendall(R1, R2) == pytest.approx(stats.kendalltau(x, y).statistic, abs=1e-13)


def test_tau_hat_against_scipy_with_ties():
    """Ties count as neither concordant nor discordant: tau hat =
    tau_b sqrt((n0 - n1)(n0 - n2)) / n0 with n1, n2 the tied pairs of each
    margin."""
    rng = np.random.default_rng(4)
    n = 500
    x = np.round(rng.standard_normal(n) * 3) / 3
    y = np.round((x + rng.standard_normal(n)) * 2) / 2
    n0 = n * (n - 1) / 2
    n1 = sum(c * (c - 1) / 2 for c in np.unique(x, return_counts=True)[1])
    n2 = sum(c * (c - 1) / 2 for c in np.unique(y, return_counts=True)[1])
    tb = stats.kendalltau(x, y, variant="b").statistic
    want = tb * math.sqrt((n0 - n1) * (n0 - n2)) / n0
    assert O.kendall(O.ranks(x), O.ranks(y)) == pytest.approx(want, abs=1e-13)


def test_row_sums_by_the_empirical_copula():
    rng = np.random.default_rng(5)
    n = 700
    x = rng.standard_normal(n)
    y = 0.6 * x + rng.standard_normal(n)
    R1, R2 = O.ranks(x), O.ranks(y)
    S = O.kendall_rows(R1, R2)
    below = (x[None, :] < x[:, None]) & (y[None, :] < y[:, None])
    LL = below.sum(axis=1)
    r1, r2 = R1 // 2, R2 // 2
    assert np.array_equal(S, 4 * LL - 2 * r1 - 2 * r2 + n + 3)


@pytest.mark.parametrize("fam,th", [("gaussian", 0.3), ("gaussian", -0.9), ("frank", 5.0), ("frank", -8.0),
                                    ("frank", 0.3), ("frank", 0.004), ("gumbel", 1.2), ("gumbel", 5.0),
                                    ("gumbel", 30.0)])
def test_inversion_round_trip(fam, th):
    t = O.tau(fam, th)
    got, st = O.kendall_theta(fam, t)
    assert st == 0
    assert got == pytest.approx(th, rel=1e-8, abs=1e-10)
    if fam == "gaussian":
        assert got == pytest.approx(math.sin(math.pi * t / 2.0), rel=1e-15)
    if fam == "gumbel":
        assert got == pytest.approx(1.0 / (1.0 - t), rel=1e-15)


def test_inversion_boundaries():
    assert O.kendall_theta("gumbel", -0.1) == (1.0, 1)
    assert O.kendall_theta("gumbel", 0.0) == (1.0, 1)
    assert O.kendall_theta("gumbel", 0.999)[1] == 2
    assert O.kendall_theta("frank", 0.9999)[1] == 2
    assert O.kendall_theta("frank", -0.9999)[1] == 2
    assert O.kendall_theta("gaussian", 1.0)[1] == 2


@pytest.mark.parametrize("fam,th", [("gaussian", 0.0), ("gaussian", 0.7), ("frank", -8.0), ("frank", 0.5),
                                    ("frank", 0.02), ("frank", 40.0), ("gumbel", 1.0), ("gumbel", 3.0)])
def test_tau_slope_against_differences(fam, th):
    h = 1e-4 * (1.0 + abs(th))
    if fam == "gumbel" and th - h < 1.0:
        d = (-3 * O.tau(fam, th) + 4 * O.tau(fam, th + h) - O.tau(fam, th + 2 * h)) / (2 * h)
    else:
        d = (O.tau(fam, th + h) - O.tau(fam, th - h)) / (2 * h)
    assert O.tau_slope(fam, th) == pytest.approx(d, rel=1e-6)


def test_tau_slope_closed_values():
    assert O.tau_slope("gaussian", 0.0) == pytest.approx(2.0 / math.pi, rel=1e-15)
    assert O.tau_slope("gumbel", 1.0) == 1.0
    assert O.tau_slope("frank", 0.0) == pytest.approx(1.0 / 9.0, rel=1e-15)
    # the series and the closed form meet at |theta| = 1e-2
    assert O.tau_slope("frank", 0.00999999) == pytest.approx(O.tau_slope("frank", 0.0100001), rel=1e-9)


def test_variance_under_independence():
    """k1(u, v) = (2u - 1)(2v - 1) at independence: var(k1) = 1/9."""
    rng = np.random.default_rng(8)
    n = 20000
    R1 = O.ranks(rng.standard_normal(n)); R2 = O.ranks(rng.standard_normal(n))
    v, zeta, t = O.kendall_var(R1, R2, "gaussian", 0.0)
    assert zeta == pytest.approx(1.0 / 9.0, rel=0.03)
    assert t == pytest.approx(O.kendall(R1, R2), abs=1e-15)
    assert n * v == pytest.approx(4.0 * zeta / (2.0 / math.pi) ** 2, rel=1e-12)


def test_tau_hat_spread_under_independence():
    """Var(tau hat) = 2 (2n + 5) / (9 n (n - 1)) exactly at independence."""
    rng = np.random.default_rng(10)
    n, S = 60, 2000
    t = [O.kendall(O.ranks(rng.standard_normal(n)), O.ranks(rng.standard_normal(n))) for _ in range(S)]
    want = 2 * (2 * n + 5) / (9 * n * (n - 1))
    assert np.var(t, ddof=1) / want == pytest.approx(1.0, abs=0.1)   # ~3 standard errors at S = 2000


@pytest.mark.parametrize("fam,th", [("gaussian", 0.6), ("frank", 5.0), ("gumbel", 2.0)])
def test_variance_against_replicate_spread(fam, th):
    n, S = 1500, 160
    est, var = [], []
    for s in range(S):
        x, y = synth.copula_pairs(fam, th, n, 61000 + s)
        R1, R2 = O.ranks(x), O.ranks(y)
        t, st = O.kendall_theta(fam, O.kendall(R1, R2))
        assert st == 0
        est.append(t)
        var.append(O.kendall_var(R1, R2, fam, t)[0])
    ratio = np.var(est, ddof=1) / np.mean(var)
    assert 0.7 <= ratio <= 1.35, ratio


def test_statuses_from_ranks():
    R = np.array([5, 5, 5, 5], dtype=np.int64)      # a margin of one value
    S2 = np.array([2, 4, 6, 8], dtype=np.int64)
    A = np.array([2, 4, 6, 8, 10, 12], dtype=np.int64)
    B = np.array([12, 4, 10, 2, 8, 6], dtype=np.int64)  # tau hat = -1/3
    sub, comb = O.kendall_fit_ranks(np.concatenate([R, A, S2[:2]]), np.concatenate([S2, B, S2[:2]]),
                                    [0, 4, 10, 12], "gumbel")
    assert sub["status"][0] == 3                                   # DEGENERATE
    assert sub["status"][1] == 1 and sub["theta"][1] == 1.0         # negative dependence: Gumbel at theta = 1
    assert sub["status"][2] == 2                                   # two concordant rows: tau = 1, box edge
    assert comb["n_used"][0] == 1
