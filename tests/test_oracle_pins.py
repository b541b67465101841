"""Pins of the FP64 CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: values the
paper prints (Sec. 2.5), library routines (scipy, mpmath), symbolic
differentiation of the printed copulas (sympy, eq. (8), (10), (11) with
eq. (5)), brute force on tiny inputs, closed forms (the Gaussian likelihood
equation, the semiparametric efficiency bound) and sampling behaviour.
"""
import math

import mpmath
import numpy as np
import pytest
import sympy as sp
from scipy.special import ndtri
from scipy.stats import multivariate_normal, norm

import oracle.oracle as O
import synth
from conftest import read_table

mpmath.mp.dps = 40


# --------------------------------------------------------------------------
# Sec. 2.5 prints Spearman's rho and Kendall's tau for the study's parameters.

@pytest.mark.parametrize("row", read_table("sec2_5_dependence.txt"))
def test_printed_dependence_values(row):
    fam, th, rho_s, tau = row[0], float(row[1]), float(row[2]), float(row[3])
    assert round(O.tau(fam, th), 2) == pytest.approx(tau, abs=1e-9)
    assert round(O.rho_s(fam, th), 2) == pytest.approx(rho_s, abs=1e-9)


def test_debye_against_quadrature():
    for k in (1, 2):
        for x in (-200.0, -20.0, -3.0, 0.5, 5.0, 40.0, 150.0, 200.0):
            ref = k / x**k * float(mpmath.quad(lambda t: t**k / mpmath.expm1(t) if t != 0 else (1 if k == 1 else 0), [0, x]))
            assert O.debye(k, x) == pytest.approx(ref, rel=1e-12)


# --------------------------------------------------------------------------
# Normal quantile (needed for eq. (8)).

def test_qnorm_against_scipy_and_mpmath():
    p = np.concatenate([np.logspace(-300, -1, 60), np.linspace(0.01, 0.99, 41)])
    z = O.qnorm(p, 1.0 - p)
    assert np.allclose(z, ndtri(p), rtol=2e-14, atol=1e-15)
    for pi, zi in zip(p[::7], z[::7]):
        ref = float(mpmath.sqrt(2) * mpmath.erfinv(2 * mpmath.mpf(pi) - 1)) if pi > 1e-15 else None
        if ref is not None:
            assert zi == pytest.approx(ref, rel=1e-14, abs=1e-15)
    # antisymmetry with the exact complement
    assert np.array_equal(O.qnorm(1.0 - p[:50], p[:50]), -z[:50])


# --------------------------------------------------------------------------
# Ranks, eq. (12), against O(n^2) brute force.

def brute_ranks(x, ties):
    n = len(x)
    R = np.empty(n, dtype=np.int64)
    for i in range(n):
        less = sum(1 for j in range(n) if x[j] < x[i])
        eq = sum(1 for j in range(n) if x[j] == x[i])
        eq_before = sum(1 for j in range(i) if x[j] == x[i])
        R[i] = 2 * less + eq + 1 if ties == "average" else 2 * (less + eq_before + 1)
    return R


@pytest.mark.parametrize("ties", ["average", "first"])
def test_ranks_brute_force(ties):
    rng = np.random.default_rng(11)
    cases = [np.array([]), np.array([1.0]), np.array([2.0, 2.0, 2.0]), np.array([0.0, -0.0, 1.0, -1.0, -0.0]),
             np.array([3.0, 1.0, 2.0, 2.0, 5.0, 1.0, 1.0])]
    for n in (2, 5, 17, 64, 200):
        cases.append(rng.standard_normal(n))
        cases.append(rng.integers(0, 5, n).astype(np.float64))  # heavy ties
        cases.append(np.float32(rng.standard_normal(n)).astype(np.float64))
    for x in cases:
        assert np.array_equal(O.ranks(x, ties), brute_ranks(list(x), ties)), x


def test_average_ranks_permutation_invariant():
    rng = np.random.default_rng(3)
    x = rng.integers(0, 30, 500).astype(np.float64)
    perm = rng.permutation(500)
    assert np.array_equal(O.ranks(x)[perm], O.ranks(x[perm]))


# --------------------------------------------------------------------------
# Densities: eq. (5) applied to the printed copulas.

def _sympy_copulas():
    t, u, v = sp.symbols("t u v", real=True)
    frank = -1 / t * sp.log(1 + (sp.exp(-t * u) - 1) * (sp.exp(-t * v) - 1) / (sp.exp(-t) - 1))
    gumbel = sp.exp(-((-sp.log(u)) ** t + (-sp.log(v)) ** t) ** (1 / t))
    out = {}
    for name, C in (("frank", frank), ("gumbel", gumbel)):
        c = sp.diff(C, u, v)
        l = sp.log(c)
        lt = sp.diff(l, t)
        exprs = [c, lt, sp.diff(lt, t), sp.diff(lt, u), sp.diff(lt, v)]
        out[name] = [sp.lambdify((t, u, v), e, "mpmath") for e in exprs]
    return out


_SYM = None


def sym():
    global _SYM
    if _SYM is None:
        _SYM = _sympy_copulas()
    return _SYM


@pytest.mark.parametrize("family,theta", [("frank", 5.0), ("frank", -8.0), ("frank", 0.3), ("frank", 30.0),
                                          ("frank", 2e-5), ("frank", -3e-4), ("frank", 2.5e-3), ("frank", -4e-3), ("gumbel", 1.0), ("gumbel", 1.7),
                                          ("gumbel", 5.0), ("gumbel", 20.0)])
def test_density_and_derivatives_match_printed_cdf(family, theta):
    """sympy mixed partial of eq. (10)/(11) and its theta/u/v derivatives."""
    fns = sym()[family]
    rng = np.random.default_rng(5)
    pts = [(0.3, 0.6), (0.01, 0.97), (0.5, 0.5), (0.999, 0.998), (0.002, 0.003)] + [tuple(rng.uniform(0.01, 0.99, 2)) for _ in range(5)]
    u = np.array([p[0] for p in pts]); v = np.array([p[1] for p in pts])
    d = O.logc_derivs(family, theta, u, 1 - u, v, 1 - v)
    for i, (ui, vi) in enumerate(pts):
        args = (mpmath.mpf(theta), mpmath.mpf(ui), mpmath.mpf(vi))
        c = fns[0](*args)
        assert math.exp(d[i, 0]) == pytest.approx(float(c), rel=1e-11)
        for k in range(1, 5):
            ref = float(fns[k](*args))
            assert d[i, k] == pytest.approx(ref, rel=1e-8, abs=1e-9 * (1 + abs(ref))), (k, ui, vi)


def _gauss_logc_mp(rho, u, v):
    # eq. (8): the integrand at the upper limits s = Phi^{-1}(u), t = Phi^{-1}(v),
    # times d Phi^{-1}/du * d Phi^{-1}/dv (fundamental theorem of calculus).
    s = mpmath.sqrt(2) * mpmath.erfinv(2 * u - 1)
    t = mpmath.sqrt(2) * mpmath.erfinv(2 * v - 1)
    f = 1 / (2 * mpmath.pi * mpmath.sqrt(1 - rho**2)) * mpmath.exp(-(s**2 - 2 * rho * s * t + t**2) / (2 * (1 - rho**2)))
    phi = lambda z: mpmath.exp(-z**2 / 2) / mpmath.sqrt(2 * mpmath.pi)
    return mpmath.log(f / (phi(s) * phi(t)))


@pytest.mark.parametrize("rho", [0.5, -0.9, 0.0, 0.95])
def test_gaussian_density_and_derivatives(rho):
    pts = [(0.3, 0.6), (0.01, 0.97), (0.5, 0.5), (0.999, 0.998), (0.2, 0.21)]
    u = np.array([p[0] for p in pts]); v = np.array([p[1] for p in pts])
    d = O.logc_derivs("gaussian", rho, u, 1 - u, v, 1 - v)
    for i, (ui, vi) in enumerate(pts):
        U, V, Rr = mpmath.mpf(ui), mpmath.mpf(vi), mpmath.mpf(rho)
        assert d[i, 0] == pytest.approx(float(_gauss_logc_mp(Rr, U, V)), rel=1e-12, abs=1e-13)
        lt = float(mpmath.diff(lambda r: _gauss_logc_mp(r, U, V), Rr))
        ltt = float(mpmath.diff(lambda r: _gauss_logc_mp(r, U, V), Rr, 2))
        ltu = float(mpmath.diff(lambda r, a: _gauss_logc_mp(r, a, V), (Rr, U), (1, 1)))
        ltv = float(mpmath.diff(lambda r, b: _gauss_logc_mp(r, U, b), (Rr, V), (1, 1)))
        for k, ref in ((1, lt), (2, ltt), (3, ltu), (4, ltv)):
            assert d[i, k] == pytest.approx(ref, rel=1e-9, abs=1e-10), (k, ui, vi)
    # and against scipy's bivariate normal CDF by a finite mixed difference
    h = 1e-3
    for ui, vi in [(0.3, 0.6), (0.5, 0.5)]:
        cdf = lambda a, b: multivariate_normal.cdf([norm.ppf(a), norm.ppf(b)], mean=[0, 0], cov=[[1, rho], [rho, 1]])
        fd = (cdf(ui + h, vi + h) - cdf(ui + h, vi - h) - cdf(ui - h, vi + h) + cdf(ui - h, vi - h)) / (4 * h * h)
        dd = O.logc_derivs("gaussian", rho, np.array([ui]), np.array([1 - ui]), np.array([vi]), np.array([1 - vi]))
        assert math.exp(dd[0, 0]) == pytest.approx(fd, rel=2e-3)


@pytest.mark.parametrize("family,theta", [("gaussian", 0.5), ("gaussian", -0.9), ("frank", 5.0), ("frank", -8.0),
                                          ("frank", 1e-5), ("gumbel", 2.0), ("gumbel", 5.0)])
def test_density_integrates_to_one(family, theta):
    """Midpoint rule on 512^2 and 1024^2 grids with Richardson extrapolation."""
    def mid(m):
        g = (np.arange(m) + 0.5) / m
        U, V = np.meshgrid(g, g, indexing="ij")
        U, V = U.ravel(), V.ravel()
        return float(np.exp(O.logc_derivs(family, theta, U, 1 - U, V, 1 - V)[:, 0]).mean())
    i1, i2 = mid(512), mid(1024)
    assert abs(i2 - 1.0) < 2e-3
    assert abs(2 * i2 - i1 - 1.0) < 1e-4


def test_uniform_margins():
    """int_0^1 c(u, v) dv = 1 for fixed u (each margin of a copula is uniform)."""
    m = 20000
    g = (np.arange(m) + 0.5) / m
    for fam, th in (("frank", 5.0), ("gumbel", 2.0), ("gaussian", 0.5)):
        for u0 in (0.2, 0.7):
            u = np.full(m, u0)
            val = np.exp(O.logc_derivs(fam, th, u, 1 - u, g, 1 - g)[:, 0]).mean()
            assert abs(val - 1.0) < 2e-3, (fam, u0, val)


def test_frank_series_continuity_and_reflection():
    u = np.array([0.1, 0.4, 0.93]); v = np.array([0.7, 0.2, 0.95])
    lo = O.logc_derivs("frank", 3e-3 * (1 - 1e-12), u, 1 - u, v, 1 - v)
    hi = O.logc_derivs("frank", 3e-3, u, 1 - u, v, 1 - v)
    # the series (below 3e-3) and the closed form (from 3e-3 on) agree at the switch
    assert np.allclose(lo[:, :2], hi[:, :2], rtol=1e-10, atol=1e-14)
    assert np.allclose(lo[:, 2:], hi[:, 2:], rtol=1e-8, atol=1e-10)
    # c(u, v; -theta) = c(u, 1 - v; theta)
    a = O.logc_derivs("frank", -6.0, u, 1 - u, v, 1 - v)
    b = O.logc_derivs("frank", 6.0, u, 1 - u, 1 - v, v)
    assert np.allclose(a[:, 0], b[:, 0], rtol=1e-13)


def test_derivatives_against_finite_differences():
    rng = np.random.default_rng(8)
    u = rng.uniform(0.02, 0.98, 20); v = rng.uniform(0.02, 0.98, 20)
    for fam, th in (("gaussian", 0.6), ("frank", -4.0), ("frank", 12.0), ("gumbel", 2.5)):
        d = O.logc_derivs(fam, th, u, 1 - u, v, 1 - v)
        h = 1e-5
        p = O.logc_derivs(fam, th + h, u, 1 - u, v, 1 - v)
        m = O.logc_derivs(fam, th - h, u, 1 - u, v, 1 - v)
        assert np.allclose((p[:, 0] - m[:, 0]) / (2 * h), d[:, 1], rtol=1e-6, atol=1e-7)
        assert np.allclose((p[:, 1] - m[:, 1]) / (2 * h), d[:, 2], rtol=1e-6, atol=1e-6)
        pu = O.logc_derivs(fam, th, u + h, 1 - u - h, v, 1 - v)
        mu = O.logc_derivs(fam, th, u - h, 1 - u + h, v, 1 - v)
        assert np.allclose((pu[:, 1] - mu[:, 1]) / (2 * h), d[:, 3], rtol=1e-5, atol=1e-6)
        pv = O.logc_derivs(fam, th, u, 1 - u, v + h, 1 - v - h)
        mv = O.logc_derivs(fam, th, u, 1 - u, v - h, 1 - v + h)
        assert np.allclose((pv[:, 1] - mv[:, 1]) / (2 * h), d[:, 4], rtol=1e-5, atol=1e-6)


# --------------------------------------------------------------------------
# Maximisation of eq. (13).

def _loglik(fam, th, R1, R2, n):
    u, omu = O.pobs_from_ranks(R1, n)
    v, omv = O.pobs_from_ranks(R2, n)
    return O.logc_derivs(fam, th, u, omu, v, omv)[:, 0].sum()


@pytest.mark.parametrize("fam,th", [("gaussian", 0.5), ("frank", 4.0), ("frank", -3.0), ("gumbel", 2.0)])
def test_mle_against_dense_grid(fam, th):
    lo, hi = {"gaussian": (-0.999, 0.999), "frank": (-60.0, 60.0), "gumbel": (1.0, 40.0)}[fam]
    for n, seed in ((5, 1), (12, 2), (30, 3), (50, 4)):
        x, y = synth.copula_pairs(fam, th, n, seed)
        sub, _ = O.fit(x, y, [0, n], fam)
        R1, R2 = O.ranks(x), O.ranks(y)
        grid = np.linspace(lo, hi, 100_001)
        u, omu = O.pobs_from_ranks(R1, n)
        v, omv = O.pobs_from_ranks(R2, n)
        ll = np.array([O.logc_derivs(fam, g, u, omu, v, omv)[:, 0].sum() for g in grid[::50]])
        j = int(np.argmax(ll)) * 50
        fine = grid[max(j - 50, 0):j + 51]
        llf = np.array([O.logc_derivs(fam, g, u, omu, v, omv)[:, 0].sum() for g in fine])
        best = fine[int(np.argmax(llf))]
        st = int(sub["status"][0])
        if st == 0:
            assert sub["loglik"][0] >= llf.max() - 1e-9
            assert abs(sub["theta"][0] - best) <= 2 * (grid[1] - grid[0])
            d = O.logc_derivs(fam, sub["theta"][0], u, omu, v, omv)
            assert abs(d[:, 1].sum()) < 1e-8 * (1 + np.abs(d[:, 1]).sum())
            assert d[:, 2].sum() < 0
        else:  # a boundary estimate: the likelihood must be monotone toward it
            assert st in (1, 2)


def test_gaussian_estimate_solves_likelihood_cubic():
    """For normal scores z the Gaussian-copula MPL equation is
    n r^3 - B r^2 + (A - n) r - B = 0, A = sum(z1^2 + z2^2), B = sum z1 z2."""
    for rho, n, seed in ((0.5, 2000, 1), (-0.8, 1500, 2), (0.05, 3000, 3)):
        x, y = synth.copula_pairs("gaussian", rho, n, seed)
        sub, _ = O.fit(x, y, [0, n], "gaussian")
        R1, R2 = O.ranks(x), O.ranks(y)
        z1 = ndtri(R1 / (2.0 * (n + 1))); z2 = ndtri(R2 / (2.0 * (n + 1)))
        A = np.sum(z1**2 + z2**2); B = np.sum(z1 * z2)
        roots = np.roots([n, -B, A - n, -B])
        real = [r.real for r in roots if abs(r.imag) < 1e-12 and -1 < r.real < 1]
        assert len(real) >= 1
        assert min(abs(sub["theta"][0] - r) for r in real) < 1e-11


@pytest.mark.parametrize("fam,th", [("gaussian", 0.7), ("frank", 5.0), ("frank", -8.0), ("gumbel", 2.0), ("gumbel", 3.0)])
def test_large_n_consistency_with_kendall_tau(fam, th):
    n = 20000
    x, y = synth.copula_pairs(fam, th, n, 77)
    sub, _ = O.fit(x, y, [0, n], fam)
    t_hat = float(sub["theta"][0]); sd = math.sqrt(float(sub["var"][0]))
    dtau = (O.tau(fam, t_hat + 1e-6) - O.tau(fam, t_hat - 1e-6)) / 2e-6
    assert abs(O.tau(fam, t_hat) - O.tau(fam, th)) <= 4 * abs(dtau) * sd


# --------------------------------------------------------------------------
# Variance (Sec. 2.3, Genest, Ghoudi & Rivest 1995).

def _ggr_bruteforce(R1, R2, fam, th, n):
    u, omu = O.pobs_from_ranks(R1, n)
    v, omv = O.pobs_from_ranks(R2, n)
    d = O.logc_derivs(fam, th, u, omu, v, omv)
    s, g1, g2 = d[:, 1], d[:, 3], d[:, 4]
    W1 = np.array([sum(g1[l] for l in range(n) if u[l] >= u[i]) / n for i in range(n)])
    W2 = np.array([sum(g2[l] for l in range(n) if v[l] >= v[i]) / n for i in range(n)])
    psi = s + W1 + W2
    nu = np.mean((psi - psi.mean()) ** 2)
    beta = np.mean(s**2)
    return nu / (n * beta**2), W1, W2


def test_ggr_against_literal_definition_with_ties():
    rng = np.random.default_rng(9)
    for fam, th in (("gaussian", 0.4), ("frank", 3.0), ("gumbel", 1.8)):
        n = 120
        x = rng.integers(0, 40, n).astype(np.float64)  # ties
        y = x + rng.integers(0, 30, n)
        R1, R2 = O.ranks(x), O.ranks(y)
        var, terms = O.ggr(R1, R2, fam, th)
        ref, W1, W2 = _ggr_bruteforce(R1, R2, fam, th, n)
        assert var == pytest.approx(ref, rel=1e-12)
        assert np.allclose(terms[:, 1], W1, rtol=1e-12, atol=1e-14)
        assert np.allclose(terms[:, 2], W2, rtol=1e-12, atol=1e-14)


def test_gaussian_variance_closed_forms():
    """Normal-scores correlation is semiparametrically efficient:
    n var_GGR -> (1 - rho^2)^2, and the inverse information is (1-rho^2)^2/(1+rho^2)."""
    n = 20000
    for rho in (0.5, 0.8):
        x, y = synth.copula_pairs("gaussian", rho, n, 31)
        sub, _ = O.fit(x, y, [0, n], "gaussian")
        sub2, _ = O.fit(x, y, [0, n], "gaussian", var="invinfo")
        r = float(sub["theta"][0])
        assert n * sub["var"][0] == pytest.approx((1 - r * r) ** 2, rel=0.06)
        assert n * sub2["var"][0] == pytest.approx((1 - r * r) ** 2 / (1 + r * r), rel=0.06)


@pytest.mark.parametrize("fam,th", [("frank", 5.0), ("gumbel", 2.0)])
def test_variance_matches_replicate_spread(fam, th):
    """Across independent replicates the spread of the estimates matches the
    mean estimated variance (ratio within sampling error)."""
    reps, n = 240, 800
    xs, ys = [], []
    for r in range(reps):
        x, y = synth.copula_pairs(fam, th, n, 10_000 + r)
        xs.append(x); ys.append(y)
    off = np.arange(reps + 1, dtype=np.int64) * n
    sub, _ = O.fit(np.concatenate(xs), np.concatenate(ys), off, fam)
    ok = sub["status"] == 0
    ratio = np.var(sub["theta"][ok]) / np.mean(sub["var"][ok])
    assert 0.75 < ratio < 1.3, ratio


# --------------------------------------------------------------------------
# Combination, eq. (15)/(16).

def test_combine_closed_forms():
    sub = np.zeros(6, dtype=O.SUBSET_DTYPE)
    sub["theta"] = [1.0, 2.0, 3.0, 4.0, 5.0, 6.0]
    sub["var"] = [1.0, 1.0, 1.0, 0.5, 0.25, 2.0]
    sub["status"] = [0, 0, 1, 0, 3, 2]
    comb = O.combine(sub, [0, 3, 6])
    assert comb["theta"][0] == pytest.approx(2.0)  # equal weights -> arithmetic mean
    assert comb["var_combined"][0] == pytest.approx(1.0 / 3.0)
    assert comb["theta"][1] == pytest.approx(4.0) and comb["n_used"][1] == 1 and comb["n_excluded"][1] == 2
    sub2 = sub.copy(); sub2["var"] *= 7.5  # common scale leaves the combined estimate unchanged
    assert O.combine(sub2, [0, 3, 6])["theta"][0] == pytest.approx(2.0)
    sub3 = sub.copy(); sub3["status"][:3] = 3
    c3 = O.combine(sub3, [0, 3])
    assert c3["status"][0] == 1 and math.isnan(c3["theta"][0])


def test_single_subset_is_full_fit():
    x, y = synth.copula_pairs("frank", 5.0, 3000, 4)
    sub, comb = O.fit(x, y, [0, 3000], "frank")
    assert comb["theta"][0] == sub["theta"][0]


# --------------------------------------------------------------------------
# Statuses forced by crafted inputs.

def test_statuses():
    rng = np.random.default_rng(2)
    x = rng.standard_normal(400); y = x + 0.3 * rng.standard_normal(400)
    xs = x.copy(); xs[250] = np.nan
    xc = x.copy(); xc[300:400] = 1.5
    off = np.array([0, 0, 1, 100, 200, 300, 400])
    sub, comb = O.fit(xs, y, off, "frank")
    assert list(sub["status"][:2]) == [3, 3]          # empty and 1-row subsets
    assert sub["status"][4] == 4                         # NaN
    sub, _ = O.fit(xc, y, off, "frank")
    assert sub["status"][5] == 3                          # constant margin
    # perfectly concordant -> the box edge
    z = np.arange(50, dtype=np.float64)
    for fam in ("gaussian", "frank", "gumbel"):
        s, _ = O.fit(z, z, [0, 50], fam)
        assert s["status"][0] == 2, fam
    # negatively dependent data under Gumbel -> theta = 1
    s, _ = O.fit(z, -z + 0.1 * rng.standard_normal(50), [0, 50], "gumbel")
    assert s["status"][0] == 1 and s["theta"][0] == 1.0 and s["var"][0] > 0
    # iteration cap
    x5, y5 = synth.copula_pairs("frank", 5.0, 500, 6)
    s, _ = O.fit(x5, y5, [0, 500], "frank", max_iter=1)
    assert s["status"][0] == 5
