"""Pins of the oracle's simulation inputs and study metrics (Sec. 2.5-2.6)
against what the mathematics fixes: the published known-answer values of
the Philox4x32-10 generator, the copulas' Kendall's tau closed forms and
normal margins for the samplers, and for the density distances of
eq. (19)-(20): zero distance to itself, unit mass, the closed forms of the
Gaussian copula density's L2 products, and library quadrature in the unit
square for the bounded Frank density."""
import math

import numpy as np
import pytest
from scipy import integrate, stats

import oracle.oracle as O

# Random123's known-answer vectors for philox4x32-10: (counter, key, output)
PHILOX_KAT = [
    ((0, 0, 0, 0), (0, 0), (0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8)),
    ((0xFFFFFFFF,) * 4, (0xFFFFFFFF,) * 2, (0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD)),
    ((0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344), (0xA4093822, 0x299F31D0),
     (0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1)),
]


@pytest.mark.parametrize("ctr,key,want", PHILOX_KAT)
def test_philox_known_answers(ctr, key, want):
    assert tuple(int(v) for v in O.philox4x32_10(ctr, key)) == want


@pytest.mark.parametrize("fam,th", [("gaussian", 0.5), ("gaussian", -0.9), ("frank", 5.0), ("frank", -8.0),
                                    ("frank", 80.0), ("frank", 0.0), ("gumbel", 2.0), ("gumbel", 1.0),
                                    ("gumbel", 20.0)])
def test_sampler_dependence_and_margins(fam, th):
    n = 20000
    x, y = O.sample(fam, th, 12345, 1000, n)
    assert np.all(np.isfinite(x)) and np.all(np.isfinite(y))
    tau = stats.kendalltau(x, y).statistic
    # standard error of Kendall's tau is below sqrt(2(2n+5)/(9n(n-1))) * 2
    se = 2.0 * math.sqrt(2.0 * (2 * n + 5) / (9.0 * n * (n - 1)))
    assert abs(tau - O.tau(fam, th)) <= 4.0 * se, (fam, th, tau, O.tau(fam, th))
    for m in (x, y):
        assert stats.kstest(m, "norm").pvalue > 1e-4
    if fam == "gaussian":
        assert abs(np.corrcoef(x, y)[0, 1] - th) <= 4.0 * (1 - th * th) / math.sqrt(n) + 1e-3


def test_sampler_rows_are_independent_of_the_range():
    a = O.sample("gumbel", 3.0, 7, 0, 500)
    b = O.sample("gumbel", 3.0, 7, 200, 100)
    assert np.array_equal(a[0][200:300], b[0]) and np.array_equal(a[1][200:300], b[1])
    c = O.sample("gumbel", 3.0, 8, 200, 100)
    assert not np.array_equal(b[0], c[0])


@pytest.mark.parametrize("fam,th", [("gaussian", 0.3), ("gaussian", -0.8), ("frank", 5.0), ("frank", -2.0),
                                    ("gumbel", 5.0), ("gumbel", 1.5)])
def test_density_mass_and_self_distance(fam, th):
    out = O.density_distance(fam, th, th, panels=128)
    assert out[0] == 0.0 and out[2] == 0.0
    assert out[1] == pytest.approx(1.0, abs=2e-9)


def gaussian_l2_products(ra, rb):
    """int c_a^2 = 1 / (1 - r^2); int c_a c_b = 1 / sqrt((1 - ra^2)(1 - rb^2) det M),
    M = inv(S_a) + inv(S_b) - I for the correlation matrices S."""
    def inv(r):
        return np.array([[1.0, -r], [-r, 1.0]]) / (1.0 - r * r)
    M = inv(ra) + inv(rb) - np.eye(2)
    cross = 1.0 / math.sqrt((1 - ra * ra) * (1 - rb * rb) * np.linalg.det(M))
    return 1.0 / (1 - ra * ra), 1.0 / (1 - rb * rb), cross


@pytest.mark.parametrize("ra,rb", [(0.3, 0.3021), (0.9, 0.895), (-0.5, -0.47)])
def test_gaussian_l2_closed_forms(ra, rb):
    out = O.density_distance("gaussian", ra, rb, panels=128)
    aa, bb, ab = gaussian_l2_products(ra, rb)
    assert out[3] == pytest.approx(aa, rel=1e-9)
    assert out[2] == pytest.approx(aa + bb - 2.0 * ab, rel=1e-6, abs=1e-14)


def frank_density(u, v, th):
    E = -math.expm1(-th)
    D = E - (1 - math.exp(-th * u)) * (1 - math.exp(-th * v))
    return th * E * math.exp(-th * (u + v)) / (D * D)


@pytest.mark.parametrize("ta,tb", [(5.0, 5.01), (-3.0, -2.95)])
def test_frank_distances_against_unit_square_quadrature(ta, tb):
    out = O.density_distance("frank", ta, tb, panels=128)
    opts = {"epsabs": 1e-12, "epsrel": 1e-10}
    l1 = integrate.dblquad(lambda v, u: abs(frank_density(u, v, ta) - frank_density(u, v, tb)), 0, 1, 0, 1,
                           **opts)[0]
    l2 = integrate.dblquad(lambda v, u: (frank_density(u, v, ta) - frank_density(u, v, tb)) ** 2, 0, 1, 0, 1,
                           **opts)[0]
    n2 = integrate.dblquad(lambda v, u: frank_density(u, v, ta) ** 2, 0, 1, 0, 1, **opts)[0]
    assert out[0] == pytest.approx(l1, rel=1e-6)
    assert out[2] == pytest.approx(l2, rel=1e-6)
    assert out[3] == pytest.approx(n2, rel=1e-8)


def test_replicate_summary_by_hand():
    comb = np.array([1.0, 2.0, 4.0, 9.0])
    full = np.array([1.5, 1.0, 4.0, 0.0])
    st = np.array([0, 0, 0, 1])
    s = O.replicate_summary(comb, st * 0, full, st)
    assert s[4] == 3
    assert s[0] == pytest.approx(7.0 / 3) and s[1] == pytest.approx(6.5 / 3)
    assert s[2] == pytest.approx(0.5 / 3) and s[3] == pytest.approx((0.25 + 1.0 + 0.0) / 3)
