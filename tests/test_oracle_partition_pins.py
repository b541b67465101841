"""Pins of the partition oracle (oracle/partition.py): hand-derived cases,
brute-force positions in x-order, and the invariants each scheme fixes; and,
through the oracle's fit, the effect the schemes are meant to show (slices of
x's range are not samples of the copula; a systematic sample across x is)."""
import os

import numpy as np
import pytest

import oracle.oracle as O
import oracle.partition as P
import synth

HERE = os.path.dirname(os.path.abspath(__file__))


def golden_cases():
    out = []
    with open(os.path.join(HERE, "golden", "partition_tiny.txt")) as f:
        for line in f:
            if not line.startswith("case "):
                continue
            xs, m, scheme, rows, offs = [s.strip() for s in line[5:].split("|")]
            out.append((np.array([float(v) for v in xs.split()]), int(m), scheme,
                        np.array([int(v) for v in rows.split()]), np.array([int(v) for v in offs.split()])))
    return out


@pytest.mark.parametrize("case", golden_cases(), ids=lambda c: f"{c[2]}-N{len(c[0])}-M{c[1]}")
def test_hand_derived_cases(case):
    x, M, scheme, rows, offs = case
    y = np.arange(len(x), dtype=np.float64)  # y records the source row
    xo, yo, got = P.partition(x, y, [0, len(x)], M, scheme)
    assert np.array_equal(yo.astype(np.int64), rows)
    assert np.array_equal(xo, x[rows])
    assert np.array_equal(got, offs)


def brute_positions(x):
    """p(i) = #{j : x_j < x_i} + #{j < i : x_j = x_i}, O(N^2)."""
    n = len(x)
    p = np.zeros(n, dtype=np.int64)
    for i in range(n):
        p[i] = int(np.sum(x < x[i])) + int(np.sum(x[:i] == x[i]))
    return p


def tied_values(rng, n, dtype):
    g = np.round(rng.standard_normal(n) * 3) / 3
    g[::11] = -0.0
    g[1::13] = 0.0
    return g.astype(dtype)


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_x_order_is_brute_force_order(dtype):
    rng = np.random.default_rng(3)
    x = tied_values(rng, 600, dtype)
    order = P.x_order(x)
    p = brute_positions(x.astype(np.float64))
    assert np.array_equal(order[p], np.arange(len(x)))


def check_invariants(x, y, rep, M, scheme, xo, yo, offs):
    R = len(rep) - 1
    assert len(offs) == R * M + 1 and offs[0] == 0 and offs[-1] == rep[-1]
    assert np.all(np.diff(offs) >= 0)
    for r in range(R):
        b, e = rep[r], rep[r + 1]
        N = e - b
        assert offs[r * M] == b and offs[(r + 1) * M] == e
        # the pairs of the replicate, each kept whole
        src = sorted(zip(x[b:e].tolist(), y[b:e].tolist()))
        dst = sorted(zip(xo[b:e].tolist(), yo[b:e].tolist()))
        assert src == dst
        sub = [xo[offs[r * M + m]:offs[r * M + m + 1]] for m in range(M)]
        sizes = np.array([len(s) for s in sub])
        if scheme in ("contiguous", "blocks"):
            assert np.array_equal(sizes, np.diff(P.even_bounds(N, M)))
        if scheme == "contiguous":
            assert np.array_equal(xo[b:e], x[b:e]) and np.array_equal(yo[b:e], y[b:e])
            continue
        for s in sub:
            assert np.all(np.diff(s.astype(np.float64)) >= 0)
        xs = np.sort(x[b:e].astype(np.float64))
        if scheme == "blocks":
            assert np.array_equal(np.concatenate(sub).astype(np.float64), xs)
        else:
            assert np.array_equal(sizes, [(N - m + M - 1) // M for m in range(M)])
            # the j-th row of subset m is position j M + m of the x-order
            for m in range(M):
                assert np.array_equal(sub[m].astype(np.float64), xs[m::M])


@pytest.mark.parametrize("scheme", P.SCHEMES)
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_scheme_invariants(scheme, dtype):
    rng = np.random.default_rng(11)
    sizes = [0, 1, 2, 5, 97, 1000, 4096, 333]
    rep = synth.offsets_from_sizes(np.array(sizes))
    x = tied_values(rng, int(rep[-1]), dtype)
    y = rng.standard_normal(int(rep[-1])).astype(dtype)
    for M in (1, 3, 7, 64):
        xo, yo, offs = P.partition(x, y, rep, M, scheme)
        check_invariants(x, y, rep, M, scheme, xo, yo, offs)


def test_rejects_unknown_scheme_and_bad_m():
    with pytest.raises(ValueError):
        P.partition(np.zeros(3), np.zeros(3), [0, 3], 2, "random")
    with pytest.raises(ValueError):
        P.partition(np.zeros(3), np.zeros(3), [0, 3], 0, "blocks")


def test_slices_of_x_bias_the_combined_estimate_and_a_systematic_sample_does_not():
    """Gaussian rho = 0.6, N = 20000, M = 10, through the oracle's fit and
    combination (eq. 13-15). A slice of 10% of x's range holds a much weaker
    rank dependence (about 0.1 in the middle slices), so the blocks scheme's
    combined estimate falls far below the full-data one; every-M-th row of the
    x-order is a sample across x's whole range, whose combined estimate stays
    within a few standard errors (sd ~ (1 - rho^2) / sqrt(N) = 0.0045) of
    the full-data estimate."""
    x, y = synth.copula_pairs("gaussian", 0.6, 20000, 8)
    full = O.fit(x, y, np.array([0, 20000]), "gaussian", nthreads=0)[1]["theta"][0]
    got = {}
    for scheme in P.SCHEMES:
        xo, yo, offs = P.partition(x, y, [0, 20000], 10, scheme)
        got[scheme] = O.fit(xo, yo, offs, "gaussian", nthreads=0)[1]["theta"][0]
    assert abs(full - 0.6) < 0.03
    assert abs(got["contiguous"] - full) < 0.02
    assert abs(got["strided"] - full) < 0.02
    assert got["blocks"] < 0.35
