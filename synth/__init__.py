"""Seeded synthetic inputs shaped like the paper's simulation study (Sec. 2.5).

This module only draws data. It holds none of the estimator's arithmetic
(no ranks, no likelihood, no variance, no combination) and is the one piece
both the CPU oracle and the GPU library are fed from. Every random number is
drawn here with numpy's PCG64 ``default_rng`` in float64.

Samplers (all with N(0, 1) margins, x = Phi^{-1}(U1), y = Phi^{-1}(U2)):

* Gaussian copula, eq. (8): Cholesky of [[1, rho], [rho, 1]].
* Frank copula, eq. (10): conditional inversion of dC/du.
* Gumbel copula, eq. (11): Marshall-Olkin with a positive-stable frailty drawn
  by Kanter's representation.

Subset splits (partition of eq. (14)): equal, Dirichlet(1) and uniform-size
splits with integer sizes by largest remainder.
"""
from __future__ import annotations

import concurrent.futures
import dataclasses
import math
import os
from typing import List, Sequence

import numpy as np
from scipy import integrate, optimize
from scipy.special import ndtri, ndtri_exp

FAMILY_CODES = {"gaussian": 0, "frank": 1, "gumbel": 2}


def _open_uniform(rng: np.random.Generator, n: int) -> np.ndarray:
    """Uniforms strictly inside (0, 1): (k + 1/2) / 2^53."""
    k = rng.integers(0, 2**53, size=n, dtype=np.int64)
    return (k.astype(np.float64) + 0.5) * (1.0 / 2**53)


def _normal_margin(u: np.ndarray, omu: np.ndarray) -> np.ndarray:
    """Phi^{-1}(u) taking the tail from the smaller of u and 1 - u."""
    out = np.empty_like(u)
    lo = u <= 0.5
    out[lo] = ndtri(u[lo])
    out[~lo] = -ndtri(omu[~lo])
    return out


def gaussian_pairs(n: int, rho: float, rng: np.random.Generator):
    g = rng.standard_normal((2, n))
    x = g[0]
    y = rho * g[0] + math.sqrt(1.0 - rho * rho) * g[1]
    return x, y


def frank_pairs(n: int, theta: float, rng: np.random.Generator):
    """Conditional inversion of dC/du = w, written so that no step cancels for
    large |theta|: e^{-theta v} = (omw e^{-theta u} + w e^{-theta}) / (w +
    omw e^{-theta u}) gives v = u - D / theta and 1 - v = (1 - u) + D / theta
    with D = log1p(w expm1(-theta (1 - u))) - log1p(omw expm1(-theta u))."""
    u = _open_uniform(rng, n)
    w = _open_uniform(rng, n)
    omu = 1.0 - u
    if abs(theta) < 1e-12:
        v, omv = w, 1.0 - w
    else:
        D = np.log1p(w * np.expm1(-theta * omu)) - np.log1p((1.0 - w) * np.expm1(-theta * u))
        v = u - D / theta
        omv = omu + D / theta
    v = np.clip(v, 2.0**-1000, 1.0 - 2.0**-53)
    omv = np.clip(omv, 2.0**-1000, 1.0 - 2.0**-53)
    return _normal_margin(u, omu), _normal_margin(v, omv)


def gumbel_pairs(n: int, theta: float, rng: np.random.Generator):
    alpha = 1.0 / theta
    Th = _open_uniform(rng, n) * math.pi
    W = rng.standard_exponential(n)
    if alpha == 1.0:
        S = np.ones(n)
    else:
        S = (np.sin(alpha * Th) / np.sin(Th) ** (1.0 / alpha)
             * (np.sin((1.0 - alpha) * Th) / W) ** ((1.0 - alpha) / alpha))
    E1 = rng.standard_exponential(n)
    E2 = rng.standard_exponential(n)
    # U_j = exp(-t_j), t_j = (E_j / S)^alpha; Phi^{-1}(exp(-t)) via ndtri_exp.
    t1 = (E1 / S) ** alpha
    t2 = (E2 / S) ** alpha
    t1 = np.maximum(t1, 1e-300)
    t2 = np.maximum(t2, 1e-300)
    return ndtri_exp(-t1), ndtri_exp(-t2)


def copula_pairs(family: str, theta: float, n: int, seed: int, dtype=np.float64):
    rng = np.random.default_rng(seed)
    if family == "gaussian":
        x, y = gaussian_pairs(n, theta, rng)
    elif family == "frank":
        x, y = frank_pairs(n, theta, rng)
    elif family == "gumbel":
        x, y = gumbel_pairs(n, theta, rng)
    else:
        raise ValueError(family)
    return np.ascontiguousarray(x, dtype=dtype), np.ascontiguousarray(y, dtype=dtype)


# ----------------------------------------------------------------------------
# Kendall tau -> theta, used only to draw per-replicate parameters.

def _frank_tau(theta: float) -> float:
    if abs(theta) < 1e-8:
        return theta / 9.0
    d1 = integrate.quad(lambda t: t / math.expm1(t) if t != 0 else 1.0, 0.0, theta,
                        epsabs=1e-14, epsrel=1e-13)[0] / theta
    return 1.0 - 4.0 / theta * (1.0 - d1)


def theta_from_tau(family: str, tau: float) -> float:
    if family == "gaussian":
        return math.sin(math.pi * tau / 2.0)
    if family == "gumbel":
        return 1.0 / (1.0 - tau)
    if family == "frank":
        return optimize.brentq(lambda th: _frank_tau(th) - tau, -500.0, 500.0, xtol=1e-14)
    raise ValueError(family)


# ----------------------------------------------------------------------------
# Splits.

def largest_remainder(n: int, weights: np.ndarray) -> np.ndarray:
    """Integer sizes summing to n: floor(n w / sum w), remainder to the largest
    fractional parts (ties to the lower index)."""
    w = np.asarray(weights, dtype=np.float64)
    share = n * w / w.sum()
    sizes = np.floor(share).astype(np.int64)
    rem = n - int(sizes.sum())
    if rem > 0:
        frac = share - sizes
        order = np.lexsort((np.arange(len(w)), -frac))
        sizes[order[:rem]] += 1
    return sizes


def offsets_from_sizes(sizes: np.ndarray) -> np.ndarray:
    off = np.zeros(len(sizes) + 1, dtype=np.int64)
    np.cumsum(sizes, out=off[1:])
    return off


def equal_offsets(n: int, K: int) -> np.ndarray:
    return np.array([(n * k) // K for k in range(K + 1)], dtype=np.int64)


def dirichlet_offsets(n: int, K: int, rng: np.random.Generator) -> np.ndarray:
    return offsets_from_sizes(largest_remainder(n, rng.standard_exponential(K)))


def uniform_size_offsets(n: int, K: int, lo: float, hi: float, rng: np.random.Generator) -> np.ndarray:
    return offsets_from_sizes(largest_remainder(n, rng.uniform(lo, hi, K)))


# ----------------------------------------------------------------------------
# Workloads.

@dataclasses.dataclass
class Workload:
    """A batch of groups; group g holds subsets [group_offsets[g], group_offsets[g+1])
    over rows [offsets[group_offsets[g]], offsets[group_offsets[g+1]])."""
    name: str
    x: np.ndarray
    y: np.ndarray
    offsets: np.ndarray
    group_offsets: np.ndarray
    families: List[str]
    thetas: List[float]
    seeds: List[int]

    @property
    def n(self) -> int:
        return int(self.offsets[-1])

    @property
    def K(self) -> int:
        return len(self.offsets) - 1

    @property
    def G(self) -> int:
        return len(self.group_offsets) - 1


def _concat(name, parts, dtype):
    xs, ys, offs, gofs = [], [], [0], [0]
    fams, ths, seeds = [], [], []
    base = 0
    for (x, y, off, fam, th, seed) in parts:
        xs.append(np.asarray(x, dtype=dtype))
        ys.append(np.asarray(y, dtype=dtype))
        offs.extend((off[1:] + base).tolist())
        base += int(off[-1])
        gofs.append(gofs[-1] + len(off) - 1)
        fams.append(fam)
        ths.append(th)
        seeds.append(seed)
    return Workload(name, np.concatenate(xs), np.concatenate(ys), np.array(offs, dtype=np.int64),
                    np.array(gofs, dtype=np.int64), fams, ths, seeds)


def gaussian_1e4(K: int) -> Workload:
    """n = 10,000 Gaussian pairs, rho = 0.5, seed 0, K in {1, 10}, FP64."""
    g = np.random.default_rng(0).standard_normal((2, 10_000))
    x = g[0]
    y = 0.5 * g[0] + math.sqrt(0.75) * g[1]
    return _concat(f"gaussian rho=0.5 n=1e4 K={K} fp64", [(x, y, equal_offsets(10_000, K), "gaussian", 0.5, 0)],
                   np.float64)


MILLION_ROW_THETA = {"gaussian": 0.7, "frank": 5.0, "gumbel": 2.0}


def one_million_rows(family: str, K: int, n: int = 1_000_000) -> Workload:
    """n = 1e6 pairs of one family (Gaussian 0.7, Frank 5, Gumbel 2), K equal subsets, FP64."""
    seed = 2000 + FAMILY_CODES[family]
    th = MILLION_ROW_THETA[family]
    x, y = copula_pairs(family, th, n, seed)
    return _concat(f"{family} theta={th} n={n} K={K} fp64", [(x, y, equal_offsets(n, K), family, th, seed)],
                   np.float64)


def replicate_batch(replicates: int = 1000, n: int = 100_000, K: int = 50, seed0: int = 3000) -> Workload:
    """Replicates of n pairs, family = r mod 3, Kendall tau ~ U[0.1, 0.8],
    K Dirichlet(1) subsets per replicate; FP32 storage. Replicates are drawn
    on a thread pool; each has its own seeds, so the result does not depend on
    the number of workers."""
    fams = ["gaussian", "frank", "gumbel"]

    def one(r):
        rng = np.random.default_rng(seed0 + r)
        fam = fams[r % 3]
        tau = rng.uniform(0.1, 0.8)
        th = theta_from_tau(fam, tau)
        x, y = copula_pairs(fam, th, n, seed0 + 100_000 + r, dtype=np.float32)
        off = dirichlet_offsets(n, K, rng)
        return (x, y, off, fam, th, seed0 + r)

    with concurrent.futures.ThreadPoolExecutor(min(16, os.cpu_count() or 1)) as ex:
        parts = list(ex.map(one, range(replicates)))
    return _concat(f"{replicates} replicates x n={n}, K={K} Dirichlet(1) fp32", parts, np.float32)


HUNDRED_MILLION_SETTINGS = [("gumbel", 3.0), ("frank", -8.0)]


def hundred_million_rows(family: str, theta: float, n: int = 100_000_000, K: int = 1000) -> Workload:
    """One family at n pairs in FP32 storage, K equal subsets."""
    seed = 4000 + FAMILY_CODES[family]
    x, y = _chunked_pairs(family, theta, n, seed, np.float32)
    return _concat(f"{family} theta={theta} n={n} K={K} fp32", [(x, y, equal_offsets(n, K), family, theta, seed)],
                   np.float32)


NINE_SETTINGS = [("frank", -10.0), ("frank", -1.0), ("frank", 0.01), ("frank", 1.0), ("frank", 10.0),
           ("frank", 30.0), ("gaussian", -0.95), ("gaussian", 0.0), ("gaussian", 0.95)]


def nine_settings(settings: Sequence = NINE_SETTINGS, n: int = 10_000_000, K: int = 1000, lo: float = 5000.0,
            hi: float = 15000.0) -> Workload:
    """Each setting: n pairs in FP32, K subsets with sizes ~ U[lo, hi] renormalised to n."""
    parts = []
    for i, (fam, th) in enumerate(settings):
        seed = 5000 + i
        x, y = _chunked_pairs(fam, th, n, seed, np.float32)
        off = uniform_size_offsets(n, K, lo, hi, np.random.default_rng(seed + 500))
        parts.append((x, y, off, fam, th, seed))
    return _concat(f"{len(settings)} settings x n={n}, K={K} U[{lo:g},{hi:g}] fp32", parts, np.float32)


def _chunked_pairs(family: str, theta: float, n: int, seed: int, dtype, chunk: int = 1 << 22,
                   workers: int = 0):
    """Draw n pairs in chunks (bounded float64 temporaries), seeded per chunk.
    Chunks are drawn on a thread pool (numpy releases the GIL in its bulk
    generators and ufuncs); every chunk has its own seed, so the result does
    not depend on the number of workers."""
    x = np.empty(n, dtype=dtype)
    y = np.empty(n, dtype=dtype)
    starts = list(range(0, n, chunk))

    def one(c):
        start = starts[c]
        m = min(chunk, n - start)
        xs, ys = copula_pairs(family, theta, m, seed * 1_000_003 + c)
        x[start:start + m] = xs
        y[start:start + m] = ys

    workers = workers or min(16, os.cpu_count() or 1)
    if workers <= 1 or len(starts) <= 1:
        for c in range(len(starts)):
            one(c)
    else:
        with concurrent.futures.ThreadPoolExecutor(workers) as ex:
            list(ex.map(one, range(len(starts))))
    return x, y
