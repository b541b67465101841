"""The simulation study of Sec. 2.5-2.6 of arXiv:1609.05530 on the device.

One cell of the study (a family at theta, full-data size N, M subsets, S
replicates): replicate s is rows [s N, (s + 1) N) of one seeded stream drawn
by the on-device sampler; every replicate is fitted on its M equal subsets
and combined (eq. 16: one cpc_fit_batched group per replicate) and on its
full data (a group of one subset); the replicate summary gives eq. (17),
(18), the estimated bias and MSE, and the densities at the two means give the
relative L1 and L2 distances of eq. (19)-(20). Every step runs in the HIP
kernels of libcpc; this module only sequences the calls.

The study grid of Sec. 2.5: Gaussian theta = 0.3, Frank theta = 5, Gumbel
theta = 5; N in {50000, 100000, 200000}; M in {10, 20, 100}; S = 50. The draws
of a (family, N) pair are shared by its three values of M.

    python -m paper_1609_05530_amd.study [--S 50] [--prec fp64]
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np
import torch

PAPER_THETA = {"gaussian": 0.3, "frank": 5.0, "gumbel": 5.0}
PAPER_N = (50_000, 100_000, 200_000)
PAPER_M = (10, 20, 100)
# Sec. 3.2: largest estimated bias and MSE over the grid per family, and the
# bound on the relative L1 / L2 errors (all families)
PAPER_BOUNDS = {"bias": {"gaussian": 0.002, "frank": 0.008, "gumbel": 0.008},
                "mse": {"gaussian": 4e-6, "frank": 7e-5, "gumbel": 9e-5},
                "l1_l2": 0.0013}


def draw(family: str, theta: float, S: int, N: int, seed: int, dtype=torch.float64, device="cuda"):
    """S replicates of N pairs (rows [s N, (s + 1) N) of the seeded stream)."""
    from . import sample
    return sample(family, theta, S * N, seed=seed, row0=0, dtype=dtype, device=device)


def fit_subsets(x, y, family: str, N: int, M: int, S: int, prec: str = "fp64"):
    """eq. (16): each replicate's M equal subsets fitted and combined (one
    group per replicate)."""
    from . import fit_batched
    if N % M:
        raise ValueError("N must be a multiple of M")
    off = np.arange(0, S * N + 1, N // M, dtype=np.int64)
    gofs = np.arange(0, S * M + 1, M, dtype=np.int64)
    return fit_batched(x, y, off, gofs, [family] * S, prec=prec)


def fit_full(x, y, family: str, N: int, S: int, prec: str = "fp64"):
    """Each replicate's full-data estimate (a group of one subset)."""
    from . import fit_batched
    off = np.arange(0, S * N + 1, N, dtype=np.int64)
    return fit_batched(x, y, off, np.arange(0, S + 1, dtype=np.int64), [family] * S, prec=prec)


def metrics(family: str, sub, full, panels: int = 256, box=None):
    """[eq. 17, eq. 18, bias, MSE, replicates used] and
    [int |c_F - c_C|, int c_F, int (c_F - c_C)^2, int c_F^2] at the two means
    (device tensors; no host round trip between the steps)."""
    from . import density_distance, replicate_summary
    summ = replicate_summary(sub.raw_comb, full.raw_comb)
    dist = density_distance(family, summ[1:2], summ[0:1], panels=panels, box=box)[0]
    return summ, dist


def run_cell(family: str, theta: float, N: int, M: int, S: int, seed: int = 1, prec: str = "fp64",
             panels: int = 256, x=None, y=None, full=None):
    dtype = torch.float64 if prec == "fp64" else torch.float32
    if x is None:
        x, y = draw(family, theta, S, N, seed, dtype=dtype)
    if full is None:
        full = fit_full(x, y, family, N, S, prec=prec)
    sub = fit_subsets(x, y, family, N, M, S, prec=prec)
    summ, dist = metrics(family, sub, full, panels=panels)
    s = summ.cpu().numpy()
    d = dist.cpu().numpy()
    return {"x": x, "y": y, "sub": sub, "full": full, "summary": s, "distance": d,
            "rel_l1": float(d[0] / d[1]), "rel_l2": float(np.sqrt(d[2] / d[3]))}


def run_grid(S: int = 50, prec: str = "fp64", seed0: int = 5000, panels: int = 256, log=sys.stderr):
    """The grid of Sec. 2.5; one row per (family, N, M) with the Sec. 2.6
    metrics and the time of the cell (its subset fits and metrics; the draw
    and the full-data fit of a (family, N) pair are timed once, on its first
    row)."""
    rows = []
    for fi, (family, theta) in enumerate(PAPER_THETA.items()):
        for N in PAPER_N:
            dtype = torch.float64 if prec == "fp64" else torch.float32
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            x, y = draw(family, theta, S, N, seed0 + 10 * fi + PAPER_N.index(N), dtype=dtype)
            full = fit_full(x, y, family, N, S, prec=prec)
            torch.cuda.synchronize()
            t_shared = time.perf_counter() - t0
            for M in PAPER_M:
                t0 = time.perf_counter()
                r = run_cell(family, theta, N, M, S, prec=prec, panels=panels, x=x, y=y, full=full)
                torch.cuda.synchronize()
                dt = time.perf_counter() - t0 + t_shared
                t_shared = 0.0
                s = r["summary"]
                row = {"family": family, "theta": theta, "N": N, "M": M, "S": int(s[4]),
                       "theta_combined_sim": float(s[0]), "theta_full_sim": float(s[1]),
                       "bias": float(s[2]), "mse": float(s[3]), "rel_l1": r["rel_l1"], "rel_l2": r["rel_l2"],
                       "seconds": dt}
                rows.append(row)
                print(f"[study] {family} N={N} M={M}: bias {s[2]:+.2e} mse {s[3]:.2e} "
                      f"L1 {r['rel_l1']:.2e} L2 {r['rel_l2']:.2e} ({dt:.3f} s)", file=log, flush=True)
            del x, y, full
    return rows


PARTITION_STUDY_SCHEMES = ("contiguous", "unequal", "blocks", "strided")


def unequal_offsets(N: int, M: int, S: int, seed: int) -> np.ndarray:
    """Subset bounds of S replicates of N rows, each split into M contiguous
    runs of unequal sizes: Dirichlet(1, ..., 1) proportions w (seeded numpy
    draws), bounds floor(N (w_1 + ... + w_m)), the last one N."""
    rng = np.random.default_rng(seed)
    out = [0]
    for s in range(S):
        c = np.floor(N * np.cumsum(rng.dirichlet(np.ones(M)))).astype(np.int64)
        c[-1] = N
        out.extend((s * N + np.maximum.accumulate(c)).tolist())
    return np.array(out, dtype=np.int64)


def partition_cell(family: str, theta: float, N: int, M: int, S: int, schemes=PARTITION_STUDY_SCHEMES,
                   seed: int = 1, prec: str = "fp64", x=None, y=None, full=None):
    """The partitioning study that Sec. 4 leaves as future work, for one
    cell: the same S replicates of N rows split into M subsets by each
    scheme, fitted and combined per replicate (eq. 16), and summarised
    against the full-data estimates like the grid (eq. 17, 18, bias, MSE);
    also the mean combined estimate's distance from theta and the spread of
    the combined estimates. Schemes: those of cpc_partition ("contiguous",
    "blocks", "strided") and "unequal" (contiguous runs of Dirichlet(1)
    sizes, the unequal subsets that Sec. 4 says the inverse-variance weights
    account for). One dict per scheme."""
    from . import fit_batched, partition, replicate_summary
    dtype = torch.float64 if prec == "fp64" else torch.float32
    if x is None:
        x, y = draw(family, theta, S, N, seed, dtype=dtype)
    if full is None:
        full = fit_full(x, y, family, N, S, prec=prec)
    rep = np.arange(0, S * N + 1, N, dtype=np.int64)
    gofs = np.arange(0, S * M + 1, M, dtype=np.int64)
    out = []
    for scheme in schemes:
        if scheme == "unequal":
            xo, yo, offs = x, y, unequal_offsets(N, M, S, seed + 7919)
        else:
            xo, yo, offs = partition(x, y, rep, M, scheme)
        sub = fit_batched(xo, yo, offs, gofs, [family] * S, prec=prec)
        s = replicate_summary(sub.raw_comb, full.raw_comb).cpu().numpy()
        comb = sub.raw_comb[:, 0].cpu().numpy()
        out.append({"scheme": scheme, "family": family, "theta": theta, "N": N, "M": M, "S": int(s[4]),
                    "theta_combined_sim": float(s[0]), "theta_full_sim": float(s[1]), "bias": float(s[2]),
                    "mse": float(s[3]), "bias_vs_theta": float(np.nanmean(comb) - theta),
                    "sd_combined": float(np.nanstd(comb))})
        del xo, yo, sub
    return out


def outside_paper_bounds(rows, slack: float = 1.0):
    """Rows whose |bias|, MSE or L1 / L2 exceed Sec. 3.2's bounds times slack."""
    bad = []
    for r in rows:
        f = r["family"]
        if (abs(r["bias"]) > slack * PAPER_BOUNDS["bias"][f] or r["mse"] > slack * PAPER_BOUNDS["mse"][f]
                or r["rel_l1"] > slack * PAPER_BOUNDS["l1_l2"] or r["rel_l2"] > slack * PAPER_BOUNDS["l1_l2"]):
            bad.append(r)
    return bad


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--S", type=int, default=50)
    ap.add_argument("--prec", default="fp64", choices=["fp64", "fp32c"])
    ap.add_argument("--panels", type=int, default=256)
    a = ap.parse_args()
    rows = run_grid(S=a.S, prec=a.prec, panels=a.panels)
    print(json.dumps({"rows": rows, "outside_paper_bounds": len(outside_paper_bounds(rows))}))


if __name__ == "__main__":
    main()
