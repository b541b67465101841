"""Row partitions of a data set into subsets (eq. 14) by different schemes:
the input side of the study of how the partitioning affects the combined
estimate, which Sec. 4 of arXiv:1609.05530 leaves as future work.

TEST INFRASTRUCTURE, like ``oracle.py``: only the test suite,
``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` may import
it. Plain numpy.

A data set holds R replicates; replicate r is rows rep_offsets[r] ..
rep_offsets[r+1] - 1 (N_r rows) and is split into M subsets, subset (r, m)
becoming rows offsets[r M + m] .. offsets[r M + m + 1] - 1 of the output
(the replicates keep their row ranges). p(i) is row i's position, from 0, in
its replicate's order of x, ties (equal values; -0 equals +0) by row order:
the ranks of eq. (12) with ties broken by row order, minus one.

  contiguous : the paper's split (Sec. 2.5: equal subsets of N/M rows), for
               any N: subset m is the stored rows floor(m N / M) ..
               floor((m + 1) N / M) - 1, rows copied in place.
  blocks     : subset m is the positions floor(m N / M) .. floor((m + 1) N / M)
               - 1 of the x-order: M disjoint slices of x's range (the
               subsets are not samples of the joint distribution).
  strided    : subset m is the positions p with p mod M = m: every M-th row
               of the x-order (a systematic sample across x's range); it has
               ceil((N - m) / M) rows.
Inside a subset the rows are in stored order (contiguous) or in x-order
(blocks, strided). x must be finite.
"""
from __future__ import annotations

import numpy as np

SCHEMES = ("contiguous", "blocks", "strided")


def even_bounds(N: int, M: int) -> np.ndarray:
    """floor(m N / M) for m = 0 .. M."""
    return np.array([(m * N) // M for m in range(M + 1)], dtype=np.int64)


def x_order(x: np.ndarray) -> np.ndarray:
    """Rows of one replicate in order of x, ties by row order (a stable sort;
    numpy compares -0 and +0 as equal)."""
    return np.argsort(np.asarray(x), kind="stable")


def split_one(x: np.ndarray, M: int, scheme: str):
    """One replicate: (rows of the output in order, subset sizes)."""
    N = len(x)
    if scheme == "contiguous":
        return np.arange(N, dtype=np.int64), np.diff(even_bounds(N, M))
    order = x_order(x)
    if scheme == "blocks":
        return order.astype(np.int64), np.diff(even_bounds(N, M))
    if scheme == "strided":
        # subset m collects order[m], order[m + M], order[m + 2M], ...
        parts = [order[m::M] for m in range(M)]
        return np.concatenate(parts).astype(np.int64) if N else np.zeros(0, np.int64), \
            np.array([len(q) for q in parts], dtype=np.int64)
    raise ValueError(f"unknown scheme {scheme!r}")


def partition(x: np.ndarray, y: np.ndarray, rep_offsets, M: int, scheme: str):
    """(x_out, y_out, offsets[R M + 1]) for every replicate of the data set."""
    if M < 1:
        raise ValueError("M must be >= 1")
    rep = np.asarray(rep_offsets, dtype=np.int64)
    x = np.asarray(x)
    y = np.asarray(y)
    xo = np.empty_like(x)
    yo = np.empty_like(y)
    offs = [0]
    for r in range(len(rep) - 1):
        b, e = int(rep[r]), int(rep[r + 1])
        rows, sizes = split_one(x[b:e], M, scheme)
        xo[b:e] = x[b:e][rows]
        yo[b:e] = y[b:e][rows]
        offs.extend((b + np.cumsum(sizes)).tolist())
    return xo, yo, np.array(offs, dtype=np.int64)
