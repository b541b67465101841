"""GPU parity inside the precision bands of the FP32-compensated path.

The FP32 row arithmetic hands over to FP64 near the family boundaries
(Sec. 2.2 parameter ranges of eq. 8, 10, 11): Frank far from independence
(|theta| > 50), the Gaussian near |rho| = 1 (FP64 rows above |rho| = 0.99,
FP64 normal scores in the sufficient statistics above |rho_S| = 0.98), and
Gumbel just above theta = 1. Each case here puts estimates inside a band,
on subsets of the workgroup path (5000..15000 rows) and of the streaming path
(more than 16384 rows), and compares every subset with the FP64 oracle at the
tolerances of the parity tests: FP32c Frank / Gumbel 1e-5 relative to
max(|theta|, 0.1), Gaussian 1e-6 relative; FP64 1e-6 relative.
"""
import numpy as np
import pytest
import torch

import oracle.oracle as O
import synth
from test_gpu_parity import compare, dev, to_np

pytestmark = pytest.mark.gpu

WG_SIZES = [5000, 9000, 15000, 12000, 7000, 11000, 6000, 14000]
BIG_SIZES = [20000, 40000, 17000]

# (family, theta, band test on the oracle's estimates)
BAND_CASES = [
    ("gumbel", 1.01, lambda t: (t > 1.0) & (t <= 1.05)),
    ("gumbel", 1.03, lambda t: (t > 1.0) & (t <= 1.05)),
    ("gumbel", 1.1, lambda t: (t > 1.05) & (t <= 1.2)),
    ("frank", -120.0, lambda t: t < -50.0),
    ("frank", 80.0, lambda t: t > 50.0),
    ("gaussian", 0.985, lambda t: (np.abs(t) > 0.98) & (np.abs(t) <= 0.99)),
    ("gaussian", 0.995, lambda t: np.abs(t) > 0.99),
    ("gaussian", -0.995, lambda t: np.abs(t) > 0.99),
]

_cache = {}


def band_case(fam, th, path):
    key = (fam, th, path)
    if key not in _cache:
        sizes = np.array(WG_SIZES if path == "workgroup" else BIG_SIZES)
        seed = 700 + int(abs(th) * 100) % 97 + (0 if path == "workgroup" else 50) + (1 if th < 0 else 0)
        x, y = synth.copula_pairs(fam, th, int(sizes.sum()), seed)
        # FP32 storage: the oracle reads the same rounded values
        x = x.astype(np.float32).astype(np.float64)
        y = y.astype(np.float32).astype(np.float64)
        off = synth.offsets_from_sizes(sizes)
        _cache[key] = (x, y, off) + O.fit(x, y, off, fam, nthreads=0)
    return _cache[key]


@pytest.mark.parametrize("path", ["workgroup", "streaming"])
@pytest.mark.parametrize("fam,th,band", BAND_CASES, ids=[f"{f}{t}" for f, t, _ in BAND_CASES])
@pytest.mark.parametrize("prec", ["fp32c", "fp64"])
def test_band_parity(fam, th, band, path, prec):
    x, y, off, sub, comb = band_case(fam, th, path)
    interior = (sub["status"] == 0) & band(sub["theta"])
    print(f"[band] {fam} {th} {path}: {int(interior.sum())} of {len(sub['theta'])} oracle estimates inside the band",
          flush=True)
    assert interior.any(), "no oracle estimate falls inside the band: the case does not test it"
    dt = torch.float32
    res = to_np(__import__("paper_1609_05530_amd").fit(dev(x, dt), dev(y, dt), off, fam, prec=prec))
    compare(res, sub, comb, prec, fam, f"band {fam} {th} {path} {prec}")
