"""The VALU issue-rate probe (include/cpc_probe.h) on the GPU: every
instruction runs, FP32 FMA sustains a large share of the FP32 vector peak
(157.3 TFLOP/s = 256 CUs x 128 FMA lanes x 2.4 GHz), and no transcendental
issues faster than FMA."""
import ctypes
import os

import pytest
import torch

from conftest import ROOT

pytestmark = pytest.mark.gpu

PEAK = 256 * 128 * 2.4e9


def test_probe_rates():
    assert torch.cuda.is_available()
    P = ctypes.CDLL(os.path.join(ROOT, "paper_1609_05530_amd", "libcpc_probe.so"))
    P.cpc_probe_valu.restype = ctypes.c_int
    P.cpc_probe_valu.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_double),
                                 ctypes.POINTER(ctypes.c_float)]
    rates = []
    for op in range(5):
        r, ms = ctypes.c_double(), ctypes.c_float()
        assert P.cpc_probe_valu(0, op, 2048, ctypes.byref(r), ctypes.byref(ms)) == 0, op
        assert ms.value > 0.0
        rates.append(r.value)
    print("[probe] lane ops/s fma exp2 log2 rcp sqrt:", " ".join(f"{v:.3e}" for v in rates), flush=True)
    assert 0.5 * PEAK <= rates[0] <= 1.05 * PEAK, rates[0]
    for v in rates[1:]:
        assert 0.0 < v <= 1.05 * rates[0]
