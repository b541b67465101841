"""The C-ABI library: it loads without a GPU, exports every entry point the
header declares, and rejects misuse on the host before touching the device."""
import ctypes
import os
import re

import pytest

from conftest import ROOT

HEADER = os.path.join(ROOT, "include", "cpc.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(cpc_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def L():
    from paper_1609_05530_amd import _lib
    return _lib.lib()


def test_exports_every_declared_symbol(L):
    names = declared_functions()
    assert len(names) >= 11
    for name in names:
        assert hasattr(L, name), name
    from paper_1609_05530_amd._lib import SIGNATURES
    assert set(SIGNATURES) == set(names)


def test_struct_sizes_match_header():
    from paper_1609_05530_amd._lib import Options
    assert ctypes.sizeof(Options) == 40


def test_defaults_and_workspace(L):
    from paper_1609_05530_amd._lib import Options
    o = Options()
    L.cpc_default_options(ctypes.byref(o))
    assert (o.prec, o.ties, o.var, o.max_iter, o.n_min, o.schedule) == (0, 0, 0, 60, 2, -1)
    a = L.cpc_workspace_bytes(1000, 10, 1, 0, ctypes.byref(o))
    b = L.cpc_workspace_bytes(2000, 10, 1, 0, ctypes.byref(o))
    assert 0 < a < b
    assert L.cpc_workspace_bytes(-1, 10, 1, 0, ctypes.byref(o)) == 0


def test_errors_before_any_device_call(L):
    import numpy as np
    from paper_1609_05530_amd._lib import Options
    o = Options()
    L.cpc_default_options(ctypes.byref(o))
    off = np.array([0, 5, 10], dtype=np.int64)
    rc = L.cpc_fit(None, 1, 1, 0, 10, off.ctypes.data, 2, 0, ctypes.byref(o), 1, 1 << 20, 1, 1, None)
    assert rc == -7  # CPC_E_HANDLE
    assert b"handle" in L.cpc_last_error()
    for code in range(-9, 1):
        assert len(L.cpc_strerror(code)) > 0
    h = ctypes.c_void_p()
    assert L.cpc_create(0, None) == -1  # CPC_E_NULL


PROBE_HEADER = os.path.join(ROOT, "include", "cpc_probe.h")


def test_probe_library_exports_its_header():
    text = re.sub(r"/\*.*?\*/", "", open(PROBE_HEADER).read(), flags=re.S)
    names = sorted(set(re.findall(r"\b(cpc_probe_[a-z_]+)\s*\(", text)))
    assert names == ["cpc_probe_valu"]
    P = ctypes.CDLL(os.path.join(ROOT, "paper_1609_05530_amd", "libcpc_probe.so"))
    for name in names:
        assert hasattr(P, name), name
    P.cpc_probe_valu.restype = ctypes.c_int
    r, ms = ctypes.c_double(), ctypes.c_float()
    # argument checks come before any device call
    assert P.cpc_probe_valu(0, 7, 16, ctypes.byref(r), ctypes.byref(ms)) == -1
    assert P.cpc_probe_valu(0, 0, 0, ctypes.byref(r), ctypes.byref(ms)) == -1


def test_workspace_follows_the_partition(L):
    """The exact workspace of a partition reserves the streaming path's
    arrays (88 bytes per row) only for the rows of subsets above 16384 rows;
    the upper bound assumes every row may be there."""
    import numpy as np
    from paper_1609_05530_amd._lib import Options
    o = Options()
    L.cpc_default_options(ctypes.byref(o))
    n = 2_000_000
    small = np.arange(0, n + 1, 10_000, dtype=np.int64)          # 200 subsets of 10000 rows
    big = np.array([0, 1_000_000, n], dtype=np.int64)             # 2 subsets of 1e6 rows
    mixed = np.array([0, 500_000] + list(range(510_000, n + 1, 10_000)), dtype=np.int64)
    bound = L.cpc_workspace_bytes(n, 200, 1, 1, ctypes.byref(o))
    e_small = L.cpc_workspace_bytes_for(small.ctypes.data, len(small) - 1, 1, 1, ctypes.byref(o))
    e_big = L.cpc_workspace_bytes_for(big.ctypes.data, len(big) - 1, 1, 1, ctypes.byref(o))
    e_mixed = L.cpc_workspace_bytes_for(mixed.ctypes.data, len(mixed) - 1, 1, 1, ctypes.byref(o))
    assert 0 < e_small < e_mixed < e_big <= bound
    assert e_small < 32 * n              # about 28 bytes per row without streaming subsets
    assert e_big >= 116 * n              # the streaming arrays for every row
    assert e_mixed - e_small >= 88 * 500_000
    bad = np.array([0, 10, 5], dtype=np.int64)
    assert L.cpc_workspace_bytes_for(bad.ctypes.data, 2, 1, 1, ctypes.byref(o)) == 0
    assert L.cpc_workspace_bytes_for(None, 2, 1, 1, ctypes.byref(o)) == 0
