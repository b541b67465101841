"""AddressSanitizer + UndefinedBehaviorSanitizer builds of the host code, run
on the CPU: the oracle (gcc, its own sanitizer runtime) over every entry
point on small inputs with ties, degenerate subsets and every family, and
the C ABI's host side (cpc_api.cpp built by hipcc with the sanitizers on its
host pass only, linked with the kernel objects of the regular build) over
the calls that run without a GPU: options, workspace sizing over valid and
invalid partitions, and the argument checks made before any device call.

Each library is loaded in a child Python process that preloads the matching
sanitizer runtime; a report (or a non-zero exit) fails the test."""
import os
import shutil
import subprocess
import sys
import textwrap

import pytest

from conftest import ROOT

ORACLE_SRC = os.path.join(ROOT, "oracle", "cpc_oracle.c")
CSRC = os.path.join(ROOT, "paper_1609_05530_amd", "csrc")
BUILD = os.path.join(ROOT, "_build")
SAN_ENV = {"ASAN_OPTIONS": "detect_leaks=0:abort_on_error=0:exitcode=23",
           "UBSAN_OPTIONS": "print_stacktrace=1:halt_on_error=1:exitcode=24"}


# first lines of every child: the sanitizer runtime is mapped into the process
_PROLOGUE = """
import sys
with open("/proc/self/maps") as _f:
    assert "asan" in _f.read(), "the sanitizer runtime is not loaded"
"""


def _run_child(script: str, preload: str, tmp_path):
    path = tmp_path / "child.py"
    path.write_text(_PROLOGUE + textwrap.dedent(script))
    env = dict(os.environ, LD_PRELOAD=preload, PYTHONPATH=ROOT, OMP_NUM_THREADS="2", **SAN_ENV)
    r = subprocess.run([sys.executable, str(path)], env=env, cwd=ROOT, capture_output=True, text=True, timeout=600)
    out = r.stdout + r.stderr
    assert "ERROR: AddressSanitizer" not in out, out[-4000:]
    assert "runtime error:" not in out, out[-4000:]
    assert r.returncode == 0, out[-4000:]
    assert "child done" in r.stdout, out[-4000:]


def test_oracle_under_asan_ubsan(tmp_path):
    rt = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    if not os.path.isabs(rt) or not os.path.exists(rt):
        pytest.skip("gcc's AddressSanitizer runtime is not installed")
    lib = tmp_path / "liboracle_san.so"
    subprocess.check_call(["gcc", "-O1", "-g", "-std=c11", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                           "-fno-omit-frame-pointer", "-o", str(lib), ORACLE_SRC, "-lm"])
    _run_child(f"""
        import numpy as np
        import oracle.oracle as O
        O.LIB = {str(lib)!r}   # the sanitized build (newer than the source: no rebuild)
        import synth
        rng = np.random.default_rng(1)
        sizes = np.array([0, 1, 2, 3, 40, 257, 1000])
        off = synth.offsets_from_sizes(sizes)
        n = int(off[-1])
        for fam, th in (("gaussian", 0.6), ("frank", -4.0), ("gumbel", 1.8)):
            x, y = synth.copula_pairs(fam, th, n, 11)
            x[off[5]:off[5] + 60] = np.round(x[off[5]:off[5] + 60])      # ties
            y[off[4]:off[5]] = 1.0                                       # a constant margin
            for ties in ("average", "first"):
                sub, comb = O.fit(x, y, off, fam, ties=ties)
            O.combine(sub, np.array([0, 3, 7]))
            R1 = np.concatenate([O.ranks(x[off[m]:off[m + 1]]) for m in range(len(sizes))])
            R2 = np.concatenate([O.ranks(y[off[m]:off[m + 1]]) for m in range(len(sizes))])
            O.spearman_fit_ranks(R1, R2, off, fam, np.array([0, 4, 7]))
            r1, r2 = R1[off[6]:], R2[off[6]:]
            O.ggr(r1, r2, fam, th)
            O.spearman_var(r1, r2, fam, th)
            O.sample(fam, th, 5, 3, 300)
            O.density_distance(fam, th, th * 1.01, box=8.0, panels=8)
            O.tau(fam, th); O.rho_s(fam, th)
        O.replicate_summary(np.array([1.0, 1.1, np.nan]), np.array([0, 0, 3], dtype=np.int32),
                            np.array([1.0, 1.2, 1.0]), np.array([0, 0, 0], dtype=np.int32))
        O.qnorm(np.array([1e-300, 0.3, 0.5, 1.0 - 1e-16]))
        O.debye(1, 3.0); O.debye(2, -150.0)
        O.philox4x32_10(np.array([1, 2, 3, 4], dtype=np.uint32), np.array([5, 6], dtype=np.uint32))
        print("child done")
    """, rt, tmp_path)


def test_abi_host_side_under_asan_ubsan(tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    rt = subprocess.run([hipcc, "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True,
                        text=True).stdout.strip()
    if not os.path.isabs(rt) or not os.path.exists(rt):
        pytest.skip("clang's AddressSanitizer runtime is not installed")
    from paper_1609_05530_amd import build as B
    kernels = [os.path.join(BUILD, os.path.splitext(s)[0] + ".o") for s in B.SOURCES if s != "cpc_api.cpp"]
    if not all(os.path.exists(k) for k in kernels):
        pytest.skip("the kernel objects are not built (python -m paper_1609_05530_amd.build)")
    obj = tmp_path / "cpc_api_san.o"
    lib = tmp_path / "libcpc_san.so"
    # sanitizers on the host pass only (the device code is unchanged)
    san = "-Xarch_host -fsanitize=address -Xarch_host -fsanitize=undefined -Xarch_host -fno-omit-frame-pointer"
    subprocess.check_call([hipcc, *B.COMMON, *san.split(), "-g", "-x", "hip", "-c",
                           os.path.join(CSRC, "cpc_api.cpp"), "-o", str(obj)])
    subprocess.check_call([hipcc, "-shared", "-shared-libsan", *"-Xarch_host -fsanitize=address".split(),
                           *"-Xarch_host -fsanitize=undefined".split(), f"--offload-arch={B.ARCH}", "-o", str(lib),
                           str(obj), *kernels])
    _run_child(f"""
        import ctypes
        import numpy as np
        from paper_1609_05530_amd._lib import SIGNATURES, Options
        L = ctypes.CDLL({str(lib)!r})
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name); f.restype = res; f.argtypes = args
        o = Options()
        L.cpc_default_options(ctypes.byref(o))
        assert L.cpc_workspace_bytes(10**6, 100, 3, 0, ctypes.byref(o)) > 0
        assert L.cpc_workspace_bytes(-1, 10, 1, 0, ctypes.byref(o)) == 0
        good = np.array([0, 5000, 5000, 40000, 41000], dtype=np.int64)
        assert L.cpc_workspace_bytes_for(good.ctypes.data, 4, 2, 0, ctypes.byref(o)) > 0
        for bad, K in ((np.array([0, 5, 3], dtype=np.int64), 2), (np.array([1, 5], dtype=np.int64), 1),
                       (np.array([0, -1], dtype=np.int64), 1), (np.array([0], dtype=np.int64), 0)):
            assert L.cpc_workspace_bytes_for(bad.ctypes.data, K, 1, 0, ctypes.byref(o)) == 0
        assert len(L.cpc_last_error()) > 0
        assert L.cpc_spearman_workspace_bytes(1000, 10, 2) > 0
        for code in range(-12, 2):
            assert len(L.cpc_strerror(code)) > 0
        off = np.array([0, 5, 10], dtype=np.int64)
        assert L.cpc_fit(None, 1, 1, 0, 10, off.ctypes.data, 2, 0, ctypes.byref(o), 1, 1 << 20, 1, 1, None) == -7
        print("child done")
    """, rt, tmp_path)
