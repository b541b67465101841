"""Builds libcpc.so (the HIP kernels + C ABI) for gfx950, in-tree.

Also builds libcpc_hostmath.so, a host-only compilation of the kernels'
per-row arithmetic used by CPU unit tests, and libcpc_probe.so, the VALU
issue-rate probe (include/cpc_probe.h) that bench.py runs.

Usage: python -m paper_1609_05530_amd.build [-v]
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libcpc.so")
HOSTMATH = os.path.join(HERE, "libcpc_hostmath.so")
PROBE = os.path.join(HERE, "libcpc_probe.so")

ARCH = "gfx950"
SOURCES = ["cpc_api.cpp", "k_rank.hip", "k_fit.hip", "k_var.hip", "k_big.hip", "k_eval.hip", "k_combine.hip",
           "k_sample.hip", "k_study.hip", "k_moment.hip", "k_gaussk.hip", "k_partition.hip"]

COMMON = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    # keep FP32 denormals (IEEE semantics on both sides of the parity tests)
    "-fno-gpu-flush-denormals-to-zero",
    # no packed FP32 instructions (their results are not trusted on this hardware)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    f"-I{INCLUDE}", f"-I{CSRC}",
]


def hipcc() -> str:
    p = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    return p


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(l for l in r.stdout.splitlines() if "packed-fp32-ops" not in l and l.strip())
    if r.returncode != 0:
        raise RuntimeError(f"build step failed ({r.returncode}): {' '.join(cmd)}\n{out}")
    if verbose and out:
        print(out)


def build(verbose: bool = False, jobs: int | None = None) -> str:
    os.makedirs(BUILD, exist_ok=True)
    objs = []
    cmds = []
    for src in SOURCES:
        obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
        objs.append(obj)
        lang = ["-x", "hip"] if src.endswith(".cpp") else []
        cmds.append([hipcc(), *COMMON, *lang, "-c", os.path.join(CSRC, src), "-o", obj])
    jobs = jobs or min(len(cmds), max(1, min(16, os.cpu_count() or 1)))
    with cf.ThreadPoolExecutor(jobs) as ex:
        list(ex.map(lambda c: _run(c, verbose), cmds))
    tmp = LIB + ".tmp"
    _run([hipcc(), "-shared", f"--offload-arch={ARCH}", "-o", tmp, *objs], verbose)
    os.replace(tmp, LIB)
    tmp = HOSTMATH + ".tmp"
    _run([hipcc(), *COMMON, "-shared", "-o", tmp, os.path.join(CSRC, "host_math_shim.hip")], verbose)
    os.replace(tmp, HOSTMATH)
    tmp = PROBE + ".tmp"
    _run([hipcc(), *COMMON, "-shared", "-o", tmp, os.path.join(CSRC, "probe_valu.hip")], verbose)
    os.replace(tmp, PROBE)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
