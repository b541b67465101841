"""Benchmark of the partition-and-combine MPL copula estimator (arXiv:1609.05530)
on one MI355X.

One step = one cpc_fit_batched over the whole workload: ranks (eq. 12), the
maximisation of eq. (13) for every subset, the Sec. 2.3 variances and the
eq. (15)/(16) combination per group, replayed as one captured hipGraph.
Inputs are resident in HBM before the timed region. Prints one JSON line.

Default workload (the shape the headline metric is quoted on, n = 1e7 per
setting): Frank theta in {-10, -1, 0.01, 1, 10, 30} and Gaussian rho in
{-0.95, 0, 0.95}, each n = 10,000,000 FP32 pairs in K = 1000 subsets with
sizes ~ U[5000, 15000] renormalised; 9 groups, 9000 subset fits per step.
"""
from __future__ import annotations

import argparse
import glob
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# VALU issue slots per row of one Newton pass (per score + Hessian row
# evaluation), counted from the FP32 row formulas: transcendentals (exp, log,
# reciprocal) issue at a quarter of the full rate and count 4 slots each.
#   Frank (|theta| >= 2):  exp x2, rcp x2 (1/b, 1/D)  -> 16 + 30 FMA/mul/add
#   Frank (|theta| <  2):  expm1 x2, rcp x1           -> 12 + 34
#   Gumbel:                exp x2, log x1, rcp x2      -> 20 + 40
#   Gaussian (one pass):   AS 241 x2 (rcp + ~10 FMA)  -> 8 + 23
SLOTS_PER_ROW_PASS = {"frank": 46.0, "gumbel": 60.0, "gaussian": 31.0}
# FP32 vector peak 157.3 TFLOP/s = 78.6 T FMA lane-operations/s (256 CUs x 128
# FMA lanes per clock x 2.4 GHz); the issue probe (libcpc_probe.so) sustains
# most of it with ordinary (non-packed) FP32 instructions.
PEAK_LANE_SLOTS = 256 * 128 * 2.4e9
PEAK_HBM = 8.0e12                       # bytes/s
# Algorithmic HBM bytes per row of the rank step: read x, y (FP32) and write
# the two u16 doubled ranks.
RANK_BYTES_PER_ROW = 4 + 4 + 2 + 2
# the rank kernel's sources (body, launch shapes and shape tables)
RANK_SOURCES = ["paper_1609_05530_amd/csrc/rank_wg.h", "paper_1609_05530_amd/csrc/block_rank.h",
                "paper_1609_05530_amd/csrc/k_rank.hip", "paper_1609_05530_amd/csrc/rank_shapes.h"]
# the fit and variance kernels' sources (bodies and the device math they use)
FIT_VAR_SOURCES = ["paper_1609_05530_amd/csrc/k_fit.hip", "paper_1609_05530_amd/csrc/k_var.hip",
                   "paper_1609_05530_amd/csrc/family_math.h", "paper_1609_05530_amd/csrc/row_eval.h",
                   "paper_1609_05530_amd/csrc/solver.h", "paper_1609_05530_amd/csrc/cpc_device.h"]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--prec", default="fp32c", choices=["fp32c", "fp64"])
    ap.add_argument("--n", type=int, default=10_000_000, help="rows per setting")
    ap.add_argument("--K", type=int, default=1000, help="subsets per setting")
    ap.add_argument("--settings", default="all", help="'all' or a comma list of indices into the 9 settings")
    ap.add_argument("--no-graph", action="store_true", help="launch eagerly instead of replaying a hipGraph")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64-compare", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=64, help="subsets per setting in the CPU-baseline sample")
    ap.add_argument("--profile", action="store_true", help="short run for a profiler (no oracle, no checks)")
    ap.add_argument("--no-small-configs", action="store_true",
                    help="skip the GPU times of the n=1e4 and n=1e6 FP64 workloads")
    ap.add_argument("--no-legs", action="store_true",
                    help="skip the n=1e8, replicate-batch and Gumbel legs")
    ap.add_argument("--legs", default="",
                    help="comma-separated names of the legs to run (default: all of them)")
    ap.add_argument("--oracle-1thread", action="store_true",
                    help="also time the oracle on one thread on the n=1e4 and n=1e6 workloads (minutes)")
    return ap.parse_args()


def source_hash(paths) -> str:
    h = hashlib.sha256()
    for p in paths:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def rank_source_hash() -> str:
    return source_hash(RANK_SOURCES)


def valu_probe():
    """Measured lane operations per second of FP32 FMA and of the FP32
    transcendental instructions (libcpc_probe.so), and each transcendental's
    cost in FMA issue slots; None if the probe library is missing."""
    import ctypes
    path = os.path.join(ROOT, "paper_1609_05530_amd", "libcpc_probe.so")
    if not os.path.exists(path):
        return None
    L = ctypes.CDLL(path)
    L.cpc_probe_valu.restype = ctypes.c_int
    L.cpc_probe_valu.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_double),
                                 ctypes.POINTER(ctypes.c_float)]
    rates = {}
    for op, name in enumerate(("fma", "exp2", "log2", "rcp", "sqrt")):
        r, ms = ctypes.c_double(), ctypes.c_float()
        if L.cpc_probe_valu(0, op, 2048, ctypes.byref(r), ctypes.byref(ms)) != 0:
            return None
        rates[name] = r.value
    return {"lane_ops_per_s": {k: v for k, v in rates.items()},
            "slots_per_op": {k: rates["fma"] / v for k, v in rates.items() if k != "fma"},
            "fma_vs_peak": rates["fma"] / PEAK_LANE_SLOTS}


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def small_configs(cpc, synth, dev, oracle_1thread):
    """The n = 1e4 Gaussian workload (K = 1, 10) and the n = 1e6 workloads of
    the three families (K = 1, 10, 100) on the FP64 GPU path: median time of
    a graph replay with inputs resident in HBM. With oracle_1thread, the
    oracle's one-thread wall time (host arrays to results) on each, all of
    them run side by side on host threads, and the GPU's error against it."""
    import torch
    cases = [synth.gaussian_1e4(K) for K in (1, 10)]
    cases += [synth.one_million_rows(f, K) for f in ("gaussian", "frank", "gumbel") for K in (1, 10, 100)]
    rows = []
    for w in cases:
        x = torch.from_numpy(w.x).to(dev)
        y = torch.from_numpy(w.y).to(dev)
        ws = torch.empty(cpc.workspace_bytes(w.n, w.K, w.G, dtype=x.dtype, offsets=w.offsets, prec="fp64"), dtype=torch.uint8,
                         device=dev)
        out = cpc.FitResult(torch.empty((w.K, 6), dtype=torch.float64, device=dev),
                            torch.empty((w.G, 5), dtype=torch.float64, device=dev))

        def step():
            cpc.fit_batched(x, y, w.offsets, w.group_offsets, w.families, workspace=ws, out=out, prec="fp64",
                            graph=True)
        for _ in range(2):
            step()
        torch.cuda.synchronize()
        evs = [torch.cuda.Event(enable_timing=True) for _ in range(11)]
        evs[0].record()
        for i in range(10):
            step()
            evs[i + 1].record()
        torch.cuda.synchronize()
        ms = float(np.median([evs[i].elapsed_time(evs[i + 1]) for i in range(10)]))
        rows.append({"workload": w.name, "gpu_ms": ms, "theta_combined": float(out.combined_theta.cpu().numpy()[0]),
                     "_theta": out.theta.cpu().numpy()})
        print(f"[small configs] {w.name}: {ms:.3f} ms", file=sys.stderr, flush=True)
        del x, y, ws, out
    if oracle_1thread:
        from concurrent.futures import ThreadPoolExecutor
        import oracle.oracle as O

        def run(w):
            t0 = time.perf_counter()
            sub, _ = O.fit(w.x, w.y, w.offsets, w.families, w.group_offsets, nthreads=1)
            dt = time.perf_counter() - t0
            print(f"[oracle 1 thread] {w.name}: {dt:.1f} s", file=sys.stderr, flush=True)
            return dt, sub["theta"]
        with ThreadPoolExecutor(max_workers=len(cases)) as ex:
            res = list(ex.map(run, cases))
        for r, (dt, th) in zip(rows, res):
            r["oracle_1thread_s"] = dt
            r["theta_max_rel_vs_oracle"] = float(np.max(np.abs(r["_theta"] - th) / np.maximum(np.abs(th), 1e-2)))
    for r in rows:
        del r["_theta"]
    return rows


def measured_rank_traffic():
    """HBM bytes per step of the rank kernels from the committed rocprofv3 PMC
    summary, if it was taken on the current rank sources (else None)."""
    for path in glob.glob(os.path.join(ROOT, "profiles", "*rank*pmc*.md")):
        with open(path) as f:
            text = f.read()
        m_hash = re.search(r"rank_source_sha256_16:\s*([0-9a-f]+)", text)
        m_bytes = re.search(r"rank_hbm_bytes_per_step:\s*([0-9.eE+]+)", text)
        if m_hash and m_bytes and m_hash.group(1) == rank_source_hash():
            return float(m_bytes.group(1))
    return None


def measured_fit_var_counters():
    """VALU instruction counts per step of the fit and variance kernels from
    the committed rocprofv3 PMC summary of the default workload, if it was
    taken on the current sources (else None)."""
    keys = ("valu", "trans_f32", "trans_f64", "f64")
    for path in glob.glob(os.path.join(ROOT, "profiles", "*fit_var*valu*.md")):
        with open(path) as f:
            text = f.read()
        m_hash = re.search(r"fit_var_source_sha256_16:\s*([0-9a-f]+)", text)
        if not m_hash or m_hash.group(1) != source_hash(FIT_VAR_SOURCES):
            continue
        out = {}
        for ph in ("fit", "var"):
            for k in keys:
                m = re.search(rf"{ph}_{k}_insts_per_step:\s*([0-9.eE+]+)", text)
                if not m:
                    break
                out[(ph, k)] = float(m.group(1))
        if len(out) == 2 * len(keys):
            return out
    return None


def issued_slots(c, phase, trans_slots):
    """Issued VALU lane-slots of one phase: 64 per wave instruction, an FP32
    transcendental weighted by its measured slot cost, FP64 FMA/MUL/ADD 2
    (half-rate), FP64 transcendentals 8."""
    v, t, t64, f64 = (c[(phase, k)] for k in ("valu", "trans_f32", "trans_f64", "f64"))
    return 64.0 * ((v - t - t64 - f64) + trans_slots * t + 2.0 * f64 + 8.0 * t64)


# FP32-compensated parity tolerances the GPU tests hold every estimate to
# (relative to max(|theta|, floor)); FP64 path: 1e-6 relative (floor 1e-3).
TOLERANCES = {
    "fp32c": {"frank": {"rel": 1e-5, "floor": 0.1}, "gumbel": {"rel": 1e-5, "floor": 0.1},
              "gaussian": {"rel": 1e-6, "floor": 1e-2}},
    "fp64": {"all": {"rel": 1e-6, "floor": 1e-3}},
}


def _fit_timed(cpc, x, y, offsets, gofs, fams, prec, reps, dev, torch):
    """Median ms of `reps` graph replays of one batched fit (inputs resident)."""
    K, G = len(offsets) - 1, len(gofs) - 1
    ws = torch.empty(cpc.workspace_bytes(x.shape[0], K, G, dtype=x.dtype, offsets=offsets, prec=prec),
                     dtype=torch.uint8, device=dev)
    out = cpc.FitResult(torch.empty((K, 6), dtype=torch.float64, device=dev),
                        torch.empty((G, 5), dtype=torch.float64, device=dev))

    def step():
        cpc.fit_batched(x, y, offsets, gofs, fams, workspace=ws, out=out, prec=prec, graph=True)
    step()
    step()
    torch.cuda.synchronize()
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(reps + 1)]
    evs[0].record()
    for i in range(reps):
        step()
        evs[i + 1].record()
    torch.cuda.synchronize()
    ms = float(np.median([evs[i].elapsed_time(evs[i + 1]) for i in range(reps)]))
    del ws
    return ms, out


def _oracle_err(O, xs, ys, offsets, picks, fam_of, theta_gpu, status_gpu):
    """Max relative error of the GPU estimates on the picked subsets against
    the oracle run on the same rows (FP32 values widened)."""
    sub_x = [xs[offsets[m]:offsets[m + 1]].astype(np.float64) for m in picks]
    sub_y = [ys[offsets[m]:offsets[m + 1]].astype(np.float64) for m in picks]
    import synth
    off = synth.offsets_from_sizes(np.array([len(v) for v in sub_x]))
    gofs = np.arange(len(picks) + 1, dtype=np.int64)
    sub, _ = O.fit(np.concatenate(sub_x), np.concatenate(sub_y), off, [fam_of[m] for m in picks], gofs)
    ok = (sub["status"] == 0) & (status_gpu[picks] == 0)
    floor = np.array([0.1 if fam_of[m] == "frank" else (1e-2 if fam_of[m] == "gaussian" else 0.1) for m in picks])
    rel = np.abs(theta_gpu[picks][ok] - sub["theta"][ok]) / np.maximum(np.abs(sub["theta"][ok]), floor[ok])
    return {"subsets_checked": int(ok.sum()), "theta_max_rel": float(rel.max(initial=0.0)),
            "status_match": bool(np.array_equal(sub["status"], status_gpu[picks]))}


def leg_gumbel_headline_shape(cpc, synth, O, dev, torch):
    """Gumbel theta = 2 at the shape of the headline workload: n = 1e7 FP32
    pairs (drawn on the GPU), K = 1000 subsets of U[5000, 15000] rows."""
    n, K = 10_000_000, 1000
    t0 = time.perf_counter()
    x, y = cpc.sample("gumbel", 2.0, n, seed=7002, dtype=torch.float32, device=dev)
    torch.cuda.synchronize()
    gen = time.perf_counter() - t0
    off = synth.uniform_size_offsets(n, K, 5000.0, 15000.0, np.random.default_rng(7003))
    gofs = np.array([0, K], dtype=np.int64)
    ms, out = _fit_timed(cpc, x, y, off, gofs, ["gumbel"], "fp32c", 10, dev, torch)
    ms64, out64 = _fit_timed(cpc, x, y, off, gofs, ["gumbel"], "fp64", 5, dev, torch)
    th, st = out.theta.cpu().numpy(), out.status.cpu().numpy()
    picks = list(range(0, K, K // 32))
    err = _oracle_err(O, x.cpu().numpy(), y.cpu().numpy(), off, picks, ["gumbel"] * K, th, st)
    return {"workload": "gumbel theta=2, n=1e7 FP32 (GPU sampler), K=1000 U[5000,15000]",
            "ms_per_fit": ms, "subset_fits_per_s": K / (ms / 1e3), "fp64_ms": ms64,
            "speedup_fp32c_over_fp64": ms64 / ms, "gen_s": gen, "err_vs_oracle": err,
            "newton_passes_mean": float(np.mean(out.iters.cpu().numpy()[st == 0]))}


def leg_replicate_batch(cpc, synth, O, dev, torch):
    """1000 replicates x 1e5 pairs, family r mod 3 with Kendall tau ~
    U[0.1, 0.8], K = 50 Dirichlet(1) subsets each (about 50,000 fits, one
    graph replay); replicates drawn on the GPU sampler."""
    R, n, K = 1000, 100_000, 50
    fams = ["gaussian", "frank", "gumbel"]
    x = torch.empty(R * n, dtype=torch.float32, device=dev)
    y = torch.empty(R * n, dtype=torch.float32, device=dev)
    offs, gofs, fam_g = [0], [0], []
    t0 = time.perf_counter()
    for r in range(R):
        rng = np.random.default_rng(3000 + r)
        fam = fams[r % 3]
        th = synth.theta_from_tau(fam, rng.uniform(0.1, 0.8))
        xr, yr = cpc.sample(fam, th, n, seed=9_000_000 + r, dtype=torch.float32, device=dev)
        x[r * n:(r + 1) * n] = xr
        y[r * n:(r + 1) * n] = yr
        o = synth.dirichlet_offsets(n, K, rng)
        offs.extend((o[1:] + r * n).tolist())
        gofs.append(gofs[-1] + K)
        fam_g.append(fam)
    torch.cuda.synchronize()
    gen = time.perf_counter() - t0
    offs = np.array(offs, dtype=np.int64)
    gofs = np.array(gofs, dtype=np.int64)
    ms, out = _fit_timed(cpc, x, y, offs, gofs, fam_g, "fp32c", 10, dev, torch)
    th, st = out.theta.cpu().numpy(), out.status.cpu().numpy()
    fam_of = [fam_g[m // K] for m in range(R * K)]
    sizes = np.diff(offs)
    picks = sorted(set([int(np.argmax(sizes))] + list(range(7, R * K, (R * K) // 30))))
    err = _oracle_err(O, x.cpu().numpy(), y.cpu().numpy(), offs, picks, fam_of, th, st)
    return {"workload": "1000 replicates x n=1e5 FP32 (GPU sampler), K=50 Dirichlet(1), family r mod 3",
            "subsets": R * K, "ms_per_fit": ms, "subset_fits_per_s": R * K / (ms / 1e3), "gen_s": gen,
            "status_counts": {str(int(s)): int(np.sum(st == s)) for s in np.unique(st)}, "err_vs_oracle": err}


def leg_partition(cpc, synth, O, dev, torch):
    """Partitioning schemes on the paper's largest study cell: 50 replicates
    of 2e5 FP64 pairs (Gaussian 0.3, GPU sampler) split into M = 100 subsets
    by cpc_partition (x-order blocks and strided: ranks of both margins with
    ties by row order, then the scatter kernel); two replicates checked bit
    for bit against the partition oracle; and the partition study of that
    cell (bias and MSE against the full-data estimates per scheme)."""
    import oracle.partition as OP
    from paper_1609_05530_amd import study
    S, N, M = 50, 200_000, 100
    x, y = cpc.sample("gaussian", 0.3, S * N, seed=4242, dtype=torch.float64, device=dev)
    rep = np.arange(0, S * N + 1, N, dtype=np.int64)
    out = {"workload": f"{S} replicates x {N} FP64 pairs, M = {M}"}
    ws = torch.empty(int(cpc._lib.lib().cpc_partition_workspace_bytes(rep.ctypes.data, S, 0, 1)),
                     dtype=torch.uint8, device=dev)
    for scheme in ("blocks", "strided"):
        for _ in range(2):
            cpc.partition(x, y, rep, M, scheme, workspace=ws)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        ms = []
        for _ in range(10):
            ev[0].record()
            xo, yo, offs = cpc.partition(x, y, rep, M, scheme, workspace=ws)
            ev[1].record()
            torch.cuda.synchronize()
            ms.append(ev[0].elapsed_time(ev[1]))
        med = float(np.median(ms))
        hx, hy = x[: 2 * N].cpu().numpy(), y[: 2 * N].cpu().numpy()
        ex, ey, _ = OP.partition(hx, hy, rep[:3], M, scheme)
        same = bool(np.array_equal(xo[: 2 * N].cpu().numpy().view(np.uint64), ex.view(np.uint64))
                    and np.array_equal(yo[: 2 * N].cpu().numpy().view(np.uint64), ey.view(np.uint64)))
        out[scheme] = {"ms": med, "rows_per_s": S * N / (med / 1e3), "bit_exact_2_replicates": same}
        del xo, yo
    for _ in range(2):
        cpc.rank(x, y, rep, ties="first")
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ms = []
    for _ in range(10):
        ev[0].record()
        cpc.rank(x, y, rep, ties="first")
        ev[1].record()
        torch.cuda.synchronize()
        ms.append(ev[0].elapsed_time(ev[1]))
    out["ranks_alone_ms"] = float(np.median(ms))
    rows = study.partition_cell("gaussian", 0.3, N, M, S, x=x, y=y)
    out["study"] = {r["scheme"]: {"bias": r["bias"], "mse": r["mse"], "bias_vs_theta": r["bias_vs_theta"],
                                  "sd_combined": r["sd_combined"], "replicates": r["S"]} for r in rows}
    return out


def leg_moment_estimators(cpc, synth, O, dev, torch, w, x, y):
    """The Spearman- and Kendall-inversion estimators on the headline
    workload's ranks (9000 subsets, 9e7 rows): median of 5 timed calls each,
    and the sampled error against the oracle (host ranks of the same rows)."""
    R1, R2 = cpc.rank(x, y, w.offsets)
    out = {}
    for name, fn in (("spearman", cpc.spearman_fit), ("kendall", cpc.kendall_fit)):
        ws = torch.empty(int(getattr(cpc._lib.lib(), f"cpc_{name}_workspace_bytes")(w.n, w.K, w.G)),
                         dtype=torch.uint8, device=dev)
        res = fn(R1, R2, w.offsets, w.families, w.group_offsets, workspace=ws)
        torch.cuda.synchronize()
        ms = []
        for _ in range(5):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            res = fn(R1, R2, w.offsets, w.families, w.group_offsets, workspace=ws)
            e1.record()
            torch.cuda.synchronize()
            ms.append(e0.elapsed_time(e1))
        med = float(np.median(ms))
        # oracle on 2 subsets per setting
        rng = np.random.default_rng(11)
        picks = np.concatenate([rng.choice(np.arange(w.group_offsets[g], w.group_offsets[g + 1]), 2, replace=False)
                                for g in range(w.G)])
        xs = [w.x[w.offsets[m]:w.offsets[m + 1]].astype(np.float64) for m in picks]
        ys = [w.y[w.offsets[m]:w.offsets[m + 1]].astype(np.float64) for m in picks]
        r1 = np.concatenate([O.ranks(v) for v in xs]); r2 = np.concatenate([O.ranks(v) for v in ys])
        off = synth.offsets_from_sizes(np.array([len(v) for v in xs]))
        fam_of = [w.families[int(np.searchsorted(w.group_offsets, m, side="right") - 1)] for m in picks]
        ofit = O.spearman_fit_ranks if name == "spearman" else O.kendall_fit_ranks
        sub, _ = ofit(r1, r2, off, fam_of, np.arange(len(picks) + 1))
        th = res.theta.cpu().numpy()[picks]
        st = res.status.cpu().numpy()[picks]
        ok = (sub["status"] == 0) & (st == 0)
        rel = np.abs(th[ok] - sub["theta"][ok]) / np.maximum(np.abs(sub["theta"][ok]), 0.1)
        out[name] = {"ms": med, "subset_fits_per_s": w.K / (med / 1e3), "rows_per_s": w.n / (med / 1e3),
                     "err_vs_oracle": {"subsets_checked": int(ok.sum()), "theta_max_rel": float(rel.max(initial=0)),
                                       "status_match": bool(np.array_equal(st, sub["status"]))}}
    out["workload"] = "ranks of the 9 x 1e7-row headline workload (K = 9000), FP64 estimator arithmetic"
    return out


def leg_adjoint(cpc, synth, O, dev, torch, w, x, y, theta):
    """The adjoint kernel (cpc_eval: per-subset sums of l, dl/dtheta and
    d2l/dtheta2 of eq. (13)) on the headline workload's ranks at the fitted
    theta, FP32c and FP64: one call per family's run of settings, median of
    5; rows evaluated per second (each row gives l, s and h once)."""
    R1, R2 = cpc.rank(x, y, w.offsets)
    th = torch.as_tensor(theta, dtype=torch.float64, device=dev)
    runs, g = [], 0
    while g < w.G:
        h = g
        while h < w.G and w.families[h] == w.families[g]:
            h += 1
        m0, m1 = int(w.group_offsets[g]), int(w.group_offsets[h])
        a, b = int(w.offsets[m0]), int(w.offsets[m1])
        runs.append((w.families[g], R1[a:b], R2[a:b], w.offsets[m0:m1 + 1] - a, th[m0:m1].contiguous()))
        g = h
    out = {}
    for prec in ("fp32c", "fp64"):
        def call():
            for fam, r1, r2, off, t in runs:
                cpc.eval_subsets(r1, r2, off, fam, t, prec=prec)
        call()
        torch.cuda.synchronize()
        ts = []
        for _ in range(5):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            call()
            e1.record()
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        ms = float(np.median(ts))
        out[prec] = {"ms": ms, "row_evals_per_s": w.n / (ms / 1e3), "subsets_per_s": w.K / (ms / 1e3)}
    out["workload"] = "9 x 1e7-row headline ranks (K = 9000) at the fitted theta; l, s, h per row"
    return out


def leg_gaussk(cpc, synth, O, dev, torch, k=8, K=500, m=10_000):
    """The k-dimensional Gaussian copula (eq. 7): K subsets of m rows of k
    margins (host-drawn N(0, R) rows, R a fixed correlation matrix), ranks of
    every margin and the fit timed separately (median of 5), and the sampled
    error against the numpy oracle."""
    from oracle import gaussk as GK
    rng = np.random.default_rng(12)
    A = rng.standard_normal((k, 2 * k))
    Sg = A @ A.T + 0.5 * np.eye(k)
    d = np.sqrt(np.diag(Sg))
    Rm = Sg / np.outer(d, d)
    n = K * m
    t0 = time.perf_counter()
    X = (rng.standard_normal((n, k)) @ np.linalg.cholesky(Rm).T).T.copy()
    gen = time.perf_counter() - t0
    off = np.arange(0, n + 1, m, dtype=np.int64)
    Xd = torch.from_numpy(X).to(dev)
    ws = torch.empty(int(cpc._lib.lib().cpc_gaussk_workspace_bytes(n, k, K, 1)), dtype=torch.uint8, device=dev)

    def med(fn):
        fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(5):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        return float(np.median(ts))
    holder = {}
    ms_rank = med(lambda: holder.__setitem__("R", cpc.rank_margins(Xd, off)))
    ms_fit = med(lambda: holder.__setitem__("res", cpc.gaussk_fit(holder["R"], off, workspace=ws)))
    res = holder["res"]
    p = k * (k - 1) // 2
    th = res.theta.cpu().numpy().reshape(p, K)
    st = res.status.cpu().numpy().reshape(p, K)
    errs = []
    for mm in (0, K - 1):
        Rs = np.stack([O.ranks(X[j, off[mm]:off[mm + 1]]) for j in range(k)], axis=1)
        tho, _, _, _, _, sto = GK.fit_subset(Rs)
        errs.append(float(np.max(np.abs(th[:, mm] - tho) / np.maximum(np.abs(tho), 0.1))) if sto == 0 else np.nan)
    comb = res.combined_theta.cpu().numpy()
    truth = np.array([Rm[j, l] for j, l in GK.pairs(k)])
    return {"workload": f"k={k} margins, K={K} subsets x {m} rows (host-drawn N(0, R)), FP64",
            "rank_ms": ms_rank, "fit_ms": ms_fit, "subset_fits_per_s": K / (ms_fit / 1e3),
            "rows_per_s_fit": n / (ms_fit / 1e3), "gen_s": gen, "status_ok": bool(np.all(st == 0)),
            "err_vs_oracle": {"subsets_checked": 2, "theta_max_rel": float(np.nanmax(errs))},
            "combined_max_abs_dev_from_R": float(np.max(np.abs(comb - truth)))}


def leg_hundred_million_rows(cpc, synth, O, dev, torch):
    """n = 1e8 FP32 pairs per family (Gumbel theta = 3, Frank theta = -8) drawn
    on the GPU, K = 1000 equal subsets: FP32c and FP64 times and errors."""
    n, K = 100_000_000, 1000
    res = []
    for fam, th in synth.HUNDRED_MILLION_SETTINGS:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x, y = cpc.sample(fam, th, n, seed=4000 + synth.FAMILY_CODES[fam], dtype=torch.float32, device=dev)
        torch.cuda.synchronize()
        gen = time.perf_counter() - t0
        off = synth.equal_offsets(n, K)
        gofs = np.array([0, K], dtype=np.int64)
        ms, out = _fit_timed(cpc, x, y, off, gofs, [fam], "fp32c", 3, dev, torch)
        th32, st = out.theta.cpu().numpy(), out.status.cpu().numpy()
        c32 = float(out.combined_theta.cpu().numpy()[0])
        ms64, out64 = _fit_timed(cpc, x, y, off, gofs, [fam], "fp64", 3, dev, torch)
        th64 = out64.theta.cpu().numpy()
        c64 = float(out64.combined_theta.cpu().numpy()[0])
        picks = list(range(0, K, K // 8))
        xs, ys = x.cpu().numpy(), y.cpu().numpy()
        err32 = _oracle_err(O, xs, ys, off, picks, [fam] * K, th32, st)
        err64 = _oracle_err(O, xs, ys, off, picks, [fam] * K, th64, out64.status.cpu().numpy())
        res.append({"workload": f"{fam} theta={th:g}, n=1e8 FP32 (GPU sampler), K=1000 x 1e5",
                    "fp32c_ms": ms, "fp64_ms": ms64, "speedup_fp32c_over_fp64": ms64 / ms,
                    "rows_per_s_fp32c": n / (ms / 1e3), "sampler_s": gen, "sampler_rows_per_s": n / gen,
                    "combined_fp32c": c32, "combined_fp64": c64,
                    "combined_rel_fp32c_vs_fp64": abs(c32 - c64) / abs(c64),
                    "err_vs_oracle_fp32c": err32, "err_vs_oracle_fp64": err64})
        del x, y, out, out64
        torch.cuda.empty_cache()
    return res


def main():
    a = parse()
    if a.gpus != 1:
        print("bench.py measures one GPU only (subsets are independent: several GPUs would each take "
              "whole subsets and all-reduce the per-group sums of eq. 15).", file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_1609_05530_amd as cpc
    import synth

    settings = synth.NINE_SETTINGS if a.settings == "all" else [synth.NINE_SETTINGS[int(i)] for i in a.settings.split(",")]
    t0 = time.time()
    w = synth.nine_settings(settings=settings, n=a.n, K=a.K)
    gen_s = time.time() - t0
    dev = torch.device("cuda:0")
    x = torch.from_numpy(w.x).to(dev)
    y = torch.from_numpy(w.y).to(dev)
    fams = w.families
    K, G, n = w.K, w.G, w.n
    graph = not a.no_graph

    def make_step(prec):
        ws = torch.empty(cpc.workspace_bytes(n, K, G, dtype=x.dtype, offsets=w.offsets, prec=prec), dtype=torch.uint8, device=dev)
        out = cpc.FitResult(torch.empty((K, 6), dtype=torch.float64, device=dev),
                            torch.empty((G, 5), dtype=torch.float64, device=dev))

        def step(**kw):
            # every step records the phase events (in graph mode the library
            # replays one graph per phase, with the events between them)
            cpc.fit_batched(x, y, w.offsets, w.group_offsets, fams, workspace=ws, out=out, prec=prec, graph=graph,
                            phase_times=True, **kw)
        return step, out

    def timed(step, steps, warmup):
        for _ in range(warmup):
            step()
        torch.cuda.synchronize()
        evs = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
        t_start = time.perf_counter()
        evs[0].record()
        for i in range(steps):
            step()
            evs[i + 1].record()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t_start
        per = np.array([evs[i].elapsed_time(evs[i + 1]) for i in range(steps)])
        return float(evs[0].elapsed_time(evs[-1]) / steps), float(np.median(per)), wall

    step, out = make_step(a.prec)
    ms_step, ms_median, wall = timed(step, a.steps, a.warmup)

    if a.profile:
        # a plain device copy of known size (x: 4 bytes x rows) to scale the
        # profiler's HBM byte counters
        xc = x.clone()
        torch.cuda.synchronize()
        del xc

    # per-phase durations of the last timed step (HIP events the library
    # records on the launch stream between the phase graphs)
    phases = np.array(cpc.phase_times(0), dtype=np.float64)

    theta = out.theta.cpu().numpy()
    iters = out.iters.cpu().numpy()
    status = out.status.cpu().numpy()
    nsub = out.n.cpu().numpy()
    fam_of = np.empty(K, dtype=object)
    for g in range(G):
        fam_of[w.group_offsets[g]:w.group_offsets[g + 1]] = fams[g]

    # algorithmic work of the fit kernels: rows x Newton passes x slots per row-pass
    slots = 0.0
    obs_evals = 0.0
    for fam in set(fams):
        sel = fam_of == fam
        passes = iters[sel].astype(np.float64)
        slots += float(np.sum(nsub[sel] * passes)) * SLOTS_PER_ROW_PASS[fam]
        obs_evals += float(np.sum(nsub[sel] * (passes + 1.0)))  # + the variance pass
    fit_s = phases[1] / 1e3
    achieved_fit = slots / fit_s if fit_s > 0 else 0.0
    rank_s = phases[0] / 1e3
    rank_bytes = float(n) * RANK_BYTES_PER_ROW
    achieved_rank = rank_bytes / rank_s if rank_s > 0 else 0.0
    traffic = measured_rank_traffic()

    line = {
        "metric": "subset-fits/sec (batched MPL copula fits, n=1e7 per setting)",
        "value": K / (ms_step / 1e3),
        "unit": "subset-fits/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms_step,
        "ms_per_step_median": ms_median,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if a.prec == "fp32c" else "f64",
        "data": "synthetic",
        "config": {
            "workload": f"{G} settings x n={a.n} FP32 pairs, K={a.K} subsets each, sizes U[5000,15000] renormalised",
            "settings": [f"{f} {t:g}" for f, t in settings],
            "subset_fits_per_step": K,
            "rows_per_step": n,
            "precision": a.prec,
            "launch": "hipGraph replay" if graph else "eager",
        },
        "obs_evals_per_s": obs_evals / (ms_step / 1e3),
        "obs_evals_per_s_eval_kernels": obs_evals / ((phases[1] + phases[2]) / 1e3),
        "phase_ms": {"rank": phases[0], "fit": phases[1], "variance": phases[2], "combine": phases[3]},
        "newton_passes_mean": float(np.mean(iters[status == 0])) if np.any(status == 0) else None,
        "status_counts": {str(int(s)): int(np.sum(status == s)) for s in np.unique(status)},
        "wall_s_timed": wall,
        "gen_s": gen_s,
        "roofline": {
            "kernel": "k_rank_wg (ranks of eq. 12; all its launches in one step)",
            "bound": "hbm",
            "achieved": achieved_rank / 1e9,
            "peak": PEAK_HBM / 1e9,
            "unit": "GB/s",
            "frac": achieved_rank / PEAK_HBM,
            "traffic": traffic,
            "algorithmic_bytes": rank_bytes,
        },
        "roofline_fit": {
            "kernel": "k_fit_wg (Newton passes of eq. 13)",
            "bound": "alu",
            "achieved": achieved_fit / 1e12,
            "peak": PEAK_LANE_SLOTS / 1e12,
            "unit": "T VALU lane-slots/s",
            "frac": achieved_fit / PEAK_LANE_SLOTS,
            "traffic": None,
        },
    }

    if not a.profile:
        probe = valu_probe()
        line["valu_probe"] = probe
        counters = measured_fit_var_counters() if (a.prec == "fp32c" and graph and a.n == 10_000_000
                                                    and a.K == 1000 and a.settings == "all") else None
        if counters is not None:
            # issued VALU slots per step from the committed counter profile of
            # this workload, over the fit and variance phase times just measured
            w_trans = probe["slots_per_op"]["exp2"] if probe else 3.2
            for ph, key, ms in (("fit", "roofline_fit", phases[1]), ("var", "roofline_var", phases[2])):
                sl = issued_slots(counters, ph, w_trans)
                rate = sl / (ms / 1e3) if ms > 0 else 0.0
                issued = {"lane_slots_per_step": sl, "achieved": rate / 1e12, "peak": PEAK_LANE_SLOTS / 1e12,
                          "unit": "T VALU lane-slots/s", "frac": rate / PEAK_LANE_SLOTS,
                          "valu_wave_insts_per_step": counters[(ph, "valu")],
                          "trans_f32_lane_ops_per_s": 64.0 * counters[(ph, "trans_f32")] / (ms / 1e3) if ms > 0 else 0.0,
                          "source": "rocprofv3 PMC counts of the committed profile x measured phase time"}
                if key == "roofline_fit":
                    line[key]["issued"] = issued
                else:
                    line[key] = {"kernel": "k_var_wg (GGR variance, Sec. 2.3)", "bound": "alu", **issued}
    if not a.profile and not a.no_small_configs:
        line["small_configs_fp64"] = small_configs(cpc, synth, dev, a.oracle_1thread)

    if not a.profile and not a.no_fp64_compare and a.prec == "fp32c":
        step64, out64 = make_step("fp64")
        ms64, med64, _ = timed(step64, max(3, a.steps // 4), 1)
        line["fp64_path"] = {"ms_per_step": ms64, "ms_per_step_median": med64,
                             "speedup_fp32c_over_fp64": ms64 / ms_step}
        theta64 = out64.theta.cpu().numpy()
    else:
        theta64 = None

    if not a.profile:
        import oracle.oracle as O
        # error vs the FP64 oracle and the oracle's own rate on a bounded sample
        pick = []
        for g in range(G):
            m0 = int(w.group_offsets[g])
            pick.extend(range(m0, m0 + a.cpu_sample))
        xs = [w.x[w.offsets[m]:w.offsets[m + 1]].astype(np.float64) for m in pick]
        ys = [w.y[w.offsets[m]:w.offsets[m + 1]].astype(np.float64) for m in pick]
        sizes = np.array([len(v) for v in xs])
        off = synth.offsets_from_sizes(sizes)
        gofs = np.arange(0, len(pick) + 1, a.cpu_sample, dtype=np.int64)
        nt = O.num_threads(0)
        t0 = time.perf_counter()
        sub, _ = O.fit(np.concatenate(xs), np.concatenate(ys), off, fams, gofs, nthreads=nt)
        cpu_s = time.perf_counter() - t0
        ref = sub["theta"]
        ok = (sub["status"] == 0) & (status[pick] == 0)
        floor = np.array([0.1 if fam_of[m] == "frank" else 1e-2 for m in pick])

        def rel_err(th):
            got = th[pick]
            return np.abs(got[ok] - ref[ok]) / np.maximum(np.abs(ref[ok]), floor[ok])
        rel = rel_err(theta)
        vrel = np.abs(out.var.cpu().numpy()[pick][ok] / sub["var"][ok] - 1.0)
        line["err_vs_oracle"] = {
            "subsets_checked": int(ok.sum()),
            "theta_max_rel": float(rel.max(initial=0)),
            "theta_median_rel": float(np.median(rel)) if rel.size else None,
            "var_max_rel": float(vrel.max(initial=0)),
            "status_match": bool(np.array_equal(sub["status"], status[pick])),
        }
        if theta64 is not None:
            rel64 = rel_err(theta64)
            line["fp64_path"]["theta_max_rel_vs_oracle"] = float(rel64.max(initial=0))
        # the combination (eq. 15) of the sampled subsets per setting, GPU vs oracle
        xs_d = torch.from_numpy(np.concatenate(xs).astype(np.float32)).to(dev)
        ys_d = torch.from_numpy(np.concatenate(ys).astype(np.float32)).to(dev)
        samp = cpc.fit_batched(xs_d, ys_d, off, gofs, fams, prec=a.prec)
        _, comb_o = O.fit(np.concatenate(xs), np.concatenate(ys), off, fams, gofs, nthreads=nt)
        cg = samp.combined_theta.cpu().numpy()
        cfl = np.array([0.1 if f == "frank" else 1e-2 for f in fams])
        line["err_vs_oracle"]["combined_max_rel"] = float(np.max(np.abs(cg - comb_o["theta"]) /
                                                                 np.maximum(np.abs(comb_o["theta"]), cfl)))
        line["err_vs_oracle"]["tolerance"] = TOLERANCES[a.prec]
        w1 = synth.gaussian_1e4(1)
        t1 = time.perf_counter()
        O.fit(w1.x, w1.y, w1.offsets, w1.families, w1.group_offsets, nthreads=1)
        line["oracle_1thread_s_gaussian_1e4_K1"] = time.perf_counter() - t1
        line["cpu_baseline"] = {
            "value": len(pick) / cpu_s,
            "unit": "subset-fits/s",
            "cores": nt,
            "cpu_model": cpu_model(),
            "kind": "oracle",
            "sample": f"{len(pick)} subsets ({a.cpu_sample} per setting, {int(sizes.sum())} rows), FP64 oracle, "
                      f"OpenMP over subsets, {cpu_s:.1f} s",
        }
    if not a.profile and not a.no_legs:
        import oracle.oracle as O
        legs = (("gumbel_theta2_1e7_k1000", leg_gumbel_headline_shape),
                ("replicate_batch_1000x1e5", leg_replicate_batch),
                ("rows_1e8", leg_hundred_million_rows),
                ("moment_estimators_9x1e7", lambda *args: leg_moment_estimators(*args, w, x, y)),
                ("gaussk_k8_500x1e4", leg_gaussk),
                ("partition_50x2e5_m100", leg_partition),
                ("adjoint_9x1e7", lambda *args: leg_adjoint(*args, w, x, y, theta)))
        pick = set(s for s in a.legs.split(",") if s)
        unknown = pick - set(name for name, _ in legs)
        if unknown:
            raise SystemExit(f"unknown legs: {sorted(unknown)}")
        for name, fn in legs:
            if pick and name not in pick:
                continue
            t0 = time.perf_counter()
            line[name] = fn(cpc, synth, O, dev, torch)
            print(f"[leg] {name}: {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
