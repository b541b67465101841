"""Full-size workloads on the GPU, checked on sampled subsets against the FP64
oracle and, at any size, against properties of the method:

* the 9 x 1e7-row FP32 workload in the launch configuration bench.py times
  (hipGraph replay, FP32-compensated rows);
* 1e8 FP32 rows per family in 1000 subsets of 1e5 (the streaming path), in
  the FP32-compensated and the FP64 path;
* 1000 replicates of 1e5 rows, each split into 50 Dirichlet(1) subsets
  (about 50,000 subsets from 0 to ~22,000 rows, all size classes at once).

Combined estimates are checked against eq. (15) evaluated on the returned
per-subset results, and the FP64 path's combined estimate against the truth
within its own standard error.
"""
import time

import numpy as np
import pytest
import torch

import oracle.oracle as O
import synth

pytestmark = pytest.mark.gpu

TOL = {("fp64", "gaussian"): (1e-6, 1e-3), ("fp64", "frank"): (1e-6, 1e-3), ("fp64", "gumbel"): (1e-6, 1e-3),
       ("fp32c", "gaussian"): (1e-6, 1e-2), ("fp32c", "frank"): (1e-5, 0.1), ("fp32c", "gumbel"): (1e-5, 0.1)}


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    assert torch.cuda.is_available(), "GPU tests need a ROCm GPU"
    import paper_1609_05530_amd  # noqa: F401  (fails loudly if libcpc.so is missing)


def cpc():
    import paper_1609_05530_amd as m
    return m


def dev(a, dtype):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype).cuda()


def to_np(res):
    torch.cuda.synchronize()
    return {k: getattr(res, k).cpu().numpy() for k in
            ("theta", "var", "loglik", "score", "n", "iters", "status",
             "combined_theta", "combined_var", "n_used", "n_excluded", "combined_status")}


def combine_closed_form(g, gofs):
    """eq. (15) from the returned per-subset results: usable = OK or BOUNDARY_NATURAL."""
    th, n_used = [], []
    for a, b in zip(gofs[:-1], gofs[1:]):
        st = g["status"][a:b]
        use = (st == 0) | (st == 1)
        w = 1.0 / g["var"][a:b][use]
        th.append(np.sum(w * g["theta"][a:b][use]) / np.sum(w) if use.any() else np.nan)
        n_used.append(int(use.sum()))
    return np.array(th), np.array(n_used)


def check_against_oracle(g, w, pick, fams_of, prec, label, nthreads=0):
    """Oracle fits of the picked subsets (each one its own group)."""
    xs = [w.x[w.offsets[m]:w.offsets[m + 1]].astype(np.float64) for m in pick]
    ys = [w.y[w.offsets[m]:w.offsets[m + 1]].astype(np.float64) for m in pick]
    off = synth.offsets_from_sizes(np.array([len(v) for v in xs]))
    fams = [fams_of[m] for m in pick]
    gofs = np.arange(len(pick) + 1, dtype=np.int64)
    sub, _ = O.fit(np.concatenate(xs), np.concatenate(ys), off, fams, gofs, nthreads=nthreads or O.num_threads(0))
    assert np.array_equal(g["status"][pick], sub["status"]), (label, g["status"][pick], sub["status"])
    worst = 0.0
    for j, m in enumerate(pick):
        st = sub["status"][j]
        if st not in (0, 1, 2):
            continue
        rt, floor = TOL[(prec, fams[j])]
        d = abs(g["theta"][m] - sub["theta"][j]) / max(abs(sub["theta"][j]), floor)
        worst = max(worst, d)
        assert d <= rt, (label, m, fams[j], g["theta"][m], sub["theta"][j])
        if st in (0, 1):
            vt = 1e-6 if prec == "fp64" else 1e-4
            assert abs(g["var"][m] / sub["var"][j] - 1.0) <= vt, (label, m, g["var"][m], sub["var"][j])
    print(f"[{label}] {len(pick)} sampled subsets vs oracle: max rel dtheta {worst:.2e}", flush=True)


def family_of_subsets(w):
    fam_of = np.empty(w.K, dtype=object)
    for gi in range(w.G):
        fam_of[w.group_offsets[gi]:w.group_offsets[gi + 1]] = w.families[gi]
    return fam_of


def test_nine_settings_full_size_bench_launch():
    m = cpc()
    w = synth.nine_settings()
    x, y = dev(w.x, torch.float32), dev(w.y, torch.float32)
    ws = torch.empty(m.workspace_bytes(w.n, w.K, w.G, dtype=torch.float32, prec="fp32c"), dtype=torch.uint8,
                     device="cuda")
    out = m.FitResult(torch.empty((w.K, 6), dtype=torch.float64, device="cuda"),
                      torch.empty((w.G, 5), dtype=torch.float64, device="cuda"))
    for _ in range(2):  # capture, then replay
        m.fit_batched(x, y, w.offsets, w.group_offsets, w.families, workspace=ws, out=out, graph=True, prec="fp32c")
    g = to_np(out)
    assert np.all(g["status"] == 0), np.unique(g["status"], return_counts=True)
    eager = to_np(m.fit_batched(x, y, w.offsets, w.group_offsets, w.families, prec="fp32c"))
    for k in g:
        assert np.array_equal(g[k], eager[k], equal_nan=True), k
    th, nu = combine_closed_form(g, w.group_offsets)
    assert np.allclose(g["combined_theta"], th, rtol=1e-12, atol=0), (g["combined_theta"], th)
    assert np.array_equal(g["n_used"], nu)
    fam_of = family_of_subsets(w)
    pick = []
    for gi in range(w.G):
        a, b = int(w.group_offsets[gi]), int(w.group_offsets[gi + 1])
        pick += [a, (a + b) // 2, b - 1]
    check_against_oracle(g, w, pick, fam_of, "fp32c", "nine_settings")


@pytest.mark.parametrize("fam,th", synth.HUNDRED_MILLION_SETTINGS)
def test_hundred_million_rows_full_size(fam, th):
    m = cpc()
    t0 = time.time()
    w = synth.hundred_million_rows(fam, th)
    gen = time.time() - t0
    x, y = dev(w.x, torch.float32), dev(w.y, torch.float32)
    fam_of = family_of_subsets(w)
    pick = [0, w.K // 2, w.K - 1]
    times = {}
    for prec in ("fp32c", "fp64"):
        ws = torch.empty(m.workspace_bytes(w.n, w.K, w.G, dtype=torch.float32, prec=prec), dtype=torch.uint8,
                         device="cuda")
        m.fit(x, y, w.offsets, fam, workspace=ws, prec=prec)  # warm-up
        torch.cuda.synchronize()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record()
        res = m.fit(x, y, w.offsets, fam, workspace=ws, prec=prec)
        ev1.record()
        g = to_np(res)
        times[prec] = ev0.elapsed_time(ev1)
        assert np.all(g["status"] == 0), (prec, np.unique(g["status"], return_counts=True))
        tc, nu = combine_closed_form(g, w.group_offsets)
        assert np.allclose(g["combined_theta"], tc, rtol=1e-12, atol=0)
        assert nu[0] == w.K
        check_against_oracle(g, w, pick, fam_of, prec, f"hundred_million_rows {fam} {prec}")
        se = float(np.sqrt(g["combined_var"][0]))
        assert abs(g["combined_theta"][0] - th) <= 6 * se, (prec, g["combined_theta"][0], th, se)
        print(f"[1e8 rows] {fam} theta={th} {prec}: combined {g['combined_theta'][0]:.6f} (se {se:.2e}), "
              f"mean Newton passes {g['iters'].mean():.2f}, {times[prec]:.1f} ms", flush=True)
        del ws
    print(f"[1e8 rows] {fam}: n={w.n} K={w.K}, FP32c {times['fp32c']:.1f} ms, FP64 {times['fp64']:.1f} ms, "
          f"speed-up {times['fp64'] / times['fp32c']:.2f}x (generation {gen:.1f} s)", flush=True)


def test_replicate_batch_full_size():
    m = cpc()
    t0 = time.time()
    w = synth.replicate_batch()
    gen = time.time() - t0
    assert w.K == 50_000 and w.G == 1000
    x, y = dev(w.x, torch.float32), dev(w.y, torch.float32)
    ws = torch.empty(m.workspace_bytes(w.n, w.K, w.G, dtype=torch.float32, prec="fp32c"), dtype=torch.uint8,
                     device="cuda")
    out = m.FitResult(torch.empty((w.K, 6), dtype=torch.float64, device="cuda"),
                      torch.empty((w.G, 5), dtype=torch.float64, device="cuda"))
    m.fit_batched(x, y, w.offsets, w.group_offsets, w.families, workspace=ws, out=out, graph=True, prec="fp32c")
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    m.fit_batched(x, y, w.offsets, w.group_offsets, w.families, workspace=ws, out=out, graph=True, prec="fp32c")
    ev1.record()
    g = to_np(out)
    ms = ev0.elapsed_time(ev1)
    sizes = np.diff(w.offsets)
    st = g["status"]
    # subsets below n_min = 2 are DEGENERATE; every other one is fitted
    assert np.all(st[sizes < 2] == 3)
    assert np.all(np.isin(st[sizes >= 2], [0, 1, 2])), np.unique(st[sizes >= 2], return_counts=True)
    th, nu = combine_closed_form(g, w.group_offsets)
    good = ~np.isnan(th)
    assert np.allclose(g["combined_theta"][good], th[good], rtol=1e-12, atol=0)
    assert np.array_equal(g["n_used"], nu)
    assert np.array_equal(g["n_used"] + g["n_excluded"], np.diff(w.group_offsets))
    fam_of = family_of_subsets(w)
    rng = np.random.default_rng(33)
    fitted = np.flatnonzero(sizes >= 2)
    pick = sorted(set(rng.choice(fitted, 30, replace=False).tolist()
                      + np.argsort(sizes)[-4:].tolist()                       # largest (streaming path)
                      + fitted[np.argsort(sizes[fitted])[:6]].tolist()))      # smallest fitted
    check_against_oracle(g, w, pick, fam_of, "fp32c", "replicate_batch")
    print(f"[replicate batch] K={w.K} subsets (sizes {sizes.min()}..{sizes.max()}), G={w.G}: "
          f"statuses {dict(zip(*np.unique(st, return_counts=True)))}, {ms:.1f} ms per graph replay "
          f"({w.K / (ms / 1e3):.0f} subset-fits/s; generation {gen:.1f} s)", flush=True)
