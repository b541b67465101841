"""GPU parity of the partitioning schemes (cpc_partition) against the
partition oracle: output rows bit for bit and subset bounds exactly, on
replicates that span the rank kernels' size classes and the streaming path
(more than 16384 rows), with ties, signed zeros, empty replicates and more
subsets than rows; the whole study cell (partition -> batched fits ->
combination) against the oracle's fits; the size of the paper's largest
study cell; and the argument checks."""
import numpy as np
import pytest
import torch

import oracle.oracle as O
import oracle.partition as OP
import synth

pytestmark = pytest.mark.gpu

SIZES = [0, 1, 2, 7, 500, 513, 2048, 4097, 16384, 16385, 30000, 12345]


def tied_values(rng, n):
    g = np.round(rng.standard_normal(n) * 40) / 40  # many exact ties
    g[::11] = -0.0
    g[1::13] = 0.0
    return g


def bits(a: np.ndarray) -> np.ndarray:
    return a.view(np.uint64 if a.dtype == np.float64 else np.uint32)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("scheme", OP.SCHEMES)
def test_partition_bit_exact(scheme, dtype):
    import paper_1609_05530_amd as m
    rng = np.random.default_rng(21)
    rep = synth.offsets_from_sizes(np.array(SIZES))
    npd = np.float64 if dtype == torch.float64 else np.float32
    x = tied_values(rng, int(rep[-1])).astype(npd)
    y = rng.standard_normal(int(rep[-1])).astype(npd)
    dx, dy = torch.as_tensor(x).cuda(), torch.as_tensor(y).cuda()
    for M in (1, 3, 10, 64, 20000):
        print(f"[partition] {scheme} {dtype} M={M}: replicates of {SIZES} rows", flush=True)
        xo, yo, offs = m.partition(dx, dy, rep, M, scheme)
        ex, ey, eoffs = OP.partition(x, y, rep, M, scheme)
        assert np.array_equal(offs, eoffs), (scheme, M)
        assert np.array_equal(bits(xo.cpu().numpy()), bits(ex)), (scheme, M)
        assert np.array_equal(bits(yo.cpu().numpy()), bits(ey)), (scheme, M)


@pytest.mark.parametrize("scheme", OP.SCHEMES)
def test_partitioned_fit_matches_oracle(scheme):
    """Gaussian 0.5 and Frank 5, 3 replicates of 6000 rows each in 10
    subsets: the GPU partition, fits and combination against the oracle's
    partition, fits and combination (FP64)."""
    import paper_1609_05530_amd as m
    S, N, M = 3, 6000, 10
    for fam, th in (("gaussian", 0.5), ("frank", 5.0)):
        x, y = synth.copula_pairs(fam, th, S * N, 40)
        rep = np.arange(0, S * N + 1, N, dtype=np.int64)
        gofs = np.arange(0, S * M + 1, M, dtype=np.int64)
        xo, yo, offs = m.partition(torch.as_tensor(x).cuda(), torch.as_tensor(y).cuda(), rep, M, scheme)
        res = m.fit_batched(xo, yo, offs, gofs, [fam] * S, prec="fp64")
        ex, ey, eoffs = OP.partition(x, y, rep, M, scheme)
        sub, comb = O.fit(ex, ey, eoffs, fam, group_offsets=gofs, nthreads=0)
        got = res.raw_comb[:, 0].cpu().numpy()
        rel = np.abs(got - comb["theta"]) / np.maximum(np.abs(comb["theta"]), 0.1)
        print(f"[partition] {scheme} {fam} {th}: combined {np.round(got, 4)}, max rel dev {rel.max():.1e}",
              flush=True)
        assert np.all(rel <= 1e-9), (scheme, fam)


def test_paper_cell_size_blocks_and_strided():
    """The paper's largest cell, 50 replicates of 200000 FP64 rows in 100
    subsets (1e7 rows, every replicate on the streaming rank path): bit-exact
    against the oracle for the two x-order schemes."""
    import paper_1609_05530_amd as m
    S, N, M = 50, 200_000, 100
    x, y = m.sample("gumbel", 5.0, S * N, seed=77, dtype=torch.float64)
    rep = np.arange(0, S * N + 1, N, dtype=np.int64)
    hx, hy = x.cpu().numpy(), y.cpu().numpy()
    for scheme in ("blocks", "strided"):
        print(f"[partition] {scheme}: {S} x {N} rows, M = {M}", flush=True)
        xo, yo, offs = m.partition(x, y, rep, M, scheme)
        ex, ey, eoffs = OP.partition(hx, hy, rep, M, scheme)
        assert np.array_equal(offs, eoffs)
        assert np.array_equal(bits(xo.cpu().numpy()), bits(ex))
        assert np.array_equal(bits(yo.cpu().numpy()), bits(ey))


def test_partition_study_effects():
    """Gaussian 0.3 (the paper's), N = 100000, M = 20 (subsets of 5000 rows,
    where the paper's contiguous split meets Sec. 3.2's bias bound of 0.002),
    S = 10: unequal Dirichlet(1) sizes stay within that bound as well (the
    inverse-variance weights of eq. 15 take the sizes into account), and so
    does every M-th row of the x-order (strided), while slices of x's range
    (blocks) pull the combined estimate far towards independence."""
    from paper_1609_05530_amd import study
    rows = {r["scheme"]: r for r in study.partition_cell("gaussian", 0.3, 100_000, 20, 10, seed=3)}
    for s, r in rows.items():
        print(f"[partition study] {s}: bias {r['bias']:+.2e} mse {r['mse']:.2e} "
              f"vs theta {r['bias_vs_theta']:+.2e} sd {r['sd_combined']:.2e}", flush=True)
    assert all(r["S"] == 10 for r in rows.values())
    assert abs(rows["contiguous"]["bias"]) < 0.002
    assert abs(rows["unequal"]["bias"]) < 0.002
    assert abs(rows["strided"]["bias"]) < 0.002
    assert rows["blocks"]["bias"] < -0.15


def test_partition_argument_errors():
    import paper_1609_05530_amd as m
    x = torch.zeros(10, dtype=torch.float64, device="cuda")
    y = torch.zeros(10, dtype=torch.float64, device="cuda")
    for bad in (dict(M=0), dict(M=1 << 31), dict(scheme=7), dict(rep=[0, 5]), dict(rep=[0, 6, 4, 10])):
        kw = dict(rep=[0, 10], M=2, scheme=1)
        kw.update(bad)
        with pytest.raises(m.CpcError):
            m.partition(x, y, kw["rep"], kw["M"], kw["scheme"])
    # outputs may not alias the inputs
    L = m._lib.lib()
    rep = np.array([0, 10], dtype=np.int64)
    offs = np.zeros(3, dtype=np.int64)
    ws = torch.empty(int(L.cpc_partition_workspace_bytes(rep.ctypes.data, 1, 0, 1)), dtype=torch.uint8,
                     device="cuda")
    xo = torch.empty_like(x)
    rc = L.cpc_partition(m._handle(x.device), x.data_ptr(), y.data_ptr(), 0, 10, rep.ctypes.data, 1, 2, 1,
                         ws.data_ptr(), ws.numel(), x.data_ptr(), xo.data_ptr(), offs.ctypes.data, None)
    assert rc == -2
