"""The allocation-free entry point cpc_fit_batched_noalloc (static device
scratch instead of a caller's workspace), called through the C ABI, against
cpc_fit_batched on the same inputs: two calls in a row, the second smaller
than the first (the scratch keeps the first call's contents), then a
partition too large for the scratch, rejected on the host."""
import ctypes

import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu


def _abi_noalloc(m, x, y, off, gofs, fams, prec):
    L = m._lib.lib()
    off = np.ascontiguousarray(off, dtype=np.int64)
    gofs = np.ascontiguousarray(gofs, dtype=np.int64)
    fam = np.ascontiguousarray([m.FAMILIES[f] for f in fams], dtype=np.int32)
    K, G = len(off) - 1, len(gofs) - 1
    o = m._options(prec=prec)
    out = m.FitResult(torch.empty((K, 6), dtype=torch.float64, device=x.device),
                      torch.empty((G, 5), dtype=torch.float64, device=x.device))
    dt = 0 if x.dtype == torch.float64 else 1
    rc = L.cpc_fit_batched_noalloc(m._handle(x.device), x.data_ptr(), y.data_ptr(), dt, x.shape[0],
                                   off.ctypes.data, K, gofs.ctypes.data, G, fam.ctypes.data, ctypes.byref(o),
                                   out.raw.data_ptr(), out.raw_comb.data_ptr(), m._stream(x.device))
    return rc, out


def _case(sizes, parts, seed, dtype):
    rng = np.random.default_rng(seed)
    xs, ys, offs, gofs, fams = [], [], [0], [0], []
    base = 0
    for k, (fam, th) in enumerate(parts):
        sz = np.asarray(sizes[k])
        x, y = synth.copula_pairs(fam, th, int(sz.sum()), int(rng.integers(1 << 30)))
        xs.append(x); ys.append(y)
        o = synth.offsets_from_sizes(sz)
        offs.extend((o[1:] + base).tolist()); base += int(o[-1])
        gofs.append(gofs[-1] + len(sz)); fams.append(fam)
    x = torch.as_tensor(np.concatenate(xs), dtype=dtype).cuda()
    y = torch.as_tensor(np.concatenate(ys), dtype=dtype).cuda()
    return x, y, np.array(offs), np.array(gofs), fams


def _same(a, b, prec):
    torch.cuda.synchronize()
    st_a, st_b = a.status.cpu().numpy(), b.status.cpu().numpy()
    assert np.array_equal(st_a, st_b)
    assert np.array_equal(a.n.cpu().numpy(), b.n.cpu().numpy())
    ok = (st_a == 0) | (st_a == 1) | (st_a == 2)
    ta, tb = a.theta.cpu().numpy()[ok], b.theta.cpu().numpy()[ok]
    tol = 1e-6 if prec == "fp64" else 1e-5
    assert np.all(np.abs(ta - tb) <= tol * np.maximum(np.abs(tb), 0.1))
    use = (st_a == 0) | (st_a == 1)
    va, vb = a.var.cpu().numpy()[use], b.var.cpu().numpy()[use]
    assert np.all(np.abs(va / vb - 1.0) <= (1e-6 if prec == "fp64" else 1e-4))
    ca, cb = a.combined_theta.cpu().numpy(), b.combined_theta.cpu().numpy()
    good = b.combined_status.cpu().numpy() == 0
    assert np.array_equal(a.combined_status.cpu().numpy(), b.combined_status.cpu().numpy())
    assert np.all(np.abs(ca[good] - cb[good]) <= tol * np.maximum(np.abs(cb[good]), 0.1))
    assert np.array_equal(a.n_used.cpu().numpy(), b.n_used.cpu().numpy())
    bitwise = np.array_equal(a.raw.cpu().numpy(), b.raw.cpu().numpy(), equal_nan=True)
    print(f"[noalloc] {prec}: {len(st_a)} subsets match (bitwise identical: {bitwise})", flush=True)


@pytest.mark.parametrize("prec", ["fp32c", "fp64"])
def test_noalloc_matches_workspace_entry_point(prec):
    import paper_1609_05530_amd as m
    dt = torch.float32 if prec == "fp32c" else torch.float64
    # first call: three groups, one with a subset of the streaming path
    x, y, off, gofs, fams = _case([[3000, 20000, 700, 12000], [5000, 9000, 1], [400, 16384, 8000]],
                                  [("frank", 6.0), ("gumbel", 2.0), ("gaussian", 0.5)], 5, dt)
    print(f"[noalloc] call 1: n={x.shape[0]} K={len(off) - 1} G={len(gofs) - 1}", flush=True)
    rc, a = _abi_noalloc(m, x, y, off, gofs, fams, prec)
    assert rc == 0, m._lib.lib().cpc_last_error()
    b = m.fit_batched(x, y, off, gofs, fams, prec=prec)
    _same(a, b, prec)
    # second call, smaller, on the same scratch
    x2, y2, off2, gofs2, fams2 = _case([[2500, 600], [4000]], [("gumbel", 1.5), ("frank", -4.0)], 6, dt)
    print(f"[noalloc] call 2: n={x2.shape[0]} K={len(off2) - 1} G={len(gofs2) - 1}", flush=True)
    rc, a2 = _abi_noalloc(m, x2, y2, off2, gofs2, fams2, prec)
    assert rc == 0, m._lib.lib().cpc_last_error()
    b2 = m.fit_batched(x2, y2, off2, gofs2, fams2, prec=prec)
    _same(a2, b2, prec)


def test_noalloc_rejects_partitions_beyond_the_scratch():
    import paper_1609_05530_amd as m
    L = m._lib.lib()
    n = 3_000_000  # ~28 bytes per row: more than the 64 MiB scratch
    off = np.linspace(0, n, 301).astype(np.int64)
    gofs = np.array([0, 300], dtype=np.int64)
    fam = np.array([1], dtype=np.int32)
    # inputs of the full size (the call is rejected on the host before any launch)
    x = torch.zeros(n, dtype=torch.float32, device="cuda")
    res = torch.empty((300, 6), dtype=torch.float64, device="cuda")
    comb = torch.empty((1, 5), dtype=torch.float64, device="cuda")
    o = m._options(prec="fp32c")
    rc = L.cpc_fit_batched_noalloc(m._handle(x.device), x.data_ptr(), x.data_ptr(), 1, n, off.ctypes.data, 300,
                                   gofs.ctypes.data, 1, fam.ctypes.data, ctypes.byref(o), res.data_ptr(),
                                   comb.data_ptr(), m._stream(x.device))
    assert rc == -5, rc  # CPC_E_WORKSPACE
    assert b"scratch" in L.cpc_last_error()
    o.flags = 1  # CPC_FLAG_GRAPH
    off_s = np.array([0, 16], dtype=np.int64)
    gofs_s = np.array([0, 1], dtype=np.int64)
    rc = L.cpc_fit_batched_noalloc(m._handle(x.device), x.data_ptr(), x.data_ptr(), 1, 16, off_s.ctypes.data, 1,
                                   gofs_s.ctypes.data, 1, fam.ctypes.data, ctypes.byref(o), res.data_ptr(),
                                   comb.data_ptr(), m._stream(x.device))
    assert rc == -8, rc  # CPC_E_OPTIONS
