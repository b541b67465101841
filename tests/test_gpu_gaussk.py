"""GPU parity of the k-dimensional Gaussian copula fit (cpc_gaussk_fit,
eq. (7)) against the numpy oracle on the same data: the GPU ranks each
margin (cpc_rank), the oracle ranks it itself (the rankings are
bit-identical, tested elsewhere). Tolerances: each correlation 1e-9 relative
to max(|r|, 0.1) (both Newton iterations stop at 1e-12; the GPU's sums of
z z' and of the per-row score products run on the FP64 matrix cores in
another order), variance 1e-8 relative, log-likelihood 1e-10 relative,
combined correlations 1e-9; statuses and subsets used exactly."""
import numpy as np
import pytest
import torch

import oracle.oracle as O
from oracle import gaussk as GK
import synth

pytestmark = pytest.mark.gpu


def corr(k, seed):
    """A random correlation matrix with correlations up to about 0.7."""
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((k, 2 * k))
    S = A @ A.T + 0.5 * np.eye(k)
    d = np.sqrt(np.diag(S))
    return S / np.outer(d, d)


def draw(Rm, n, seed):
    rng = np.random.default_rng(seed)
    X = rng.multivariate_normal(np.zeros(len(Rm)), Rm, size=n)
    X[:, 0] = np.exp(X[:, 0])  # any increasing transform of a margin leaves the ranks alone
    return X


def gpu_fit(X, off, gofs=None):
    import paper_1609_05530_amd as m
    Xd = torch.as_tensor(np.ascontiguousarray(X.T), dtype=torch.float64).cuda()
    R = m.rank_margins(Xd, off)
    res = m.gaussk_fit(R, off, gofs)
    torch.cuda.synchronize()
    return {k: getattr(res, k).cpu().numpy() for k in
            ("theta", "var", "loglik", "status", "iters", "combined_theta", "n_used", "combined_status")}


def oracle_fit(X, off, gofs=None):
    R = np.stack([np.concatenate([O.ranks(X[off[m]:off[m + 1], j]) for m in range(len(off) - 1)])
                  for j in range(X.shape[1])], axis=1)
    return GK.fit_ranks(R, off, gofs)


def compare(g, sub, comb, label):
    p, K = sub.shape
    st = sub["status"].ravel()
    assert np.array_equal(g["status"], st), (label, g["status"].reshape(p, K), sub["status"])
    ok = st == 0
    th_o = sub["theta"].ravel()
    fitted = ok | (st == 2) | (st == 5)
    dth = np.abs(g["theta"][fitted] - th_o[fitted]) / np.maximum(np.abs(th_o[fitted]), 0.1)
    dvar = np.abs(g["var"][ok] / sub["var"].ravel()[ok] - 1.0)
    dll = np.abs(g["loglik"][ok] / sub["loglik"].ravel()[ok] - 1.0)
    cth = comb["theta"].ravel()
    good = comb["status"].ravel() == 0
    dc = np.abs(g["combined_theta"][good] - cth[good]) / np.maximum(np.abs(cth[good]), 0.1)
    print(f"[gaussk] {label}: p={p} K={K} max dtheta {dth.max(initial=0):.2e} dvar {dvar.max(initial=0):.2e} "
          f"dloglik {dll.max(initial=0):.2e} dcomb {dc.max(initial=0):.2e}", flush=True)
    assert dth.max(initial=0) <= 1e-9, label
    assert dvar.max(initial=0) <= 1e-8, label
    assert dll.max(initial=0) <= 1e-10, label
    assert np.array_equal(g["n_used"], comb["n_used"].ravel()), label
    assert dc.max(initial=0) <= 1e-9, label


@pytest.mark.parametrize("k", [2, 3, 5, 8])
def test_gaussk_parity(k):
    sizes = np.array([3000, 1500, 700, 5000, 20000, 257])
    off = synth.offsets_from_sizes(sizes)
    X = draw(corr(k, 10 + k), int(sizes.sum()), 20 + k)
    print(f"[gaussk] k={k}: n={len(X)} K={len(sizes)}", flush=True)
    sub, comb = oracle_fit(X, off)
    assert np.all(sub["status"] == 0)
    compare(gpu_fit(X, off), sub, comb, f"k={k}")


def test_gaussk_large_subsets_and_tied_margins():
    """Subsets past the size up to which tie-free margins are found in LDS
    (24575 rows: their bins are all added atomically) beside smaller ones, one
    with a tied margin (its bins added atomically, the others stored)."""
    k = 5
    sizes = np.array([24575, 24576, 30000, 6000])
    off = synth.offsets_from_sizes(sizes)
    X = draw(corr(k, 41), int(sizes.sum()), 42)
    X[off[3]:off[4], 1] = np.round(X[off[3]:off[4], 1] * 8) / 8  # ties in one margin
    print(f"[gaussk] large subsets: n={len(X)} K={len(sizes)}", flush=True)
    sub, comb = oracle_fit(X, off)
    assert np.all(sub["status"] == 0)
    compare(gpu_fit(X, off), sub, comb, "large subsets, tied margin")


def test_gaussk_groups_ties_and_statuses():
    """Groups, tied margins, too few rows (n <= k), a constant margin and two
    nearly collinear margins. (A margin repeated exactly gives a normalised
    Gram matrix whose correlation is 1 only up to the rounding of its sums,
    so the status at that edge is not compared here; the oracle pins it.)"""
    k = 4
    sizes = np.array([900, 4, 3, 1200, 800, 600, 2500, 1000])
    off = synth.offsets_from_sizes(sizes)
    X = draw(corr(k, 31), int(sizes.sum()), 32)
    a, b = off[3], off[4]
    X[a:b, 2] = np.round(X[a:b, 2] * 2) / 2           # heavy ties
    X[off[4]:off[5], 1] = 0.25                        # a constant margin
    X[off[5]:off[6], 3] = X[off[5]:off[6], 0] + 0.05 * np.random.default_rng(33).standard_normal(off[6] - off[5])
    gofs = np.array([0, 3, 6, 8])
    print(f"[gaussk] groups: n={len(X)} K={len(sizes)}", flush=True)
    sub, comb = oracle_fit(X, off, gofs)
    st = sub["status"][0]
    assert list(st) == [0, 3, 3, 0, 3, 0, 0, 0], st
    compare(gpu_fit(X, off, gofs), sub, comb, "groups, ties, statuses")


def test_gaussk_rejects_bad_k():
    import paper_1609_05530_amd as m
    R = torch.full((9, 10), 2, dtype=torch.int32, device="cuda")
    with pytest.raises(m.CpcError) as e:
        m.gaussk_fit(R, np.array([0, 10]))
    assert e.value.code == -9  # CPC_E_UNSUPPORTED
    with pytest.raises(m.CpcError) as e:
        m.gaussk_fit(R[:1], np.array([0, 10]))
    assert e.value.code == -2  # CPC_E_SIZE
