"""GPU parity of the Spearman-inversion estimator (cpc_spearman_fit) against
the FP64 oracle on the same data: the GPU ranks each subset (cpc_rank), the
oracle ranks it itself (the two rankings are bit-identical, tested
elsewhere). Tolerances: rho_S hat 1e-12 (an exact integer sum divided once),
theta 1e-6 relative to max(|theta|, 0.1) (the FP64 bar; the two sides
integrate rho_S(theta) by different rules), variance 1e-5 relative (the
oracle's slope of rho_S is a central difference), combined 1e-6."""
import numpy as np
import pytest
import torch

import oracle.oracle as O
import synth

pytestmark = pytest.mark.gpu

SIZES = [3000, 20000, 700, 12000, 40, 2, 9000, 2100]
CASES = [("gaussian", 0.5), ("gaussian", -0.8), ("frank", 5.0), ("frank", -8.0), ("frank", 0.3),
         ("gumbel", 2.0), ("gumbel", 1.02), ("gumbel", 8.0)]


def compare(g, sub, comb, label):
    st = sub["status"]
    assert np.array_equal(g["status"], st), (label, g["status"], st)
    fitted = (st == 0) | (st == 1) | (st == 2)
    dth = np.abs(g["theta"][fitted] - sub["theta"][fitted]) / np.maximum(np.abs(sub["theta"][fitted]), 0.1)
    drho = np.abs(g["loglik"][fitted] - sub["loglik"][fitted])
    use = (st == 0) | (st == 1)
    dvar = np.abs(g["var"][use] / sub["var"][use] - 1.0)
    dc = np.abs(g["combined_theta"] - comb["theta"]) / np.maximum(np.abs(comb["theta"]), 0.1)
    print(f"[spearman] {label}: max dtheta {dth.max(initial=0):.2e} drho {drho.max(initial=0):.2e} "
          f"dvar {dvar.max(initial=0):.2e} dcomb {np.nanmax(dc, initial=0):.2e}", flush=True)
    assert dth.max(initial=0) <= 1e-6, label
    assert drho.max(initial=0) <= 1e-12, label
    assert dvar.max(initial=0) <= 1e-5, label
    assert np.array_equal(g["n_used"], comb["n_used"]), label
    good = comb["status"] == 0
    assert np.all(dc[good] <= 1e-6), label


def gpu_fit(x, y, off, fams, gofs=None):
    import paper_1609_05530_amd as m
    dt = torch.float64
    R1, R2 = m.rank(torch.as_tensor(x, dtype=dt).cuda(), torch.as_tensor(y, dtype=dt).cuda(), off)
    res = m.spearman_fit(R1, R2, off, fams, gofs)
    torch.cuda.synchronize()
    return {k: getattr(res, k).cpu().numpy() for k in
            ("theta", "var", "loglik", "status", "combined_theta", "n_used", "combined_status")}


def oracle_fit(x, y, off, fams, gofs=None):
    R1 = np.concatenate([O.ranks(x[off[m]:off[m + 1]]) for m in range(len(off) - 1)])
    R2 = np.concatenate([O.ranks(y[off[m]:off[m + 1]]) for m in range(len(off) - 1)])
    return O.spearman_fit_ranks(R1, R2, off, fams, gofs)


@pytest.mark.parametrize("fam,th", CASES)
def test_spearman_fit_parity(fam, th):
    n = int(sum(SIZES))
    x, y = synth.copula_pairs(fam, th, n, 800 + int(abs(th) * 10))
    off = synth.offsets_from_sizes(np.array(SIZES))
    sub, comb = oracle_fit(x, y, off, fam)
    compare(gpu_fit(x, y, off, fam), sub, comb, f"{fam} {th}")


def test_spearman_groups_ties_and_statuses():
    """Several groups of different families in one call, tied margins, a
    constant margin (DEGENERATE) and negative dependence under Gumbel
    (theta = 1, BOUNDARY_NATURAL)."""
    parts = [("frank", 4.0), ("gumbel", 2.5), ("gaussian", 0.6), ("gumbel", 3.0)]
    xs, ys, offs, gofs = [], [], [0], [0]
    rng = np.random.default_rng(5)
    base = 0
    for k, (fam, th) in enumerate(parts):
        sizes = rng.integers(500, 6000, 5)
        x, y = synth.copula_pairs(fam, th, int(sizes.sum()), 900 + k)
        o = synth.offsets_from_sizes(sizes)
        if k == 0:
            x[o[1]:o[3]] = np.round(x[o[1]:o[3]] * 4) / 4  # heavy ties
        if k == 1:
            x[o[2]:o[3]] = 1.5                             # a constant margin
        if k == 3:
            y[o[0]:o[1]] = -x[o[0]:o[1]]                    # negative dependence
        xs.append(x); ys.append(y)
        offs.extend((o[1:] + base).tolist()); base += int(o[-1])
        gofs.append(gofs[-1] + len(sizes))
    x = np.concatenate(xs); y = np.concatenate(ys)
    offs = np.array(offs); gofs = np.array(gofs)
    fams = [p[0] for p in parts]
    sub, comb = oracle_fit(x, y, offs, fams, gofs)
    assert 3 in sub["status"] and 1 in sub["status"]
    compare(gpu_fit(x, y, offs, fams, gofs), sub, comb, "groups, ties, statuses")
