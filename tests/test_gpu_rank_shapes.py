"""Every launch shape of the workgroup rank kernel (the radix variants, the
one-wave merge sort and the truncated sorts the autotuner chooses among),
forced for the size class of its capacity: ranks bit-exact against the
oracle for sizes spanning the class (ragged, powers of two and one past
them), FP32 margins with ties, +-0, values of one sign, two values, uniform
values, a narrow cluster and a cluster a few ulps wide beside an outlier
(long runs of equal leading bits: a truncated sort falls back to the full
sort), values rounded to 1e-5 (exact ties inside short runs), and both tie
rules; and a whole batched
fit under each forced shape is bitwise identical to the built-in shapes (the
sorted positions and tie starts are those of the stable order whatever the
sort)."""
import numpy as np
import pytest
import torch

import oracle.oracle as O
import synth

pytestmark = pytest.mark.gpu

# (threads, items) of each shape, in the library's shape order; 14 is the
# merge sort, 15 the truncated sort
SHAPES = [(64, 8), (256, 8), (128, 16), (512, 16), (256, 32), (1024, 16), (512, 32),
          (64, 8), (256, 8), (128, 16), (512, 16), (256, 32), (1024, 16), (512, 32),
          (64, 8), (64, 8)]
CLASS_OF_CAP = {512: (1, 512), 2048: (513, 2048), 8192: (2049, 8192), 16384: (8193, 16384)}


def class_range(shape):
    t, e = SHAPES[shape]
    return CLASS_OF_CAP[t * e]


def margins(sizes, rng):
    xs, ys = [], []
    for i, m in enumerate(sizes):
        g = rng.standard_normal(m)
        kind = i % 9
        if kind == 1:
            x = np.round(g * 4) / 4                     # heavy ties
        elif kind == 2:
            x = np.abs(g)                               # one sign
        elif kind == 3:
            x = g.copy(); x[::7] = 0.0; x[1::7] = -0.0  # signed zeros
        elif kind == 4:
            x = np.where(g > 0.3, 1.0, 2.0)             # two values
        elif kind == 5:
            x = rng.random(m)                           # uniform on [0, 1)
        elif kind == 6:
            x = 1.0 + 1e-3 * g                          # a narrow cluster
        elif kind == 7:
            x = np.round(g, 5)                          # exact ties among nearby values
        elif kind == 8:
            x = 1.0 + rng.integers(0, 64, m) * 2.0 ** -23  # a cluster a few ulps wide ...
            x[0] = -1e4                                 # ... beside an outlier
        else:
            x = g
        xs.append(x)
        ys.append(rng.permutation(x) + (0.0 if kind in (4, 8) else 0.5 * rng.standard_normal(m)))
    return np.concatenate(xs).astype(np.float32), np.concatenate(ys).astype(np.float32)


def test_shape_table_matches_library():
    import paper_1609_05530_amd as m
    with pytest.raises(m.CpcError):
        m.rank(torch.zeros(4, device="cuda"), torch.zeros(4, device="cuda"), [0, 4], schedule=len(SHAPES) + 1)


@pytest.mark.parametrize("ties", ["average", "first"])
@pytest.mark.parametrize("shape", range(len(SHAPES)))
def test_forced_shape_ranks_bit_exact(shape, ties):
    import paper_1609_05530_amd as m
    lo, hi = class_range(shape)
    rng = np.random.default_rng(100 + shape)
    pw = [s for s in (512, 1024, 2048, 4096, 8192, 16384) if lo <= s <= hi]
    sizes = sorted(set([lo, lo + 1, hi, *pw, *[min(p + 1, hi) for p in pw], *rng.integers(lo, hi + 1, 6).tolist()]))
    x, y = margins(sizes, rng)
    off = synth.offsets_from_sizes(np.array(sizes))
    dev = lambda a: torch.as_tensor(a, dtype=torch.float32).cuda()
    print(f"[shapes] shape {shape} {SHAPES[shape]} ties={ties}: {len(sizes)} subsets of {lo}..{hi} rows", flush=True)
    R1, R2 = m.rank(dev(x), dev(y), off, ties=ties, schedule=1 + shape)
    R1 = R1.cpu().numpy().astype(np.int64); R2 = R2.cpu().numpy().astype(np.int64)
    xd, yd = x.astype(np.float64), y.astype(np.float64)
    for k in range(len(sizes)):
        a, b = off[k], off[k + 1]
        assert np.array_equal(R1[a:b], O.ranks(xd[a:b], ties)), (shape, sizes[k])
        assert np.array_equal(R2[a:b], O.ranks(yd[a:b], ties)), (shape, sizes[k])


def test_fit_with_forced_shapes_equals_built_in_shapes():
    import paper_1609_05530_amd as m
    rng = np.random.default_rng(7)
    sizes = np.concatenate([rng.integers(3, 512, 40), rng.integers(513, 2048, 30), rng.integers(2049, 8192, 20),
                            rng.integers(8193, 16384, 12)])
    off = synth.offsets_from_sizes(sizes)
    x, y = m.sample("frank", 4.0, int(off[-1]), seed=9, dtype=torch.float32)
    gofs = np.array([0, len(sizes)])
    ref = m.fit_batched(x, y, off, gofs, ["frank"], prec="fp32c", schedule=0)
    ref_raw = ref.raw.cpu().numpy().copy()
    for shape in range(len(SHAPES)):
        got = m.fit_batched(x, y, off, gofs, ["frank"], prec="fp32c", schedule=1 + shape)
        assert np.array_equal(got.raw.cpu().numpy(), ref_raw, equal_nan=True), shape
    # graph mode, the schedule changing between calls (each schedule captures its own launches)
    for sched in (0, 15, 16, 0):
        got = m.fit_batched(x, y, off, gofs, ["frank"], prec="fp32c", graph=True, schedule=sched)
        assert np.array_equal(got.raw.cpu().numpy(), ref_raw, equal_nan=True), sched
