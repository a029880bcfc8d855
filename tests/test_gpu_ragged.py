"""GPU parity of ragged plans (one recorded HIP graph, one launch) against the FP64 oracle.

Covers mixed square blocks, rectangles and whole images (including the non-power-of-two
384 axis, computed from the dense Q_n), the forward / inverse / fused round trip,
replays on the same and on a different buffer, and the planner's error paths.
"""
import numpy as np
import pytest

import oracle
import workloads
from tests.gpu_util import GATE

pytestmark = pytest.mark.gpu
DIRS = ("forward", "inverse", "roundtrip")


def _lib():
    import paper_2609_28519_amd as dct
    dct.init(0)
    return dct


def _check(rg: workloads.Ragged, out: np.ndarray, direction: str, idx=None, label=""):
    """Scores every listed item against the oracle, batched by shape."""
    idx = np.arange(rg.count) if idx is None else np.asarray(idx)
    worst = 0.0
    shapes = {}
    for i in idx:
        shapes.setdefault((int(rg.rows[i]), int(rg.cols[i])), []).append(int(i))
    for (h, w), items in shapes.items():
        x = np.stack([rg.item(i) for i in items])
        y = np.stack([rg.item(i, out) for i in items])
        if direction == "forward":
            ref = oracle.forward(x)
        elif direction == "inverse":
            ref = oracle.inverse(x)
        else:
            ref = x.astype(np.float64)
        e = oracle.e_rel(y, ref, x)
        assert e.max() <= GATE[direction], "%s %s %dx%d: %.3e" % (label, direction, h, w, e.max())
        worst = max(worst, float(e.max()))
    return worst


def _small_ragged(seed=11):
    # image axes: even/odd dense passes (1024, 512, 384, 64, 40, 24) and the plain dense
    # pass (12, 20: half-lengths not multiples of 4)
    images = ((1024, 1024), (512, 384), (384, 512), (256, 128), (64, 1024), (40, 24), (12, 20))
    return workloads.c4_ragged(blocks=3000, images=images, seed=seed)


@pytest.mark.parametrize("direction", DIRS)
@pytest.mark.parametrize("precision", ("fp32", "auto"))
def test_ragged_small_every_item(direction, precision):
    import torch
    dct = _lib()
    rg = _small_ragged()
    plan = dct.RaggedPlan(rg.offsets, rg.rows, rg.cols, direction, precision)
    info = plan.info()
    assert info["items"] == rg.count
    assert info["classes"] == len(set(zip(rg.rows.tolist(), rg.cols.tolist())))
    assert info["graph_nodes"] >= info["classes"]
    buf = torch.from_numpy(rg.data).cuda()
    plan.execute(buf)
    torch.cuda.synchronize()
    worst = _check(rg, buf.cpu().numpy(), direction, label=precision)
    print("ragged %s %s worst e_rel %.3e" % (direction, precision, worst))
    plan.close()


def test_ragged_replay_same_and_new_buffer():
    """The recorded graph replays on the same buffer and on a different one (base slot update)."""
    import torch
    dct = _lib()
    rg = _small_ragged(seed=12)
    plan = dct.RaggedPlan(rg.offsets, rg.rows, rg.cols, "forward", "fp32")
    a = torch.from_numpy(rg.data).cuda()
    b = torch.from_numpy(rg.data).cuda()
    plan.execute(a)
    plan.execute(b)
    torch.cuda.synchronize()
    ya = a.cpu().numpy()
    assert np.array_equal(ya, b.cpu().numpy())
    a.copy_(torch.from_numpy(rg.data))
    plan.execute(a)  # back to the first buffer
    torch.cuda.synchronize()
    assert np.array_equal(a.cpu().numpy(), ya)
    _check(rg, ya, "forward", label="replay")
    plan.close()


def test_ragged_guards_untouched():
    """Gaps between items (guard values) survive the graph, including the image workspace passes."""
    import torch
    dct = _lib()
    rows = np.array([8, 16, 512, 32, 64, 256, 1024], np.int32)
    cols = np.array([8, 16, 384, 32, 64, 256, 1024], np.int32)
    gap = 16
    offsets = np.zeros(rows.size, np.int64)
    pos = gap
    for i in range(rows.size):
        offsets[i] = pos
        pos += int(rows[i]) * int(cols[i]) + gap
    g = np.random.default_rng(4)
    data = np.full(pos + gap, np.float32(-7.25), np.float32)
    for i in range(rows.size):
        data[offsets[i]:offsets[i] + rows[i] * cols[i]] = g.standard_normal(rows[i] * cols[i])
    rg = workloads.Ragged(data, offsets, rows, cols, np.zeros(rows.size, bool))
    plan = dct.RaggedPlan(offsets, rows, cols, "roundtrip", "fp32")
    buf = torch.from_numpy(data).cuda()
    plan.execute(buf)
    torch.cuda.synchronize()
    out = buf.cpu().numpy()
    mask = np.ones(out.size, bool)
    for i in range(rows.size):
        mask[offsets[i]:offsets[i] + rows[i] * cols[i]] = False
    assert np.all(out[mask] == np.float32(-7.25))
    _check(rg, out, "roundtrip", label="guards")
    plan.close()


def test_ragged_plan_errors():
    dct = _lib()
    with pytest.raises(dct.DCT2DError) as e:
        dct.RaggedPlan([2], [8], [8])  # offset not a multiple of 4
    assert e.value.code == -4
    with pytest.raises(dct.DCT2DError) as e:
        dct.RaggedPlan([0, 32], [8, 8], [8, 8])  # overlapping
    assert e.value.code == -1
    with pytest.raises(dct.DCT2DError) as e:
        dct.RaggedPlan([0], [2048], [8])  # axis too long
    assert e.value.code == -2
    with pytest.raises(dct.DCT2DError) as e:
        dct.RaggedPlan([0], [8], [8], "forward", "bf16x3")  # not a float32-accurate path
    assert e.value.code == -5


@pytest.mark.parametrize("direction", ("forward", "roundtrip"))
def test_c4_full_ragged_sampled(direction):
    """The full ragged configuration (200k blocks + 4 x 1024^2 + 4 x 512x384, 5% x 1e30), one graph
    launch; every image and a seeded sample of 3000 blocks (plus every 1e30 block of the sample
    classes 128/256) checked against the oracle."""
    import torch
    dct = _lib()
    rg = workloads.c4_ragged()
    plan = dct.RaggedPlan(rg.offsets, rg.rows, rg.cols, direction, "auto")
    buf = torch.from_numpy(rg.data).cuda()
    plan.execute(buf)
    torch.cuda.synchronize()
    out = buf.cpu().numpy()
    g = np.random.default_rng(2026)
    nblocks = rg.count - 8
    sample = np.unique(np.concatenate([g.integers(0, nblocks, 3000), np.arange(nblocks, rg.count),
                                       np.flatnonzero(rg.scaled[:nblocks] & (rg.rows[:nblocks] >= 128))[:40]]))
    worst = _check(rg, out, direction, idx=sample, label="c4")
    print("c4 %s sampled %d items, worst e_rel %.3e" % (direction, sample.size, worst))
    plan.close()


@pytest.mark.parametrize("direction", DIRS)
def test_ragged_every_wave_variant(direction):
    """Ragged plans reach the wave-local kernels through offset lists and the plan's base
    slot; every variant of the 8..64 classes (grid-stride, staged, occupancy-capped) is
    recorded and checked, including each class's partial last tile."""
    import torch
    dct = _lib()
    mix = {8: 0.4, 16: 0.3, 32: 0.2, 64: 0.1}
    rg = workloads.c4_ragged(blocks=1203, images=(), seed=24, mix=mix)  # 476, 350, 253, 124 blocks
    sizes = sorted(mix)
    keep = {n: dct.get_variant(n, n, direction, "fp32") for n in sizes}
    nv = dct.variant_count(8, 8, direction, "fp32")
    try:
        for v in [0] + list(range(3, nv)):
            for n in sizes:
                dct.set_variant(n, n, direction, "fp32", v)
            plan = dct.RaggedPlan(rg.offsets, rg.rows, rg.cols, direction, "fp32")
            buf = torch.from_numpy(rg.data).cuda()
            plan.execute(buf)
            torch.cuda.synchronize()
            _check(rg, buf.cpu().numpy(), direction, label="v%d" % v)
            plan.close()
    finally:
        for n in sizes:
            dct.set_variant(n, n, direction, "fp32", keep[n])


@pytest.mark.parametrize("direction", DIRS)
def test_ragged_non_power_of_two_axes_beyond_384(direction):
    """Whole images with non-power-of-two axes above 384 (computed exactly from the dense Q_n
    of eq. 1, no zero-padding; Section 7.1 rejects such axes in the paper's library): 1000,
    600, 520, 700, 768 and 1020, with even/odd passes where the axis divides by 8 and the
    plain dense pass otherwise, beside a few hundred blocks."""
    import torch
    dct = _lib()
    images = ((1000, 600), (600, 1000), (520, 700), (768, 768), (8, 1000), (1020, 12))
    rg = workloads.c4_ragged(blocks=300, images=images, seed=29)
    plan = dct.RaggedPlan(rg.offsets, rg.rows, rg.cols, direction, "fp32")
    buf = torch.from_numpy(rg.data).cuda()
    plan.execute(buf)
    torch.cuda.synchronize()
    worst = _check(rg, buf.cpu().numpy(), direction, label="beyond 384")
    print("ragged beyond-384 %s worst e_rel %.3e" % (direction, worst))
    plan.close()
