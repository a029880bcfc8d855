"""GPU parity of the float32 path against the FP64 oracle (Section 6 eq. 5 metric).

Gates: normwise relative error per array <= 2e-6 for forward and inverse and
<= 4e-6 for the fused round trip, whose reference is the input itself (the exact
round trip is the identity, Section 2.1).  Inputs come from the seeded generators
in ``workloads``; expected values come only from the oracle.
"""
import numpy as np
import pytest

import oracle
import workloads
from tests.gpu_util import GATE, assert_parity, errors, run, to_gpu

pytestmark = pytest.mark.gpu
SIZES = (8, 16, 32, 64, 128, 256)
DIRS = ("forward", "inverse", "roundtrip")


def _lib():
    import paper_2609_28519_amd as dct
    dct.init(0)
    return dct


@pytest.mark.parametrize("direction", DIRS)
def test_c1_uniform8(direction):
    """4096 blocks of 8x8 U[-1,1] (the small configuration), every block checked."""
    _lib()
    x = workloads.c1_uniform8().x
    y = run(x, direction)
    e = assert_parity(x, y, direction, label="c1")
    assert e.max() < 5e-7  # far inside the gate: float32 error is ~1e-7 (Section 6 Table 3 band)


def test_c1_two_call_roundtrip():
    """The materialised round trip (forward then inverse calls) also meets the gate (Section 4.2)."""
    _lib()
    x = workloads.c1_uniform8().x
    y = run(run(x, "forward"), "inverse")
    assert_parity(x, y, "roundtrip", label="c1 two-call")


@pytest.mark.parametrize("n", SIZES)
@pytest.mark.parametrize("direction", DIRS)
def test_square_sizes_ragged_tail(n, direction):
    """Batches spanning several tiles plus a ragged tail, N(0,1)."""
    _lib()
    batch = {8: 1001, 16: 523, 32: 131, 64: 37, 128: 11, 256: 5}[n]
    x = workloads.c3_normal(n, batch=batch, seed=1234 + n).x
    y = run(x, direction)
    assert_parity(x, y, direction, label="N=%d" % n)


@pytest.mark.parametrize("h,w", [(8, 16), (16, 8), (8, 64), (64, 8), (32, 128), (128, 32), (128, 64),
                                 (8, 256), (256, 8), (16, 256), (256, 16), (32, 256), (256, 32), (64, 256),
                                 (256, 64), (128, 256), (256, 128)])
@pytest.mark.parametrize("direction", DIRS)
def test_rectangles(h, w, direction):
    """Rectangular arrays Q_h X Q_w^T (Section 7.1)."""
    _lib()
    g = np.random.default_rng(h * 1000 + w)
    x = g.standard_normal((7, h, w)).astype(np.float32)
    y = run(x, direction)
    assert_parity(x, y, direction, label="%dx%d" % (h, w))


LONG_SHAPES = [(512, 512), (1024, 1024), (8, 1024), (1024, 8), (1024, 16), (16, 512), (256, 512), (512, 64),
               (512, 1024), (1024, 512), (128, 1024)]


@pytest.mark.parametrize("h,w", LONG_SHAPES)
@pytest.mark.parametrize("direction", DIRS)
def test_long_axes_basic_calls(h, w, direction):
    """Axes of 512 and 1024 through the in-place basic calls (two passes whose long-axis lines
    are shared by two or four wavefronts): a batch whose line count leaves a partial group of 64
    lines, every array checked against the oracle."""
    import torch
    dct = _lib()
    g = np.random.default_rng(h + 7 * w)
    batch = max(3, min(9, (1 << 22) // (h * w)))
    x = g.standard_normal((batch, h, w)).astype(np.float32)
    t = to_gpu(x)
    {"forward": dct.forward_, "inverse": dct.inverse_, "roundtrip": dct.roundtrip_}[direction](t)
    torch.cuda.synchronize()
    assert_parity(x, t.cpu().numpy(), direction, label="%dx%d" % (h, w))


@pytest.mark.parametrize("h,w", [(512, 512), (8, 1024), (1024, 64)])
@pytest.mark.parametrize("direction", DIRS)
def test_long_axes_out_of_place(h, w, direction):
    """The same out of place: the input is left untouched and the output matches the oracle."""
    import torch
    dct = _lib()
    g = np.random.default_rng(3 * h + w)
    x = g.standard_normal((5, h, w)).astype(np.float32)
    t = to_gpu(x)
    out = dct.transform(t, None, direction, "fp32")
    torch.cuda.synchronize()
    assert np.array_equal(t.cpu().numpy(), x), "out-of-place call modified its input"
    assert_parity(x, out.cpu().numpy(), direction, label="%dx%d" % (h, w))


def test_long_axes_other_precisions_rejected():
    """Only the float32 path exists for axes of 512 and 1024."""
    dct = _lib()
    x = to_gpu(np.zeros((2, 512, 512), np.float32))
    with pytest.raises(dct.DCT2DError) as e:
        dct.transform(x, None, "forward", "bf16")
    assert e.value.code == -5  # DCT2D_ERR_PRECISION


@pytest.mark.parametrize("n", (8, 64, 256))
def test_inverse_of_stored_spectrum(n):
    """Inverse applied to fl32(C(X)) recovers X (the inverse's own input is the spectrum)."""
    _lib()
    x = workloads.c3_normal(n, batch=9, seed=77).x
    spec = oracle.forward(x).astype(np.float32)
    y = run(spec, "inverse")
    assert_parity(spec, y, "inverse", label="spectrum N=%d" % n)
    assert oracle.e_rel(y, x, x).max() < 4e-6


@pytest.mark.parametrize("n", (16, 64, 256))
def test_strided_batch_and_guards(n):
    """stride > rows*cols: the gaps between arrays are guard values that must stay untouched."""
    import torch
    import paper_2609_28519_amd as dct
    _lib()
    batch, gap = 9, 12
    stride = n * n + gap
    g = np.random.default_rng(n)
    x = g.standard_normal((batch, n, n)).astype(np.float32)
    buf = np.full(batch * stride + 64, np.float32(1234.5), np.float32)
    for b in range(batch):
        buf[b * stride:b * stride + n * n] = x[b].ravel()
    t = to_gpu(buf)
    dct.forward_(t, rows=n, cols=n, stride=stride)
    torch.cuda.synchronize()
    out = t.cpu().numpy()
    y = np.stack([out[b * stride:b * stride + n * n].reshape(n, n) for b in range(batch)])
    assert_parity(x, y, "forward", label="strided")
    mask = np.ones(out.size, bool)
    for b in range(batch):
        mask[b * stride:b * stride + n * n] = False
    assert np.all(out[mask] == np.float32(1234.5)), "guard values overwritten"


@pytest.mark.parametrize("n", (8, 32, 128, 256))
def test_out_of_place_leaves_input_unchanged(n):
    _lib()
    x = workloads.c3_normal(n, batch=6, seed=5).x
    t = to_gpu(x)
    import torch
    import paper_2609_28519_amd as dct
    for d in DIRS:
        out = dct.transform(t, None, d, "fp32")
        torch.cuda.synchronize()
        assert np.array_equal(t.cpu().numpy(), x)
        assert_parity(x, out.cpu().numpy(), d, label="oop")


def test_zero_and_extreme_blocks():
    """Zero blocks give exact zeros (absolute check); 2^+-100 and 1e30 blocks meet the gate."""
    _lib()
    g = np.random.default_rng(3)
    for n in SIZES:
        x = g.uniform(-1, 1, (6, n, n))
        x[0] = 0.0
        x[1] *= 2.0 ** 100
        x[2] *= 2.0 ** -100
        x[3] *= 1e30
        x = x.astype(np.float32)
        for d in DIRS:
            y = run(x, d)
            assert np.all(y[0] == 0.0)
            assert_parity(x, y, d, label="extreme N=%d" % n)


def test_batch_zero_and_one():
    import torch
    import paper_2609_28519_amd as dct
    _lib()
    t = torch.zeros((0, 16, 16), device="cuda")
    dct.forward_(t)
    x = workloads.c3_normal(32, batch=1, seed=9).x
    assert_parity(x, run(x, "forward"), "forward")


def test_determinism_bitwise():
    """The same call on the same input gives bitwise-identical output."""
    _lib()
    for n in (8, 64, 256):
        x = workloads.c3_normal(n, batch=33, seed=n).x
        a = run(x, "roundtrip")
        b = run(x, "roundtrip")
        assert np.array_equal(a, b)


@pytest.mark.parametrize("direction", DIRS)
def test_c2_mixture_fp32(direction):
    """65536 16x16 tiles of the mixed configuration on the float32 path, per category."""
    _lib()
    bt = workloads.c2_mixture16()
    y = run(bt.x, direction)
    e = errors(bt.x, y, direction)
    for c in np.unique(bt.category):
        assert e[bt.category == c].max() <= GATE[direction], "category %d" % c


def _full_batch_check(dct, n, x_dev, xs, idx, refs, label, call):
    """Runs `call(direction, tensor)` on a fresh full-size copy per direction and checks: the
    sampled arrays against the oracle (forward, inverse: the input read as a spectrum) or the
    input (round trip); every array of the batch against a closed form that needs no oracle
    (round trip: the input itself; forward and inverse: Parseval's norm identity)."""
    import torch
    from tests.gpu_util import parseval_rel, per_array_rel
    sel = torch.from_numpy(idx).cuda()
    for d in DIRS:
        t = x_dev.clone()
        call(d, t)
        torch.cuda.synchronize()
        y = t[sel].cpu().numpy()
        e = oracle.e_rel(y, refs[d], xs)
        assert np.isfinite(e).all() and e.max() <= GATE[d], "%s %s: sampled max e_rel %.3e at array %d" % (
            label, d, e.max(), idx[int(np.argmax(e))])
        if d == "roundtrip":
            whole = per_array_rel(t, x_dev)
            gate = GATE[d]
        else:
            whole = parseval_rel(t, x_dev)
            gate = GATE[d]
        assert np.isfinite(whole).all() and whole.max() <= gate, "%s %s: array %d off by %.3e (all %d arrays)" % (
            label, d, int(np.argmax(whole)), whole.max(), whole.size)
        del t
    torch.cuda.empty_cache()


def _sample_refs(xs):
    return {"forward": oracle.forward(xs), "inverse": oracle.inverse(xs), "roundtrip": xs.astype(np.float64)}


@pytest.mark.parametrize("n", SIZES)
def test_full_size_c3_sampled(n):
    """Full 512 MiB batch (2^27/N^2 arrays of N(0,1)), in place through the three basic calls
    (forward_, inverse_ and the fused roundtrip_), in the launch configuration the benchmark
    times.  About 200 arrays spread over the whole batch (one per segment, the first and the last
    among them) are checked against the oracle; every array is checked against a closed form."""
    from tests.gpu_util import spread
    dct = _lib()
    bt = workloads.c3_normal(n)
    batch = bt.x.shape[0]
    idx = spread(batch, 200, seed=n)
    xs = bt.x[idx].copy()
    x_dev = to_gpu(bt.x)
    del bt
    calls = {"forward": dct.forward_, "inverse": dct.inverse_, "roundtrip": dct.roundtrip_}
    _full_batch_check(dct, n, x_dev, xs, idx, _sample_refs(xs), "full N=%d" % n, lambda d, t: calls[d](t))


@pytest.mark.parametrize("n,variants", [(256, (0, 1, 2, 3, 4)), (128, (0, 3, 4, 5))])
def test_full_batch_every_looping_variant(n, variants):
    """The variants whose workgroups loop over several arrays (N = 256: one resident workgroup per
    CU walks about eight arrays; N = 128 variants 0 and 3: grid-stride loops), and their
    one-array-per-workgroup siblings, at the full 512 MiB batch, every direction, in place:
    arrays from every pass of each loop are checked against the oracle, and every array against
    its closed form."""
    from tests.gpu_util import spread
    dct = _lib()
    bt = workloads.c3_normal(n, seed=4321 + n)
    batch = bt.x.shape[0]
    idx = spread(batch, 160, seed=7 * n)
    xs = bt.x[idx].copy()
    refs = _sample_refs(xs)
    x_dev = to_gpu(bt.x)
    del bt
    keep = {d: dct.get_variant(n, n, d, "fp32") for d in DIRS}
    try:
        for v in variants:
            for d in DIRS:
                dct.set_variant(n, n, d, "fp32", v)
            _full_batch_check(dct, n, x_dev, xs, idx, refs, "N=%d v%d" % (n, v),
                              lambda d, t: dct.transform(t, t, d, "fp32"))
    finally:
        for d in DIRS:
            dct.set_variant(n, n, d, "fp32", keep[d])


@pytest.mark.parametrize("h,w", [(8, 256), (256, 8), (16, 256), (256, 32), (64, 256), (256, 64), (128, 256)])
def test_rect256_every_variant_many_tiles(h, w):
    """Rectangles with a 256 axis in every variant, at a batch of about three tiles per CU plus a
    ragged last tile (a tile is 64 long lines: 64 / short-axis arrays, or one array for a short
    axis of 64 or 128), so that the persistent schedules (one or two resident workgroups per CU,
    one of them double-buffered) run every stage of their loops, in place, every direction:
    sampled arrays against the oracle, every array against its closed form."""
    from tests.gpu_util import spread
    dct = _lib()
    s = w if h == 256 else h
    per_tile = max(1, 64 // s) if s <= 64 else 1
    batch = per_tile * (3 * 256 + 5) - (per_tile - 1 if per_tile > 1 else 0)
    g = np.random.default_rng(h * 7 + w)
    x = g.standard_normal((batch, h, w)).astype(np.float32)
    idx = spread(batch, 120, seed=h + w)
    xs = x[idx].copy()
    refs = _sample_refs(xs)
    x_dev = to_gpu(x)
    del x
    keep = {d: dct.get_variant(h, w, d, "fp32") for d in DIRS}
    try:
        for v in range(dct.variant_count(h, w, "forward", "fp32")):
            for d in DIRS:
                dct.set_variant(h, w, d, "fp32", v)
            _full_batch_check(dct, s, x_dev, xs, idx, refs, "%dx%d v%d" % (h, w, v),
                              lambda d, t: dct.transform(t, t, d, "fp32"))
    finally:
        for d in DIRS:
            dct.set_variant(h, w, d, "fp32", keep[d])


@pytest.mark.parametrize("h,w", [(8, 8), (16, 16), (32, 32), (64, 64), (128, 128), (256, 256), (8, 64), (64, 16),
                                 (128, 32), (256, 64), (8, 256), (128, 256), (256, 16)])
@pytest.mark.parametrize("direction", DIRS)
def test_every_variant(h, w, direction):
    """Every kernel variant the autotuner may pick meets the gate (the policy only changes speed)."""
    dct = _lib()
    g = np.random.default_rng(h + 3 * w)
    x = g.standard_normal(((2048 // h) + 3, h, w)).astype(np.float32)
    nv = dct.variant_count(h, w, direction, "fp32")
    assert nv >= 1
    keep = dct.get_variant(h, w, direction, "fp32")
    try:
        for v in range(nv):
            dct.set_variant(h, w, direction, "fp32", v)
            assert_parity(x, run(x, direction), direction, label="%dx%d v%d" % (h, w, v))
    finally:
        dct.set_variant(h, w, direction, "fp32", keep)


@pytest.mark.parametrize("h,w", [(8, 8), (16, 16), (32, 32), (64, 64), (8, 64), (64, 16)])
@pytest.mark.parametrize("direction", DIRS)
def test_wave_variants_many_tiles(h, w, direction):
    """The wave-local variants (0: grid-stride over several tiles per workgroup, 4: tiles
    staged through LDS with whole-tile 16-byte moves, 7 and 12: plain and staged with the
    resident workgroups per CU capped) and, at 64 x 64, the two-wavefront split kernel (13)
    on a 64 MiB batch plus a ragged tail; about 500 sampled arrays (the first, the last and
    the tail among them) are checked."""
    import torch
    dct = _lib()
    batch = (1 << 24) // (h * w) + 5
    g = np.random.default_rng(7 * h + w)
    x = g.standard_normal((batch, h, w)).astype(np.float32)
    idx = np.unique(np.concatenate([g.integers(0, batch, 500), np.arange(batch - 6, batch), [0]]))
    xs = x[idx].copy()
    ref = oracle.forward(xs) if direction == "forward" else oracle.inverse(xs) if direction == "inverse" else xs
    keep = dct.get_variant(h, w, direction, "fp32")
    t = torch.from_numpy(x).cuda()
    out = torch.empty_like(t)
    try:
        for v in (0, 4, 7, 12) + ((13, 15) if h == w == 64 else ()):
            dct.set_variant(h, w, direction, "fp32", v)
            out.fill_(float("nan"))
            dct.transform(t, out, direction, "fp32")
            torch.cuda.synchronize()
            y = out[torch.from_numpy(idx).cuda()].cpu().numpy()
            e = oracle.e_rel(y, ref, xs)
            assert np.isfinite(e).all() and e.max() <= GATE[direction], "%dx%d v%d %s: %.3e" % (
                h, w, v, direction, e.max())
    finally:
        dct.set_variant(h, w, direction, "fp32", keep)
