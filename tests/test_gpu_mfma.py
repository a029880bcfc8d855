"""GPU parity of the dense matrix (MFMA) paths, N = 8, 16, 32, against the FP64 oracle.

Gated (float32-accurate) paths: split bf16 with three-way splits and six products
("bf16x6") and split fp16 with per-block power-of-two scaling ("fp16x3"), at
2e-6 (forward/inverse) and 4e-6 (round trip).  The two-way bf16 split with three
products ("bf16x3") carries about 16 significant bits and is reported, not gated; the
single-pass bf16 / fp16 / fp8 paths are reported, not gated.  Every path is held to a
loose band that any layout or indexing mistake would break.
"""
import numpy as np
import pytest

import oracle
import workloads
from tests.gpu_util import GATE, assert_parity, errors, run

pytestmark = pytest.mark.gpu
DIRS = ("forward", "inverse", "roundtrip")
GATED = ("bf16x6", "fp16x3")
# loose sanity bands for ungated paths (normwise relative error per array)
BAND = {"bf16x3": 5e-5, "bf16": 2e-2, "fp16": 3e-3, "fp8": 0.25}


def _lib():
    import paper_2609_28519_amd as dct
    dct.init(0)
    return dct


def _limit(prec, direction):
    return GATE[direction] if prec in GATED else BAND[prec] * (2 if direction == "roundtrip" else 1)


@pytest.mark.parametrize("prec", ["bf16x6", "fp16x3", "bf16x3", "bf16", "fp16", "fp8"])
@pytest.mark.parametrize("n", (8, 16, 32, 64))
@pytest.mark.parametrize("direction", DIRS)
def test_paths_normal_inputs(prec, n, direction):
    _lib()
    batch = {8: 1003, 16: 517, 32: 131, 64: 71}[n]  # several waves plus a ragged tail
    x = workloads.c3_normal(n, batch=batch, seed=99 + n).x
    y = run(x, direction, prec)
    e = errors(x, y, direction)
    print("%-7s N=%-3d %-9s max %.3e median %.3e" % (prec, n, direction, e.max(), np.median(e)))
    assert e.max() <= _limit(prec, direction), "%s N=%d %s: %.3e" % (prec, n, direction, e.max())


@pytest.mark.parametrize("prec", GATED)
@pytest.mark.parametrize("n", (8, 16, 32, 64))
def test_gated_paths_extreme_blocks(prec, n):
    """Power-of-two scaling per block: 2^+-100, 1e30 and zero blocks meet the gate."""
    _lib()
    g = np.random.default_rng(n)
    x = g.uniform(-1, 1, (12, n, n))
    x[0] = 0.0
    x[1] *= 2.0 ** 100
    x[2] *= 2.0 ** -100
    x[3] *= 1e30
    x[4] *= 2.0 ** 60
    x[5] *= 2.0 ** -60
    x[6] = 3.0  # constant: DC only
    x = x.astype(np.float32)
    for d in DIRS:
        y = run(x, d, prec)
        assert np.all(y[0] == 0.0)
        assert_parity(x, y, d, label="%s extreme N=%d" % (prec, n))


@pytest.mark.parametrize("prec", ("bf16x3", "bf16x6", "fp16x3"))
@pytest.mark.parametrize("direction", DIRS)
def test_c2_mixture_split_paths(prec, direction):
    """The 16x16 mixed configuration on the split-precision matrix paths, per category."""
    _lib()
    bt = workloads.c2_mixture16()
    y = run(bt.x, direction, prec)
    e = errors(bt.x, y, direction)
    lim = _limit(prec, direction)
    for c in np.unique(bt.category):
        print("%s %s category %d: max %.3e" % (prec, direction, c, e[bt.category == c].max()))
        assert e[bt.category == c].max() <= lim


@pytest.mark.parametrize("prec", ("bf16x6", "fp16x3", "fp8"))
@pytest.mark.parametrize("n", (8, 16, 32))
def test_every_unroll_variant(prec, n):
    dct = _lib()
    x = workloads.c3_normal(n, batch=777, seed=5).x
    keep = dct.get_variant(n, n, "forward", prec)
    try:
        for v in range(dct.variant_count(n, n, "forward", prec)):
            dct.set_variant(n, n, "forward", prec, v)
            y = run(x, "forward", prec)
            assert errors(x, y, "forward").max() <= _limit(prec, "forward")
    finally:
        dct.set_variant(n, n, "forward", prec, keep)


def test_mfma_determinism_and_unsupported_sizes():
    import torch
    dct = _lib()
    x = workloads.c3_normal(16, batch=100, seed=1).x
    assert np.array_equal(run(x, "forward", "bf16x6"), run(x, "forward", "bf16x6"))
    t = torch.zeros((4, 128, 128), device="cuda")
    with pytest.raises(dct.DCT2DError):
        dct.transform(t, None, "forward", "bf16x6")  # matrix paths exist for N <= 64 only
    t = torch.zeros((4, 8, 16), device="cuda")
    with pytest.raises(dct.DCT2DError):
        dct.transform(t, None, "forward", "fp16x3")  # squares only


def test_weak_component_reported():
    """Weak cosine component (amplitude 1e-6 on an O(1) ramp): its relative error is reported
    (Section 6: the norm criterion can hide weak-component loss); not gated."""
    _lib()
    bt = workloads.c2_mixture16(batch=4096)
    idx = np.flatnonzero(bt.category == workloads.CAT_RAMP_WEAK)[:64]
    x = bt.x[idx]
    ref = oracle.forward(x)
    for prec in ("fp32", "bf16x6", "fp16x3", "bf16x3"):
        y = run(x, "forward", prec)
        rel = [oracle.weak_component_error(y[i], ref[i], *bt.weak_kl[idx[i]]) for i in range(len(idx))]
        print("weak component %s: median %.3e max %.3e" % (prec, np.median(rel), np.max(rel)))
        assert np.all(np.isfinite(rel))
