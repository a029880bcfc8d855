"""Argument checks of the Python binding and the autotuner's correctness guard, on the GPU.

The binding hands raw device pointers to the C ABI, so it must refuse any buffer the
kernels would misuse: a host tensor, another dtype, another device, a ragged base too
short for its plan.  The tuner must freeze only variants that pass its own guard
(the candidate composed with the opposite transform returns the input on arrays
spread over the whole batch), so a tuned policy meets parity on a batch larger than
one pass of any looping schedule.
"""
import ctypes

import numpy as np
import pytest

import oracle
import workloads
from tests.gpu_util import GATE, spread

pytestmark = pytest.mark.gpu


def _lib():
    import paper_2609_28519_amd as dct
    dct.init(0)
    return dct


def test_transform_rejects_bad_output_buffers():
    import torch
    dct = _lib()
    x = torch.zeros((3, 16, 16), device="cuda")
    with pytest.raises(TypeError):
        dct.transform(x, torch.zeros((3, 16, 16)), "forward", "fp32")  # host tensor
    with pytest.raises(TypeError):
        dct.transform(x, torch.zeros((3, 16, 16), device="cuda", dtype=torch.float16), "forward", "fp32")
    with pytest.raises(ValueError):
        dct.transform(x, torch.zeros((3, 16, 8), device="cuda"), "forward", "fp32")
    with pytest.raises(TypeError):
        dct.filter(x, torch.ones((16, 16)), out=x)  # host multipliers
    with pytest.raises(TypeError):
        dct.filter(x, torch.ones((16, 16), device="cuda"), out=torch.zeros((3, 16, 16)))


def test_in_place_with_different_strides_is_rejected():
    """in == out with in_stride != out_stride would write array b over another array's input."""
    import torch
    dct = _lib()
    buf = torch.zeros(4 * 80, device="cuda")
    lam = torch.ones(64, device="cuda")
    p = ctypes.c_void_p(buf.data_ptr())
    lib = dct.load()
    assert lib.dct2d_transform_ex(0, p, p, 3, 8, 8, 80, 64, 0, None) == -1
    assert lib.dct2d_filter(p, p, 3, 8, 8, 64, 80, ctypes.c_void_p(lam.data_ptr()), 0, None) == -1
    assert lib.dct2d_transform_ex(0, p, p, 1, 8, 8, 80, 64, 0, None) == 0  # one array: no conflict
    torch.cuda.synchronize()


def test_ragged_plan_checks_its_base():
    import torch
    dct = _lib()
    offsets = [0, 64, 64 + 256]
    rows, cols = [8, 16, 8], [8, 16, 8]
    plan = dct.RaggedPlan(offsets, rows, cols, "forward", "fp32")
    try:
        assert plan.extent == 64 + 256 + 64
        with pytest.raises(ValueError):
            plan.execute(torch.zeros(plan.extent - 1, device="cuda"))
        with pytest.raises(TypeError):
            plan.execute(torch.zeros(plan.extent, device="cuda", dtype=torch.float64))
        with pytest.raises(TypeError):
            plan.execute(torch.zeros(plan.extent))
        base = torch.zeros(plan.extent, device="cuda")
        plan.execute(base)
        torch.cuda.synchronize()
    finally:
        plan.close()


@pytest.mark.parametrize("n,direction", [(256, "roundtrip"), (256, "forward"), (128, "inverse"),
                                         (64, "roundtrip"), (16, "forward")])
def test_tuned_variant_meets_parity_across_the_batch(n, direction):
    """Tune on a batch of several loop passes plus a tail, then check arrays spread over a fresh
    batch of that size against the oracle in the frozen variant."""
    import torch
    dct = _lib()
    keep = dct.get_variant(n, n, direction, "fp32")
    batch = {256: 3 * 256 + 5, 128: 9 * 256 + 3}.get(n, (1 << 22) // (n * n) + 7)
    try:
        ms = dct.tune(n, n, direction, "fp32", batch=batch)
        assert ms > 0
        v = dct.get_variant(n, n, direction, "fp32")
        assert 0 <= v < dct.variant_count(n, n, direction, "fp32")
        x = workloads.c3_normal(n, batch=batch, seed=99 + n).x
        idx = spread(batch, 64, seed=n)
        t = torch.from_numpy(x).cuda()
        dct.transform(t, t, direction, "fp32")
        torch.cuda.synchronize()
        y = t[torch.from_numpy(idx).cuda()].cpu().numpy()
        xs = x[idx]
        ref = {"forward": oracle.forward, "inverse": oracle.inverse}.get(direction, lambda a: a.astype(np.float64))(xs)
        e = oracle.e_rel(y, ref, xs)
        assert e.max() <= GATE[direction], "tuned v%d: %.3e" % (v, e.max())
    finally:
        dct.set_variant(n, n, direction, "fp32", keep)
