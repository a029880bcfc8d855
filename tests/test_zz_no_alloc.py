"""dct2d_image_transform_noalloc against dct2d_image_transform (through the C ABI).

The no-allocation entry point runs the same kernels with its dense Q tables and workspace in
the library's fixed device scratch, so its output must equal the allocating entry point's
bit for bit, and meet the oracle's gates.  Two calls in a row, the second with a smaller
input, check that nothing a call leaves in the shared scratch leaks into the next; the
first call spans more than one chunk of the scratch.
"""
import ctypes

import numpy as np
import pytest

import oracle
from tests.gpu_util import GATE

pytestmark = pytest.mark.gpu


def _call(name, d, t, out, batch, h, w):
    import paper_2609_28519_amd as dct
    fn = getattr(dct.load(), name)
    rc = fn(d, ctypes.c_void_p(t.data_ptr()), ctypes.c_void_p(out.data_ptr()), batch, h, w, h * w, h * w, None)
    assert rc == 0, "%s returned %d" % (name, rc)


@pytest.mark.parametrize("direction", (0, 1, 2))
def test_noalloc_equals_allocating_entry_point(direction):
    import torch
    import paper_2609_28519_amd as dct
    dct.init(0)
    gate = GATE[("forward", "inverse", "roundtrip")[direction]]
    # first call: 20 images of 1024 x 1024 (80 MiB, two chunks of the 64 MiB scratch);
    # second call: 3 images of 600 x 1000, smaller, another pair of dense tables
    for h, w, batch in ((1024, 1024, 20), (600, 1000, 3)):
        g = np.random.default_rng(h + w + direction)
        x = g.uniform(-1, 1, (batch, h, w)).astype(np.float32)
        t = torch.from_numpy(x).cuda()
        ref = torch.full_like(t, float("nan"))
        got = torch.full_like(t, float("nan"))
        _call("dct2d_image_transform", direction, t, ref, batch, h, w)
        _call("dct2d_image_transform_noalloc", direction, t, got, batch, h, w)
        torch.cuda.synchronize()
        a, b = ref.cpu().numpy(), got.cpu().numpy()
        assert np.isfinite(b).all()
        assert np.array_equal(a, b), "%dx%d: differs from the allocating entry point" % (h, w)
        pick = [0, batch - 1]
        xs = x[pick]
        exp = {0: oracle.forward, 1: oracle.inverse}.get(direction, lambda v: v.astype(np.float64))(xs)
        e = oracle.e_rel(b[pick], exp, xs)
        assert e.max() <= gate, "%dx%d: %.3e" % (h, w, e.max())
