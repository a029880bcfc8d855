"""GPU parity of dct2d_image_transform: batched whole images of any shape with both axes in
[8, 1024] (Section 2.1 eq. 1-2 on rectangles, Section 7.1), against the FP64 oracle.

Shapes outside the fast kernels (512, 1024, and lengths that are not powers of two: 384,
600, 1000, 12 x ...) go through the dense Q_n passes; power-of-two shapes up to 256 through
the basic calls' kernels.  Gates as everywhere: 2e-6 forward and inverse, 4e-6 round trip.
"""
import numpy as np
import pytest

import oracle
from tests.gpu_util import GATE

pytestmark = pytest.mark.gpu
DIRS = ("forward", "inverse", "roundtrip")


def _lib():
    import paper_2609_28519_amd as dct
    dct.init(0)
    return dct


def _ref(x, d):
    return {"forward": oracle.forward, "inverse": oracle.inverse}.get(d, lambda a: a.astype(np.float64))(x)


@pytest.mark.parametrize("h,w,batch", [(1024, 1024, 2), (512, 512, 3), (512, 384, 3), (384, 512, 3),
                                       (600, 1000, 2), (1000, 600, 2), (12, 20, 37), (8, 1024, 9), (1024, 8, 9),
                                       (520, 768, 2), (256, 256, 3), (16, 64, 17)])
@pytest.mark.parametrize("direction", DIRS)
def test_image_transform_matches_oracle(h, w, batch, direction):
    import torch
    dct = _lib()
    g = np.random.default_rng(h * 3 + w)
    x = g.uniform(-1, 1, (batch, h, w)).astype(np.float32)
    x[0] *= np.float32(1e30)
    t = torch.from_numpy(x).cuda()
    y = dct.image_transform(t, None, direction)
    torch.cuda.synchronize()
    e = oracle.e_rel(y.cpu().numpy(), _ref(x, direction), x)
    assert e.max() <= GATE[direction], "%dx%d %s: %.3e" % (h, w, direction, e.max())
    assert np.array_equal(t.cpu().numpy(), x)  # out of place leaves the input alone
    dct.image_transform(t, t, direction)       # in place gives the same result
    torch.cuda.synchronize()
    assert np.array_equal(t.cpu().numpy(), y.cpu().numpy())


def test_image_transform_strided_through_the_c_abi():
    """stride > rows*cols: the gaps are guard values that must stay untouched."""
    import ctypes

    import torch
    dct = _lib()
    h, w, batch, gap = 384, 512, 3, 36
    n = h * w
    s = n + gap
    x = np.random.default_rng(5).standard_normal((batch, h, w)).astype(np.float32)
    buf = np.full(batch * s, np.float32(-7.25), np.float32)
    for b in range(batch):
        buf[b * s:b * s + n] = x[b].ravel()
    t = torch.from_numpy(buf).cuda()
    rc = dct.load().dct2d_image_transform(0, ctypes.c_void_p(t.data_ptr()), ctypes.c_void_p(t.data_ptr()), batch,
                                          h, w, s, s, None)
    assert rc == 0
    torch.cuda.synchronize()
    out = t.cpu().numpy()
    y = np.stack([out[b * s:b * s + n].reshape(h, w) for b in range(batch)])
    assert oracle.e_rel(y, oracle.forward(x), x).max() <= GATE["forward"]
    mask = np.ones(out.size, bool)
    for b in range(batch):
        mask[b * s:b * s + n] = False
    assert np.all(out[mask] == np.float32(-7.25))
