"""Section 6 on the HIP path: fault injection on real GPU outputs, and boundary diagnostics.

Fault injection (Section 6, fault-injection protocol): correct outputs of the HIP
kernels are perturbed on the host by the faults an implementation can plausibly
have: a uniform scale error of 1e-5, one coefficient with its sign flipped, the
output transposed (orientation), the other direction's transform in place of this
one (swapped direction), and one lost component.  For every size and direction the
eq. 5 criterion with its gate must flag every fault on at least one input, and pass
the unperturbed output.

Boundary diagnostics (Section 6: subnormal inputs, extreme finite amplitudes, and
non-finite values) are reported, not gated, as the paper does: the printed table is
the report.  What the test does assert is isolation: a non-finite or overflowing
array never changes its neighbours in the batch, and a NaN input yields a NaN output.
"""
import numpy as np
import pytest

import oracle
from tests.gpu_util import GATE, run

pytestmark = pytest.mark.gpu
SIZES = (8, 16, 32, 64, 128, 256)
DIRS = ("forward", "inverse", "roundtrip")


def _lib():
    import paper_2609_28519_amd as dct
    dct.init(0)
    return dct


def _reference(x, d):
    if d == "forward":
        return oracle.forward(x)
    if d == "inverse":
        return oracle.inverse(x)
    return x.astype(np.float64)


def _other(x, d):
    """The wrong direction's exact result: the swapped-direction fault."""
    if d == "forward":
        return oracle.inverse(x)
    if d == "inverse":
        return oracle.forward(x)
    return oracle.forward(x)  # a round trip that skipped its inverse half


@pytest.mark.parametrize("n", SIZES)
@pytest.mark.parametrize("direction", DIRS)
def test_injected_faults_on_gpu_outputs_are_detected(n, direction):
    _lib()
    g = np.random.default_rng(1000 + n)
    x = g.standard_normal((3, n, n)).astype(np.float32)
    y = run(x, direction).astype(np.float64)
    ref = _reference(x, direction)
    e0 = oracle.e_rel(y, ref, x)
    assert e0.max() <= GATE[direction], "unperturbed output fails: %.3e" % e0.max()
    big = np.unravel_index(np.argmax(np.abs(y[0])), y[0].shape)
    faults = {}
    faults["scale"] = y * (1 + 1e-5)
    sgn = y.copy()
    sgn[0][big] = -sgn[0][big]
    faults["sign"] = sgn
    faults["orientation"] = np.ascontiguousarray(np.swapaxes(y, 1, 2))
    faults["swapped_direction"] = _other(x, direction)
    lost = y.copy()
    lost[0][big] = 0.0
    faults["component_loss"] = lost
    report = {}
    for name, yf in faults.items():
        e = oracle.e_rel(yf, ref, x)
        report[name] = float(e.max())
        assert e.max() > GATE[direction], "N=%d %s: %s fault not detected (e_rel %.3e)" % (
            n, direction, name, e.max())
    print("faults N=%d %-9s" % (n, direction), " ".join("%s=%.2e" % kv for kv in report.items()))


def _rel(y, ref, x):
    with np.errstate(all="ignore"):
        return float(oracle.e_rel(y, ref, x).max())


@pytest.mark.parametrize("n", SIZES)
def test_boundary_diagnostics_reported(n):
    """The boundary set of workloads.boundary_set (normal, subnormal, amplitude FLT_MAX / n with a
    representable exact result, a 3e38 impulse, one NaN, one +Inf), followed by a normal array.
    Errors and non-finite fractions are printed, not gated; the normal arrays on either side must
    stay within the gate whatever their neighbours hold, and the NaN array's output must hold a
    NaN."""
    import workloads
    _lib()
    bs = workloads.boundary_set(n)
    extra = np.random.default_rng(n).uniform(-1, 1, (1, n, n)).astype(np.float32)
    x = np.concatenate([bs.x, extra])
    names = workloads.BOUNDARY_CASES + ("normal_after",)
    finite = [i for i in range(len(names)) if np.isfinite(x[i]).all()]
    rows = []
    for d in DIRS:
        y = run(x, d)
        ref = dict(zip(finite, _reference(x[finite], d)))
        for b in (0, len(names) - 1):
            e = oracle.e_rel(y[b], ref[b], x[b])[0]
            assert e <= GATE[d], "N=%d %s: normal array %d disturbed (%.3e)" % (n, d, b, e)
        assert np.isnan(y[names.index("nan")]).any(), "N=%d %s: NaN input did not propagate" % (n, d)
        cells = []
        for i, name in enumerate(names[1:-1], start=1):
            fin = float(np.isfinite(y[i]).mean())
            e = _rel(y[i], ref[i], x[i]) if i in ref and fin == 1.0 else float("nan")
            cells.append("%s: finite %.3f e_rel %s" % (name, fin, "%.2e" % e if e == e else "n/a"))
        rows.append("boundary N=%d %s | %s" % (n, d, " | ".join(cells)))
    print("\n" + "\n".join(rows))
