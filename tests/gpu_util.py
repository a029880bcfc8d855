"""Helpers for the GPU parity tests: run the HIP path through the C ABI and score it
against the FP64 oracle with the acceptance metric of Section 6 eq. 5."""
import numpy as np

import oracle

GATE = {"forward": 2e-6, "inverse": 2e-6, "roundtrip": 4e-6}


def to_gpu(x: np.ndarray):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def run(x: np.ndarray, direction: str, precision: str = "fp32", inplace: bool = True) -> np.ndarray:
    import torch
    import paper_2609_28519_amd as dct
    t = to_gpu(x)
    if inplace:
        dct.transform(t, t, direction, precision)
        out = t
    else:
        out = dct.transform(t, None, direction, precision)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def reference(x: np.ndarray, direction: str) -> np.ndarray:
    if direction == "forward":
        return oracle.forward(x)
    if direction == "inverse":
        return oracle.inverse(x)
    return x.astype(np.float64)  # the exact round trip is the input itself (Section 2.1)


def errors(x: np.ndarray, y: np.ndarray, direction: str) -> np.ndarray:
    return oracle.e_rel(y, reference(x, direction), x)


def assert_parity(x: np.ndarray, y: np.ndarray, direction: str, gate: float | None = None, label: str = ""):
    e = errors(x, y, direction)
    g = GATE[direction] if gate is None else gate
    worst = int(np.argmax(e))
    assert e.max() <= g, "%s %s: max e_rel %.3e at block %d (gate %.1e)" % (label, direction, e.max(), worst, g)
    return e
