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


def spread(batch: int, k: int, seed: int = 0) -> np.ndarray:
    """About k distinct array indices spread over the whole batch: one random index in each of k
    equal segments, plus the first and the last array.  Every pass of a grid-stride or persistent
    schedule (a contiguous run of grid-size arrays) is hit once k exceeds batch / grid."""
    g = np.random.default_rng(seed)
    k = max(1, min(k, batch))
    edges = np.linspace(0, batch, k + 1).astype(np.int64)
    idx = [int(g.integers(lo, hi)) for lo, hi in zip(edges[:-1], edges[1:]) if hi > lo]
    return np.unique(np.array(idx + [0, batch - 1], dtype=np.int64))


def per_array_rel(a, b):
    """||a_i - b_i|| / ||b_i|| for every array i of two (batch, rows, cols) CUDA tensors, in
    float64 on the GPU (a closed-form reference such as the round trip's input needs no oracle)."""
    import torch
    d = (a.double() - b.double()).reshape(a.shape[0], -1)
    n = b.double().reshape(b.shape[0], -1)
    return (torch.linalg.vector_norm(d, dim=1) / torch.linalg.vector_norm(n, dim=1)).cpu().numpy()


def parseval_rel(y, x):
    """| ||y_i|| - ||x_i|| | / ||x_i|| per array (the orthonormal transforms preserve the norm)."""
    import torch
    ny = torch.linalg.vector_norm(y.double().reshape(y.shape[0], -1), dim=1)
    nx = torch.linalg.vector_norm(x.double().reshape(x.shape[0], -1), dim=1)
    return ((ny - nx).abs() / nx).cpu().numpy()
