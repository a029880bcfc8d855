"""Seeded synthetic inputs for the batched 2D DCT (shared by tests, oracle runs and bench).

This module only draws random numbers and lays them out; it holds none of the
transform's arithmetic.  The one signal it synthesises beyond noise is a
sampled separable cosine ("single cosine basis component" of the mixtures),
built here from numpy's cos and normalised to unit Frobenius norm by its own
measured norm, so it never relies on the transform's scale factors.

Every generator draws in float64 from numpy's PCG64 and rounds to float32 with
round-to-nearest-even, as one stream per call, so the same seed always gives
the same arrays.

The paper verifies on a 474-array dataset that is not available here
(Section 6).  These synthetic families stand in for it: uniform and normal
noise, smooth ramps with weak components, constants with weak perturbations,
and extreme power-of-two amplitudes (the categories listed in Section 6).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

SIZES = (8, 16, 32, 64, 128, 256)
SEED_BASE = 260928519
SEEDS = {"c1": SEED_BASE + 1, "c2": SEED_BASE + 2, "c3": SEED_BASE + 3,
         "c4": SEED_BASE + 4, "c5": SEED_BASE + 5, "tune": SEED_BASE + 99}

# category codes used in metadata
CAT_UNIFORM, CAT_NORMAL, CAT_RAMP_WEAK, CAT_EXTREME, CAT_WEAK_CONST, CAT_SCALED = 0, 1, 2, 3, 4, 5


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def cosine_image(h: int, w: int, k: int, l: int) -> np.ndarray:
    """Sampled separable cosine cos(pi(2i+1)k/(2h)) cos(pi(2j+1)l/(2w)), unit Frobenius norm."""
    i = np.arange(h, dtype=np.float64)
    j = np.arange(w, dtype=np.float64)
    img = np.outer(np.cos(np.pi * (2 * i + 1) * k / (2 * h)), np.cos(np.pi * (2 * j + 1) * l / (2 * w)))
    return img / np.sqrt(np.sum(img * img))


@dataclass
class Batch:
    """A packed batch of equal-shape arrays plus per-array metadata."""
    x: np.ndarray                      # (batch, rows, cols) float32
    category: np.ndarray | None = None  # int8 per array
    weak_kl: np.ndarray | None = None   # (batch, 2) int32, -1 where not applicable
    meta: dict = field(default_factory=dict)


def c1_uniform8(batch: int = 4096, seed: int = SEEDS["c1"]) -> Batch:
    """4096 row-major 8x8 blocks, i.i.d. U[-1,1]."""
    g = rng(seed)
    x = g.uniform(-1.0, 1.0, size=(batch, 8, 8)).astype(np.float32)
    return Batch(x, np.full(batch, CAT_UNIFORM, np.int8))


def c2_mixture16(batch: int = 65536, seed: int = SEEDS["c2"], n: int = 16) -> Batch:
    """16x16 tiles: 40% U[-1,1], 30% N(0,1), 20% ramp + 1e-6 cosine component, 10% U[-1,1]*2^(+-100).

    Ramp tiles: a + g_r*r/(n-1) + g_c*c/(n-1), a, g_r, g_c ~ U[-1/2, 1/2], plus 1e-6 times a unit-norm
    sampled cosine of random frequency (k,l) != (0,0).
    """
    g = rng(seed)
    cat = g.choice(np.array([CAT_UNIFORM, CAT_NORMAL, CAT_RAMP_WEAK, CAT_EXTREME], np.int8),
                   size=batch, p=[0.4, 0.3, 0.2, 0.1])
    x = np.empty((batch, n, n), dtype=np.float64)
    weak = np.full((batch, 2), -1, np.int32)
    iu = np.flatnonzero(cat == CAT_UNIFORM)
    x[iu] = g.uniform(-1.0, 1.0, size=(iu.size, n, n))
    inn = np.flatnonzero(cat == CAT_NORMAL)
    x[inn] = g.standard_normal(size=(inn.size, n, n))
    ir = np.flatnonzero(cat == CAT_RAMP_WEAK)
    coef = g.uniform(-0.5, 0.5, size=(ir.size, 3))
    r = np.arange(n, dtype=np.float64)[:, None] / (n - 1)
    c = np.arange(n, dtype=np.float64)[None, :] / (n - 1)
    kl = g.integers(0, n, size=(ir.size, 2))
    zero = (kl[:, 0] == 0) & (kl[:, 1] == 0)
    kl[zero, 1] = g.integers(1, n, size=int(zero.sum()))
    for t, idx in enumerate(ir):
        x[idx] = coef[t, 0] + coef[t, 1] * r + coef[t, 2] * c + 1e-6 * cosine_image(n, n, kl[t, 0], kl[t, 1])
    weak[ir] = kl
    ie = np.flatnonzero(cat == CAT_EXTREME)
    sgn = np.where(g.uniform(size=ie.size) < 0.5, -100.0, 100.0)
    x[ie] = g.uniform(-1.0, 1.0, size=(ie.size, n, n)) * np.exp2(sgn)[:, None, None]
    return Batch(x.astype(np.float32), cat, weak)


def c3_normal(n: int, batch: int | None = None, seed: int | None = None) -> Batch:
    """N x N blocks, i.i.d. N(0,1); default batch 2^27/N^2 (512 MiB of float32)."""
    if batch is None:
        batch = (1 << 27) // (n * n)
    g = rng(SEEDS["c3"] + n if seed is None else seed)
    out = np.empty((batch, n, n), dtype=np.float32)
    chunk = max(1, (1 << 22) // (n * n))
    for s in range(0, batch, chunk):
        e = min(batch, s + chunk)
        out[s:e] = g.standard_normal(size=(e - s, n, n))
    return Batch(out, np.full(batch, CAT_NORMAL, np.int8))


C4_MIX = {8: 0.40, 16: 0.30, 32: 0.15, 64: 0.10, 128: 0.04, 256: 0.01}
C4_IMAGES = ((1024, 1024),) * 4 + ((512, 384),) * 4


@dataclass
class Ragged:
    """A ragged batch packed in one float32 buffer.

    offsets[i] is the element offset of item i in `data`; rows/cols its shape
    (row-major, pitch = cols).  `scaled` flags the items multiplied by 1e30.
    """
    data: np.ndarray
    offsets: np.ndarray
    rows: np.ndarray
    cols: np.ndarray
    scaled: np.ndarray

    @property
    def count(self) -> int:
        return int(self.offsets.size)

    def item(self, i: int, buf: np.ndarray | None = None) -> np.ndarray:
        b = self.data if buf is None else buf
        o, h, w = int(self.offsets[i]), int(self.rows[i]), int(self.cols[i])
        return b[o:o + h * w].reshape(h, w)


def c4_ragged(blocks: int = 200_000, images=C4_IMAGES, seed: int = SEEDS["c4"],
              p_scaled: float = 0.05, mix=None) -> Ragged:
    """Ragged batch: square blocks with sizes drawn from the mix, in random order, then the images.

    Values U[-1,1]; each item (block or image) is multiplied by 1e30 with probability p_scaled.
    """
    mix = C4_MIX if mix is None else mix
    g = rng(seed)
    sizes = np.array(sorted(mix), np.int32)
    probs = np.array([mix[s] for s in sorted(mix)], np.float64)
    probs = probs / probs.sum()
    n = g.choice(sizes, size=blocks, p=probs).astype(np.int32)
    rows = np.concatenate([n, np.array([h for h, _ in images], np.int32)])
    cols = np.concatenate([n, np.array([w for _, w in images], np.int32)])
    count = rows.size
    elems = rows.astype(np.int64) * cols
    offsets = np.zeros(count, np.int64)
    offsets[1:] = np.cumsum(elems)[:-1]
    total = int(elems.sum())
    data = np.empty(total, np.float32)
    chunk = 1 << 24
    for s in range(0, total, chunk):
        e = min(total, s + chunk)
        data[s:e] = g.uniform(-1.0, 1.0, size=e - s)
    scaled = g.uniform(size=count) < p_scaled
    for i in np.flatnonzero(scaled):
        o = offsets[i]
        data[o:o + elems[i]] *= np.float32(1e30)
    return Ragged(data, offsets, rows, cols, scaled)


def c5_ladder(n: int, batch: int = 1 << 18, seed: int | None = None) -> Batch:
    """Precision-ladder blocks: 80% N(0,1); 10% N(0,1)*2^(+-60); 10% A*1 + 1e-7*|A|*n*cosine(k,l).

    The weak blocks are a constant A ~ N(0,1) plus a unit-norm sampled cosine of amplitude
    1e-7*|A|*n, i.e. 1e-7 relative to the constant's Frobenius norm |A|*n.
    """
    g = rng(SEEDS["c5"] + n if seed is None else seed)
    cat = g.choice(np.array([CAT_NORMAL, CAT_SCALED, CAT_WEAK_CONST], np.int8), size=batch,
                   p=[0.8, 0.1, 0.1])
    out = np.empty((batch, n, n), dtype=np.float32)
    weak = np.full((batch, 2), -1, np.int32)
    chunk = max(1, (1 << 22) // (n * n))
    for s in range(0, batch, chunk):
        e = min(batch, s + chunk)
        out[s:e] = g.standard_normal(size=(e - s, n, n))
    isc = np.flatnonzero(cat == CAT_SCALED)
    ex = np.where(g.uniform(size=isc.size) < 0.5, -60.0, 60.0)
    out[isc] = (out[isc].astype(np.float64) * np.exp2(ex)[:, None, None]).astype(np.float32)
    iw = np.flatnonzero(cat == CAT_WEAK_CONST)
    a = g.standard_normal(size=iw.size)
    kl = g.integers(0, n, size=(iw.size, 2))
    zero = (kl[:, 0] == 0) & (kl[:, 1] == 0)
    kl[zero, 0] = g.integers(1, n, size=int(zero.sum()))
    for t, idx in enumerate(iw):
        blk = a[t] + 1e-7 * abs(a[t]) * n * cosine_image(n, n, kl[t, 0], kl[t, 1])
        out[idx] = blk.astype(np.float32)
    weak[iw] = kl
    return Batch(out, cat, weak)


BOUNDARY_CASES = ("normal", "subnormal", "large", "impulse_3e38", "nan", "inf")


def boundary_set(n: int, seed: int = SEED_BASE + 6) -> Batch:
    """Boundary diagnostics (Section 6: subnormals, extreme finite amplitudes), one n x n array per
    case, in the order of BOUNDARY_CASES: U[-1,1]; U[-1,1] * 1e-40 (subnormal float32); U[-1,1] *
    FLT_MAX / n, whose exact orthonormal transform is still representable (its Frobenius norm is at
    most FLT_MAX / sqrt(3)) while unnormalised intermediate sums need not be; a single impulse of
    3e38; U[-1,1] with one NaN; U[-1,1] with one +Inf."""
    g = rng(seed + n)
    x = g.uniform(-1.0, 1.0, size=(len(BOUNDARY_CASES), n, n))
    x[1] *= 1e-40
    x[2] *= float(np.finfo(np.float32).max) / n
    x[3] = 0.0
    x[3, n // 3, n // 5] = 3e38
    x[4, n // 3, n // 5] = np.nan
    x[5, n // 2, 1] = np.inf
    return Batch(x.astype(np.float32), np.arange(len(BOUNDARY_CASES), dtype=np.int8))
