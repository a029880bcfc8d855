"""Planted-mistake check of the oracle's pins (CPU only).

A copy of the oracle's C source is edited to carry one plausible mistake (a wrong
scale factor, a dropped half-sample shift, a transposed operand, a dropped term,
a wrong sign), built into a temporary library, and the pins of test_oracle.py
are re-run on it: every planted mistake must be caught by at least one of them.
The real oracle is never modified.
"""
import json
import os
import subprocess

import numpy as np
import pytest
import scipy.fft

import oracle
from tests.test_oracle_filter import neumann_laplacian, poisson_multipliers

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(os.path.dirname(HERE), "oracle", "dct_oracle.c")
GOLD = os.path.join(HERE, "golden", "closed_forms.json")

MUTATIONS = {
    "alpha0_wrong": ("sqrt(1.0 / (double)n)", "sqrt(2.0 / (double)n)"),
    "half_shift_dropped": ("(int64_t)(2 * j + 1) * k", "(int64_t)(2 * j) * k"),
    "second_product_transposed": ("s += qh[(int64_t)k * h + r] * t[(int64_t)r * w + l]",
                                  "s += qh[(int64_t)r * h + k] * t[(int64_t)r * w + l]"),
    "inverse_not_transposed": ("s += qh[(int64_t)k * h + r] * t[(int64_t)k * w + c]",
                               "s += qh[(int64_t)r * h + k] * t[(int64_t)k * w + c]"),
    "dropped_term": ("for (int32_t c = 0; c < w; ++c) s += x",
                     "for (int32_t c = 0; c < w - 1; ++c) s += x"),
    "wrong_quadrant_sign": ("sign = -1.0", "sign = 1.0"),
    "zero_not_exact": ("if (m == n) return 0.0;", "if (m == n) return 1e-9;"),
    "filter_multiplier_transposed": ("t2[i] *= lam[i];",
                                     "t2[i] *= lam[(i % job->cols) * job->rows + i / job->cols];"),
    "filter_multiplier_dropped": ("t2[i] *= lam[i];", "t2[i] *= 1.0;"),
    "filter_per_array_operator_ignored": ("job->lam + b * job->lam_stride", "job->lam"),
}


def _pins_pass(orc: oracle.Oracle) -> bool:
    """The pins of test_oracle.py, condensed; True only if all hold."""
    gold = json.load(open(GOLD))
    q8 = orc.qmatrix(8)
    for e in gold["q8_entries"]:
        if abs(q8[e["k"], e["j"]] - e["value"]) > 2e-16:
            return False
    for n in (12, 24):
        q = orc.qmatrix(n)
        for k in range(n):
            for j in range(n):
                if ((2 * j + 1) * k) % (2 * n) == n and q[k, j] != 0.0:
                    return False
    g = np.random.default_rng(0)
    for h, w in ((8, 8), (16, 32), (64, 64)):
        x = g.standard_normal((2, h, w)).astype(np.float32)
        xd = x.astype(np.float64)
        ys = scipy.fft.dctn(xd, type=2, norm="ortho", axes=(1, 2))
        if np.abs(orc.forward(x) - ys).max() > 1e-12 * np.abs(ys).max():
            return False
        xs = scipy.fft.idctn(xd, type=2, norm="ortho", axes=(1, 2))
        if np.abs(orc.inverse(x) - xs).max() > 1e-12 * np.abs(xs).max():
            return False
        if np.abs(orc.roundtrip(x) - xd).max() > 1e-13:
            return False
    # the spectral filter: Neumann Poisson solve (test_oracle_filter.py)
    for h, w in ((8, 32), (32, 8)):
        x = g.standard_normal((3, h, w)).astype(np.float32)
        xd = x.astype(np.float64)
        lam = poisson_multipliers(h, w)
        for op in (lam, np.broadcast_to(lam, (3, h, w)).copy()):
            u = orc.filter(x, op)
            r = neumann_laplacian(u) - (xd - xd.mean(axis=(1, 2), keepdims=True))
            if not np.all(np.isfinite(r)) or np.abs(r).max() > 1e-11 * np.abs(xd).max() * 64:
                return False
        # one constant operator per array: array b scaled by c[b]
        c = np.array([1.0, -2.0, 0.5])[:, None, None] * np.ones((3, h, w))
        if np.abs(orc.filter(x, c) - c * xd).max() > 1e-12 * np.abs(xd).max():
            return False
    return True


def test_real_oracle_passes_condensed_pins():
    assert _pins_pass(oracle.Oracle(oracle.build()))


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_mistake_is_caught(name, tmp_path):
    old, new = MUTATIONS[name]
    src = open(SRC).read()
    assert old in src, "mutation anchor not found: %s" % name
    mutated = tmp_path / ("oracle_%s.c" % name)
    mutated.write_text(src.replace(old, new))
    lib = tmp_path / ("liboracle_%s.so" % name)
    subprocess.run(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-pthread", str(mutated), "-o", str(lib),
                    "-lm"], check=True)
    assert not _pins_pass(oracle.Oracle(str(lib))), "pins missed planted mistake %s" % name
