"""Pins for the oracle's two error measures (CPU only).

``oracle.e_rel`` is the acceptance metric of Section 6 eq. 5: per array, the
Frobenius norm of the output error divided by the Frobenius norm of that
transform's own input.  ``oracle.weak_component_error`` is the relative error of
one spectral coefficient (Section 6: a strong constant can hide the loss of a weak
component that the norm criterion passes).

The expected values below are worked out by hand from those definitions on inputs
chosen so that a plausible slip (the output's norm as the denominator, one norm for
the whole batch, a dropped square root, the max-abs norm, a transposed coefficient
index, a missing absolute value) gives a different number.  The last test plants
each of those slips in a copy of the function and checks that a pin catches it.
"""
import inspect
import math

import numpy as np
import pytest

import oracle


def _two_array_case():
    """x: arrays of norm 16 and 1600; y: the references, norms 8 and 24 (different from x's);
    yhat: y with one entry off by 0.004 (array 0) and 0.04 (array 1)."""
    x = np.empty((2, 8, 8))
    x[0] = 2.0          # ||x0|| = sqrt(64 * 4) = 16
    x[1] = 200.0        # ||x1|| = 1600
    y = np.empty((2, 8, 8))
    y[0] = 1.0          # ||y0|| = 8
    y[1] = 3.0          # ||y1|| = 24
    yhat = y.copy()
    yhat[0, 1, 2] += 0.004
    yhat[1, 5, 6] += 0.04
    return yhat, y, x


def _e_rel_pins(e_rel) -> list[str]:
    """Names of the e_rel pins that fail for this implementation (empty: all hold)."""
    bad = []
    yhat, y, x = _two_array_case()
    e = np.asarray(e_rel(yhat, y, x))
    # per array, denominator ||x_b||: 0.004 / 16 and 0.04 / 1600
    if e.shape != (2,) or abs(e[0] - 2.5e-4) > 1e-15 or abs(e[1] - 2.5e-5) > 1e-16:
        bad.append("two_arrays")
    # uniform relative scaling: ||y (1 + d) - y|| / ||x|| = d ||y|| / ||x|| exactly
    g = np.random.default_rng(1)
    xs = g.standard_normal((3, 16, 8))
    ys = 0.5 * xs
    for d in (1e-5, 1e-8, 1e-12):
        es = np.asarray(e_rel(ys * (1 + d), ys, xs))
        if es.shape != (3,) or np.abs(es / (0.5 * d) - 1).max() > 1e-3:
            bad.append("scale_%g" % d)
    # an exact result scores 0
    if np.any(np.asarray(e_rel(ys, ys, xs)) != 0.0):
        bad.append("exact_is_zero")
    # a zero input falls back to the absolute error: 3-4-5 triangle in one array
    z = np.zeros((1, 4, 4))
    r = np.zeros((1, 4, 4))
    rh = r.copy()
    rh[0, 0, 0], rh[0, 3, 1] = 3e-9, -4e-9
    ez = np.asarray(e_rel(rh, r, z))
    if ez.shape != (1,) or abs(ez[0] - 5e-9) > 1e-22:
        bad.append("zero_input_absolute")
    # a single 2-D array is a batch of one
    e1 = np.asarray(e_rel(yhat[0], y[0], x[0]))
    if e1.shape != (1,) or abs(e1[0] - 2.5e-4) > 1e-15:
        bad.append("single_array")
    return bad


def _weak_pins(wce) -> list[str]:
    """Names of the weak_component_error pins that fail for this implementation."""
    bad = []
    k, l = 2, 5
    y = np.zeros((8, 8))
    y[k, l] = 1e-6
    y[l, k] = 5.0         # a strong coefficient at the transposed index
    yhat = y.copy()
    yhat[k, l] += 1e-8
    yhat[0, 0] += 1.0     # errors elsewhere do not count
    yhat[l, k] += 0.5
    if abs(wce(yhat, y, k, l) - 1e-2) > 1e-9:
        bad.append("relative")
    neg = -y
    negh = -yhat
    if abs(wce(negh, neg, k, l) - 1e-2) > 1e-9:
        bad.append("negative_reference")
    flip = y.copy()
    flip[k, l] = -1e-6    # the component's sign lost: error 2
    if abs(wce(flip, y, k, l) - 2.0) > 1e-12:
        bad.append("sign_flip")
    y0 = np.zeros((8, 8))
    h0 = y0.copy()
    h0[k, l] = -3e-9      # a zero reference falls back to the absolute error
    if abs(wce(h0, y0, k, l) - 3e-9) > 1e-24:
        bad.append("zero_reference")
    return bad


def test_e_rel_pins_hold():
    assert _e_rel_pins(oracle.e_rel) == []


def test_weak_component_error_pins_hold():
    assert _weak_pins(oracle.weak_component_error) == []


@pytest.mark.parametrize("h,w,k,l", [(8, 8, 3, 1), (16, 16, 0, 7), (32, 8, 5, 2)])
def test_weak_component_through_the_oracle(h, w, k, l):
    """X = c + eps * B_kl, with B_kl the unit-norm sampled cosine of frequency (k, l), has
    coefficient (k, l) = eps exactly (eq. 1-2: B_kl is the outer product of rows k and l of
    the orthonormal Q, and the constant contributes only to (0, 0)); an output with that
    coefficient off by delta scores delta / eps, whatever the strong constant does."""
    if (k, l) == (0, 0):
        pytest.skip("the weak component is not the DC term")
    eps, delta, c = 1e-6, 2e-9, 3.0
    i = np.arange(h)[:, None]
    j = np.arange(w)[None, :]
    b = np.cos(np.pi * (2 * i + 1) * k / (2 * h)) * np.cos(np.pi * (2 * j + 1) * l / (2 * w))
    b /= np.sqrt((b * b).sum())
    x = c + eps * b
    y = oracle.forward(x)  # double input: no float32 rounding of the weak component
    assert y[k, l] == pytest.approx(eps, rel=1e-8)
    yhat = y.copy()
    yhat[k, l] += delta
    yhat[0, 0] *= 1 + 1e-7  # the strong DC term's error is irrelevant to this measure
    assert oracle.weak_component_error(yhat, y, k, l) == pytest.approx(delta / eps, rel=1e-6)
    # while the norm criterion of eq. 5 barely notices the component's 0.2 % error
    assert oracle.e_rel(yhat, y, x)[0] < 1e-6


# Plausible slips, each planted in a copy of the function's source.
E_REL_MUTATIONS = {
    "denominator_is_reference_norm": ("den = np.sqrt(np.sum(x * x, axis=(1, 2)))",
                                      "den = np.sqrt(np.sum(y * y, axis=(1, 2)))"),
    "denominator_is_output_norm": ("den = np.sqrt(np.sum(x * x, axis=(1, 2)))",
                                   "den = np.sqrt(np.sum(yhat * yhat, axis=(1, 2)))"),
    "batch_wide_denominator": ("den = np.sqrt(np.sum(x * x, axis=(1, 2)))",
                               "den = np.full(x.shape[0], np.sqrt(np.sum(x * x)))"),
    "batch_wide_numerator": ("num = np.sqrt(np.sum((yhat - y) ** 2, axis=(1, 2)))",
                             "num = np.full(y.shape[0], np.sqrt(np.sum((yhat - y) ** 2)))"),
    "squared_norms": ("num = np.sqrt(np.sum((yhat - y) ** 2, axis=(1, 2)))",
                      "num = np.sum((yhat - y) ** 2, axis=(1, 2))"),
    "max_abs_norm": ("num = np.sqrt(np.sum((yhat - y) ** 2, axis=(1, 2)))",
                     "num = np.abs(yhat - y).max(axis=(1, 2))"),
    "zero_input_scored_relative": ("out = np.where(den > 0, num / np.where(den > 0, den, 1.0), num)",
                                   "out = np.where(den > 0, num / np.where(den > 0, den, 1.0), 0.0)"),
}
WEAK_MUTATIONS = {
    "transposed_index": ("ref = float(y[k, l])", "ref = float(y[l, k])"),
    "relative_to_output": ("/ abs(ref)", "/ abs(float(yhat[k, l]))"),
    "no_absolute_value": ("abs(float(yhat[k, l]) - ref) / abs(ref)", "(float(yhat[k, l]) - ref) / ref"),
}


def _mutant(fn, old, new):
    src = inspect.getsource(fn)
    assert old in src, "mutation anchor not found: %r" % old
    ns = {"np": np, "math": math}
    exec(compile(src.replace(old, new), "<mutant>", "exec"), ns)
    return ns[fn.__name__]


@pytest.mark.parametrize("name", sorted(E_REL_MUTATIONS))
def test_planted_e_rel_mistake_is_caught(name):
    old, new = E_REL_MUTATIONS[name]
    assert _e_rel_pins(_mutant(oracle.e_rel, old, new)), "pins missed %s" % name


@pytest.mark.parametrize("name", sorted(WEAK_MUTATIONS))
def test_planted_weak_component_mistake_is_caught(name):
    old, new = WEAK_MUTATIONS[name]
    assert _weak_pins(_mutant(oracle.weak_component_error, old, new)), "pins missed %s" % name
