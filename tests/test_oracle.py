"""Pins for the FP64 oracle: it is checked against things other than itself.

Each test cites what fixes the expected value: the paper's definitions
(Section 2.1 eq. 1-2, Section 7.1 rectangles), closed forms that follow from
them, orthonormality invariants, an explicit O(N^4) brute force, and SciPy's
independent orthonormal DCT (one of the systems the paper compares against,
Section 4.2 Table 1) used as a black box.
"""
import json
import math
import os

import numpy as np
import pytest
import scipy.fft

import oracle
import workloads

GOLD = os.path.join(os.path.dirname(__file__), "golden", "closed_forms.json")
SIZES = (8, 16, 32, 64, 128, 256)


def _rng(s=1):
    return np.random.default_rng(s)


def test_q_matrix_matches_golden_entries():
    """Section 2.1 eq. 1: hand-evaluated entries of Q_8 and Q_16."""
    gold = json.load(open(GOLD))
    q8 = oracle.qmatrix(8)
    for e in gold["q8_entries"]:
        assert q8[e["k"], e["j"]] == pytest.approx(e["value"], abs=2e-16), e["why"]
    q16 = oracle.qmatrix(16)
    for e in gold["q16_entries"]:
        assert q16[e["k"], e["j"]] == pytest.approx(e["value"], abs=2e-16), e["why"]


@pytest.mark.parametrize("n", SIZES + (384, 512, 1024, 26, 12))
def test_q_is_orthogonal(n):
    """eq. 1 defines an orthonormal matrix: Q Q^T = I (Section 2.1)."""
    q = oracle.qmatrix(n)
    assert np.abs(q @ q.T - np.eye(n)).max() < 1e-13


@pytest.mark.parametrize("n", (8, 16, 64, 256, 12, 384))
def test_q_exact_zeros_and_symmetry(n):
    """eq. 1: cos(pi/2)=0 exactly at (2j+1)k = n mod 2n; Q[k][n-1-j] = (-1)^k Q[k][j].

    Power-of-two n has no such zeros; n = 12 and 384 (the image axis) do.
    """
    q = oracle.qmatrix(n)
    zeros = 0
    for k in range(n):
        for j in range(n):
            if ((2 * j + 1) * k) % (2 * n) == n:
                assert q[k, j] == 0.0
                zeros += 1
            assert q[k, n - 1 - j] == (-1) ** k * q[k, j]
    assert (zeros > 0) == (n & (n - 1) != 0)


def test_impulse_and_constant_closed_forms():
    """eq. 2 closed forms: DC of a unit impulse is 1/sqrt(hw); a constant c maps to c*sqrt(hw) e00."""
    gold = json.load(open(GOLD))
    for e in gold["impulse_dc"]:
        x = np.zeros((e["rows"], e["cols"]))
        x[3, 5] = 1.0
        assert oracle.forward(x)[0, 0] == pytest.approx(e["value"], rel=1e-15), e["why"]
    for e in gold["constant_dc"]:
        x = np.full((e["rows"], e["cols"]), e["c"])
        y = oracle.forward(x)
        assert y[0, 0] == pytest.approx(e["value"], rel=1e-14), e["why"]
        y[0, 0] = 0.0
        assert np.abs(y).max() < 1e-14 * abs(e["value"])


@pytest.mark.parametrize("n", SIZES)
def test_constant_gives_dc_only(n):
    """A constant block has only a DC coefficient, c*n (eq. 2 with Q 1 = sqrt(n) e_0)."""
    x = np.full((n, n), np.float32(0.75), dtype=np.float32)
    y = oracle.forward(x)
    assert y[0, 0] == pytest.approx(0.75 * n, rel=1e-14)
    y[0, 0] = 0
    assert np.abs(y).max() < 1e-13


@pytest.mark.parametrize("h,w", [(8, 8), (16, 16), (32, 8), (64, 64), (16, 128), (256, 256)])
def test_single_cosine_gives_one_coefficient(h, w):
    """A unit-norm sampled cosine of frequency (k,l) maps to exactly one unit coefficient.

    The cosine is built by the input generator from numpy's cos and normalised by its own
    norm; discrete orthogonality of the cosines (a textbook fact behind eq. 1) fixes the
    result as e_k e_l^T.
    """
    g = _rng(h * 7 + w)
    for _ in range(4):
        k, l = int(g.integers(0, h)), int(g.integers(0, w))
        x = workloads.cosine_image(h, w, k, l)
        y = oracle.forward(x)
        assert y[k, l] == pytest.approx(1.0, abs=1e-13)
        y[k, l] = 0
        assert np.abs(y).max() < 1e-13


@pytest.mark.parametrize("h,w", [(8, 8), (16, 16), (8, 64), (64, 8), (128, 128)])
def test_cosine_along_rows_closed_form(h, w):
    """X_ij = cos(pi(2i+1)k/(2h)) (constant along j): Y_k0 = sqrt(h/2) sqrt(w), all else 0."""
    k = h // 2 - 1
    i = np.arange(h)
    x = np.repeat(np.cos(np.pi * (2 * i + 1) * k / (2 * h))[:, None], w, axis=1)
    y = oracle.forward(x)
    assert y[k, 0] == pytest.approx(math.sqrt(h / 2) * math.sqrt(w), rel=1e-13)
    y[k, 0] = 0
    assert np.abs(y).max() < 1e-12


@pytest.mark.parametrize("n", SIZES)
def test_parseval(n):
    """Orthonormal scaling preserves the Frobenius norm (Section 2.1; Section 6 after eq. 5)."""
    x = _rng(n).standard_normal((4, n, n)).astype(np.float32)
    y = oracle.forward(x)
    assert np.allclose(np.linalg.norm(y, axis=(1, 2)), np.linalg.norm(x.astype(np.float64), axis=(1, 2)),
                       rtol=1e-13, atol=0)


@pytest.mark.parametrize("h,w", [(8, 8), (32, 32), (256, 256), (8, 64), (64, 16)])
def test_roundtrip_is_identity(h, w):
    """The exact round trip C^-1(C(X)) is X (Section 2.1)."""
    x = _rng(h + w).uniform(-1, 1, (3, h, w)).astype(np.float32)
    assert np.abs(oracle.roundtrip(x) - x).max() < 1e-13


@pytest.mark.parametrize("h,w", [(8, 8), (16, 32), (128, 128)])
def test_inverse_is_adjoint(h, w):
    """<C(X), Y> = <X, C^-1(Y)>: the inverse is the Frobenius adjoint (Section 2.1, Prop. 2)."""
    g = _rng(3)
    x = g.standard_normal((h, w))
    yy = g.standard_normal((h, w))
    lhs = np.sum(oracle.forward(x) * yy)
    rhs = np.sum(x * oracle.inverse(yy))
    assert lhs == pytest.approx(rhs, rel=1e-12, abs=1e-12)


def _brute_forward(x):
    """O(h^2 w^2) quadruple sum of eq. 1-2 with math.cos, written independently of the oracle."""
    h, w = x.shape
    y = np.zeros((h, w))
    for k in range(h):
        ak = math.sqrt((1.0 if k == 0 else 2.0) / h)
        for l in range(w):
            al = math.sqrt((1.0 if l == 0 else 2.0) / w)
            s = 0.0
            for i in range(h):
                ci = math.cos(math.pi * (i + 0.5) * k / h)
                for j in range(w):
                    s += x[i, j] * ci * math.cos(math.pi * (j + 0.5) * l / w)
            y[k, l] = ak * al * s
    return y


def _brute_inverse(y):
    h, w = y.shape
    x = np.zeros((h, w))
    for i in range(h):
        for j in range(w):
            s = 0.0
            for k in range(h):
                ak = math.sqrt((1.0 if k == 0 else 2.0) / h)
                ck = math.cos(math.pi * (i + 0.5) * k / h)
                for l in range(w):
                    al = math.sqrt((1.0 if l == 0 else 2.0) / w)
                    s += y[k, l] * ak * al * ck * math.cos(math.pi * (j + 0.5) * l / w)
            x[i, j] = s
    return x


@pytest.mark.parametrize("h,w", [(8, 8), (8, 16)])
def test_bruteforce_n8(h, w):
    """Explicit O(N^4) evaluation of eq. 2 agrees with the separable oracle."""
    x = _rng(11).uniform(-1, 1, (h, w)).astype(np.float32)
    assert np.abs(oracle.forward(x) - _brute_forward(x.astype(np.float64))).max() < 1e-14
    assert np.abs(oracle.inverse(x) - _brute_inverse(x.astype(np.float64))).max() < 1e-14


@pytest.mark.parametrize("h,w", [(n, n) for n in SIZES] + [(512, 384), (384, 512), (16, 32), (8, 64), (64, 8),
                                                            (1024, 1024), (32, 26)])
def test_matches_scipy_orthonormal_dct(h, w):
    """SciPy's dctn/idctn(type 2, norm='ortho') is an independent implementation of eq. 2."""
    b = 2 if h * w <= 65536 else 1
    x = _rng(h * w).standard_normal((b, h, w)).astype(np.float32)
    xd = x.astype(np.float64)
    y = oracle.forward(x)
    ys = scipy.fft.dctn(xd, type=2, norm="ortho", axes=(1, 2))
    assert np.abs(y - ys).max() < 1e-12 * max(1.0, np.abs(ys).max())
    xi = oracle.inverse(x)
    xs = scipy.fft.idctn(xd, type=2, norm="ortho", axes=(1, 2))
    assert np.abs(xi - xs).max() < 1e-12 * max(1.0, np.abs(xs).max())


def test_threads_do_not_change_result():
    x = _rng(5).standard_normal((37, 32, 32)).astype(np.float32)
    a = oracle.forward(x, threads=1)
    b = oracle.forward(x, threads=8)
    assert np.array_equal(a, b)


def test_zero_block_and_metric():
    """Zero input gives exactly zero; eq. 5 falls back to an absolute check on zero inputs."""
    x = np.zeros((2, 16, 16), np.float32)
    y = oracle.forward(x)
    assert np.all(y == 0)
    e = oracle.e_rel(y + 1e-9, y, x)
    assert np.allclose(e, 1e-9 * 16)


def test_extreme_amplitudes_exact_scaling():
    """Power-of-two scaling commutes with the linear map exactly in double (2^+-100, 1e30 inputs)."""
    x = _rng(9).uniform(-1, 1, (16, 16)).astype(np.float32)
    y = oracle.forward(x)
    for p in (-100, 100, 60, -60):
        xs = (x.astype(np.float64) * 2.0 ** p).astype(np.float32)
        assert np.array_equal(oracle.forward(xs), y * 2.0 ** p)


@pytest.mark.parametrize("n", (8, 16, 32, 64, 128, 256))
def test_fault_injection_is_detected(n):
    """Section 6: injected scaling, sign, orientation and component-loss faults exceed the gate.

    Faults are applied to correct oracle outputs; the criterion of eq. 5 with the 2e-6
    gate must flag every one of them on at least one input (here: on this input).
    """
    x = _rng(n).standard_normal((n, n)).astype(np.float32)
    y = oracle.forward(x)
    faults = {
        "scale": y * (1 + 1e-5),
        "sign": y * np.where(np.arange(n * n).reshape(n, n) == 1, -1, 1),
        "orientation": y.T.copy(),
        "component_loss": np.where(np.arange(n * n).reshape(n, n) == n + 1, 0.0, y),
    }
    for name, yf in faults.items():
        assert oracle.e_rel(yf, y, x)[0] > 2e-6, name
    assert oracle.e_rel(y, y, x)[0] == 0.0
