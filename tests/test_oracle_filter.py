"""Pins of the oracle's spectral filter (CPU only).

The filter is the transform-operator-inverse composition of Prop. 1 / eq. 4 in the
orthonormal form: X' = Q_h^T (L o (Q_h X Q_w^T)) Q_w, with L an array of multipliers
on the 2D coefficients.  Each pin below fixes it by something other than the oracle
itself:

* L = 1 gives X (orthonormality, Section 2.1); L = c gives c X.
* L = indicator of (0, 0) gives the array mean everywhere (Q_n's row 0 is constant).
* L = indicator of (k, l) gives the projection onto the separable basis image built
  from scipy's orthonormal inverse DCT of unit vectors (a library routine).
* The Neumann Poisson solve: the DCT-II basis vectors are the eigenvectors of the
  second difference with mirrored (half-sample) boundaries, eigenvalue 2 cos(pi k / n) - 2.
  With L = 1 / (2 cos(pi k / h) + 2 cos(pi l / w) - 4) and L[0][0] = 0 the filter solves
  the 5-point Laplace equation, checked with a plain stencil: Lap(X') = X - mean(X) and
  mean(X') = 0.  A transposed multiplier index on a rectangle fails it.
"""
import numpy as np
import pytest
import scipy.fft

import oracle


def _x(seed, shape):
    return np.random.default_rng(seed).standard_normal(shape).astype(np.float32)


def neumann_laplacian(u):
    """5-point Laplacian with mirrored boundaries (ghost cell = edge cell)."""
    p = np.pad(u, ((0, 0), (1, 1), (1, 1)), mode="edge")
    return p[:, :-2, 1:-1] + p[:, 2:, 1:-1] + p[:, 1:-1, :-2] + p[:, 1:-1, 2:] - 4.0 * u


def poisson_multipliers(h, w):
    k = np.arange(h)[:, None]
    l = np.arange(w)[None, :]
    mu = 2.0 * np.cos(np.pi * k / h) + 2.0 * np.cos(np.pi * l / w) - 4.0
    lam = np.zeros((h, w))
    lam[mu != 0] = 1.0 / mu[mu != 0]
    return lam


@pytest.mark.parametrize("h,w", [(8, 8), (8, 16), (32, 16), (64, 64)])
def test_identity_and_constant_operators(h, w):
    x = _x(1, (3, h, w))
    xd = x.astype(np.float64)
    assert np.abs(oracle.filter(x, np.ones((h, w))) - xd).max() <= 1e-13 * max(1.0, np.abs(xd).max())
    c = np.array([2.5, -0.75, 0.0])[:, None, None] * np.ones((3, h, w))
    got = oracle.filter(x, c)
    assert np.abs(got - c * xd).max() <= 1e-13 * max(1.0, np.abs(xd).max()) * 2.5
    assert np.all(got[2] == 0.0)


@pytest.mark.parametrize("h,w", [(8, 8), (16, 8), (64, 32)])
def test_dc_operator_gives_mean(h, w):
    x = _x(2, (2, h, w))
    lam = np.zeros((h, w))
    lam[0, 0] = 1.0
    got = oracle.filter(x, lam)
    mean = x.astype(np.float64).mean(axis=(1, 2))
    assert np.abs(got - mean[:, None, None]).max() <= 1e-14 * np.abs(x).max() * 10


@pytest.mark.parametrize("h,w,k,l", [(8, 8, 3, 5), (16, 32, 7, 30), (32, 8, 31, 1)])
def test_single_coefficient_is_a_projection(h, w, k, l):
    x = _x(3, (2, h, w)).astype(np.float32)
    lam = np.zeros((h, w))
    lam[k, l] = 1.0
    got = oracle.filter(x, lam)
    ek = np.zeros(h); ek[k] = 1.0
    el = np.zeros(w); el[l] = 1.0
    basis = np.outer(scipy.fft.idct(ek, type=2, norm="ortho"), scipy.fft.idct(el, type=2, norm="ortho"))
    coef = np.einsum("brc,rc->b", x.astype(np.float64), basis)
    want = coef[:, None, None] * basis[None]
    assert np.abs(got - want).max() <= 1e-13 * max(1.0, np.abs(x).max())


@pytest.mark.parametrize("h,w", [(8, 8), (8, 32), (32, 8), (16, 64), (64, 64)])
def test_neumann_poisson_solve(h, w):
    x = _x(4, (2, h, w))
    xd = x.astype(np.float64)
    u = oracle.filter(x, poisson_multipliers(h, w))
    resid = neumann_laplacian(u) - (xd - xd.mean(axis=(1, 2), keepdims=True))
    scale = np.sqrt((xd * xd).sum(axis=(1, 2))).max()
    assert np.sqrt((resid * resid).sum(axis=(1, 2))).max() <= 1e-11 * scale
    assert np.abs(u.mean(axis=(1, 2))).max() <= 1e-12 * np.abs(u).max()


def test_random_multipliers_against_scipy():
    h, w = 16, 32
    x = _x(5, (4, h, w))
    lam = np.random.default_rng(6).uniform(-2.0, 2.0, (4, h, w))
    got = oracle.filter(x, lam)
    ys = scipy.fft.dctn(x.astype(np.float64), type=2, norm="ortho", axes=(1, 2))
    want = scipy.fft.idctn(lam * ys, type=2, norm="ortho", axes=(1, 2))
    assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max()


def test_bad_multiplier_shape_rejected():
    x = _x(7, (2, 8, 8))
    with pytest.raises(ValueError):
        oracle.filter(x, np.ones((8, 16)))
