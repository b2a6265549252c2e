"""Pins of the oracle's Chebyshev filter, Rayleigh-Ritz and Lanczos (Sec. 3.4,
Sec. 4 solver settings) against direct spectral evaluation, brute-force
diagonalisation, interlacing and closed-form spectra.  CPU only."""
import math

import numpy as np
import pytest
from numpy.polynomial import chebyshev as npcheb

from oracle.fd import Grid, apply_H, dense_H
from oracle.cell import local_potential, projectors
from oracle.chefsi import (cheb_filter, cheb_direct, chebyshev_value, rayleigh_ritz,
                           lanczos_bounds, filter_center_halfwidth)


def _cell(k=(0.0, 0.0, 0.0), n=(8, 9, 10), L=(4.8, 5.4, 6.0), ls=(0, 1), seed=11):
    rng = np.random.default_rng(seed)
    R = rng.uniform(0, 1, (3, 3)) * np.array(L)
    grid = Grid(n=n, L=L, k=k)
    V = local_potential(grid, R, rng.uniform(2, 6, 3), rng.uniform(0.8, 1.5, 3))
    ca = np.repeat(np.arange(3), len(ls))
    cl = np.tile(ls, 3)
    P = projectors(grid, R, ca, cl, rng.uniform(0.5, 2, len(ca)), np.full(len(ca), 1.8))
    return grid, V, P


def test_chebyshev_value_matches_numpy():
    t = np.linspace(-3, 3, 601)
    for m in (1, 2, 5, 20, 24):
        c = np.zeros(m + 1)
        c[m] = 1.0
        np.testing.assert_allclose(chebyshev_value(m, t), npcheb.chebval(t, c), rtol=1e-9, atol=1e-12)


@pytest.mark.parametrize("k,degree", [((0.0, 0.0, 0.0), 20), ((0.3, -0.4, 0.2), 11), ((0.0, 0.0, 0.0), 1)])
def test_filter_recurrence_vs_direct(k, degree):
    grid, V, P = _cell(k=k)
    H = dense_H(grid, V, P)
    lam = np.linalg.eigvalsh(H)
    rng = np.random.default_rng(3)
    X = rng.standard_normal((grid.n_d, 5))
    if not grid.is_gamma:
        X = X + 1j * rng.standard_normal((grid.n_d, 5))
    lcut, lmax = lam[12], lam[-1] * 1.01
    Yr = cheb_filter(X, grid, V, P, degree, lcut, lmax)
    Yd = cheb_direct(X, grid, V, P, degree, lcut, lmax)
    err = np.linalg.norm(Yr - Yd, axis=0) / np.linalg.norm(Yd, axis=0)
    assert err.max() < 1e-11


def test_rayleigh_ritz_interlacing_and_orthonormality():
    grid, V, P = _cell(k=(0.2, 0.1, -0.3))
    lam = np.linalg.eigvalsh(dense_H(grid, V, P))
    rng = np.random.default_rng(5)
    X = rng.standard_normal((grid.n_d, 9)) + 1j * rng.standard_normal((grid.n_d, 9))
    theta, Xr = rayleigh_ritz(X, grid, V, P)
    assert np.all(theta >= lam[:9] - 1e-10)            # Cauchy interlacing
    assert np.all(theta <= lam[-9:] + 1e-10)
    np.testing.assert_allclose(Xr.conj().T @ Xr, np.eye(9), atol=1e-12)
    # the rotated block diagonalises the projected operator
    Hs = Xr.conj().T @ apply_H(Xr, grid, V, P)
    np.testing.assert_allclose(Hs, np.diag(theta), atol=1e-10)


@pytest.mark.parametrize("k", [(0.0, 0.0, 0.0), (0.25, -0.35, 0.15)])
def test_chefsi_converges_to_dense_spectrum(k):
    """Repeated filter + Rayleigh-Ritz passes reach the lowest eigenvalues of
    the dense H (brute force) for the states below the filter cut."""
    grid, V, P = _cell(k=k)
    lam = np.linalg.eigvalsh(dense_H(grid, V, P))
    rng = np.random.default_rng(7)
    ns = 12
    X = rng.standard_normal((grid.n_d, ns))
    if not grid.is_gamma:
        X = X + 1j * rng.standard_normal((grid.n_d, ns))
    v0 = rng.standard_normal(grid.n_d)
    lmin, lmax = lanczos_bounds(grid, V, P, v0, 30)
    theta = None
    for it in range(12):
        lcut = 0.5 * (lmin + lmax) if theta is None else theta[-1]
        Xf = cheb_filter(X, grid, V, P, 20, lcut, lmax)
        theta, X = rayleigh_ritz(Xf, grid, V, P)
    np.testing.assert_allclose(theta[:8], lam[:8], atol=1e-8)


def test_lanczos_bounds_bracket():
    grid, V, P = _cell(k=(0.1, 0.0, 0.2))
    lam = np.linalg.eigvalsh(dense_H(grid, V, P))
    v0 = np.random.default_rng(1).standard_normal(grid.n_d)
    lmin, lmax = lanczos_bounds(grid, V, P, v0, 20)
    assert lmax >= lam[-1]
    assert lmin >= lam[0] - 1e-10
    assert lmax <= lam[-1] * 1.2 + 1.0


def test_free_electron_chefsi_24():
    """CheFSI on the empty 24^3 / L = 12 cell reproduces the closed-shell
    free-electron levels 0 (x1), 0.137078 (x6), 0.274156 (x12), 0.411234 (x8),
    0.548311 (x6)."""
    grid = Grid(n=(24, 24, 24), L=(12.0, 12.0, 12.0))
    V = np.zeros(grid.n_d)
    rng = np.random.default_rng(0)
    ns = 40
    X = rng.standard_normal((grid.n_d, ns))
    lmax = 3.53647 * 3 / 0.25 * 1.01          # kinetic bound: 3 directions x T(pi)/h^2
    theta = None
    for it in range(8):
        lcut = 2.0 if theta is None else theta[-1]
        theta, X = rayleigh_ritz(cheb_filter(X, grid, V, (), 20, lcut, lmax), grid, V, ())
    ref = [0.0] + [0.137078] * 6 + [0.274156] * 12 + [0.411234] * 8 + [0.548311] * 6
    np.testing.assert_allclose(theta[:33], ref, atol=2e-6)


def test_filter_center_halfwidth():
    c, e = filter_center_halfwidth(1.0, 9.0)
    assert (c, e) == (5.0, 4.0)
