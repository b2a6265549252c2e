"""Pins of the band-structure and density-of-states oracle (Sec. 4) against the
free-electron closed form, time reversal, the reciprocal-lattice period and the
normalisation of the density of states.  CPU only."""
import math

import numpy as np
import pytest

from oracle.fd import laplacian_weights
from oracle.bands import bands, dos


def _fd_free_levels(n, L, k, n_o, count):
    """Sorted -1/2 Lap_h symbols of the Bloch plane waves e^{i(k+G).x} of the grid."""
    vals = []
    ranges = [range(-(n[s] // 2), n[s] - n[s] // 2) for s in range(3)]
    sym = []
    for s in range(3):
        h = L[s] / n[s]
        w0, w = laplacian_weights(n_o, h)
        q = np.array([k[s] + 2 * math.pi * m / L[s] for m in ranges[s]])
        sym.append(-0.5 * (2 * w0 + 2 * sum(w[p - 1] * np.cos(p * q * h) for p in range(1, n_o + 1))))
    tot = sym[0][:, None, None] + sym[1][None, :, None] + sym[2][None, None, :]
    return np.sort(tot.ravel())[:count]


def test_empty_cell_free_electron_bands():
    n, L = (8, 9, 10), (4.0, 4.5, 5.0)
    ks = np.array([[0.0, 0.0, 0.0], [0.3, -0.2, 0.1], [math.pi / 4.0, 0.0, 0.0]])
    got = bands(n, L, ks, np.zeros(int(np.prod(n))), None, 12)
    for b, k in enumerate(ks):
        np.testing.assert_allclose(got[b], _fd_free_levels(n, L, k, 6, 12), atol=1e-10)


def test_time_reversal_and_reciprocal_period():
    rng = np.random.default_rng(21)
    n, L = (9, 8, 10), (4.5, 4.0, 5.0)
    R = rng.uniform(0, 1, (2, 3)) * np.asarray(L)
    atoms = (R, np.array([0, 1, 1]), np.array([0, 0, 1]), np.array([1.1, 0.8, 1.3]), np.array([1.8, 1.8, 1.8]))
    veff = -1.5 * np.exp(-rng.uniform(0, 1, int(np.prod(n))))
    k = np.array([0.21, -0.37, 0.15])
    G = np.array([2 * math.pi / L[0], 0.0, -2 * math.pi / L[2]])
    e = bands(n, L, np.stack([k, -k, k + G]), veff, atoms, 10)
    np.testing.assert_allclose(e[1], e[0], atol=1e-10)
    np.testing.assert_allclose(e[2], e[0], atol=1e-10)


def test_dos_normalisation_and_single_level():
    eig = np.array([[-1.0, 0.2, 0.5], [-0.8, 0.1, 0.9]])
    wk = np.array([0.25, 0.75])
    E = np.linspace(-3.0, 3.0, 6001)
    D = dos(eig, wk, E, 0.05)
    assert np.trapezoid(D, E) == pytest.approx(2.0 * 3 * wk.sum(), rel=1e-9)
    one = dos(np.array([[0.3]]), np.array([1.0]), np.array([0.3, 0.35]), 0.05)
    np.testing.assert_allclose(one, [2.0 / (0.05 * math.sqrt(2 * math.pi)),
                                     2.0 * math.exp(-0.5) / (0.05 * math.sqrt(2 * math.pi))], rtol=1e-14)
