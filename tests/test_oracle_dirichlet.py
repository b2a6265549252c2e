"""Pins of the zero-Dirichlet boundaries of the oracle (Sec. 3.1: values at indices
outside the grid are zero in a Dirichlet direction; slabs and wires): the Kronecker
form of the empty-cell Hamiltonian built from banded Toeplitz blocks, the closed-form
levels of the second-order stencil, the local potential without images across a
Dirichlet direction (brute force), projector supports inside the grid, and the force
identities with Dirichlet directions.  CPU only."""
import math

import numpy as np
import pytest

from oracle.fd import Grid, dense_H, laplacian_weights
from oracle.cell import local_potential, projectors
from oracle.forces import (local_energy, local_force, nonlocal_force, nonlocal_force_on_projectors)


def _toeplitz_1d(n, L, n_o, kL, dirichlet):
    """-1/2 d^2/dx^2 of Sec. 3.1 on n nodes as a dense matrix: a banded Toeplitz matrix
    (Dirichlet) or its Bloch-periodic wrap (periodic)."""
    h = L / n
    w0, w = laplacian_weights(n_o, h)
    T = np.zeros((n, n), dtype=np.complex128)
    for i in range(n):
        T[i, i] += 2 * w0
        for p in range(1, n_o + 1):
            for sgn in (1, -1):
                j = i + sgn * p
                if 0 <= j < n:
                    T[i, j] += w[p - 1]
                elif not dirichlet:
                    T[i, j % n] += w[p - 1] * np.exp(1j * kL * (j // n))
    return -0.5 * T


@pytest.mark.parametrize("bc", [(0, 0, 1), (0, 1, 1), (1, 1, 1)])
def test_empty_cell_kronecker_form(bc):
    n, L, k = (6, 5, 7), (3.0, 2.5, 3.5), (0.4, -0.3, 0.2)
    k = tuple(0.0 if bc[s] else k[s] for s in range(3))
    grid = Grid(n=n, L=L, n_o=6, k=k, bc=bc)
    H = dense_H(grid, np.zeros(grid.n_d))
    T = [_toeplitz_1d(n[s], L[s], 6, k[s] * L[s], bc[s] == 1) for s in range(3)]
    I = [np.eye(n[s]) for s in range(3)]
    # flattened index g = i + n1 (j + n2 k): Kronecker order (z, y, x)
    ref = np.kron(np.kron(I[2], I[1]), T[0]) + np.kron(np.kron(I[2], T[1]), I[0]) + np.kron(np.kron(T[2], I[1]), I[0])
    np.testing.assert_allclose(H, ref, atol=1e-12)


def test_second_order_dirichlet_levels():
    """n_o = 1, Dirichlet in z: levels (1/h^2)(1 - cos q h) per direction, with
    q_z h_z = pi m / (n_z + 1) (sine modes) and q = k + G in the periodic directions."""
    n, L, k = (5, 4, 6), (2.5, 2.0, 3.5), (0.3, -0.2, 0.0)
    grid = Grid(n=n, L=L, n_o=1, k=k, bc=(0, 0, 1))
    ev = np.linalg.eigvalsh(dense_H(grid, np.zeros(grid.n_d)))
    lev = []
    for a in range(n[0]):
        for b in range(n[1]):
            for m in range(1, n[2] + 1):
                qx = k[0] + 2 * math.pi * (a - n[0] // 2) / L[0]
                qy = k[1] + 2 * math.pi * (b - n[1] // 2) / L[1]
                hx, hy, hz = L[0] / n[0], L[1] / n[1], L[2] / n[2]
                lev.append((1 - math.cos(qx * hx)) / hx ** 2 + (1 - math.cos(qy * hy)) / hy ** 2
                           + (1 - math.cos(math.pi * m / (n[2] + 1))) / hz ** 2)
    np.testing.assert_allclose(ev, np.sort(lev), atol=1e-11)


def test_local_potential_without_dirichlet_images():
    rng = np.random.default_rng(41)
    grid = Grid(n=(8, 7, 9), L=(4.0, 3.5, 4.5), bc=(0, 0, 1))
    R = rng.uniform(0, 1, (2, 3)) * np.asarray(grid.L)
    D, W = np.array([2.5, 3.5]), np.array([0.9, 1.2])
    V = local_potential(grid, R, D, W)
    x = grid.coords()
    ref = np.zeros(grid.n_d)
    for J in range(2):
        for a in range(-4, 5):
            for b in range(-4, 5):
                d = x - (R[J] + np.array([a * grid.L[0], b * grid.L[1], 0.0]))
                r2 = np.sum(d * d, axis=1)
                ref += np.where(r2 <= (10 * W[J]) ** 2, -D[J] * np.exp(-r2 / (2 * W[J] ** 2)), 0.0)
    np.testing.assert_allclose(V, ref, atol=1e-13)


def test_projector_support_and_force_identities_with_dirichlet():
    """Supports stay inside the grid across the Dirichlet direction (no wrap), the
    summation-by-parts identity of the non-local force holds (the central stencil
    with zero padding is still skew-adjoint), and the local force is the derivative
    of the local energy."""
    rng = np.random.default_rng(42)
    grid = Grid(n=(10, 9, 12), L=(5.0, 4.5, 6.0), k=(0.2, -0.3, 0.0), bc=(0, 0, 1))
    R = np.array([[1.0, 2.0, 0.6], [3.5, 1.0, 5.2]])        # both near a Dirichlet face
    ca, cl, cg, crc = np.array([0, 1, 1]), np.array([0, 0, 1]), np.array([1.1, 0.9, 1.3]), np.full(3, 2.0)
    P = projectors(grid, R, ca, cl, cg, crc)
    for p in P:
        kz = p["idx"] // (grid.n[0] * grid.n[1])
        z = kz * grid.h[2]
        assert np.all(np.abs(z - R[p["atom"], 2]) <= 2.0 + 1e-12)
    X = np.linalg.qr(rng.standard_normal((grid.n_d, 5)) + 1j * rng.standard_normal((grid.n_d, 5)))[0]
    occ = rng.uniform(0, 1, (1, 5))
    F = nonlocal_force([grid], [P], [X], occ, 2)
    F2 = nonlocal_force_on_projectors([grid], [P], [X], occ, 2)
    assert np.abs(F).max() > 1e-4
    np.testing.assert_allclose(F, F2, atol=1e-11 * np.abs(F).max())
    D, W = np.array([3.0, 2.0]), np.array([1.0, 0.8])
    rho = rng.uniform(0, 1, grid.n_d)
    Fl = local_force(grid, R, D, W, rho)
    d = 1e-4
    for J, s in [(0, 2), (1, 0)]:
        Rp, Rm = R.copy(), R.copy()
        Rp[J, s] += d
        Rm[J, s] -= d
        fd = -(local_energy(grid, rho, local_potential(grid, Rp, D, W))
               - local_energy(grid, rho, local_potential(grid, Rm, D, W))) / (2 * d)
        assert Fl[J, s] == pytest.approx(fd, rel=1e-6, abs=1e-9)
