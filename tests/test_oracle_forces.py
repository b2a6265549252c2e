"""Pins of the atomic-force oracle (Sec. 2 atomic forces, Sec. 3.6 local and
non-local components) against closed forms, exact discrete identities and
finite differences of the energy.  CPU only."""
import math

import numpy as np
import pytest

from oracle.fd import Grid
from oracle.cell import local_potential, projectors
from oracle.forces import (fd_gradient, local_energy, local_force, nonlocal_energy, nonlocal_force,
                           nonlocal_force_on_projectors)
from oracle.scf import sad_density, scf


def _orth(rng, n_d, n_s, cplx):
    A = rng.standard_normal((n_d, n_s))
    if cplx:
        A = A + 1j * rng.standard_normal((n_d, n_s))
    Q, _ = np.linalg.qr(A)
    return Q


def _atoms(rng, n_atoms, L):
    R = rng.uniform(0, 1, (n_atoms, 3)) * np.asarray(L)[None, :]
    depth = rng.uniform(2.0, 6.0, n_atoms)
    width = rng.uniform(0.8, 1.5, n_atoms)
    return R, depth, width


@pytest.mark.parametrize("k", [(0.0, 0.0, 0.0), (0.31, -0.17, 0.42)])
def test_gradient_symbol_on_bloch_waves(k):
    """grad_h e^{i(k+G).x} = i sigma(k+G) e^{i(k+G).x} with the closed-form symbol
    sigma_s(q) = 2 sum_p w~_p sin(p q h_s) (w~_p of Sec. 3.1); the Bloch map
    psi(i + n) = e^{ikL} psi(i) holds for these waves, so the wrap is exercised."""
    grid = Grid(n=(10, 12, 9), L=(5.0, 6.6, 4.5), n_o=6, k=k)
    x = grid.coords()
    fn = math.factorial(6)
    for m in [(0, 0, 0), (1, -2, 1), (3, 2, -4)]:
        q = np.array([k[s] + 2 * math.pi * m[s] / grid.L[s] for s in range(3)])
        f = np.exp(1j * (x @ q))
        g = fd_gradient(f, grid)
        for s in range(3):
            h = grid.h[s]
            sig = 2.0 * sum((-1) ** (p + 1) * fn * fn / (h * p * math.factorial(6 - p) * math.factorial(6 + p))
                            * math.sin(p * q[s] * h) for p in range(1, 7))
            np.testing.assert_allclose(g[s], 1j * sig * f, atol=1e-12 * max(1.0, abs(sig)))
        # the symbol approaches the exact derivative for well-resolved waves
        if m == (1, -2, 1):
            np.testing.assert_allclose(g, 1j * q[:, None] * f[None, :], atol=1e-3 * np.abs(q).max())


def test_local_force_is_minus_energy_derivative():
    """f_loc = -dE_loc/dR at fixed density: central differences of
    E_loc = h^3 sum rho V_loc(R) over every atom and direction."""
    rng = np.random.default_rng(11)
    grid = Grid(n=(14, 12, 13), L=(7.0, 6.0, 6.5))
    R, depth, width = _atoms(rng, 3, grid.L)
    rho = rng.uniform(0.0, 1.0, grid.n_d)
    F = local_force(grid, R, depth, width, rho)
    d = 1e-4
    for J in range(3):
        for s in range(3):
            Rp, Rm = R.copy(), R.copy()
            Rp[J, s] += d
            Rm[J, s] -= d
            Ep = local_energy(grid, rho, local_potential(grid, Rp, depth, width))
            Em = local_energy(grid, rho, local_potential(grid, Rm, depth, width))
            assert F[J, s] == pytest.approx(-(Ep - Em) / (2 * d), rel=1e-6, abs=1e-8 * np.abs(F).max())


@pytest.mark.parametrize("cplx", [False, True])
def test_nonlocal_force_summation_by_parts(cplx):
    """The paper's form (gradient on the orbitals) equals the sums with the FD
    gradient moved onto the projectors, exactly (the central stencil is
    skew-adjoint on the Bloch-periodic grid); two k-points when complex."""
    rng = np.random.default_rng(12)
    L = (6.0, 5.5, 6.5)
    R, _, _ = _atoms(rng, 2, L)
    ks = [(0.21, -0.1, 0.3), (-0.2, 0.15, 0.05)] if cplx else [(0.0, 0.0, 0.0)]
    grids = [Grid(n=(12, 11, 13), L=L, n_o=6, k=k) for k in ks]
    ca, cl = np.array([0, 0, 1]), np.array([0, 1, 1])
    cg, crc = np.array([1.3, 0.7, 1.1]), np.array([2.5, 2.5, 2.8])
    pk = [projectors(g, R, ca, cl, cg, crc) for g in grids]
    Xs = [_orth(rng, grids[0].n_d, 6, cplx) for _ in grids]
    occ = rng.uniform(0, 1, (len(grids), 6)) / len(grids)
    F = nonlocal_force(grids, pk, Xs, occ, 2)
    F2 = nonlocal_force_on_projectors(grids, pk, Xs, occ, 2)
    assert np.abs(F).max() > 1e-3
    np.testing.assert_allclose(F, F2, rtol=0, atol=1e-11 * np.abs(F).max())


def test_nonlocal_force_matches_energy_derivative():
    """f_nloc against central differences of E_nl at fixed orbitals, the
    projectors rebuilt at the displaced position.  The orbitals are localised
    inside the projector spheres, so that the cutoff of the synthetic projectors
    (a jump of e^{-8} of their peak at r_c, which the derivative of a truncated
    function does not see) does not enter; what remains is the FD-gradient
    error of moving the derivative onto the orbitals (Sec. 2), about 1e-4 here."""
    rng = np.random.default_rng(13)
    L = (6.4, 6.4, 6.4)
    grid = Grid(n=(20, 20, 20), L=L)
    R, _, _ = _atoms(rng, 2, L)
    ca, cl = np.array([0, 1, 1]), np.array([0, 0, 1])
    cg, crc = np.array([1.2, 0.9, 1.4]), np.array([3.0, 3.0, 3.0])
    x = grid.coords()
    cols = []
    for J in range(2):
        for off in ([0.2, -0.1, 0.15], [-0.25, 0.2, 0.05], [0.1, 0.3, -0.2]):
            dx = x - (R[J] + np.array(off))
            dx = dx - np.round(dx / 6.4) * 6.4
            cols.append(np.exp(-np.sum(dx * dx, axis=1) / (2 * 0.6 ** 2)) * (1 + 0.3 * dx[:, 0]))
    Xs = [np.linalg.qr(np.stack(cols, axis=1))[0]]
    occ = rng.uniform(0.2, 1.0, (1, 6))
    F = nonlocal_force([grid], [projectors(grid, R, ca, cl, cg, crc)], Xs, occ, 2)
    d = 1e-4
    Ffd = np.zeros_like(F)
    for J in range(2):
        for s in range(3):
            Rp, Rm = R.copy(), R.copy()
            Rp[J, s] += d
            Rm[J, s] -= d
            Ep = nonlocal_energy(grid, projectors(grid, Rp, ca, cl, cg, crc), Xs, occ)
            Em = nonlocal_energy(grid, projectors(grid, Rm, ca, cl, cg, crc), Xs, occ)
            Ffd[J, s] = -(Ep - Em) / (2 * d)
    scale = np.abs(Ffd).max()
    assert scale > 0.1
    np.testing.assert_allclose(F, Ffd, rtol=0, atol=5e-4 * scale)


def test_inversion_symmetric_pair():
    """Two identical atoms at R and -R (mod L) on a grid mapped onto itself by
    x -> -x, with an inversion-even density and inversion-even orbitals: the
    forces are opposite (local and non-local, to rounding)."""
    rng = np.random.default_rng(14)
    grid = Grid(n=(12, 12, 12), L=(6.0, 6.0, 6.0))
    R1 = np.array([1.3, 0.8, 2.1])
    R = np.stack([R1, np.mod(-R1, 6.0)])
    depth, width = np.array([3.0, 3.0]), np.array([1.1, 1.1])
    n = grid.n[0]
    inv = lambda f: f.reshape(n, n, n)[np.ix_((-np.arange(n)) % n, (-np.arange(n)) % n, (-np.arange(n)) % n)].reshape(-1)
    rho = rng.uniform(0, 1, grid.n_d)
    rho = rho + inv(rho)
    Fl = local_force(grid, R, depth, width, rho)
    np.testing.assert_allclose(Fl[0], -Fl[1], atol=1e-12 * np.abs(Fl).max())
    A = rng.standard_normal((grid.n_d, 4))
    A = A + np.stack([inv(A[:, j]) for j in range(4)], axis=1)
    X = np.linalg.qr(A)[0]
    ca, cl = np.array([0, 0, 1, 1]), np.array([0, 1, 0, 1])
    cg, crc = np.array([1.2, 0.8, 1.2, 0.8]), np.full(4, 2.6)
    Fn = nonlocal_force([grid], [projectors(grid, R, ca, cl, cg, crc)], [X], rng.uniform(0, 1, (1, 4)), 2)
    assert np.abs(Fn).max() > 1e-4
    np.testing.assert_allclose(Fn[0], -Fn[1], atol=1e-11 * np.abs(Fn).max())


def test_total_force_matches_scf_energy_derivative():
    """Sec. 2: f_J = -dF/dR_J.  The local plus non-local force at the converged
    SCF state against central differences of the converged Harris-Foulkes free
    energy, on a small two-atom cell.  The synthetic projectors end at r_c with a
    jump of e^{-8} of their peak, so the energy moves in steps of ~1e-7 Ha as
    nodes cross a cutoff sphere and its central differences carry ~3e-4 Ha/bohr
    of noise; the bound is 1e-3 Ha/bohr, far below the non-local term itself
    (-0.046 on the first checked component), so a wrong sign or factor fails."""
    L = (5.6, 5.6, 5.6)
    R = np.array([[1.2, 1.9, 2.4], [3.9, 3.1, 4.4]])
    depth, width, Z = np.array([3.5, 2.5]), np.array([0.9, 1.1]), np.array([2.0, 2.0])
    ca, cl = np.array([0, 1]), np.array([0, 0])
    cg, crc = np.array([1.5, 1.0]), np.array([2.4, 2.4])
    grid = Grid(n=(16, 16, 16), L=L)
    X0 = np.random.default_rng(15).standard_normal((grid.n_d, 8))

    def run(Rx):
        v = local_potential(grid, Rx, depth, width)
        pj = projectors(grid, Rx, ca, cl, cg, crc)
        rho0 = sad_density(grid, Rx, width, Z, 4.0)
        out = scf(grid, v, pj, X0, 4.0, degree=14, kT=0.01, mix=0.3, tol=1e-10, max_iter=200,
                  n_first_passes=6, rho_init=rho0, mix_history=5)
        assert out["converged"]
        return out, pj

    out, pj = run(R)
    lam = out["ritz"]
    from oracle.scf import occupations
    g = occupations(lam, out["mu"], 0.01)
    rho_out = 2.0 * (np.abs(out["X"]) ** 2) @ g / grid.dV
    F = local_force(grid, R, depth, width, rho_out) + nonlocal_force([grid], [pj], [out["X"]], g[None, :], 2)
    d = 2e-3
    for J, s in [(0, 0), (1, 2)]:
        Rp, Rm = R.copy(), R.copy()
        Rp[J, s] += d
        Rm[J, s] -= d
        Ffd = -(run(Rp)[0]["energy"] - run(Rm)[0]["energy"]) / (2 * d)
        print(f"atom {J} dir {s}: force {F[J, s]:.6e}, -dF/dR {Ffd:.6e}")
        assert abs(F[J, s] - Ffd) < 1e-3
