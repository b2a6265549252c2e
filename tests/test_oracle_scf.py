"""Pins of the oracle's occupations, density, Poisson solve, exchange and SCF
(Sec. 2-3.5, reduced model) against conservation laws, closed forms and the
stencil.  CPU only."""
import math
import os

import numpy as np
import pytest

from oracle.fd import Grid, minus_half_laplacian
from oracle.scf import (occupations, fermi_level, density, poisson, slater, entropy_term,
                        harris_foulkes, sad_density, anderson_update, kerker, scf)
from oracle.chefsi import rayleigh_ritz

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_fermi_charge_and_monotone():
    rng = np.random.default_rng(0)
    lam = np.sort(rng.uniform(-2, 1, (3, 10)), axis=1)
    wk = np.array([0.5, 0.25, 0.25])
    mu = fermi_level(lam, wk, 7.0, 0.01)
    assert 2 * np.sum(wk[:, None] * occupations(lam, mu, 0.01)) == pytest.approx(7.0, rel=1e-12)
    mu2 = fermi_level(lam, wk, 9.0, 0.01)
    assert mu2 > mu
    g = occupations(np.array([mu - 100.0, mu, mu + 100.0]), mu, 0.01)
    np.testing.assert_allclose(g, [1.0, 0.5, 0.0], atol=1e-300)
    # the tanh form equals the logistic form where the latter does not overflow
    x = np.linspace(-0.2, 0.2, 41)
    np.testing.assert_allclose(occupations(x, 0.0, 0.01), 1.0 / (1.0 + np.exp(x / 0.01)), rtol=0, atol=1e-15)


def test_fermi_level_meets_the_charge_in_a_gap():
    """Sec. 3.4 electron-count constraint at the returned mu, also where a gap makes
    the count flat (every mu inside the gap is a root)."""
    lam = np.array([[-1.0, -0.9, 0.8, 0.9, 1.0, 1.5]])
    for kT in (0.001, 0.01, 0.2):
        mu = fermi_level(lam, np.array([1.0]), 4.0, kT)
        assert 2 * np.sum(occupations(lam, mu, kT)) == pytest.approx(4.0, rel=1e-12)
    assert -0.9 < fermi_level(lam, np.array([1.0]), 4.0, 0.001) < 0.8


def test_density_conservation_and_uniform_shell():
    """dV sum rho = N_e, rho >= 0, and a fully occupied closed shell of plane
    waves (any unitary mix inside the shell) gives a uniform density."""
    grid = Grid(n=(12, 12, 12), L=(6.0, 6.0, 6.0))
    x = grid.coords()
    ms = [(0, 0, 0), (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)]
    W = np.stack([np.exp(1j * x @ (2 * math.pi / 6.0 * np.array(m))) for m in ms], axis=1)
    W /= np.linalg.norm(W, axis=0)
    Q, _ = np.linalg.qr(np.random.default_rng(1).standard_normal((7, 7)))
    X = W @ Q
    occ = np.ones((1, 7))
    rho = density([X], occ, grid.dV)
    assert grid.dV * rho.sum() == pytest.approx(14.0, rel=1e-13)
    np.testing.assert_allclose(rho, 14.0 / 216.0, rtol=1e-12)
    rng = np.random.default_rng(2)
    Xr, _ = np.linalg.qr(rng.standard_normal((grid.n_d, 5)))
    w = rng.uniform(0, 1, (1, 5))
    r2 = density([Xr], w, grid.dV)
    assert np.all(r2 >= 0) and grid.dV * r2.sum() == pytest.approx(2 * w.sum(), rel=1e-12)


@pytest.mark.parametrize("n_o", [6, 2])
def test_poisson_against_stencil(n_o):
    """-Lap_h V_H = 4 pi (rho - mean rho), checked with the stencil itself
    (a different code path from the FFT diagonalisation); mean V_H = 0."""
    grid = Grid(n=(12, 14, 10), L=(6.0, 7.7, 5.0), n_o=n_o)
    rho = np.random.default_rng(3).uniform(0, 1, grid.n_d)
    vh = poisson(rho, grid)
    lap = -2.0 * minus_half_laplacian(vh, grid)
    np.testing.assert_allclose(-lap, 4 * math.pi * (rho - rho.mean()), atol=1e-10)
    assert abs(vh.mean()) < 1e-12


def test_poisson_continuum_plane_wave():
    """A smooth cosine density: V_H = 4 pi cos(G.x)/|G|^2 up to the O(h^12)
    discretisation error."""
    grid = Grid(n=(24, 24, 24), L=(12.0, 12.0, 12.0))
    x = grid.coords()
    G = 2 * math.pi / 12.0 * np.array([1.0, 0.0, 1.0])
    rho = 1.0 + 0.3 * np.cos(x @ G)
    vh = poisson(rho, grid)
    np.testing.assert_allclose(vh, 4 * math.pi * 0.3 * np.cos(x @ G) / (G @ G), atol=1e-8)


def test_slater_constants_and_derivative():
    gold = {}
    for line in open(os.path.join(GOLD, "slater_constants.txt")):
        if line.strip() and not line.startswith("#"):
            k, v = line.split()
            gold[k] = float(v)
    eps, vx = slater(np.array([1.0]))
    assert eps[0] == pytest.approx(gold["eps_coef"], rel=1e-15)
    assert vx[0] == pytest.approx(gold["v_coef"], rel=1e-15)
    # V_x = d(rho eps_x)/d rho by central differences
    r = np.array([0.013, 0.2, 1.7])
    d = 1e-6 * r
    e1, _ = slater(r + d)
    e0, _ = slater(r - d)
    _, v = slater(r)
    np.testing.assert_allclose(((r + d) * e1 - (r - d) * e0) / (2 * d), v, rtol=1e-8)


def test_entropy_limits():
    assert entropy_term(np.array([[0.0, 1.0]]), np.array([1.0]), 0.01) == 0.0
    val = entropy_term(np.array([[0.5]]), np.array([1.0]), 0.01)
    assert val == pytest.approx(2 * 0.01 * math.log(0.5), rel=1e-14)


def test_uniform_gas_fixed_point():
    """Empty cell, closed shell of 7 states (14 electrons) on a 12^3 / L = 6
    grid: a uniform density is a fixed point; one SCF step converges, and F is
    the closed form 2 sum g T + Omega eps_x(rho) rho + entropy."""
    grid = Grid(n=(12, 12, 12), L=(6.0, 6.0, 6.0))
    rho0 = np.full(grid.n_d, 14.0 / 216.0)
    X0 = np.random.default_rng(4).standard_normal((grid.n_d, 10))
    v0 = np.random.default_rng(5).standard_normal(grid.n_d)
    out = scf(grid, np.zeros(grid.n_d), (), X0, 14.0, degree=20, rho_init=rho0, lanczos_v0=v0,
              n_first_passes=8, tol=1e-9)
    assert out["converged"] and out["iterations"] == 1
    T1 = 0.0
    # closed-form kinetic levels (exact rational weights at h = 0.5)
    from fractions import Fraction
    h = 0.5
    w = [float(Fraction(2 * (-1) ** (p + 1) * 720 ** 2, p * p * math.factorial(6 - p) * math.factorial(6 + p))) / h ** 2
         for p in range(1, 7)]
    w0 = -float(sum(Fraction(1, q * q) for q in range(1, 7))) / h ** 2
    q = 2 * math.pi / 6.0
    T1 = -(w0 + sum(w[p - 1] * math.cos(p * q * h) for p in range(1, 7))) - 2 * (w0 + sum(w))
    rb = 14.0 / 216.0
    eps = -0.7385587663820223 * rb ** (1 / 3)
    vx = -0.9847450218426965 * rb ** (1 / 3)
    lam = np.array([0.0] + [T1] * 6) + vx
    np.testing.assert_allclose(out["ritz"][:7], lam, atol=1e-9)
    mu = out["mu"]
    g = 0.5 * (1 - np.tanh((out["ritz"] - mu) / 0.02))
    ent = entropy_term(g[None, :], np.array([1.0]), 0.01)
    F = 2 * np.sum(g * (out["ritz"] - vx)) + 216.0 * eps * rb + ent
    assert out["energy"] == pytest.approx(F, abs=1e-10)


def test_sad_normalisation():
    grid = Grid(n=(16, 16, 16), L=(8.0, 8.0, 8.0))
    R = np.array([[1.0, 2.0, 7.5], [4.0, 4.0, 4.0]])
    rho = sad_density(grid, R, [0.9, 1.2], [2.0, 2.0], 4.0)
    assert grid.dV * rho.sum() == pytest.approx(4.0, rel=1e-13)
    assert np.all(rho >= 0)


def test_sad_brute_force_image_sum():
    """The superposition of atomic densities at sampled nodes against a brute-force
    sum over 7^3 periodic images of the closed-form normalised Gaussian
    Z (2 pi w^2)^{-3/2} exp(-r^2 / (2 w^2)), no cutoff.  The widths are resolved by
    the grid (w/h >= 1.8), so the node sum of each image-summed Gaussian is Z to
    e^{-2 pi^2 w^2 / h^2} < 1e-25 (Poisson summation), and the renormalisation to N_e
    is the factor N_e / sum Z.  Atoms at a corner and on faces make the images count;
    a wrong width convention, a dropped image or a per-atom amplitude error fails."""
    grid = Grid(n=(18, 16, 20), L=(9.0, 8.0, 10.0))
    R = np.array([[0.1, 0.2, 9.8], [4.5, 7.9, 5.0], [8.8, 3.0, 0.05]])
    w = np.array([0.9, 1.2, 1.4])
    Z = np.array([2.0, 3.0, 1.0])
    ne = 7.5
    rho = sad_density(grid, R, w, Z, ne)
    rng = np.random.default_rng(12)
    nodes = np.concatenate([rng.integers(0, grid.n_d, 40), [0, grid.n_d - 1]])
    X = grid.coords()[nodes]
    ref = np.zeros(len(nodes))
    for J in range(3):
        for a in range(-3, 4):
            for b in range(-3, 4):
                for c in range(-3, 4):
                    d = X - R[J] - np.array([a * 9.0, b * 8.0, c * 10.0])
                    r2 = np.sum(d * d, axis=1)
                    ref += Z[J] * (2 * math.pi * w[J] ** 2) ** -1.5 * np.exp(-r2 / (2 * w[J] ** 2))
    ref *= ne / Z.sum()
    np.testing.assert_allclose(rho[nodes], ref, rtol=1e-12, atol=1e-14 * ref.max())


def test_anderson_linear_map_terminates():
    """For a linear fixed-point map x -> M x + c, Anderson extrapolation with a
    history at least the dimension minimises the residual over the affine span of
    all iterates, which is the Krylov space of GMRES (Walker and Ni, 2011): the
    iterate reaches the fixed point after d + 1 residual evaluations, for any
    relaxation.  A sign error, a dropped dX gamma term or a misaligned history
    breaks the finite termination."""
    rng = np.random.default_rng(1)
    d = 6
    M = rng.standard_normal((d, d))
    M *= 0.9 / np.max(np.abs(np.linalg.eigvals(M)))
    c = rng.standard_normal(d)
    xs = np.linalg.solve(np.eye(d) - M, c)
    for beta in (0.3, 1.0):
        x = np.zeros(d)
        hx, hf = [], []
        errs = []
        for _ in range(d + 1):
            x = anderson_update(x, M @ x + c - x, hx, hf, beta, d)
            errs.append(np.linalg.norm(x - xs))
        assert errs[-1] < 1e-10 * np.linalg.norm(xs)
        assert errs[-2] > 1e-6
    # m = 0 is plain linear mixing
    x = rng.standard_normal(d)
    f = M @ x + c - x
    np.testing.assert_array_equal(anderson_update(x, f, [], [], 0.3, 0), x + 0.3 * f)


def test_kerker_plane_waves_textbook_symbol():
    """Kerker filter on plane waves of a second-order grid (n_o = 1): the factor
    sigma / (sigma + k0^2) with the textbook symbol of the 3-point Laplacian,
    sigma(G) = sum_s (4 / h_s^2) sin^2(G_s h_s / 2); a constant is removed."""
    grid = Grid(n=(10, 12, 9), L=(5.0, 7.2, 4.5), n_o=1)
    X = grid.coords()
    k0 = 0.9
    for m in ((1, 0, 0), (2, -3, 1), (0, 1, 4)):
        G = np.array([2 * math.pi * m[s] / grid.L[s] for s in range(3)])
        f = np.cos(X @ G + 0.3)
        sig = sum(4.0 / grid.h[s] ** 2 * math.sin(G[s] * grid.h[s] / 2) ** 2 for s in range(3))
        np.testing.assert_allclose(kerker(f, grid, k0), sig / (sig + k0 * k0) * f, atol=1e-13)
    np.testing.assert_allclose(kerker(np.full(grid.n_d, 2.5), grid, k0), 0.0, atol=1e-13)


def test_anderson_preconditioned_linear_map_terminates():
    """With a fixed nonsingular linear preconditioner P the update
    x_bar + beta P f_bar spans the Krylov space of P (M - I): finite termination as in
    the unpreconditioned case (a wrong placement of P breaks it)."""
    rng = np.random.default_rng(6)
    d = 6
    M = rng.standard_normal((d, d))
    M *= 0.9 / np.max(np.abs(np.linalg.eigvals(M)))
    c = rng.standard_normal(d)
    B = rng.standard_normal((d, d))
    Pm = B @ B.T + 0.5 * np.eye(d)
    xs = np.linalg.solve(np.eye(d) - M, c)
    x = np.zeros(d)
    hx, hf = [], []
    for _ in range(d + 1):
        x = anderson_update(x, M @ x + c - x, hx, hf, 0.4, d, lambda f: Pm @ f)
    assert np.linalg.norm(x - xs) < 1e-9 * np.linalg.norm(xs)


def test_anderson_constrained_form():
    """Anderson's original form: the extrapolated point is sum_i a_i x_i over the
    last m + 1 iterates with sum_i a_i = 1 and a minimising ||sum_i a_i f_i||, then
    relaxed by beta times that residual combination.  Solved here through its
    KKT system on a nonlinear map, step by step with history m = 3 (so the window
    slides), against anderson_update."""
    rng = np.random.default_rng(4)
    d, m, beta = 8, 3, 0.4
    A = rng.standard_normal((d, d)) / 3.0
    c = rng.standard_normal(d)
    g = lambda x: np.tanh(A @ x) + c
    x = rng.standard_normal(d)
    hx, hf, xs, fs = [], [], [], []
    for step in range(8):
        f = g(x) - x
        xs.append(x.copy())
        fs.append(f.copy())
        Xw, Fw = np.array(xs[-(m + 1):]).T, np.array(fs[-(m + 1):]).T
        k = Xw.shape[1]
        K = np.zeros((k + 1, k + 1))
        K[:k, :k] = 2.0 * Fw.T @ Fw
        K[:k, k] = 1.0
        K[k, :k] = 1.0
        rhs = np.zeros(k + 1)
        rhs[k] = 1.0
        a = np.linalg.lstsq(K, rhs, rcond=None)[0][:k]
        ref = Xw @ a + beta * (Fw @ a)
        x = anderson_update(x, f, hx, hf, beta, m)
        np.testing.assert_allclose(x, ref, rtol=1e-9, atol=1e-11)


@pytest.mark.slow
def test_scf_small_cell_converges():
    """A small cell with two wells and s projectors reaches self-consistency and
    the converged density is reproduced by the final orbitals."""
    from oracle.cell import local_potential, projectors
    grid = Grid(n=(16, 16, 16), L=(8.0, 8.0, 8.0))
    rng = np.random.default_rng(8)
    R = rng.uniform(0, 8.0, (2, 3))
    vloc = local_potential(grid, R, [3.0, 4.0], [1.0, 1.2])
    P = projectors(grid, R, [0, 1], [0, 0], [1.0, 0.8], [3.0, 3.0])
    rho0 = sad_density(grid, R, [1.0, 1.2], [2.0, 2.0], 4.0)
    X0 = rng.standard_normal((grid.n_d, 8))
    out = scf(grid, vloc, P, X0, 4.0, degree=20, rho_init=rho0,
              lanczos_v0=rng.standard_normal(grid.n_d), tol=1e-7)
    assert out["converged"]
    assert grid.dV * out["rho"].sum() == pytest.approx(4.0, rel=1e-10)
