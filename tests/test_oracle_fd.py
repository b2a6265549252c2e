"""Pins of the oracle's discrete operators (Sec. 3.1) against closed forms,
exact rationals, invariants and brute force.  CPU only."""
import math
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle.fd import Grid, laplacian_weights, gradient_weights, apply_H, dense_H, minus_half_laplacian
from oracle.cell import local_potential, projectors

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    out = {}
    for line in open(os.path.join(GOLD, name)):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        k, *vals = line.split()
        out[k] = [float(Fraction(v)) for v in vals]
    return out


def test_weights_exact_no6():
    g = _golden("fd_weights_no6.txt")
    w0, w = laplacian_weights(6, 1.0)
    assert w0 == pytest.approx(g["lap_w0"][0], rel=1e-15)
    np.testing.assert_allclose(w, g["lap_w"], rtol=1e-14)
    np.testing.assert_allclose(gradient_weights(6, 1.0), g["grad_w"], rtol=1e-14)


def test_weights_textbook_low_order():
    g = _golden("fd_weights_no6.txt")
    w0, w = laplacian_weights(1, 1.0)
    assert 2 * w0 == pytest.approx(g["lap1_centre"][0]) and w[0] == pytest.approx(g["lap1_w"][0])
    w0, w = laplacian_weights(2, 1.0)
    assert 2 * w0 == pytest.approx(g["lap2_centre"][0])
    np.testing.assert_allclose(w, g["lap2_w"], rtol=1e-15)


@pytest.mark.parametrize("n_o", [1, 2, 3, 4, 6, 8])
def test_weights_moment_conditions(n_o):
    """The 2n_o-order stencil is exact on even polynomials up to x^{2 n_o}:
    sum rule, second moment 1 (second derivative of x^2 is 2), higher even
    moments 0; the gradient is exact up to x^{2 n_o - 1}."""
    h = 0.37
    w0, w = laplacian_weights(n_o, h)
    p = np.arange(1, n_o + 1, dtype=np.float64)
    assert abs(2 * w0 + 2 * w.sum()) * h * h < 1e-13
    assert np.sum(2 * p ** 2 * w) * h * h == pytest.approx(2.0, rel=1e-13)
    for j in range(2, n_o + 1):
        assert abs(np.sum(p ** (2 * j) * w)) * h * h < 1e-9 * np.sum(p ** (2 * j) * np.abs(w)) * h * h
    wt = gradient_weights(n_o, h)
    assert np.sum(2 * p * wt) * h == pytest.approx(1.0, rel=1e-13)
    for j in range(1, n_o):
        assert abs(np.sum(p ** (2 * j + 1) * wt)) < 1e-9 * np.sum(p ** (2 * j + 1) * np.abs(wt))


def _symbol(q, grid):
    """Closed form of -1/2 Lap_h on e^{iq.x}: T(q) = -sum_s [w0_s + sum_p w_p,s cos(p q_s h_s)],
    evaluated from exact rational weights (independent of the oracle's float weights)."""
    T = 0.0
    for s in range(3):
        hs = grid.h[s]
        no = grid.n_o
        w0 = -float(sum(Fraction(1, r * r) for r in range(1, no + 1))) / hs ** 2
        acc = w0
        for pp in range(1, no + 1):
            wp = float(Fraction(2 * (-1) ** (pp + 1) * math.factorial(no) ** 2,
                                pp * pp * math.factorial(no - pp) * math.factorial(no + pp))) / hs ** 2
            acc += wp * math.cos(pp * q[s] * hs)
        T -= acc
    return T


@pytest.mark.parametrize("n,L,n_o,k", [
    ((12, 12, 12), (6.0, 6.0, 6.0), 6, (0.0, 0.0, 0.0)),
    ((7, 12, 13), (3.5, 5.0, 6.2), 6, (0.3, -0.2, 0.11)),
    ((5, 6, 9), (2.0, 3.0, 4.0), 6, (0.9, 0.4, -0.7)),     # n < 2 n_o + 1: multiple wraps
    ((8, 9, 10), (4.0, 4.5, 5.0), 2, (0.25, 0.0, -0.5)),
    ((8, 9, 10), (4.0, 4.5, 5.0), 1, (0.1, 0.2, 0.3)),
])
def test_plane_wave_symbol(n, L, n_o, k):
    """psi = e^{i q.x} with q = 2 pi m / L + k is Bloch-periodic and an exact
    eigenvector of the FD kinetic operator with eigenvalue T(q)."""
    grid = Grid(n=n, L=L, n_o=n_o, k=k)
    x = grid.coords()
    rng = np.random.default_rng(5)
    for _ in range(4):
        m = rng.integers(-3, 4, size=3)
        q = np.array([2 * math.pi * m[s] / L[s] + k[s] for s in range(3)])
        psi = np.exp(1j * x @ q)
        Tpsi = minus_half_laplacian(psi, grid)
        np.testing.assert_allclose(Tpsi, _symbol(q, grid) * psi, rtol=0, atol=1e-11 * max(1, abs(_symbol(q, grid))))


def test_free_electron_levels_24():
    """The 33 lowest free-electron levels of the 24^3 / L = 12 cell (Gamma) from
    the closed form, against the tabulated values with their degeneracies."""
    grid = Grid(n=(24, 24, 24), L=(12.0, 12.0, 12.0))
    levels = []
    for a in range(-3, 4):
        for b in range(-3, 4):
            for c in range(-3, 4):
                q = np.array([a, b, c]) * 2 * math.pi / 12.0
                levels.append(_symbol(q, grid))
    levels = np.sort(levels)[:33]
    ref = []
    for line in open(os.path.join(GOLD, "free_electron_24.txt")):
        if line.startswith("#") or not line.strip():
            continue
        v, d = line.split()
        ref += [float(v)] * int(d)
    np.testing.assert_allclose(levels, ref, atol=6e-7)


def _small_cell(n=(8, 9, 10), L=(4.8, 5.4, 6.0), k=(0.0, 0.0, 0.0), ls=(0, 1), seed=3, n_atoms=2, rc=1.8):
    rng = np.random.default_rng(seed)
    R = rng.uniform(0, 1, (n_atoms, 3)) * np.array(L)
    depth = rng.uniform(2, 6, n_atoms)
    width = rng.uniform(0.8, 1.5, n_atoms)
    chan_atom = np.repeat(np.arange(n_atoms), len(ls))
    chan_l = np.tile(ls, n_atoms)
    gam = rng.uniform(0.5, 2.0, len(chan_atom))
    grid = Grid(n=n, L=L, k=k)
    V = local_potential(grid, R, depth, width)
    P = projectors(grid, R, chan_atom, chan_l, gam, np.full(len(chan_atom), rc))
    return grid, V, P, (R, depth, width, chan_atom, chan_l, gam, rc)


@pytest.mark.parametrize("k", [(0.0, 0.0, 0.0), (0.31, -0.22, 0.4)])
def test_hermitian(k):
    grid, V, P, _ = _small_cell(k=k)
    rng = np.random.default_rng(1)
    X = rng.standard_normal((grid.n_d, 3)) + 1j * rng.standard_normal((grid.n_d, 3))
    Y = rng.standard_normal((grid.n_d, 3)) + 1j * rng.standard_normal((grid.n_d, 3))
    lhs = X.conj().T @ apply_H(Y, grid, V, P)
    rhs = apply_H(X, grid, V, P).conj().T @ Y
    np.testing.assert_allclose(lhs, rhs, rtol=1e-12, atol=1e-10)
    if grid.is_gamma:
        Hr = apply_H(X.real, grid, V, P)
        assert not np.iscomplexobj(Hr)


def test_time_reversal_and_reciprocal_shift():
    """H(-k) = conj H(k) for a real potential, and H(k + G) = H(k)."""
    k = (0.31, -0.22, 0.4)
    grid, V, P, prm = _small_cell(k=k)
    R, depth, width, ca, cl, gam, rc = prm
    rng = np.random.default_rng(2)
    X = rng.standard_normal((grid.n_d, 2)) + 1j * rng.standard_normal((grid.n_d, 2))
    gm = Grid(n=grid.n, L=grid.L, k=tuple(-x for x in k))
    Pm = projectors(gm, R, ca, cl, gam, np.full(len(ca), rc))
    np.testing.assert_allclose(apply_H(X.conj(), gm, V, Pm), apply_H(X, grid, V, P).conj(), atol=1e-11)
    G = tuple(k[s] + 2 * math.pi / grid.L[s] * (s + 1) for s in range(3))
    gG = Grid(n=grid.n, L=grid.L, k=G)
    PG = projectors(gG, R, ca, cl, gam, np.full(len(ca), rc))
    np.testing.assert_allclose(apply_H(X, gG, V, PG), apply_H(X, grid, V, P), atol=1e-10)


@pytest.mark.parametrize("k", [(0.0, 0.0, 0.0), (0.45, -0.3, 0.2)])
def test_translation_covariance(k):
    """Moving every atom by whole grid steps (so that projector supports and
    wells cross the cell boundary) is a unitary Bloch translation of H(k): the
    spectrum must not change.  A wrong Bloch phase on the wrapped part of a
    projector, of the potential or of the stencil breaks this."""
    n, L = (8, 8, 8), (4.8, 4.8, 4.8)
    rng = np.random.default_rng(9)
    R = np.array([[0.4, 0.7, 1.1]])
    depth, width = np.array([4.0]), np.array([0.9])
    ca, cl, gam = np.array([0, 0]), np.array([0, 1]), np.array([1.3, 0.7])
    spectra = []
    for shift in [(0, 0, 0), (5, 3, 6), (7, 1, 2)]:
        Rs = (R + np.array(shift) * 0.6) % 4.8
        grid = Grid(n=n, L=L, k=k)
        V = local_potential(grid, Rs, depth, width)
        P = projectors(grid, Rs, ca, cl, gam, np.full(2, 1.9))
        spectra.append(np.linalg.eigvalsh(dense_H(grid, V, P)))
    np.testing.assert_allclose(spectra[1], spectra[0], atol=1e-10)
    np.testing.assert_allclose(spectra[2], spectra[0], atol=1e-10)


def test_projector_normalisation_and_symmetry():
    """h^3 sum |chi|^2 = 1 when r_c < L/2; an s projector centred on a node is
    symmetric under reflections, a p_x projector odd under x -> -x."""
    grid = Grid(n=(16, 16, 16), L=(8.0, 8.0, 8.0))
    R = np.array([[4.0, 4.0, 4.0]])
    P = projectors(grid, R, [0, 0], [0, 1], [1.0, 1.0], [3.0, 3.0])
    for p in P:
        assert grid.dV * np.sum(np.abs(p["val"]) ** 2) == pytest.approx(1.0, rel=1e-13)
    full = [np.zeros(grid.n_d) for _ in P]
    for f, p in zip(full, P):
        f[p["idx"]] = p["val"]
    s3 = full[0].reshape(16, 16, 16)
    px = full[1].reshape(16, 16, 16)
    # reflection x -> 2*8 - x about node 8 (index map i -> 16 - i mod 16)
    ref = (-np.arange(16)) % 16
    np.testing.assert_allclose(s3[:, :, ref], s3, atol=1e-15)
    np.testing.assert_allclose(px[:, :, ref], -px, atol=1e-15)
    np.testing.assert_allclose(s3.transpose(0, 2, 1), s3, atol=1e-15)
    assert px[8, 8, 9] > 0 and s3[8, 8, 8] == np.max(s3)


def test_rank_one_projector_secular_equation():
    """One normalised projector in an empty cell is a rank-1 update
    T + gamma h^3 chi~ chi~^H of the plane-wave-diagonal kinetic operator: its
    eigenvalues are the levels T_m (multiplicity d-1 per d-fold level) and the
    roots of 1 = gamma h^3 sum_m |v_m^H chi~|^2 / (lambda - T_m), with v_m the
    normalised plane waves (computed here by the FFT, not by the stencil)."""
    for k in [(0.0, 0.0, 0.0), (0.37, -0.21, 0.13)]:
        n, L = (8, 8, 8), (4.0, 4.0, 4.0)
        grid = Grid(n=n, L=L, k=k)
        gamma = 1.7
        P = projectors(grid, np.array([[1.23, 3.1, 0.4]]), [0], [0], [gamma], [1.9])
        chi = np.zeros(grid.n_d, dtype=complex)
        chi[P[0]["idx"]] = P[0]["val"]
        H = dense_H(grid, np.zeros(grid.n_d), P)
        lam = np.linalg.eigvalsh(H)
        # plane-wave coefficients of chi (psi-form: v_m = e^{i(G_m + k).x}/sqrt(N_d))
        x = grid.coords()
        c3 = (chi * np.exp(-1j * x @ np.array(k))).reshape(n[2], n[1], n[0])
        coef = np.fft.fftn(c3) / math.sqrt(grid.n_d)            # v_m^H chi
        Gz = 2 * math.pi * np.fft.fftfreq(n[2], d=grid.h[2])
        Gy = 2 * math.pi * np.fft.fftfreq(n[1], d=grid.h[1])
        Gx = 2 * math.pi * np.fft.fftfreq(n[0], d=grid.h[0])
        T = np.zeros(c3.shape)
        for a in range(n[2]):
            for b in range(n[1]):
                for c in range(n[0]):
                    T[a, b, c] = _symbol(np.array([Gx[c] + k[0], Gy[b] + k[1], Gz[a] + k[2]]), grid)
        T, wgt = T.ravel(), gamma * grid.dV * np.abs(coef.ravel()) ** 2
        # group numerically equal levels
        order = np.argsort(T)
        T, wgt = T[order], wgt[order]
        levels, weights, mult = [], [], []
        for t, w in zip(T, wgt):
            if levels and abs(t - levels[-1]) < 1e-9:
                weights[-1] += w
                mult[-1] += 1
            else:
                levels.append(t)
                weights.append(w)
                mult.append(1)
        levels, weights = np.array(levels), np.array(weights)
        expect = []
        for lv, m in zip(levels, mult):
            expect += [lv] * (m - 1)

        def f(x):
            return 1.0 - np.sum(weights / (x - levels))
        # one root above each coupled level (gamma > 0): in (level_i, level_{i+1})
        for i in range(len(levels)):
            lo = levels[i]
            hi = levels[i + 1] if i + 1 < len(levels) else levels[i] + np.sum(weights) + 1.0
            if weights[i] < 1e-28:
                expect.append(levels[i])
                continue
            a, b = lo + 1e-14 * max(1, abs(lo)), hi - 1e-14 * max(1, abs(hi))
            for _ in range(200):
                mid = 0.5 * (a + b)
                if f(mid) < 0:
                    a = mid
                else:
                    b = mid
            expect.append(0.5 * (a + b))
        np.testing.assert_allclose(np.sort(expect), lam, atol=2e-9)


def test_dense_matches_apply():
    grid, V, P, _ = _small_cell(k=(0.1, 0.2, -0.3))
    H = dense_H(grid, V, P)
    rng = np.random.default_rng(4)
    X = rng.standard_normal((grid.n_d, 2)) + 1j * rng.standard_normal((grid.n_d, 2))
    np.testing.assert_allclose(H @ X, apply_H(X, grid, V, P), atol=1e-11)
    np.testing.assert_allclose(H, H.conj().T, atol=1e-12)


def test_local_potential_image_sum():
    """A single well: V at a node equals -D exp(-d^2/2w^2) summed over the
    periodic images within the cutoff (brute force over many images)."""
    grid = Grid(n=(10, 10, 10), L=(5.0, 5.0, 5.0))
    R = np.array([[0.3, 4.9, 2.5]])
    V = local_potential(grid, R, [3.0], [1.2]).reshape(10, 10, 10)
    for (i, j, kk) in [(0, 0, 0), (9, 1, 5), (4, 4, 4)]:
        x = np.array([i, j, kk]) * 0.5
        acc = 0.0
        for a in range(-5, 6):
            for b in range(-5, 6):
                for c in range(-5, 6):
                    d = np.linalg.norm(x - R[0] - 5.0 * np.array([a, b, c]))
                    if d <= 12.0:
                        acc -= 3.0 * math.exp(-d * d / (2 * 1.44))
        assert V[kk, j, i] == pytest.approx(acc, rel=1e-13)
