"""Pins of the pseudocharge oracle (Sec. 2 electrostatic reformulation; Sec. 3.2,
Algorithm 1 and the truncation rule; Appendix A, E_c and f_c; Sec. 3.6 local force)
against what the mathematics fixes:
  * the synthetic potential solves the radial Poisson equation of its charge, is
    continuous with its derivative at rc, and the charge integrates to -Z (quadrature);
  * the closed-form self energy and background integral against quadrature;
  * b^h equals -(1/4pi) times the FD Laplacian operator of Sec. 3.1 (the Hamiltonian's
    kinetic stencil) applied to the sampled potential;
  * the chosen truncation box is the smallest that meets eps_b (brute force over boxes);
  * E_self^h converges to the closed form as h -> 0;
  * the textbook Ewald sum of point charges in a uniform background (written here,
    independently of the oracle): E_el + E_c and f_loc + f_c of overlapping
    pseudocharges with a uniform electron density equal the point-charge energy and
    forces (plus the closed-form background term), to the discretisation error;
  * the exact discrete identity E_el(b) + E_c = E_el(b~) - h^3 <rho, V_c>;
  * f_loc + f_c against central differences of E_el + E_c at fixed density;
  * an oracle SCF with pseudocharges converges and its total force is the slope of
    its free energy.
"""
import math

import numpy as np
import pytest
from scipy import integrate
from scipy.special import erfc

from oracle import pseudocharge as pc
from oracle.fd import Grid, apply_H


def ewald(R, q, L, eta=None, nr=4, ng=12):
    """Energy and forces of point charges q at R in a periodic cuboid with a uniform
    neutralising background (real-space erfc sum, reciprocal sum, self and
    background terms)."""
    L = np.asarray(L, float)
    om = float(L.prod())
    N = len(q)
    eta = 5.0 / L.min() if eta is None else eta
    E = 0.0
    F = np.zeros((N, 3))
    rng = range(-nr, nr + 1)
    for a in rng:
        for b in rng:
            for c in rng:
                sh = np.array([a, b, c]) * L
                for i in range(N):
                    for j in range(N):
                        if a == b == c == 0 and i == j:
                            continue
                        d = R[i] - R[j] - sh
                        r = float(np.linalg.norm(d))
                        E += 0.5 * q[i] * q[j] * erfc(eta * r) / r
                        F[i] += q[i] * q[j] * (erfc(eta * r) / r ** 2
                                               + 2 * eta / math.sqrt(math.pi) * math.exp(-(eta * r) ** 2) / r) * d / r
    rg = range(-ng, ng + 1)
    for a in rg:
        for b in rg:
            for c in rg:
                if a == b == c == 0:
                    continue
                G = 2 * math.pi * np.array([a, b, c]) / L
                G2 = float(G @ G)
                f = math.exp(-G2 / (4 * eta * eta)) / G2
                S = np.sum(q * np.exp(1j * (R @ G)))
                E += 2 * math.pi / om * f * abs(S) ** 2
                for i in range(N):
                    F[i] += 4 * math.pi / om * q[i] * f * G * np.imag(np.exp(1j * (R[i] @ G)) * np.conj(S))
    E += -eta / math.sqrt(math.pi) * float(np.sum(q * q)) - math.pi * float(q.sum()) ** 2 / (2 * om * eta * eta)
    return E, F


CELL = dict(R=np.array([[1.1, 2.3, 3.7], [3.9, 3.2, 4.6], [6.0, 6.9, 1.5]]),
            Z=np.array([2.0, 3.0, 1.0]), rc=np.array([2.2, 2.4, 1.8]), rr=np.array([1.0, 1.1, 0.9]),
            L=(9.0, 9.0, 9.0))


def _setup(grid, c, eps_b=1e-8):
    bx = pc.truncation_boxes(grid, c["R"], c["Z"], c["rc"], eps_b)
    bxr = pc.truncation_boxes(grid, c["R"], c["Z"], c["rr"], eps_b)
    return bx, bxr, pc.electrostatics_setup(grid, c["R"], c["Z"], c["rc"], c["rr"], bx, bxr)


def test_potential_solves_radial_poisson():
    Z, rc = 2.5, 1.7
    dr = 1e-3
    for r in (0.2, 0.7, 1.3, 1.69, 1.71, 2.5, 4.0):
        f = lambda x: pc.v_pseudo(x, Z, rc)
        lap = ((r + dr) ** 2 * (f(r + 2 * dr) - f(r)) / (2 * dr)
               - (r - dr) ** 2 * (f(r) - f(r - 2 * dr)) / (2 * dr)) / (2 * dr) / r ** 2
        assert abs(-lap / (4 * math.pi) - pc.b_continuous(r, Z, rc)) < 1e-5 * Z / rc ** 3
    # value and slope continuous at rc, Coulomb outside
    assert abs(pc.v_pseudo(rc * (1 - 1e-12), Z, rc) + Z / rc) < 1e-10
    slope_in = (pc.v_pseudo(rc - 1e-6, Z, rc) - pc.v_pseudo(rc - 2e-6, Z, rc)) / 1e-6
    assert abs(slope_in - Z / rc ** 2) < 1e-5
    assert pc.v_pseudo(3.0, Z, rc) == -Z / 3.0
    q, _ = integrate.quad(lambda r: 4 * math.pi * r * r * pc.b_continuous(r, Z, rc), 0, rc)
    assert abs(q + Z) < 1e-12


def test_closed_forms_against_quadrature():
    for Z, rc in ((1.0, 1.0), (2.0, 2.3), (3.0, 1.4)):
        es, _ = integrate.quad(lambda r: 0.5 * 4 * math.pi * r * r * pc.b_continuous(r, Z, rc)
                               * pc.v_pseudo(r, Z, rc), 0, rc, epsabs=1e-14)
        assert abs(pc.self_energy_continuous(Z, rc) - es) < 1e-12
        bg, _ = integrate.quad(lambda r: 4 * math.pi * r * r * (pc.v_pseudo(r, Z, rc) + Z / r), 0, rc, epsabs=1e-14)
        assert abs(pc.background_integral(Z, rc) - bg) < 1e-12


def test_pseudocharge_is_fd_laplacian_of_sampled_potential():
    """One atom in a zero-Dirichlet cell: inside its box, away from the faces, b^h equals
    -(1/4pi) Lap_h V with Lap_h = -2 (H with zero potential and no projectors)."""
    grid = Grid((30, 28, 32), (10.0, 9.8, 10.4), bc=(1, 1, 1))
    R = np.array([[5.13, 4.77, 5.31]])
    Z, rc = np.array([2.0]), np.array([2.1])
    box = pc.truncation_boxes(grid, R, Z, rc, 1e-8)
    b, eself = pc._pseudocharge_sum(grid, R, Z, rc, box)
    x = grid.coords()
    V = pc.v_pseudo(np.linalg.norm(x - R[0], axis=1), 2.0, 2.1)
    lapV = -2.0 * apply_H(V[:, None], grid, np.zeros(grid.n_d), [])[:, 0]
    n1, n2, n3 = grid.n
    h = grid.h
    inner = np.ones(grid.n_d, bool)
    for s, idx in enumerate((np.arange(grid.n_d) % n1, (np.arange(grid.n_d) // n1) % n2,
                             np.arange(grid.n_d) // (n1 * n2))):
        u = R[0][s] / h[s]
        inner &= (idx >= math.ceil(u) - box[0][s]) & (idx <= math.floor(u) + box[0][s])
        inner &= (idx >= grid.n_o) & (idx < grid.n[s] - grid.n_o)
    assert inner.sum() > 1000
    np.testing.assert_allclose(b[inner], -lapV[inner] / (4 * math.pi), rtol=0, atol=1e-12 * np.abs(b).max())
    assert abs(eself - 0.5 * grid.dV * float(np.sum(b * V))) < 1e-12


def test_truncation_box_is_smallest_meeting_eps_b():
    grid = Grid((36, 36, 36), (12.0, 12.0, 12.0), bc=(1, 1, 1))
    R = np.array([[6.07, 5.88, 6.21]])
    for Z, rc, eps in ((2.0, 2.0, 1e-8), (3.0, 1.5, 1e-6), (1.0, 2.6, 1e-10)):
        m = pc.truncation_box(grid, R[0], Z, rc, eps)
        q = lambda mm: grid.dV * pc._pseudocharge_sum(grid, R, np.array([Z]), np.array([rc]), [mm])[0].sum()
        assert abs(q(m) + Z) < eps * Z
        if m[0] > math.ceil(rc / grid.h[0]):
            assert abs(q(tuple(v - 1 for v in m)) + Z) >= eps * Z


def test_self_energy_converges_to_closed_form():
    Z, rc = 2.0, 2.0
    errs = []
    for n in (16, 24, 32):
        grid = Grid((n, n, n), (8.0, 8.0, 8.0))
        R = np.array([[3.91, 4.17, 4.03]])
        box = pc.truncation_boxes(grid, R, np.array([Z]), np.array([rc]), 1e-10)
        _, es = pc._pseudocharge_sum(grid, R, np.array([Z]), np.array([rc]), box)
        errs.append(abs(es - pc.self_energy_continuous(Z, rc)))
    assert errs[2] < errs[0] and errs[2] < 1e-5 * pc.self_energy_continuous(Z, rc)


@pytest.fixture(scope="module")
def ewald_case():
    c = CELL
    grid = Grid((24, 24, 24), c["L"])
    bx, bxr, st = _setup(grid, c)
    rho0 = c["Z"].sum() / np.prod(c["L"])
    rho = np.full(grid.n_d, rho0)
    phi = pc.electrostatic_potential(grid, rho, st["b"])
    return grid, bx, bxr, st, rho, phi


def test_energy_matches_ewald(ewald_case):
    grid, bx, bxr, st, rho, phi = ewald_case
    c = CELL
    assert abs(grid.dV * st["b"].sum() + c["Z"].sum()) < 1e-8 * c["Z"].sum()
    E = pc.electrostatic_energy(grid, rho, st, phi)
    Ee, _ = ewald(c["R"], c["Z"], c["L"])
    ref = Ee + rho[0] * sum(pc.background_integral(c["Z"][j], c["rc"][j]) for j in range(3))
    assert abs(st["ec"]) > 5e-4            # the pseudocharges overlap: the correction matters
    assert abs(E - ref) < 5e-7
    assert abs(E - st["ec"] - ref) > 5e-4


def test_forces_match_ewald(ewald_case):
    grid, bx, bxr, st, rho, phi = ewald_case
    c = CELL
    Fl = pc.local_force(grid, c["R"], c["Z"], c["rc"], bx, phi)
    Fc = pc.correction_force(grid, c["R"], c["Z"], c["rc"], c["rr"], bx, bxr, st)
    _, Fe = ewald(c["R"], c["Z"], c["L"])
    assert np.abs(Fc).max() > 2e-3
    assert np.abs(Fl + Fc - Fe).max() < 1e-4
    assert np.abs(Fl - Fe).max() > 2e-3


def test_correction_identity(ewald_case):
    """E_el(b) + E_c = E_el(b~) - h^3 <rho, V_c> (b~ - b = -Lap_h V_c / 4pi up to the
    truncated tails), with a non-uniform neutral density."""
    grid, bx, bxr, st, _, _ = ewald_case
    x = grid.coords()
    rho = np.exp(-np.sum((x - 4.5) ** 2, axis=1) / 6.0) + 0.05
    rho *= CELL["Z"].sum() / (grid.dV * rho.sum())
    lhs = pc.electrostatic_energy(grid, rho, st)
    phir = pc.electrostatic_potential(grid, rho, st["bref"])
    rhs = 0.5 * grid.dV * float(np.dot(rho + st["bref"], phir)) - st["eself_ref"] - grid.dV * float(np.dot(rho, st["vc"]))
    assert abs(lhs - rhs) < 1e-7


def test_forces_match_energy_differences_at_fixed_density():
    c = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in CELL.items()}
    grid = Grid((24, 24, 24), c["L"])
    x = grid.coords()
    rho = np.exp(-np.sum((x - np.array([4.0, 5.0, 4.4])) ** 2, axis=1) / 5.0) + 0.03
    rho *= c["Z"].sum() / (grid.dV * rho.sum())

    def energy(cc):
        _, _, st = _setup(grid, cc)
        return pc.electrostatic_energy(grid, rho, st)

    bx, bxr, st = _setup(grid, c)
    phi = pc.electrostatic_potential(grid, rho, st["b"])
    F = pc.local_force(grid, c["R"], c["Z"], c["rc"], bx, phi) + pc.correction_force(
        grid, c["R"], c["Z"], c["rc"], c["rr"], bx, bxr, st)
    d = 1e-3
    for J, s in ((0, 0), (1, 2)):
        e = []
        for sign in (1, -1):
            cc = dict(c, R=c["R"].copy())
            cc["R"][J, s] += sign * d
            e.append(energy(cc))
        fd = -(e[0] - e[1]) / (2 * d)
        assert abs(F[J, s]) > 1e-2
        assert abs(F[J, s] - fd) < 2e-4 * max(1.0, abs(fd))


def test_oracle_scf_with_pseudocharges_forces_are_energy_slopes():
    """The oracle SCF in pseudocharge mode converges, and the total force on one atom
    (f_loc + f_c + f_nloc on its converged state) is the slope of its free energy to the
    FD-gradient error of the projector cut-off (bound 1e-3 Ha/bohr)."""
    from oracle.forces import nonlocal_force
    from oracle.scf import scf, sad_density
    from paper_1603_04339_amd import workloads as wl
    from tests.helpers import oracle_setup

    base, rng = wl.draw_cell(95, 0, 20, 7.0, 2, (0,), 2.4, 8)
    X0 = wl.draw_orbitals(rng, base.n_d, 8).T
    v0 = wl.lanczos_start(rng, base.n_d)

    def run(cell):
        grid, _, P = oracle_setup(cell)
        bx = pc.truncation_boxes(grid, cell.positions, cell.Z, cell.psd_rc, 1e-8)
        bxr = pc.truncation_boxes(grid, cell.positions, cell.Z, cell.psd_rc_ref, 1e-8)
        st = pc.electrostatics_setup(grid, cell.positions, cell.Z, cell.psd_rc, cell.psd_rc_ref, bx, bxr)
        rho0 = sad_density(grid, cell.positions, cell.width, cell.Z, cell.n_elec)
        out = scf(grid, np.zeros(grid.n_d), P, X0, cell.n_elec, 16, kT=0.01, mix=0.3, tol=1e-9, max_iter=100,
                  n_first_passes=6, rho_init=rho0, lanczos_v0=v0, mix_history=7, psd=st)
        assert out["converged"]
        return out, grid, P, bx, bxr, st

    out, grid, P, bx, bxr, st = run(base)
    c = base
    F = (pc.local_force(grid, c.positions, c.Z, c.psd_rc, bx, out["phi"])
         + pc.correction_force(grid, c.positions, c.Z, c.psd_rc, c.psd_rc_ref, bx, bxr, st)
         + nonlocal_force([grid], [P], [out["X"]], out["occ"][None, :], 2))
    assert np.abs(F.sum(axis=0)).max() < 1e-4
    d = 2e-3
    e = []
    for sign in (1, -1):
        cc = wl.Cell(**{**base.__dict__, "positions": base.positions.copy()})
        cc.positions[0, 2] += sign * d
        e.append(run(cc)[0]["energy"])
    fd = -(e[0] - e[1]) / (2 * d)
    assert abs(F[0, 2]) > 3e-3
    assert abs(F[0, 2] - fd) < 1e-3
