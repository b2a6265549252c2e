"""Zero-Dirichlet directions on the GPU (Sec. 3.1: slabs and wires) against the
oracle: H X for every tile shape (slab and wire, real and Bloch-complex, FP64 and
FP32), the Chebyshev filter, a batched plan mixing a slab with a periodic cell, the
band structure of a slab, the atomic forces, the atomic superposition, and the
argument errors."""
import math
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle.bands import bands as oracle_bands
from oracle.chefsi import cheb_filter
from oracle.fd import apply_H, Grid
from oracle.forces import local_force, nonlocal_force
from oracle.scf import sad_density
from paper_1603_04339_amd import sparc as sp
from paper_1603_04339_amd import workloads as wl
from tests.helpers import oracle_setup, colnorm_err, to_dev, block_to_oracle

pytestmark = pytest.mark.gpu
N_TILE_SHAPES = 7


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = sp.Context(0)
    yield c
    c.close()


@pytest.fixture
def tile_env():
    old = os.environ.get("SPARC_HSTEP_TILE")
    yield
    if old is None:
        os.environ.pop("SPARC_HSTEP_TILE", None)
    else:
        os.environ["SPARC_HSTEP_TILE"] = old


def _cell(seed, bc, n=(37, 29, 21), L=(14.8, 11.6, 8.4), ls=(0, 1)):
    cell, rng = wl.draw_cell(97, seed, n, L, 3, ls, 2.2, 0)
    cell.bc = tuple(bc)
    # keep the atoms off the Dirichlet faces by a cutoff radius, as in a slab with vacuum
    for s in range(3):
        if bc[s]:
            cell.positions[:, s] = 2.5 + (L[s] - 5.0) * (cell.positions[:, s] / L[s])
    return cell, rng


@pytest.mark.parametrize("bc,dt", [((0, 0, 1), "r64"), ((0, 1, 1), "r64"), ((0, 0, 1), "c128"),
                                   ((0, 1, 1), "c128"), ((1, 1, 1), "r32"), ((0, 0, 1), "c64")])
def test_apply_every_tile(ctx, tile_env, bc, dt):
    cplx = dt.startswith("c")
    k = tuple(0.0 if bc[s] else (0.21, -0.13, 0.3)[s] for s in range(3)) if cplx else (0.0, 0.0, 0.0)
    cell, rng = _cell(1 + 3 * cplx + bc[1], bc)
    grid, V, P = oracle_setup(cell, k)
    X = rng.standard_normal((3, grid.n_d))
    if cplx:
        X = X + 1j * rng.standard_normal((3, grid.n_d))
    tdt = {"r64": torch.float64, "c128": torch.complex128, "r32": torch.float32, "c64": torch.complex64}[dt]
    ham = sp.Hamiltonian(ctx, cell, {"r64": sp.R64, "c128": sp.C128, "r32": sp.R32, "c64": sp.C64}[dt], kpt=k)
    vl = torch.zeros(grid.n_d, dtype=torch.float64, device="cuda:0")
    ham.get_vloc(vl)
    np.testing.assert_allclose(vl.cpu().numpy(), V, atol=1e-12)
    Xd = to_dev(X, tdt)
    Xr = block_to_oracle(Xd).astype(np.complex128 if cplx else np.float64)
    ref = apply_H(Xr, grid, V, P)
    w = sp.workspace(ham, 3, sp.OP_APPLY)
    single = dt in ("r32", "c64")
    for t in range(N_TILE_SHAPES):
        os.environ["SPARC_HSTEP_TILE"] = str(t)
        Y = torch.zeros_like(Xd)
        sp.fd_hamiltonian_apply(ham, Xd, Y, w)
        err = colnorm_err(block_to_oracle(Y).astype(Xr.dtype), ref)
        assert err < (2e-5 if single else 1e-12), (t, err)


def test_filter_and_mixed_batch(ctx):
    slab, rng = _cell(7, (0, 0, 1))
    per, _ = wl.draw_cell(97, 8, (24, 20, 18), (9.6, 8.0, 7.2), 2, (0,), 2.2, 0)
    k = (0.17, -0.09, 0.0)
    probs = []
    for c, kk in [(slab, k), (per, (0.1, 0.2, -0.15))]:
        grid, V, P = oracle_setup(c, kk)
        X0 = rng.standard_normal((4, grid.n_d)) + 1j * rng.standard_normal((4, grid.n_d))
        probs.append((c, kk, grid, V, P, X0))
    hams = [sp.Hamiltonian(ctx, p[0], sp.C128, kpt=p[1]) for p in probs]
    Xs = [to_dev(p[5]) for p in probs]
    plan = sp.FilterPlan(ctx, hams, Xs, [5, 4], use_graph=True)
    plan.run([3.0, 2.0], [60.0, 50.0])
    for i, (p, Xd) in enumerate(zip(probs, Xs)):
        ref = cheb_filter(p[5].T, p[2], p[3], p[4], [5, 4][i], [3.0, 2.0][i], [60.0, 50.0][i])
        assert colnorm_err(block_to_oracle(Xd), ref) < 1e-11
    plan.close()


def test_slab_band_structure(ctx):
    cell, rng = _cell(9, (0, 0, 1), n=(10, 11, 12), L=(5.0, 5.5, 6.0))
    grid = Grid(n=cell.n, L=cell.L, bc=cell.bc)
    from oracle.cell import local_potential
    veff = local_potential(grid, cell.positions, cell.depth, cell.width)
    ks = np.array([[0.0, 0.0, 0.0], [math.pi / 5.0, 0.0, 0.0], [0.2, -0.3, 0.0]])
    Xs = [torch.from_numpy(rng.standard_normal((14, cell.n_d)) + 1j * rng.standard_normal((14, cell.n_d))).cuda()
          for _ in ks]
    eig, passes, st = sp.band_structure(ctx, cell, torch.from_numpy(veff).cuda(), ks, Xs, n_bands=7, degree=16,
                                        max_passes=200, tol=1e-11)
    assert st == sp.OK
    ref = oracle_bands(cell.n, cell.L, ks, veff,
                       (cell.positions, cell.chan_atom, cell.chan_l, cell.chan_gamma, cell.chan_rc), 7, bc=cell.bc)
    np.testing.assert_allclose(eig, ref, atol=1e-8)


def test_forces_and_sad_with_dirichlet(ctx):
    cell, rng = _cell(10, (0, 1, 1), n=(20, 18, 22), L=(8.0, 7.2, 8.8))
    grid, V, P = oracle_setup(cell)
    rho = rng.uniform(0.0, 0.5, grid.n_d)
    ham = sp.Hamiltonian(ctx, cell, sp.R64)
    F = torch.zeros(3, 3, dtype=torch.float64, device="cuda:0")
    sp.forces_local(ham, to_dev(rho), F)
    X = np.linalg.qr(rng.standard_normal((grid.n_d, 9)))[0]
    occ = rng.uniform(0, 1, 9)
    sp.forces_nonlocal(ham, to_dev(np.ascontiguousarray(X.T)), to_dev(occ), F, sp.workspace(ham, 9, sp.OP_FORCES))
    ref = (local_force(grid, cell.positions, cell.depth, cell.width, rho)
           + nonlocal_force([grid], [P], [X], occ[None, :], 3))
    np.testing.assert_allclose(F.cpu().numpy(), ref, atol=1e-11 * np.abs(ref).max())
    r = torch.zeros(grid.n_d, dtype=torch.float64, device="cuda:0")
    sp.sad_density(ctx, cell, r)
    np.testing.assert_allclose(r.cpu().numpy(), sad_density(grid, cell.positions, cell.width, cell.Z, cell.n_elec),
                               rtol=1e-12, atol=1e-14)


def test_dirichlet_argument_errors(ctx):
    cell, rng = _cell(11, (0, 0, 1), n=(12, 10, 11), L=(6.0, 5.0, 5.5))
    with pytest.raises(sp.SparcError) as e:
        sp.Hamiltonian(ctx, cell, sp.C128, kpt=(0.1, 0.0, 0.2))
    assert e.value.status == sp.EINVAL
    cell.bc = (0, 0, 2)
    with pytest.raises(sp.SparcError) as e:
        sp.Hamiltonian(ctx, cell, sp.R64)
    assert e.value.status == sp.EINVAL
    cell.bc = (0, 0, 1)
    prm = dict(n_s=8, degree=10, n_first_passes=2, max_iter=2, lanczos_steps=10, mix_history=0, kT=0.01, mix=0.3,
               tol=1e-6, n_elec=cell.n_elec, poisson_tol=1e-10, filt=sp.R64, rr=sp.GEMM_NATIVE, final_fp64_pass=0,
               rho_init_dev=None, x0_dev=torch.zeros(8, cell.n_d, dtype=torch.float64, device="cuda:0"),
               lanczos_v0_dev=torch.ones(cell.n_d, dtype=torch.float64, device="cuda:0"))
    rho = torch.zeros(cell.n_d, dtype=torch.float64, device="cuda:0")
    ritz = torch.zeros(8, dtype=torch.float64, device="cuda:0")
    with pytest.raises(sp.SparcError) as e:
        sp.sparc_scf_run(ctx, cell, prm, rho, ritz)
    assert e.value.status == sp.EINVAL
