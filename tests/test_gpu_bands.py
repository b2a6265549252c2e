"""GPU band structure at fixed potential (sparc_band_structure: the CheFSI steps of
Sec. 3.4 repeated at every k-point, all k-points batched) against the oracle's dense
H(k) eigenvalues (Sec. 4 band structure), 1e-8 Ha; the free-electron levels of an
empty cell; the non-converged status and argument errors."""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle.bands import bands as oracle_bands
from oracle.cell import local_potential
from oracle.fd import Grid
from paper_1603_04339_amd import sparc as sp
from paper_1603_04339_amd import workloads as wl
from tests.test_oracle_bands import _fd_free_levels

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = sp.Context(0)
    yield c
    c.close()


def _starts(rng, nk, ns, nd):
    return [torch.from_numpy(rng.standard_normal((ns, nd)) + 1j * rng.standard_normal((ns, nd))).cuda()
            for _ in range(nk)]


def test_bands_match_dense_eigenvalues(ctx):
    cell, rng = wl.draw_cell(96, 0, (12, 10, 11), (6.0, 5.0, 5.5), 2, (0, 1), 2.2, 16)
    grid = Grid(n=cell.n, L=cell.L)
    veff = local_potential(grid, cell.positions, cell.depth, cell.width) + 0.3 * np.sin(
        grid.coords() @ np.array([2 * math.pi / 6.0, 0.0, 2 * math.pi / 5.5]))
    ks = np.array([[0.0, 0.0, 0.0], [math.pi / 6.0, 0.0, 0.0], [0.21, -0.33, 0.17], [-0.21, 0.33, -0.17]])
    Xs = _starts(rng, len(ks), 16, cell.n_d)
    eig, passes, st = sp.band_structure(ctx, cell, torch.from_numpy(veff).cuda(), ks, Xs, n_bands=8, degree=16,
                                        max_passes=150, tol=1e-11)
    assert st == sp.OK
    ref = oracle_bands(cell.n, cell.L, ks, veff,
                       (cell.positions, cell.chan_atom, cell.chan_l, cell.chan_gamma, cell.chan_rc), 8)
    print("passes", passes.tolist(), "max err", np.abs(eig - ref).max())
    np.testing.assert_allclose(eig, ref, atol=1e-8)
    np.testing.assert_allclose(eig[3], eig[2], atol=1e-8)        # time reversal
    # the Ritz vectors are orthonormal
    X = Xs[2].cpu().numpy()
    np.testing.assert_allclose(X.conj() @ X.T, np.eye(16), atol=1e-10)


def test_empty_cell_free_electron_levels(ctx):
    n, L = (10, 9, 8), (5.0, 4.5, 4.0)
    cell = wl.Cell(n=n, L=L, positions=np.zeros((0, 3)), depth=np.zeros(0), width=np.zeros(0),
                   chan_atom=np.zeros(0, np.int32), chan_l=np.zeros(0, np.int32), chan_gamma=np.zeros(0),
                   chan_rc=np.zeros(0), Z=np.zeros(0), n_s=20)
    ks = np.array([[0.1, -0.2, 0.3], [math.pi / 5.0, math.pi / 4.5, 0.0]])
    rng = np.random.default_rng(5)
    eig, passes, st = sp.band_structure(ctx, cell, torch.zeros(cell.n_d, dtype=torch.float64, device="cuda:0"), ks,
                                        _starts(rng, 2, 20, cell.n_d), n_bands=7, degree=16, max_passes=200,
                                        tol=1e-11)
    assert st == sp.OK
    for b, k in enumerate(ks):
        np.testing.assert_allclose(eig[b], _fd_free_levels(n, L, k, 6, 7), atol=1e-8)


def test_not_converged_and_errors(ctx):
    cell, rng = wl.draw_cell(96, 1, (12, 10, 11), (6.0, 5.0, 5.5), 2, (0,), 2.2, 8)
    grid = Grid(n=cell.n, L=cell.L)
    veff = torch.from_numpy(local_potential(grid, cell.positions, cell.depth, cell.width)).cuda()
    ks = np.zeros((1, 3))
    eig, passes, st = sp.band_structure(ctx, cell, veff, ks, _starts(rng, 1, 8, cell.n_d), n_bands=4, max_passes=1)
    assert st == sp.ENOCONV and passes.tolist() == [1] and np.all(np.isfinite(eig))
    with pytest.raises(sp.SparcError) as e:
        sp.band_structure(ctx, cell, veff, ks, _starts(rng, 1, 8, cell.n_d), n_bands=9)
    assert e.value.status == sp.ESHAPE
