"""Edge cases of the GPU path against the oracle: Rayleigh-Ritz with one and three
states (real and complex), Rayleigh-Ritz on FP32 blocks (FP32 MFMA contractions,
FP64 Cholesky and eigensolver), a 64-state block (the blocked tridiagonal
reduction and the multisection eigenvalues on their smallest size), a filter
plan holding a single problem of degree 1, and the Bloch factor at the zone
boundary k = pi / L in FP32, and every stencil tile shape (single and batched)."""
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle.fd import apply_H
from oracle.chefsi import cheb_filter, rayleigh_ritz
from paper_1603_04339_amd import sparc as sp
from paper_1603_04339_amd import workloads as wl
from tests.helpers import oracle_setup, colnorm_err, to_dev, block_to_oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = sp.Context(0)
    yield c
    c.close()


def _cell(seed, n=(12, 10, 11), L=(6.0, 5.0, 5.5)):
    cell, rng = wl.draw_cell(93, seed, n, L, 3, (0, 1), 2.0, 0)
    return cell, rng


@pytest.mark.parametrize("ns,cplx", [(1, False), (3, False), (1, True), (3, True)])
def test_rayleigh_ritz_few_states(ctx, ns, cplx):
    k = (0.2, -0.1, 0.3) if cplx else (0.0, 0.0, 0.0)
    cell, rng = _cell(ns + 10 * cplx)
    grid, V, P = oracle_setup(cell, k)
    X = rng.standard_normal((ns, grid.n_d))
    if cplx:
        X = X + 1j * rng.standard_normal((ns, grid.n_d))
    Xf = cheb_filter(X.T, grid, V, P, 6, 5.0, 80.0)
    lam, _ = rayleigh_ritz(Xf, grid, V, P)
    ham = sp.Hamiltonian(ctx, cell, sp.C128 if cplx else sp.R64, kpt=k)
    Xd = to_dev(np.ascontiguousarray(Xf.T))
    ritz = torch.zeros(ns, dtype=torch.float64, device="cuda:0")
    sp.rayleigh_ritz(ham, Xd, ritz, sp.workspace(ham, ns, sp.OP_RR))
    np.testing.assert_allclose(ritz.cpu().numpy(), lam, atol=1e-8)
    Xo = block_to_oracle(Xd)
    np.testing.assert_allclose(Xo.conj().T @ Xo, np.eye(ns), atol=1e-10)


def test_rayleigh_ritz_64_states(ctx):
    cell, rng = _cell(20, n=(16, 14, 15), L=(8.0, 7.0, 7.5))
    grid, V, P = oracle_setup(cell)
    X = rng.standard_normal((64, grid.n_d))
    Xf = cheb_filter(X.T, grid, V, P, 10, 3.0, 60.0)
    lam, _ = rayleigh_ritz(Xf, grid, V, P)
    ham = sp.Hamiltonian(ctx, cell, sp.R64)
    Xd = to_dev(np.ascontiguousarray(Xf.T))
    ritz = torch.zeros(64, dtype=torch.float64, device="cuda:0")
    sp.rayleigh_ritz(ham, Xd, ritz, sp.workspace(ham, 64, sp.OP_RR))
    np.testing.assert_allclose(ritz.cpu().numpy(), lam, atol=1e-8)


@pytest.mark.parametrize("cplx", [False, True])
def test_rayleigh_ritz_fp32(ctx, cplx):
    """FP32 block: Ritz values within 1e-4 Ha of the FP64 oracle for a mildly
    filtered block (cond ~ 1e2), orthonormal to FP32 accuracy."""
    k = (0.15, 0.0, -0.2) if cplx else (0.0, 0.0, 0.0)
    cell, rng = _cell(30 + cplx)
    grid, V, P = oracle_setup(cell, k)
    ns = 12
    X = rng.standard_normal((ns, grid.n_d))
    if cplx:
        X = X + 1j * rng.standard_normal((ns, grid.n_d))
    Xf = cheb_filter(X.T, grid, V, P, 3, 10.0, 80.0)
    lam, _ = rayleigh_ritz(Xf, grid, V, P)
    ham = sp.Hamiltonian(ctx, cell, sp.C64 if cplx else sp.R32, kpt=k)
    Xd = to_dev(np.ascontiguousarray(Xf.T), torch.complex64 if cplx else torch.float32)
    ritz = torch.zeros(ns, dtype=torch.float64, device="cuda:0")
    sp.rayleigh_ritz(ham, Xd, ritz, sp.workspace(ham, ns, sp.OP_RR))
    err = np.abs(ritz.cpu().numpy() - lam).max()
    print(f"FP32 Ritz max error {err:.2e} Ha")
    assert err < 1e-4 * max(1.0, np.abs(lam).max())
    Xo = block_to_oracle(Xd).astype(np.complex128 if cplx else np.float64)
    np.testing.assert_allclose(Xo.conj().T @ Xo, np.eye(ns), atol=1e-5)


def test_single_problem_plan_degree_one(ctx):
    cell, rng = _cell(40)
    grid, V, P = oracle_setup(cell)
    X0 = rng.standard_normal((5, grid.n_d))
    ham = sp.Hamiltonian(ctx, cell, sp.R64)
    Xd = to_dev(X0)
    plan = sp.FilterPlan(ctx, [ham], [Xd], [1], use_graph=True)
    for lc, lm in [(1.0, 50.0), (4.0, 40.0)]:
        Xd.copy_(to_dev(X0))
        plan.run([lc], [lm])
        ref = cheb_filter(X0.T, grid, V, P, 1, lc, lm)
        assert colnorm_err(block_to_oracle(Xd), ref) < 1e-12
    plan.close()


def test_zone_boundary_bloch_fp32(ctx):
    """k_s = pi / L_s: the wrap factor is -1 in every direction."""
    cell, rng = _cell(50)
    k = tuple(np.pi / l for l in cell.L)
    grid, V, P = oracle_setup(cell, k)
    X = (rng.standard_normal((4, grid.n_d)) + 1j * rng.standard_normal((4, grid.n_d)))
    ham = sp.Hamiltonian(ctx, cell, sp.C64, kpt=k)
    Xd = to_dev(X, torch.complex64)
    Y = torch.zeros_like(Xd)
    sp.fd_hamiltonian_apply(ham, Xd, Y, sp.workspace(ham, 4, sp.OP_APPLY))
    ref = apply_H(X.T.astype(np.complex64).astype(np.complex128), grid, V, P)
    assert colnorm_err(block_to_oracle(Y).astype(np.complex128), ref) < 2e-5


N_TILE_SHAPES = 7   # stencil tile shapes the library can launch (indices 0..6)


@pytest.fixture
def tile_env():
    old = os.environ.get("SPARC_HSTEP_TILE")
    yield
    if old is None:
        os.environ.pop("SPARC_HSTEP_TILE", None)
    else:
        os.environ["SPARC_HSTEP_TILE"] = old


@pytest.mark.parametrize("dt", ["r64", "c128", "r32", "c64"])
def test_every_tile_shape(ctx, tile_env, dt):
    """Every tile shape on a grid that none of them
    divides, with Bloch phases for the complex types, against the oracle."""
    cplx = dt.startswith("c")
    k = (0.21, -0.13, 0.3) if cplx else (0.0, 0.0, 0.0)
    cell, rng = _cell(60, n=(37, 29, 21), L=(14.8, 11.6, 8.4))
    grid, V, P = oracle_setup(cell, k)
    X = rng.standard_normal((3, grid.n_d))
    if cplx:
        X = X + 1j * rng.standard_normal((3, grid.n_d))
    single = dt in ("r32", "c64")
    tdt = {"r64": torch.float64, "c128": torch.complex128, "r32": torch.float32, "c64": torch.complex64}[dt]
    ham = sp.Hamiltonian(ctx, cell, {"r64": sp.R64, "c128": sp.C128, "r32": sp.R32, "c64": sp.C64}[dt], kpt=k)
    Xd = to_dev(X, tdt)
    Xr = block_to_oracle(Xd).astype(np.complex128 if cplx else np.float64)
    ref = apply_H(Xr, grid, V, P)
    w = sp.workspace(ham, 3, sp.OP_APPLY)
    for t in range(N_TILE_SHAPES):
        os.environ["SPARC_HSTEP_TILE"] = str(t)
        Y = torch.zeros_like(Xd)
        sp.fd_hamiltonian_apply(ham, Xd, Y, w)
        err = colnorm_err(block_to_oracle(Y).astype(Xr.dtype), ref)
        print(f"{dt} tile {t}: {err:.2e}")
        assert err < (2e-5 if single else 1e-12)


def test_every_tile_shape_batched(ctx, tile_env):
    """Batched filter plans with every tile shape: two uneven real problems."""
    probs = []
    for s, (n, L) in enumerate([((37, 29, 21), (14.8, 11.6, 8.4)), ((24, 20, 18), (9.6, 8.0, 7.2))]):
        cell, rng = _cell(70 + s, n=n, L=L)
        grid, V, P = oracle_setup(cell)
        probs.append((cell, grid, V, P, rng.standard_normal((4 + s, grid.n_d))))
    for t in range(N_TILE_SHAPES):
        os.environ["SPARC_HSTEP_TILE"] = str(t)
        hams = [sp.Hamiltonian(ctx, p[0], sp.R64) for p in probs]
        Xs = [to_dev(p[4]) for p in probs]
        plan = sp.FilterPlan(ctx, hams, Xs, [4, 3], use_graph=False)
        plan.run([2.0, 3.0], [60.0, 50.0])
        for i, (p, Xd) in enumerate(zip(probs, Xs)):
            ref = cheb_filter(p[4].T, p[1], p[2], p[3], [4, 3][i], [2.0, 3.0][i], [60.0, 50.0][i])
            err = colnorm_err(block_to_oracle(Xd), ref)
            print(f"batched tile {t} problem {i}: {err:.2e}")
            assert err < 1e-12
        plan.close()


@pytest.mark.parametrize("dt,k,bc", [("r64", (0.0, 0.0, 0.0), (0, 0, 1)), ("c128", (0.21, -0.13, 0.3), (0, 0, 0)),
                                     ("r32", (0.0, 0.0, 0.0), (1, 0, 0)), ("c64", (0.17, 0.0, -0.29), (0, 1, 0))],
                         ids=["r64_zslab", "c128_bloch", "r32_xslab", "c64_bloch_yslab"])
def test_point_form_matches_tiled_and_oracle(ctx, tile_env, dt, k, bc):
    """A step whose tiled launch would leave CUs idle runs one thread per (node,
    orbital); a forced tile shape keeps the tiled kernel.  Both against the oracle H X
    on a grid no tile divides, with Bloch phases and a Dirichlet direction, and against
    each other."""
    cplx = dt.startswith("c")
    cell, rng = _cell(61, n=(37, 29, 21), L=(14.8, 11.6, 8.4))
    cell.bc = bc
    kk = tuple(0.0 if b else kv for kv, b in zip(k, bc))
    grid, V, P = oracle_setup(cell, kk)
    X = rng.standard_normal((3, grid.n_d))
    if cplx:
        X = X + 1j * rng.standard_normal((3, grid.n_d))
    single = dt in ("r32", "c64")
    tdt = {"r64": torch.float64, "c128": torch.complex128, "r32": torch.float32, "c64": torch.complex64}[dt]
    ham = sp.Hamiltonian(ctx, cell, {"r64": sp.R64, "c128": sp.C128, "r32": sp.R32, "c64": sp.C64}[dt], kpt=kk)
    Xd = to_dev(X, tdt)
    Xr = block_to_oracle(Xd).astype(np.complex128 if cplx else np.float64)
    ref = apply_H(Xr, grid, V, P)
    w = sp.workspace(ham, 3, sp.OP_APPLY)
    os.environ.pop("SPARC_HSTEP_TILE", None)
    Yp = torch.zeros_like(Xd)
    sp.fd_hamiltonian_apply(ham, Xd, Yp, w)   # 3 orbitals on a small grid: the point form
    os.environ["SPARC_HSTEP_TILE"] = "1"
    Yt = torch.zeros_like(Xd)
    sp.fd_hamiltonian_apply(ham, Xd, Yt, w)   # the tiled kernel, 32 x 16
    ep = colnorm_err(block_to_oracle(Yp).astype(Xr.dtype), ref)
    et = colnorm_err(block_to_oracle(Yt).astype(Xr.dtype), ref)
    ept = colnorm_err(block_to_oracle(Yp).astype(Xr.dtype), block_to_oracle(Yt).astype(Xr.dtype))
    print(f"{dt} bc={bc}: point {ep:.2e}, tiled {et:.2e}, point vs tiled {ept:.2e}")
    tol = 2e-5 if single else 1e-12
    assert ep < tol and et < tol and ept < tol
