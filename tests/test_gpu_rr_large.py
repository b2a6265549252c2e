"""Rayleigh-Ritz (Sec. 3.4: projected pencil, orbital transformation) against the
oracle at the state counts of the large workloads, so that every kernel of the
GPU reduction runs under test:

* N_s 65, 200 and 512 in FP64: several 128 x 128 Gram tiles (upper triangle and its
  mirror), multi-column-tile rotations, the blocked Cholesky (panel and trailing
  update kernels, more than one 64-column block) and the blocked tridiagonal
  reduction;
* N_s 128 in complex128 at a Bloch k: the complex blocked tridiagonalisation
  (n >= 64) and the complex multi-tile contractions;
* N_s 256 in FP32 with native FP32 contractions and with split-BF16 x3 products
  (pre-split rotations, n_s a multiple of 16);
* N_s 63 (real and complex128) and 2: the LDS tridiagonal reduction of n < 64.

Blocks are filtered by the oracle and handed to both sides: either the steady state
of CheFSI (condition number ~1e2-1e3) or a random block after one strong filter pass
(~1e4).  FP64 bars: Ritz
values within 1e-8 Ha, X^H X = I within 1e-10, X^H H X diagonal within 1e-8 Ha.
Single-precision forms are compared with the oracle's Rayleigh-Ritz of the same
rounded block in FP64, as fractions of the spectral width."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle.fd import apply_H
from oracle.chefsi import cheb_filter, rayleigh_ritz, lanczos_bounds
from paper_1603_04339_amd import sparc as sp
from paper_1603_04339_amd import workloads as wl
from tests.helpers import oracle_setup, to_dev, block_to_oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = sp.Context(0)
    yield c
    c.close()


def _filtered(n, L, n_atoms, ns, cplx, k, seed, hard=False):
    """An oracle-filtered block (N_d x ns) of a drawn cell.  Mild: one degree-4 pass
    and a Rayleigh-Ritz rotation, then degree 10 cut just above the ns-th Ritz value
    (the steady state of CheFSI).  Hard: the random block filtered once with degree
    16 and the cut at the ns/4-th Ritz value, so that only a quarter of the states
    is damped and the columns align (condition number ~1e4: the first passes from a
    random start)."""
    cell, rng = wl.draw_cell(94, seed, n, L, n_atoms, (0, 1), 2.5, 0)
    grid, V, P = oracle_setup(cell, k)
    X = rng.standard_normal((grid.n_d, ns))
    if cplx:
        X = X + 1j * rng.standard_normal((grid.n_d, ns))
    v0 = rng.standard_normal(grid.n_d) + (1j * rng.standard_normal(grid.n_d) if cplx else 0.0)
    lmin, lmax = lanczos_bounds(grid, V, P, v0, 20)
    lam0, Xr = rayleigh_ritz(cheb_filter(X, grid, V, P, 4, 0.5 * (lmin + lmax), lmax), grid, V, P)
    if hard:
        Xf = cheb_filter(X, grid, V, P, 16, float(lam0[ns // 4]), lmax)
    else:
        Xf = cheb_filter(Xr, grid, V, P, 10, float(lam0[-1]), lmax)
    return cell, grid, V, P, Xf


def _check_fp64(ctx, cell, grid, V, P, Xf, k, dt):
    ns = Xf.shape[1]
    cond = np.linalg.cond(Xf)
    lam_ref, _ = rayleigh_ritz(Xf, grid, V, P)
    ham = sp.Hamiltonian(ctx, cell, dt, kpt=k)
    X = to_dev(np.ascontiguousarray(Xf.T))
    ritz = torch.zeros(ns, dtype=torch.float64, device="cuda:0")
    sp.rayleigh_ritz(ham, X, ritz, sp.workspace(ham, ns, sp.OP_RR))
    lam = ritz.cpu().numpy()
    Xo = block_to_oracle(X)
    orth = np.abs(Xo.conj().T @ Xo - np.eye(ns)).max()
    Hs = Xo.conj().T @ apply_H(Xo, grid, V, P)
    offd = np.abs(Hs - np.diag(np.diag(Hs))).max()
    dlam = np.abs(lam - lam_ref).max()
    print(f"n={grid.n} n_s={ns} dtype={dt} cond={cond:.2e}: max |dritz| {dlam:.2e} Ha, "
          f"orthonormality {orth:.2e}, off-diagonal of X^H H X {offd:.2e}", flush=True)
    np.testing.assert_allclose(lam, lam_ref, atol=1e-8, rtol=0)
    assert orth < 1e-10
    assert offd < 1e-8
    np.testing.assert_allclose(np.real(np.diag(Hs)), lam_ref, atol=1e-8, rtol=0)


@pytest.mark.parametrize("ns,n,hard", [(65, (12, 12, 12), True), (200, (14, 14, 14), True),
                                       (512, (16, 16, 16), False)], ids=["ns65-hard", "ns200-hard", "ns512"])
def test_rr_fp64_large(ctx, ns, n, hard):
    print(f"\n[rr fp64] n={n} n_s={ns} hard={hard}", flush=True)
    L = tuple(0.5 * m for m in n)
    cell, grid, V, P, Xf = _filtered(n, L, 4, ns, False, (0.0, 0.0, 0.0), ns, hard)
    _check_fp64(ctx, cell, grid, V, P, Xf, (0.0, 0.0, 0.0), sp.R64)


@pytest.mark.parametrize("ns,cplx", [(63, False), (63, True), (2, False)], ids=["ns63", "ns63-c128", "ns2"])
def test_rr_small_tridiagonalisation(ctx, ns, cplx):
    """N_s below 64: the tridiagonal reduction with the matrix in LDS (four waves, the
    columns dealt out mod 4, including a last partial round), the back-transformation
    with the column in registers, at the largest size of that path (63, real and
    complex at a Bloch k) and at the smallest with a reflector (2)."""
    k = (0.2, -0.15, 0.3) if cplx else (0.0, 0.0, 0.0)
    n = (12, 12, 12)
    print(f"\n[rr small] n={n} n_s={ns} complex={cplx}", flush=True)
    cell, grid, V, P, Xf = _filtered(n, (6.0, 6.0, 6.0), 3, ns, cplx, k, 11 + ns, hard=(ns > 8))
    _check_fp64(ctx, cell, grid, V, P, Xf, k, sp.C128 if cplx else sp.R64)


def test_rr_complex128_ns128(ctx):
    k = (0.2, -0.15, 0.3)
    n = (12, 12, 14)
    print(f"\n[rr c128] n={n} n_s=128 k={k}", flush=True)
    cell, grid, V, P, Xf = _filtered(n, (6.0, 6.0, 7.0), 3, 128, True, k, 7, hard=True)
    _check_fp64(ctx, cell, grid, V, P, Xf, k, sp.C128)


def test_rr_fp32_ns256(ctx):
    """FP32 block, N_s 256: native FP32 contractions within 1e-5 and split-BF16 x3
    within 1e-4 of the spectral width of the FP64 result on the same rounded block;
    orthonormality within 1e-5 / 1e-4."""
    n = (16, 16, 16)
    print(f"\n[rr fp32] n={n} n_s=256", flush=True)
    cell, grid, V, P, Xf = _filtered(n, (8.0, 8.0, 8.0), 4, 256, False, (0.0, 0.0, 0.0), 3)
    Xf = Xf / np.linalg.norm(Xf, axis=0)
    X32 = Xf.astype(np.float32)
    lam_ref, _ = rayleigh_ritz(X32.astype(np.float64), grid, V, P)
    width = float(lam_ref[-1] - lam_ref[0])
    ham = sp.Hamiltonian(ctx, cell, sp.R32)
    res = {}
    for name, mode in (("native", sp.GEMM_NATIVE), ("x3", sp.GEMM_BF16X3)):
        X = to_dev(np.ascontiguousarray(X32.T))
        ritz = torch.zeros(256, dtype=torch.float64, device="cuda:0")
        sp.rayleigh_ritz(ham, X, ritz, sp.workspace(ham, 256, sp.OP_RR), mode)
        lam = ritz.cpu().numpy()
        Xo = block_to_oracle(X).astype(np.float64)
        err = float(np.abs(lam - lam_ref).max() / width)
        orth = float(np.abs(Xo.T @ Xo - np.eye(256)).max())
        res[name] = (err, orth)
        print(f"fp32 n_s=256 {name}: max |dritz| / width {err:.2e}, orthonormality {orth:.2e}", flush=True)
    assert res["native"][0] < 1e-5 and res["native"][1] < 1e-5
    assert res["x3"][0] < 1e-4 and res["x3"][1] < 1e-4


@pytest.mark.parametrize("well", [True, False], ids=["one_pass", "two_passes"])
def test_rr_pass_selection(ctx, well):
    """The number of Cholesky-QR passes follows the conditioning of the column-scaled
    Gram matrix: a block with orthogonal columns (scaled over six decades) takes one
    pass (two N-long Grams plus the small projected product), an aligned block two
    (three plus one); both meet the FP64 bars against the oracle."""
    cell, grid, V, P, Xf = _filtered((12, 12, 14), (6.0, 6.0, 7.0), 4, 65, False, (0.0, 0.0, 0.0), 7,
                                     hard=not well)
    if well:
        Q, _ = np.linalg.qr(Xf)
        Xf = Q * np.logspace(-3, 3, Q.shape[1])[None, :]
    G = Xf.T @ Xf
    d = 1.0 / np.sqrt(np.diag(G))
    kappa = np.linalg.cond(G * d[:, None] * d[None, :])
    ns = Xf.shape[1]
    lam_ref, _ = rayleigh_ritz(Xf, grid, V, P)
    ham = sp.Hamiltonian(ctx, cell, sp.R64)
    X = to_dev(np.ascontiguousarray(Xf.T))
    ritz = torch.zeros(ns, dtype=torch.float64, device="cuda:0")
    ctx.set_timing(True)
    sp.rayleigh_ritz(ham, X, ritz, sp.workspace(ham, ns, sp.OP_RR))
    torch.cuda.synchronize()
    _, n_gram = ctx.kernel_time("gram")
    ctx.set_timing(False)
    lam = ritz.cpu().numpy()
    Xo = block_to_oracle(X)
    orth = np.abs(Xo.T @ Xo - np.eye(ns)).max()
    Hs = Xo.T @ apply_H(Xo, grid, V, P)
    offd = np.abs(Hs - np.diag(np.diag(Hs))).max()
    dlam = np.abs(lam - lam_ref).max()
    print(f"\n[rr passes] well={well} kappa(scaled Gram)={kappa:.2e} grams={n_gram}: |dritz| {dlam:.2e}, "
          f"orthonormality {orth:.2e}, off-diagonal {offd:.2e}", flush=True)
    if well:
        assert kappa < 10 and n_gram == 3
    else:
        assert kappa > 1e3 and n_gram == 4
    assert dlam < 1e-8 and orth < 1e-10 and offd < 1e-8
