"""The allocation-free H X entry point (projections held in the library's static device
array) against fd_hamiltonian_apply with a caller workspace, on two calls in a row, the
second with a smaller input, for real and Bloch-complex Hamiltonians and with the
projector scatter inside the stencil step; sizes beyond the array are refused."""
import ctypes as C
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle.fd import apply_H
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


def _ham(ctx, cell, dt, k, fused=None):
    old = os.environ.get("SPARC_NL_FUSED")
    if fused is not None:
        os.environ["SPARC_NL_FUSED"] = "1" if fused else "0"
    try:
        return sp.Hamiltonian(ctx, cell, dt, kpt=k)
    finally:
        if old is None:
            os.environ.pop("SPARC_NL_FUSED", None)
        else:
            os.environ["SPARC_NL_FUSED"] = old


def _pair(ham, X):
    """Y from the workspace entry point and from the allocation-free one."""
    ns = X.shape[0]
    Y0 = torch.full_like(X, float("nan"))
    sp.fd_hamiltonian_apply(ham, X, Y0, sp.workspace(ham, ns, sp.OP_APPLY))
    Y1 = torch.full_like(X, float("nan"))
    sp.fd_hamiltonian_apply_noalloc(ham, X, Y1)
    torch.cuda.synchronize()
    return block_to_oracle(Y0), block_to_oracle(Y1)


CASES = [(sp.R64, (0.0, 0.0, 0.0), None, 1e-12), (sp.C128, (0.2, -0.1, 0.3), None, 1e-12),
         (sp.R32, (0.0, 0.0, 0.0), None, 2e-5), (sp.R64, (0.0, 0.0, 0.0), True, 1e-12)]


@pytest.mark.parametrize("dt,k,fused,tol", CASES, ids=["r64", "c128", "r32", "r64_fused"])
def test_noalloc_matches_workspace_entry_point(ctx, dt, k, fused, tol):
    cplx = dt in (sp.C128, sp.C64)
    tdt = sp.TORCH_DTYPE[dt]
    # first call: six s+p atoms (24 projectors) on a 16x16x18 grid, 40 states
    cell, rng = wl.draw_cell(97, 1, (16, 16, 18), (8.0, 8.0, 9.0), 6, (0, 1), 3.5, 0)
    ham = _ham(ctx, cell, dt, k, fused)
    grid, V, P = oracle_setup(cell, k)
    X = rng.standard_normal((40, grid.n_d)) + (1j * rng.standard_normal((40, grid.n_d)) if cplx else 0.0)
    Xd = to_dev(X, tdt)
    print(f"\n[noalloc] dtype={dt} fused={fused} call 1: grid {cell.n}, n_s 40", flush=True)
    Y0, Y1 = _pair(ham, Xd)
    d = colnorm_err(Y1, Y0)
    print(f"call 1: vs workspace entry point {d:.2e} (bit-identical: {np.array_equal(Y0, Y1)})", flush=True)
    assert np.all(np.isfinite(Y1)) and d <= tol
    Xref = Xd.cpu().numpy().astype(np.complex128 if cplx else np.float64).T
    assert colnorm_err(Y1.astype(Xref.dtype), apply_H(Xref, grid, V, P)) < tol
    # second call, smaller input: three s atoms on a 12x14x10 grid, 9 states
    cell2, rng2 = wl.draw_cell(97, 2, (12, 14, 10), (6.0, 7.0, 5.0), 3, (0,), 2.5, 0)
    ham2 = _ham(ctx, cell2, dt, k, fused)
    grid2, V2, P2 = oracle_setup(cell2, k)
    X2 = rng2.standard_normal((9, grid2.n_d)) + (1j * rng2.standard_normal((9, grid2.n_d)) if cplx else 0.0)
    X2d = to_dev(X2, tdt)
    print(f"[noalloc] call 2: grid {cell2.n}, n_s 9", flush=True)
    Y0, Y1 = _pair(ham2, X2d)
    d = colnorm_err(Y1, Y0)
    print(f"call 2: vs workspace entry point {d:.2e} (bit-identical: {np.array_equal(Y0, Y1)})", flush=True)
    assert np.all(np.isfinite(Y1)) and d <= tol
    X2ref = X2d.cpu().numpy().astype(np.complex128 if cplx else np.float64).T
    assert colnorm_err(Y1.astype(X2ref.dtype), apply_H(X2ref, grid2, V2, P2)) < tol


def test_noalloc_refuses_projections_beyond_the_array(ctx):
    """64 s+p atoms (256 projectors): the projections of 8200 FP64 states need 16.8 MB,
    more than the 16 MiB array; the call is refused before any launch, Y stays as it
    was, and the next call of a fitting size still agrees with the workspace form."""
    limit = sp.noalloc_max_bytes()
    assert limit == 16 << 20
    cell, rng = wl.draw_cell(97, 3, (12, 12, 12), (6.0, 6.0, 6.0), 64, (0, 1), 2.0, 0)
    ham = sp.Hamiltonian(ctx, cell, sp.R64)
    nd = int(np.prod(cell.n))
    ns = 8200
    need = sp.load().sparc_workspace_bytes(ham.handle, ns, sp.OP_APPLY)
    print(f"\n[noalloc] refusal: n_s {ns}, projections {need} bytes, limit {limit}", flush=True)
    assert need > limit
    X = torch.zeros((ns, nd), dtype=torch.float64, device="cuda:0")
    Y = torch.full_like(X, 7.0)
    with pytest.raises(sp.SparcError) as ei:
        sp.fd_hamiltonian_apply_noalloc(ham, X, Y)
    assert ei.value.status == sp.ENOMEM and "static scratch" in str(ei.value)
    torch.cuda.synchronize()
    assert bool((Y == 7.0).all())
    del X, Y
    Xs = to_dev(rng.standard_normal((33, nd)))
    Y0, Y1 = _pair(ham, Xs)
    assert colnorm_err(Y1, Y0) <= 1e-12
