"""The projector term of H (Sec. 3.1, discrete non-local operator) applied inside the
stencil step against the oracle, with the fused path forced on (SPARC_NL_FUSED=1) and
off (=0) for every element type: H X, the Chebyshev filter (where a step's projector
terms are accumulated one plane ahead) and the batched filter.  The dense cell puts
more (node, atom) entries on one tile plane than the work-group has threads, so the
overflow loop runs too; a slab cell covers Dirichlet faces."""
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle.fd import apply_H
from oracle.chefsi import cheb_filter
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


def _ham(ctx, cell, dt, k, fused):
    old = os.environ.get("SPARC_NL_FUSED")
    os.environ["SPARC_NL_FUSED"] = "1" if fused else "0"
    try:
        return sp.Hamiltonian(ctx, cell, dt, kpt=k)
    finally:
        if old is None:
            del os.environ["SPARC_NL_FUSED"]
        else:
            os.environ["SPARC_NL_FUSED"] = old


DTYPES = [(sp.R64, 1e-12, (0.0, 0.0, 0.0)), (sp.R32, 2e-5, (0.0, 0.0, 0.0)),
          (sp.C128, 1e-12, (0.2, -0.1, 0.3)), (sp.C64, 2e-5, (0.2, -0.1, 0.3))]


@pytest.mark.parametrize("fused", [True, False], ids=["fused", "separate"])
@pytest.mark.parametrize("dt,tol,k", DTYPES, ids=["r64", "r32", "c128", "c64"])
def test_apply_and_filter_dense_projectors(ctx, dt, tol, k, fused):
    """Six s+p atoms with r_c 3.5 in an 8 bohr cube: up to ~900 (node, atom) entries
    on one tile plane."""
    print(f"\n[nl fused={fused}] dtype={dt} k={k}", flush=True)
    cell, rng = wl.draw_cell(95, 1, (16, 16, 18), (8.0, 8.0, 9.0), 6, (0, 1), 3.5, 0)
    grid, V, P = oracle_setup(cell, k)
    cplx = dt in (sp.C128, sp.C64)
    ns = 5
    X = rng.standard_normal((ns, grid.n_d)) + (1j * rng.standard_normal((ns, grid.n_d)) if cplx else 0.0)
    ham = _ham(ctx, cell, dt, k, fused)
    tdt = sp.TORCH_DTYPE[dt]
    Xd = to_dev(X, tdt)
    Xref = Xd.cpu().numpy().astype(np.complex128 if cplx else np.float64).T
    Y = torch.zeros_like(Xd)
    sp.fd_hamiltonian_apply(ham, Xd, Y, sp.workspace(ham, ns, sp.OP_APPLY))
    err = colnorm_err(block_to_oracle(Y).astype(Xref.dtype), apply_H(Xref, grid, V, P))
    print(f"H X colnorm err {err:.2e}", flush=True)
    assert err < tol
    sp.chebyshev_filter(ham, Xd, 5, 3.0, 70.0, sp.workspace(ham, ns, sp.OP_FILTER))
    ferr = colnorm_err(block_to_oracle(Xd).astype(Xref.dtype), cheb_filter(Xref, grid, V, P, 5, 3.0, 70.0))
    print(f"filter colnorm err {ferr:.2e}", flush=True)
    assert ferr < 10 * tol


@pytest.mark.parametrize("fused", [True, False], ids=["fused", "separate"])
def test_batched_filter_mixed_problems(ctx, fused):
    """Batched FP64 plan over a dense s+p cell, an s-only cell and a Dirichlet slab,
    each against the oracle filter."""
    cells = [wl.draw_cell(95, 2, (16, 16, 18), (8.0, 8.0, 9.0), 6, (0, 1), 3.5, 0),
             wl.draw_cell(95, 3, (20, 12, 14), (10.0, 6.0, 7.0), 3, (0,), 2.5, 0)]
    slab, rs = wl.draw_cell(95, 4, (14, 16, 20), (7.0, 8.0, 10.0), 3, (0, 1), 2.5, 0)
    slab.bc = (0, 0, 1)
    cells.append((slab, rs))
    hams, Xs, refs, degs = [], [], [], [4, 7, 5]
    for (cell, rng), deg in zip(cells, degs):
        grid, V, P = oracle_setup(cell)
        X = rng.standard_normal((4, grid.n_d))
        hams.append(_ham(ctx, cell, sp.R64, (0.0, 0.0, 0.0), fused))
        Xs.append(to_dev(X))
        refs.append(cheb_filter(X.T, grid, V, P, deg, 2.0, 60.0))
    sp.chebyshev_filter_batched(ctx, hams, Xs, degs, [2.0] * 3, [60.0] * 3)
    torch.cuda.synchronize()
    for i, (Xd, ref) in enumerate(zip(Xs, refs)):
        err = colnorm_err(block_to_oracle(Xd), ref)
        print(f"batched problem {i} fused={fused}: oracle err {err:.2e}")
        assert err < 1e-11
