"""Batched CheFSI (several (cell, k) problems per launch) through the C ABI:
the batched filter, with and without a captured HIP graph, against the oracle
filter of each problem (column-normwise 1e-10) and against the one-problem GPU
filter (1e-13); graph replays with new bounds and new blocks between them,
each checked; batched Rayleigh-Ritz against the oracle; the FP32 batched form;
the tile autotuner; error paths."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

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


def _problems(ctx, dt=sp.C128):
    """Three k-points of one cell plus a second, uneven cell (other grid, other
    n_s, ragged leading dimension)."""
    cell_a, rng = wl.draw_cell(92, 0, (14, 12, 13), (7.0, 6.0, 6.5), 3, (0, 1), 2.2, 0)
    cell_b, _ = wl.draw_cell(92, 1, (9, 16, 11), (4.5, 8.0, 5.5), 2, (0,), 2.0, 0)
    specs = [(cell_a, (0.0, 0.0, 0.0), 6, 0), (cell_a, (0.25, -0.3, 0.1), 6, 0),
             (cell_a, (0.5, 0.5, -0.5), 6, 0), (cell_b, (0.1, 0.2, 0.3), 5, 3)]
    cplx = dt in (sp.C128, sp.C64)
    out = []
    for cell, k, ns, pad in specs:
        grid, V, P = oracle_setup(cell, k)
        X = rng.standard_normal((ns, grid.n_d + pad))
        if cplx:
            X = X + 1j * rng.standard_normal((ns, grid.n_d + pad))
        ham = sp.Hamiltonian(ctx, cell, dt, kpt=k)
        out.append((grid, V, P, X, ham))
    return out


@pytest.fixture(scope="module")
def probs(ctx):
    return _problems(ctx)


DEG = [7, 4, 1, 10]   # odd and even degrees, one problem that ends early
BOUNDS = [(1.0, 60.0), (2.0, 55.0), (0.5, 70.0), (3.0, 50.0)]


def _oracle(pr, deg, bounds):
    return [cheb_filter(X[:, :g.n_d].T, g, V, P, d, lc, lm)
            for (g, V, P, X, _), d, (lc, lm) in zip(pr, deg, bounds)]


def _single(ctx, pr, deg, bounds):
    res = []
    for (g, V, P, X, ham), d, (lc, lm) in zip(pr, deg, bounds):
        Xd = to_dev(X)
        sp.chebyshev_filter(ham, Xd, d, lc, lm, sp.workspace(ham, X.shape[0], sp.OP_FILTER))
        res.append(block_to_oracle(Xd)[:g.n_d])
    return res


def test_batched_filter_matches_oracle(ctx, probs):
    Xs = [to_dev(p[3]) for p in probs]
    sp.chebyshev_filter_batched(ctx, [p[4] for p in probs], Xs, DEG, [b[0] for b in BOUNDS], [b[1] for b in BOUNDS])
    torch.cuda.synchronize()
    ref = _oracle(probs, DEG, BOUNDS)
    single = _single(ctx, probs, DEG, BOUNDS)
    for i, (p, Xd) in enumerate(zip(probs, Xs)):
        got = block_to_oracle(Xd)
        err = colnorm_err(got[:p[0].n_d], ref[i])
        print(f"problem {i}: n={p[0].n} deg={DEG[i]} oracle err {err:.2e}")
        assert err < 1e-10
        assert colnorm_err(got[:p[0].n_d], single[i]) < 1e-13
        if got.shape[0] > p[0].n_d:   # padding rows untouched
            np.testing.assert_array_equal(got[p[0].n_d:], p[3][:, p[0].n_d:].T)


def test_batched_filter_zchunked_oracle(ctx):
    """Batched filter over two Bloch k-points of a long n_o = 6 cell (16 x 16 x 98,
    3 states: every problem's launch splits z into 4 chunks) and a small second cell,
    each against the oracle filter directly."""
    cell_a, rng = wl.draw_cell(92, 5, (16, 16, 98), (8.0, 8.0, 49.0), 3, (0, 1), 2.5, 0)
    cell_b, _ = wl.draw_cell(92, 6, (10, 9, 12), (5.0, 4.5, 6.0), 2, (0,), 2.0, 0)
    specs = [(cell_a, (0.1, -0.2, 0.35), 3, 6), (cell_a, (-0.3, 0.15, 0.05), 3, 5), (cell_b, (0.2, 0.0, -0.1), 4, 7)]
    hams, Xs, refs = [], [], []
    for cell, k, ns, deg in specs:
        grid, V, P = oracle_setup(cell, k)
        X = rng.standard_normal((ns, grid.n_d)) + 1j * rng.standard_normal((ns, grid.n_d))
        hams.append(sp.Hamiltonian(ctx, cell, sp.C128, kpt=k))
        Xs.append(to_dev(X))
        refs.append(cheb_filter(X.T, grid, V, P, deg, 2.0, 60.0))
    sp.chebyshev_filter_batched(ctx, hams, Xs, [s[3] for s in specs], [2.0] * 3, [60.0] * 3)
    torch.cuda.synchronize()
    for i, (Xd, ref) in enumerate(zip(Xs, refs)):
        err = colnorm_err(block_to_oracle(Xd), ref)
        print(f"z-chunked batch problem {i}: oracle err {err:.2e}")
        assert err < 1e-11


def test_graph_replays(ctx, probs):
    """One captured graph, three replays with different bounds and blocks;
    eager torch work and a synchronisation between replays."""
    Xs = [to_dev(p[3]) for p in probs]
    plan = sp.FilterPlan(ctx, [p[4] for p in probs], Xs, DEG, use_graph=True)
    rng = np.random.default_rng(7)
    for rep in range(3):
        bounds = [(lc + 0.5 * rep, lm - 2.0 * rep) for lc, lm in BOUNDS]
        news = []
        for p, Xd in zip(probs, Xs):
            Xn = p[3] * (1.0 + rep) + 0.1 * rep * rng.standard_normal(p[3].shape)
            Xd.copy_(to_dev(Xn))
            news.append(Xn)
        torch.cuda.synchronize()
        plan.run([b[0] for b in bounds], [b[1] for b in bounds])
        pr = [(p[0], p[1], p[2], Xn, p[4]) for p, Xn in zip(probs, news)]
        ref = _single(ctx, pr, DEG, bounds)
        orc = _oracle(pr, DEG, bounds)
        for i, (p, Xd) in enumerate(zip(pr, Xs)):
            got = block_to_oracle(Xd)[:p[0].n_d]
            e1, e2 = colnorm_err(got, ref[i]), colnorm_err(got, orc[i])
            print(f"replay {rep} problem {i}: vs single {e1:.2e}, vs oracle {e2:.2e}")
            assert e1 < 1e-13 and e2 < 1e-10
    plan.close()


def test_plan_without_graph_reuse(ctx, probs):
    Xs = [to_dev(p[3]) for p in probs]
    plan = sp.FilterPlan(ctx, [p[4] for p in probs], Xs, DEG, use_graph=False)
    for rep in range(2):
        for p, Xd in zip(probs, Xs):
            Xd.copy_(to_dev(p[3]))
        plan.run([b[0] for b in BOUNDS], [b[1] for b in BOUNDS])
        ref = _oracle(probs, DEG, BOUNDS)
        for i, (p, Xd) in enumerate(zip(probs, Xs)):
            assert colnorm_err(block_to_oracle(Xd)[:p[0].n_d], ref[i]) < 1e-10
    plan.close()


def test_batched_rr(ctx, probs):
    deg = [8, 8, 8, 8]
    bounds = [(5.0, 80.0)] * 4
    filt = _oracle(probs, deg, bounds)
    Xs = [to_dev(np.ascontiguousarray(Y.T)) for Y in filt]
    ritz = [torch.zeros(Y.shape[1], dtype=torch.float64, device="cuda:0") for Y in filt]
    sp.rayleigh_ritz_batched(ctx, [p[4] for p in probs], Xs, ritz)
    for i, p in enumerate(probs):
        lam, _ = rayleigh_ritz(filt[i], p[0], p[1], p[2])
        np.testing.assert_allclose(ritz[i].cpu().numpy(), lam, atol=1e-8)
        Xo = block_to_oracle(Xs[i])
        np.testing.assert_allclose(Xo.conj().T @ Xo, np.eye(Xo.shape[1]), atol=1e-10)


def test_batched_filter_single_precision(ctx):
    pr = _problems(ctx, sp.C64)
    Xs = [to_dev(p[3], torch.complex64) for p in pr]
    deg = [5, 5, 3, 6]
    plan = sp.FilterPlan(ctx, [p[4] for p in pr], Xs, deg, use_graph=True)
    bounds = [(20.0, 60.0)] * 4
    plan.run([b[0] for b in bounds], [b[1] for b in bounds])
    ref = _oracle(pr, deg, bounds)
    for i, (p, Xd) in enumerate(zip(pr, Xs)):
        err = colnorm_err(block_to_oracle(Xd)[:p[0].n_d].astype(np.complex128), ref[i])
        print(f"fp32 problem {i}: {err:.2e}")
        assert err < 1e-4
    plan.close()


def test_autotune_same_result(ctx):
    cell, X0, rng = wl.config_cell("c1")
    ham = sp.Hamiltonian(ctx, cell, sp.R64)
    X = to_dev(X0)
    Y0 = torch.zeros_like(X)
    Y1 = torch.zeros_like(X)
    w = sp.workspace(ham, X0.shape[0], sp.OP_APPLY)
    sp.fd_hamiltonian_apply(ham, X, Y0, w)
    sp.set_autotune(ctx, True)
    try:
        sp.fd_hamiltonian_apply(ham, X, Y1, w)   # tunes, then applies with the chosen tile
        sp.fd_hamiltonian_apply(ham, X, Y1, w)   # cached choice
    finally:
        sp.set_autotune(ctx, False)
    torch.cuda.synchronize()
    assert colnorm_err(block_to_oracle(Y1), block_to_oracle(Y0)) < 1e-14


def test_batch_error_paths(ctx, probs):
    cell, _ = wl.draw_cell(92, 2, (8, 8, 8), (4.0, 4.0, 4.0), 1, (0,), 1.5, 0)
    h32 = sp.Hamiltonian(ctx, cell, sp.R32)
    X0 = to_dev(probs[0][3])
    X1 = torch.zeros(2, 512, dtype=torch.float32, device="cuda:0")
    with pytest.raises(sp.SparcError) as e:
        sp.chebyshev_filter_batched(ctx, [probs[0][4], h32], [X0, X1], [3, 3], [1.0, 1.0], [2.0, 2.0])
    assert e.value.status == sp.EINVAL
    with pytest.raises(sp.SparcError) as e:
        sp.chebyshev_filter_batched(ctx, [probs[0][4]], [X0], [0], [1.0], [2.0])
    assert e.value.status == sp.EINVAL
    with pytest.raises(sp.SparcError) as e:
        sp.chebyshev_filter_batched(ctx, [probs[0][4]], [X0], [3], [2.0], [1.0])
    assert e.value.status == sp.EINVAL
