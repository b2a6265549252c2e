"""Pins of the learned-density oracle against facts that do not come from it:
the circular-correlation theorem (FFT), shift and linearity special cases,
finite differences of the training loss, the closed form of Adam's first
step, and the charge / fallback rules of the prediction."""
import numpy as np
import pytest

from oracle import density_net as dn


def _fft_correlate(x, w, q=1):
    """y[m] = sum_d w[d] x[m + q d] for a 3x3x3 kernel with dilation q on a periodic
    grid, via the correlation theorem: y = ifft( fft(x) * conj(fft(K)) ), K[q d] = w[d]."""
    K = np.zeros_like(x)
    for kz in range(3):
        for ky in range(3):
            for kx in range(3):
                K[(q * (kz - 1)) % x.shape[0], (q * (ky - 1)) % x.shape[1], (q * (kx - 1)) % x.shape[2]] += w[kz, ky, kx]
    return np.real(np.fft.ifftn(np.fft.fftn(x) * np.conj(np.fft.fftn(K))))


@pytest.mark.parametrize("q", [1, 2, 3])
def test_conv_single_channel_matches_fft(q):
    rng = np.random.default_rng(0)
    x = rng.standard_normal((9, 10, 11))
    w = rng.standard_normal((3, 3, 3))
    y = dn.conv3d(x[None], w[None, None], np.array([0.25]), q)[0]
    np.testing.assert_allclose(y, _fft_correlate(x, w, q) + 0.25, atol=1e-12)


def test_conv_multichannel_is_sum_of_correlations():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((3, 4, 5, 6))
    W = rng.standard_normal((2, 3, 3, 3, 3))
    b = rng.standard_normal(2)
    y = dn.conv3d(x, W, b, 2)
    for co in range(2):
        ref = b[co] + sum(_fft_correlate(x[ci], W[co, ci], 2) for ci in range(3))
        np.testing.assert_allclose(y[co], ref, atol=1e-11)


def test_conv_shift_and_identity_taps():
    rng = np.random.default_rng(2)
    x = rng.standard_normal((1, 4, 5, 6))
    W = np.zeros((1, 1, 3, 3, 3))
    W[0, 0, 1, 1, 1] = 1.0
    np.testing.assert_array_equal(dn.conv3d(x, W, np.zeros(1)), x)
    W[:] = 0
    W[0, 0, 2, 1, 0] = 1.0          # reads x at offset q (+1, 0, -1)
    k, j, i = 1, 2, 3
    y = dn.conv3d(x, W, np.zeros(1))
    assert y[0, k, j, i] == x[0, (k + 1) % 4, j, (i - 1) % 6]
    y = dn.conv3d(x, W, np.zeros(1), 4)
    assert y[0, k, j, i] == x[0, (k + 4) % 4, j, (i - 4) % 6]


def test_param_count():
    assert dn.num_params() == 880 + 13856 + 27680 + 865 == 43281


def _small_net(rng, channels=(2, 3, 4, 2, 1)):
    theta = dn.init_params(rng, channels)
    theta += 0.05 * rng.standard_normal(theta.size)   # non-zero biases too
    return theta, channels


def test_loss_gradient_finite_differences():
    rng = np.random.default_rng(3)
    theta, ch = _small_net(rng)
    dil = (1, 2, 1, 2)
    xs = [np.abs(rng.standard_normal((5, 6, 4))) * 2 for _ in range(2)]
    us = [rng.standard_normal((5, 6, 4)) for _ in range(2)]
    ys = [x + 0.3 * rng.standard_normal(x.shape) for x in xs]
    L0, g = dn.loss_and_grad(theta, xs, us, ys, ch, dil)
    idx = rng.choice(theta.size, 40, replace=False)
    h = 1e-6
    for i in idx:
        tp = theta.copy()
        tp[i] += h
        tm = theta.copy()
        tm[i] -= h
        fd = (dn.loss_and_grad(tp, xs, us, ys, ch, dil)[0] - dn.loss_and_grad(tm, xs, us, ys, ch, dil)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])) + 1e-8, (i, fd, g[i])


def test_input_gradient_of_conv_finite_differences():
    rng = np.random.default_rng(4)
    x = rng.standard_normal((2, 3, 4, 5))
    W = rng.standard_normal((3, 2, 3, 3, 3))
    gy = rng.standard_normal((3, 3, 4, 5))
    gx, gW, gb = dn.conv3d_backward(x, W, gy, 2)
    f = lambda xx: float((gy * dn.conv3d(xx, W, np.zeros(3), 2)).sum())
    for _ in range(10):
        c = tuple(rng.integers(0, s) for s in x.shape)
        xp = x.copy()
        xp[c] += 1e-6
        xm = x.copy()
        xm[c] -= 1e-6
        assert abs((f(xp) - f(xm)) / 2e-6 - gx[c]) < 1e-6
    np.testing.assert_allclose(gb, gy.sum(axis=(1, 2, 3)))


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(5)
    theta = rng.standard_normal(50)
    g = rng.standard_normal(50)
    lr, eps = 1e-3, 1e-8
    t1, m, v = dn.adam_step(theta, g, np.zeros(50), np.zeros(50), 1, lr, eps=eps)
    # bias-corrected moments of the first step are g and g^2
    np.testing.assert_allclose(t1, theta - lr * g / (np.abs(g) + eps), rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(m, 0.1 * g)
    np.testing.assert_allclose(v, 0.001 * g * g)


def test_predict_zero_correction_returns_sad():
    """With every weight zero the correction is a constant (the last bias), which
    the mean subtraction removes: the prediction is the SAD density itself."""
    rng = np.random.default_rng(6)
    rho = np.abs(rng.standard_normal((6, 5, 4)))
    dV = 0.125
    n_elec = float(rho.sum() * dV)
    theta = np.zeros(dn.num_params())
    theta[-1] = 3.0
    out, used = dn.predict_density(theta, rho, -rho, n_elec, dV)
    assert used
    np.testing.assert_allclose(out, rho, rtol=1e-12)


def test_predict_renormalises_and_falls_back():
    rng = np.random.default_rng(7)
    rho = np.abs(rng.standard_normal((6, 5, 4))) * 1.25 + 0.01
    dV = 0.2
    n_elec = 10.0
    theta = dn.init_params(rng) * 0.01
    vloc = -np.abs(rng.standard_normal(rho.shape))
    out, used = dn.predict_density(theta, rho * (n_elec / (rho.sum() * dV)), vloc, n_elec, dV, charge_tol=0.5)
    assert used and abs(out.sum() * dV - n_elec) < 1e-10 and np.all(out >= 0)
    bad = theta.copy()
    bad[5] = np.nan
    out, used = dn.predict_density(bad, rho, vloc, n_elec, dV)
    assert not used and np.array_equal(out, rho)
    # a correction that the final ReLU clips changes the charge: pass-through layers
    # give d = -2 x, so relu(x + d - mean(d)) = relu(2 - x) (x has mean 1) loses the
    # charge of the points with x > 2
    L = dn.unpack(np.zeros(dn.num_params()))
    L[0][0][0, 0, 1, 1, 1] = 1.0
    L[1][0][0, 0, 1, 1, 1] = 1.0
    L[2][0][0, 0, 1, 1, 1] = 1.0
    L[3][0][0, 0, 1, 1, 1] = -2.0
    rho_n = rho * (n_elec / (rho.sum() * dV))
    x = rho_n / (n_elec / (rho.size * dV))
    lost = np.maximum(x - 2.0, 0.0).sum() / x.sum()
    assert lost > 0.01
    out, used = dn.predict_density(dn.pack(L), rho_n, vloc, n_elec, dV, charge_tol=1e-2)
    assert not used and np.array_equal(out, rho_n)
    out, used = dn.predict_density(dn.pack(L), rho_n, vloc, n_elec, dV, charge_tol=0.5)
    assert used
    np.testing.assert_allclose(out, np.maximum(2.0 - x, 0.0) * n_elec / (np.maximum(2.0 - x, 0.0).sum() * dV),
                               rtol=1e-12)


def test_bf16_round_matches_torch_bfloat16():
    """The oracle's bfloat16 rounding (from the definition: 8 significant bits, ties to
    even) against torch's own float32 -> bfloat16 conversion, on values over many
    decades, exact ties, their neighbours, zeros and the subnormal range."""
    torch = pytest.importorskip("torch")
    from oracle.density_net import bf16_round
    rng = np.random.default_rng(5)
    v = rng.standard_normal(20000) * np.exp(rng.uniform(-30, 30, 20000))
    base = (rng.integers(128, 256, 200) / 128.0) * 2.0 ** rng.integers(-20, 20, 200)
    ties = base * (1.0 + 2.0 ** -9)            # halfway between two bfloat16 values
    near = np.concatenate([ties * (1 + 2.0 ** -20), ties * (1 - 2.0 ** -20)])
    tiny = rng.uniform(-1, 1, 500) * 2.0 ** -128
    x = np.concatenate([v, -v[:100], base, ties, -ties, near, tiny, [0.0, -0.0, 1.0, -1.0]]).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    got = bf16_round(x)
    assert np.array_equal(got, ref)
    # and the ties really were ties: rounding moved them by exactly half a spacing
    assert np.all(np.abs(bf16_round(ties) - ties) == np.abs(ties) * 2.0 ** -9 / (1.0 + 2.0 ** -9))


def test_forward_bf16_is_the_rounded_network():
    """precision 'bf16' equals the FP32-mode forward of the rounded weights on the
    rounded input when the hidden activations happen to be bfloat16 numbers already
    (one layer: a 2 -> 1 network with rounded inputs), and differs from the FP32 form
    by about the bfloat16 resolution on a full network."""
    from oracle.density_net import bf16_round, forward, init_params
    rng = np.random.default_rng(9)
    n = (10, 9, 8)
    x = rng.uniform(0, 3, n)
    u = rng.uniform(-2, 2, n)
    theta = init_params(rng)
    y32, c32 = forward(theta, x, u)
    y16, c16 = forward(theta, x, u, precision="bf16")
    d32, d16 = c32[1][-1][0], c16[1][-1][0]
    rel = np.linalg.norm(d16 - d32) / np.linalg.norm(d32)
    assert 1e-4 < rel < 3e-2
    ch = (2, 1)
    th1 = rng.standard_normal(27 * 2 + 1)
    xr, ur = bf16_round(x), bf16_round(u)
    ya, ca = forward(th1, xr, ur, ch, (1,), precision="bf16")
    yb, cb = forward(bf16_round(th1), xr, ur, ch, (1,))
    assert np.array_equal(ca[1][-1], cb[1][-1])
