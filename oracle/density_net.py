"""Oracle of the learned initial density (test infrastructure only: imported by
tests/, by the package's smoke check and by the benchmark's CPU baseline, never
by the library path).

The paper starts every SCF from the superposition of atomic densities (SAD,
Sec. 3.4 and the SCF description of Sec. 4).  The learned part replaces that
first guess by

    rho_0 = renorm( relu( x + (d - mean(d)) ) * rho_bar ),   x = rho_SAD / rho_bar,
    d = f_theta(x, u),   u = -V_loc (Ha),

where rho_bar = N_e / (N_d dV) is the mean density and f_theta is a small 3-D
convolutional network: four 3x3x3 convolutions with periodic (circular)
padding and dilations 1, 2, 4, 8 (receptive field 31 points), channels
2 -> 16 -> 32 -> 32 -> 1, ReLU after the first three.  The second input
channel is the local potential: the atomic superposition of these synthetic
cells does not depend on the well depths, which shape the converged density.
Subtracting mean(d) makes the correction charge-neutral, so only the final
ReLU can change the charge; renorm scales to h^3 sum rho = N_e.  The network is
trained on (SAD, converged plain-SCF density) pairs by the mean squared error
of s = x + d - mean(d) against y = rho_SCF / rho_bar, with Adam (the loss is
taken before the ReLU so that negative values of s are penalised: the charge
they would add under the ReLU is what the fallback rule measures).  Prediction
falls back to the SAD density when any value is not finite or when the charge
before renormalisation is off by more than charge_tol * N_e.

Parity of the network's *effect* is unpinned (it is assessed by the SCF it
starts); the functions here are pinned by the circular-correlation theorem
(FFT), by finite differences of the loss, and by the closed form of Adam's
first step.

Array layout: a field of C channels is (C, n3, n2, n1) in C order, so the
flattened voxel index is i + n1 (j + n2 k) with x fastest.  A convolution
weight is W[co, ci, kz, ky, kx]; with dilation q, tap (kz, ky, kx) reads the
input at offset q (kz - 1, ky - 1, kx - 1) (cross-correlation).  The flat parameter vector holds,
layer by layer, W (C order) then b.
"""
from __future__ import annotations

import numpy as np

CHANNELS = (2, 16, 32, 32, 1)
DILATIONS = (1, 2, 4, 8)


def layer_shapes(channels=CHANNELS):
    return [((co, ci, 3, 3, 3), (co,)) for ci, co in zip(channels[:-1], channels[1:])]


def num_params(channels=CHANNELS):
    return sum(int(np.prod(w)) + b[0] for w, b in layer_shapes(channels))


def unpack(theta, channels=CHANNELS):
    """Flat parameter vector -> [(W, b), ...]."""
    out, o = [], 0
    for ws, bs in layer_shapes(channels):
        nw = int(np.prod(ws))
        W = np.asarray(theta[o:o + nw], dtype=np.float64).reshape(ws)
        o += nw
        b = np.asarray(theta[o:o + bs[0]], dtype=np.float64)
        o += bs[0]
        out.append((W, b))
    return out


def pack(layers):
    return np.concatenate([np.concatenate([W.ravel(), b.ravel()]) for W, b in layers])


def init_params(rng, channels=CHANNELS):
    """He-normal weights (std sqrt(2 / (27 C_in))), zero biases; the last layer
    is scaled by 0.1 so the untrained correction is small."""
    layers = []
    shapes = layer_shapes(channels)
    for l, (ws, bs) in enumerate(shapes):
        std = np.sqrt(2.0 / (27 * ws[1]))
        if l == len(shapes) - 1:
            std *= 0.1
        layers.append((rng.standard_normal(ws) * std, np.zeros(bs)))
    return pack(layers)


def _shifted(x, kz, ky, kx, q=1):
    """xs[c, k, j, i] = x[c, k + q(kz - 1), j + q(ky - 1), i + q(kx - 1)] (periodic)."""
    return np.roll(x, shift=(q * (1 - kz), q * (1 - ky), q * (1 - kx)), axis=(1, 2, 3))


def conv3d(x, W, b, q=1):
    """Circular 3x3x3 cross-correlation with dilation q:
    y[co] = b[co] + sum_ci sum_taps W x(shifted)."""
    y = np.empty((W.shape[0],) + x.shape[1:])
    y[:] = b[:, None, None, None]
    for kz in range(3):
        for ky in range(3):
            for kx in range(3):
                y += np.tensordot(W[:, :, kz, ky, kx], _shifted(x, kz, ky, kx, q), axes=(1, 0))
    return y


def conv3d_backward(x, W, gy, q=1):
    """Gradients of sum(gy * conv3d(x, W, b, q)) with respect to x, W and b."""
    gx = np.zeros_like(x)
    gW = np.zeros_like(W)
    for kz in range(3):
        for ky in range(3):
            for kx in range(3):
                gW[:, :, kz, ky, kx] = np.tensordot(gy, _shifted(x, kz, ky, kx, q), axes=([1, 2, 3], [1, 2, 3]))
                # adjoint of the shift: gy moved by +offset
                gys = np.roll(gy, shift=(q * (kz - 1), q * (ky - 1), q * (kx - 1)), axis=(1, 2, 3))
                gx += np.tensordot(W[:, :, kz, ky, kx].T, gys, axes=(1, 0))
    gb = gy.sum(axis=(1, 2, 3))
    return gx, gW, gb


def bf16_round(a):
    """Nearest bfloat16 value (8 significant bits, ties to even, the FP32 exponent range)
    of each element, after rounding it to FP32 (the values being rounded are FP32
    numbers in the BF16 inference form).  From the definition: x = m 2^e with
    0.5 <= |m| < 1, m is rounded to a multiple of 2^-8 (numpy's round is ties-to-even);
    below 2^-126 the spacing is the fixed 2^-133 of the subnormal range."""
    f = np.asarray(a, dtype=np.float32).astype(np.float64)
    out = np.array(f, copy=True)
    fin = np.isfinite(f) & (f != 0.0)
    m, e = np.frexp(f[fin])
    r = np.ldexp(np.round(np.ldexp(m, 8)), e - 8)
    tiny = np.abs(f[fin]) < 2.0 ** -126
    r[tiny] = np.round(f[fin][tiny] * 2.0 ** 133) * 2.0 ** -133
    out[fin] = r
    return out


def forward(theta, x, u, channels=CHANNELS, dilations=DILATIONS, precision="fp32"):
    """x: (n3, n2, n1) scaled SAD density of one cell, u: -V_loc on the same grid.
    precision "bf16": the weights and every layer's input are rounded to bfloat16
    (bf16_round) and the sums are exact; the last layer's output and the head are
    not rounded.  Returns (yhat, cache)."""
    layers = unpack(theta, channels)
    rnd = bf16_round if precision == "bf16" else (lambda v: v)
    if precision == "bf16":
        layers = [(rnd(W), rnd(b)) for W, b in layers]
    a = [np.stack([x, u])]
    for l, (W, b) in enumerate(layers):
        z = conv3d(rnd(a[-1]), W, b, dilations[l])
        a.append(np.maximum(z, 0.0) if l < len(layers) - 1 else z)
    d = a[-1][0]
    s = x + (d - d.mean())
    yhat = np.maximum(s, 0.0)
    return yhat, (layers, a, s)


def loss_and_grad(theta, xs, us, ys, channels=CHANNELS, dilations=DILATIONS):
    """Mean squared error over a batch (lists of (n3, n2, n1) arrays) and its
    gradient with respect to the flat parameters."""
    B = len(xs)
    nv = xs[0].size
    total = 0.0
    grads = None
    for x, u, y in zip(xs, us, ys):
        _, (layers, a, s) = forward(theta, x, u, channels, dilations)
        r = s - y
        total += float((r * r).sum())
        g = 2.0 * r / (B * nv)
        g = g - g.mean()                 # through d - mean(d)
        ga = g[None]
        lg = []
        for l in range(len(layers) - 1, -1, -1):
            W, _ = layers[l]
            gx, gW, gb = conv3d_backward(a[l], W, ga, dilations[l])
            lg.append((gW, gb))
            if l > 0:
                ga = gx * (a[l] > 0)     # through the ReLU of layer l-1
        gflat = pack(lg[::-1])
        grads = gflat if grads is None else grads + gflat
    return total / (B * nv), grads


def adam_step(theta, g, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba): returns (theta, m, v) after step t (1-based)."""
    m = beta1 * m + (1 - beta1) * g
    v = beta2 * v + (1 - beta2) * g * g
    mh = m / (1 - beta1 ** t)
    vh = v / (1 - beta2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def predict_density(theta, rho_sad, vloc, n_elec, dV, charge_tol=1e-2, channels=CHANNELS, dilations=DILATIONS,
                    precision="fp32"):
    """Learned first density, or the SAD density as the fallback.
    Returns (rho, used_net)."""
    nv = rho_sad.size
    rho_bar = n_elec / (nv * dV)
    x = rho_sad / rho_bar
    with np.errstate(all="ignore"):
        yhat, _ = forward(theta, x, -vloc, channels, dilations, precision)
        charge = float(yhat.sum()) * rho_bar * dV
    if not np.all(np.isfinite(yhat)) or not np.isfinite(charge) or abs(charge - n_elec) > charge_tol * n_elec:
        return rho_sad.copy(), False
    return yhat * rho_bar * (n_elec / charge), True
