"""Chebyshev-filtered subspace iteration (Sec. 3.4, Electron density calculation)
and the Lanczos estimate of the spectral bounds (Sec. 4, solver settings).

Test infrastructure (see oracle/__init__.py); never imported by the product path.
"""
from __future__ import annotations

import numpy as np

from .fd import apply_H, dense_H


def filter_center_halfwidth(lambda_cut: float, lambda_max: float):
    """c = (lambda_max + lambda_c)/2 and e = (lambda_max - lambda_c)/2 of the
    filter polynomial p_m(t) = C_m((t - c)/e) (Sec. 3.4, Chebyshev filter)."""
    return 0.5 * (lambda_max + lambda_cut), 0.5 * (lambda_max - lambda_cut)


def cheb_filter(X, grid, veff, projs, degree, lambda_cut, lambda_max, apply=None):
    """U_f = C_m((H - c)/e) U by the three-term recurrence of the Chebyshev
    polynomials (Sec. 3.4): Y_0 = X, Y_1 = (H - c) X / e,
    Y_{j+1} = 2 (H - c) Y_j / e - Y_{j-1}; returns Y_m (m = degree >= 1)."""
    if apply is None:
        def apply(Z):
            return apply_H(Z, grid, veff, projs)
    c, e = filter_center_halfwidth(lambda_cut, lambda_max)
    Y0 = np.array(X, copy=True)
    Y1 = (apply(Y0) - c * Y0) / e
    for _ in range(1, degree):
        Y2 = 2.0 * (apply(Y1) - c * Y1) / e - Y0
        Y0, Y1 = Y1, Y2
    return Y1


def chebyshev_value(m: int, t):
    """C_m(t) from its closed forms: cos(m arccos t) for |t| <= 1 and
    sign(t)^m cosh(m arccosh |t|) otherwise."""
    t = np.asarray(t, dtype=np.float64)
    out = np.empty_like(t)
    inside = np.abs(t) <= 1.0
    out[inside] = np.cos(m * np.arccos(t[inside]))
    ta = np.abs(t[~inside])
    out[~inside] = np.sign(t[~inside]) ** m * np.cosh(m * np.arccosh(ta))
    return out


def cheb_direct(X, grid, veff, projs, degree, lambda_cut, lambda_max):
    """The same filter by explicit spectral evaluation: V diag(C_m((lambda - c)/e)) V^H X
    with (lambda, V) = eigh of the dense H (small grids only)."""
    H = dense_H(grid, veff, projs)
    lam, V = np.linalg.eigh(H)
    c, e = filter_center_halfwidth(lambda_cut, lambda_max)
    p = chebyshev_value(degree, (lam - c) / e)
    return V @ (p[:, None] * (V.conj().T @ X))


def rayleigh_ritz(Xf, grid, veff, projs, apply=None):
    """Projection of H onto span(U_f) and subspace rotation (Sec. 3.4,
    subspace generalized eigenproblem and orbital transformation).

    The generalized problem H~ y = lambda M~ y with H~ = U_f^H H U_f and
    M~ = U_f^H U_f is reduced with an orthonormal basis Q of span(U_f) from a
    Householder QR, U_f = Q R, so that H~ = R^H (Q^H H Q) R and M~ = R^H R; the
    Ritz pairs of Q^H H Q are those of the pencil.  Returns (ritz ascending,
    rotated orbitals Q Z with Z the eigenvectors, i.e. U_f Y)."""
    if apply is None:
        def apply(Z):
            return apply_H(Z, grid, veff, projs)
    Q, _ = np.linalg.qr(Xf)
    Hs = Q.conj().T @ apply(Q)
    Hs = 0.5 * (Hs + Hs.conj().T)
    lam, Z = np.linalg.eigh(Hs)
    return lam, Q @ Z


def lanczos(grid, veff, projs, v0, steps: int, apply=None):
    """Plain Lanczos with full reorthogonalisation (the Lanczos method named in
    Sec. 4 for the extremal eigenvalues of H).  Returns (alpha, beta, theta,
    S) with T the tridiagonal of alpha (diag) and beta (off-diag), theta its
    eigenvalues ascending and S its eigenvectors."""
    if apply is None:
        def apply(z):
            return apply_H(z, grid, veff, projs)
    v = np.asarray(v0, dtype=np.complex128 if not grid.is_gamma else np.float64)
    v = v / np.linalg.norm(v)
    V = [v]
    alpha, beta = [], []
    for j in range(steps):
        w = apply(V[j])
        a = np.real(np.vdot(V[j], w))
        alpha.append(a)
        w = w - a * V[j]
        if j > 0:
            w = w - beta[j - 1] * V[j - 1]
        for q in V:                      # full reorthogonalisation
            w = w - np.vdot(q, w) * q
        b = np.linalg.norm(w)
        beta.append(b)
        if j + 1 < steps:
            V.append(w / b)
    T = np.diag(alpha) + np.diag(beta[:-1], 1) + np.diag(beta[:-1], -1)
    theta, S = np.linalg.eigh(T)
    return np.array(alpha), np.array(beta), theta, S


def lanczos_bounds(grid, veff, projs, v0, steps: int = 20, margin: float = 0.01, apply=None):
    """Filter bounds from Lanczos: lambda_min = smallest Ritz value, and
    lambda_max = theta_max + |beta_k s_k| (the residual bound of the largest Ritz
    pair), enlarged by `margin` times its magnitude."""
    alpha, beta, theta, S = lanczos(grid, veff, projs, v0, steps, apply)
    upper = theta[-1] + abs(beta[-1] * S[-1, -1])
    upper = upper + margin * abs(upper)
    return float(theta[0]), float(upper)
