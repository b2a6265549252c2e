"""Finite-difference operators of Section 3.1 (Finite-difference discretization).

Test infrastructure (see oracle/__init__.py); never imported by the product path.

Conventions
  grid nodes (i, j, k), 0-based, flattened x-fastest: g = i + n1*(j + n2*k);
  a block of orbitals X is a numpy array of shape (N_d, N_s), column n = orbital n;
  a column reshaped to 3-D is f3[k, j, i] (C order), so axis 2 = x, 1 = y, 0 = z.

Bloch form (reading of Sec. 2 "Electronic ground-state" with the periodic index
map of Sec. 3.1): the operator acts on psi = e^{ik.x} u, and an index that leaves
the cell is mapped to its periodic image with the Bloch factor
psi(i + n_s) = e^{i k_s L_s} psi(i).  Then H = -1/2 Lap_h + V_eff + V_nl.
A direction with zero Dirichlet conditions (slabs and wires, Sec. 3.1) sets every
value at an index outside the grid to zero instead.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Grid:
    """Uniform periodic grid on an axis-aligned cuboid cell (Sec. 3.1)."""

    n: tuple            # (n1, n2, n3)
    L: tuple            # (L1, L2, L3) in bohr
    n_o: int = 6        # half-width of the stencil (12th order: n_o = 6, Sec. 4)
    k: tuple = (0.0, 0.0, 0.0)  # Bloch wavevector (bohr^-1)
    bc: tuple = (0, 0, 0)       # per direction: 0 Bloch-periodic, 1 zero Dirichlet

    @property
    def h(self):
        return tuple(self.L[s] / self.n[s] for s in range(3))

    @property
    def n_d(self):
        return int(self.n[0] * self.n[1] * self.n[2])

    @property
    def dV(self):
        h = self.h
        return h[0] * h[1] * h[2]

    @property
    def is_gamma(self):
        return all(float(x) == 0.0 for x in self.k)

    def coords(self):
        """Node positions x_g = (i h1, j h2, k h3), shape (N_d, 3), g x-fastest."""
        h = self.h
        kk, jj, ii = np.meshgrid(np.arange(self.n[2]), np.arange(self.n[1]),
                                 np.arange(self.n[0]), indexing="ij")
        return np.stack([ii.ravel() * h[0], jj.ravel() * h[1], kk.ravel() * h[2]], axis=1)


def laplacian_weights(n_o: int, h: float):
    """Weights of the central FD Laplacian along one direction (Sec. 3.1,
    weights of the Laplacian): w_0 = -(1/h^2) sum_{q=1}^{n_o} 1/q^2 and
    w_p = 2 (-1)^{p+1} (n_o!)^2 / (h^2 p^2 (n_o-p)! (n_o+p)!), p = 1..n_o.

    The stencil sums p = 0..n_o of w_p (f^{+p} + f^{-p}), so the centre
    coefficient of one direction is 2 w_0.
    Returns (w0, w) with w[p-1] = w_p.
    """
    w0 = -sum(1.0 / (q * q) for q in range(1, n_o + 1)) / (h * h)
    fn = math.factorial(n_o)
    w = np.array([2.0 * (-1) ** (p + 1) * fn * fn
                  / (h * h * p * p * math.factorial(n_o - p) * math.factorial(n_o + p))
                  for p in range(1, n_o + 1)])
    return w0, w


def gradient_weights(n_o: int, h: float):
    """Weights of the central FD gradient (Sec. 3.1, gradient weights):
    w~_p = (-1)^{p+1} (n_o!)^2 / (h p (n_o-p)! (n_o+p)!), p = 1..n_o."""
    fn = math.factorial(n_o)
    return np.array([(-1) ** (p + 1) * fn * fn
                     / (h * p * math.factorial(n_o - p) * math.factorial(n_o + p))
                     for p in range(1, n_o + 1)])


def bloch_shift(f3: np.ndarray, p: int, axis: int, n: int, kL: float, dirichlet: bool = False):
    """Return g with g(i) = f(i + p) along `axis` (length n), mapping an index
    outside 0..n-1 to its periodic image and multiplying by the Bloch factor
    e^{i kL w}, w = floor((i+p)/n) the number of cell lengths crossed; with a
    zero Dirichlet condition such values are 0 (Sec. 3.1)."""
    idx = np.arange(n) + p
    wraps = np.floor_divide(idx, n)
    src = np.mod(idx, n)
    out = np.take(f3, src, axis=axis)
    if dirichlet:
        shape = [1, 1, 1]
        shape[axis] = n
        return out * (wraps == 0).reshape(shape)
    if kL != 0.0 and np.any(wraps != 0):
        fac = np.exp(1j * kL * wraps)
        shape = [1, 1, 1]
        shape[axis] = n
        out = out * fac.reshape(shape)
    return out


def minus_half_laplacian(f: np.ndarray, grid: Grid):
    """-1/2 Lap_h f for one grid function f (length N_d), Sec. 3.1 stencil with
    the Bloch-periodic index map."""
    n1, n2, n3 = grid.n
    f3 = f.reshape(n3, n2, n1)
    h = grid.h
    axes = (2, 1, 0)          # direction s = 1, 2, 3 -> numpy axis
    lap = np.zeros_like(f3, dtype=np.result_type(f3.dtype, np.float64)
                        if grid.is_gamma else np.complex128)
    for s in range(3):
        w0, w = laplacian_weights(grid.n_o, h[s])
        kL = grid.k[s] * grid.L[s]
        lap = lap + 2.0 * w0 * f3
        for p in range(1, grid.n_o + 1):
            lap = lap + w[p - 1] * (bloch_shift(f3, p, axes[s], grid.n[s], kL, grid.bc[s] == 1)
                                    + bloch_shift(f3, -p, axes[s], grid.n[s], kL, grid.bc[s] == 1))
    return (-0.5 * lap).reshape(-1)


def nonlocal_apply(X: np.ndarray, grid: Grid, projs):
    """Discrete non-local operator of Sec. 3.1 (V_nl with the trapezoidal rule):
    V_nl X = h1 h2 h3 sum_J gamma_J chi~_J (chi~_J^H X), with chi~_J the
    Bloch-phased image sum of the projector (values on its support)."""
    cplx = np.iscomplexobj(X) or any(np.iscomplexobj(p["val"]) for p in projs)
    Y = np.zeros(X.shape, dtype=np.complex128 if cplx else np.float64)
    for p in projs:
        idx, val = p["idx"], p["val"]
        alpha = grid.dV * (np.conj(val) @ X[idx, :])
        np.add.at(Y, idx, p["gamma"] * np.outer(val, alpha))
    return Y


def apply_H(X: np.ndarray, grid: Grid, veff: np.ndarray, projs=()):
    """H X = -1/2 Lap_h X + V_eff X + V_nl X for a block of orbitals
    (Sec. 2 Kohn-Sham equations in Bloch form, discretised as in Sec. 3.1)."""
    X = np.asarray(X)
    squeeze = X.ndim == 1
    if squeeze:
        X = X[:, None]
    cplx = (not grid.is_gamma) or np.iscomplexobj(X) or any(np.iscomplexobj(p["val"]) for p in projs)
    Y = np.zeros(X.shape, dtype=np.complex128 if cplx else np.float64)
    for c in range(X.shape[1]):
        Y[:, c] = minus_half_laplacian(X[:, c], grid) + veff * X[:, c]
    if projs:
        Y = Y + nonlocal_apply(X, grid, projs)
    return Y[:, 0] if squeeze else Y


def dense_H(grid: Grid, veff: np.ndarray, projs=()):
    """The matrix H(k) in C^{N_d x N_d} (Sec. 3.1) built column by column by
    applying H to the unit vectors; for small grids (N_d <= 12^3) only."""
    nd = grid.n_d
    if nd > 12 ** 3:
        raise ValueError("dense_H is for small grids only")
    eye = np.eye(nd)
    return apply_H(eye, grid, veff, projs)
