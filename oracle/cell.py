"""Synthetic periodic cell: local potential and Kleinman-Bylander projectors on
the grid (Sec. 2 non-local energy and Sec. 3.1 discrete non-local operator).

Test infrastructure (see oracle/__init__.py); never imported by the product path.

The paper's Troullier-Martins pseudopotentials are not available, so the cell is
synthetic (readings of the paper where its data are not available):
  V_loc(x)  = - sum_J sum_L D_J exp(-|x - R_J - L|^2 / (2 w_J^2)), every image L
              with |x - R_J - L| <= 10 w_J;
  chi_s(r)  = c exp(-r^2/(2 sigma^2)) [r <= r_c],  sigma = r_c / 4;
  chi_pm(r) = c (r_m / sigma) exp(-r^2/(2 sigma^2)) [r <= r_c], m = x, y, z;
  c normalises h1 h2 h3 sum over the unwrapped grid of chi^2 to 1.
The projector seen by a Bloch function at wavevector k is the image sum
chi~(x) = sum_L e^{i k.L} chi(x - R - L) (Sec. 2, non-local operator with the
phase factors e^{-ik.(R_J - R_J')}).
"""
from __future__ import annotations

import math

import numpy as np

from .fd import Grid

VLOC_CUTOFF_WIDTHS = 10.0


def _box_range(c: float, rcut: float, h: float, n: int):
    """Node indices i in [0, n) with |i h - c| <= rcut (may be empty)."""
    lo = max(0, math.ceil((c - rcut) / h - 1e-9))
    hi = min(n - 1, math.floor((c + rcut) / h + 1e-9))
    return np.arange(lo, hi + 1)


def _images(grid: Grid, rcut: float):
    """Integer image multiples (a, b, c) that can bring a point within rcut; none
    across a direction with zero Dirichlet conditions (the cell is not repeated)."""
    M = [0 if grid.bc[s] == 1 else int(math.ceil(rcut / grid.L[s])) + 1 for s in range(3)]
    for c in range(-M[2], M[2] + 1):
        for b in range(-M[1], M[1] + 1):
            for a in range(-M[0], M[0] + 1):
                yield (a, b, c)


def local_potential(grid: Grid, R, depth, width):
    """V_loc on the grid nodes (length N_d), summed over all atoms and images."""
    n1, n2, n3 = grid.n
    h = grid.h
    V = np.zeros((n3, n2, n1))
    for J in range(len(depth)):
        D, w = float(depth[J]), float(width[J])
        rcut = VLOC_CUTOFF_WIDTHS * w
        for img in _images(grid, rcut):
            c = [R[J][s] + img[s] * grid.L[s] for s in range(3)]
            ii = _box_range(c[0], rcut, h[0], n1)
            jj = _box_range(c[1], rcut, h[1], n2)
            kk = _box_range(c[2], rcut, h[2], n3)
            if len(ii) == 0 or len(jj) == 0 or len(kk) == 0:
                continue
            dx = ii * h[0] - c[0]
            dy = jj * h[1] - c[1]
            dz = kk * h[2] - c[2]
            r2 = dz[:, None, None] ** 2 + dy[None, :, None] ** 2 + dx[None, None, :] ** 2
            val = np.where(r2 <= rcut * rcut, -D * np.exp(-r2 / (2.0 * w * w)), 0.0)
            V[np.ix_(kk, jj, ii)] += val
    return V.reshape(-1)


def _channel_shapes(l: int):
    """Angular factors of the synthetic projector channels: l = 0 gives one s
    function, l = 1 gives three real p functions (x, y, z)."""
    if l == 0:
        return [None]
    if l == 1:
        return [0, 1, 2]
    raise ValueError("only l = 0 and l = 1 channels are synthesised")


def projectors(grid: Grid, R, chan_atom, chan_l, chan_gamma, chan_rc):
    """Kleinman-Bylander projectors chi~_{Jlm} on the grid for Bloch vector grid.k.

    Returns a list of dicts {atom, l, m, gamma, idx, val}: idx the grid nodes
    of the support (ascending, unique), val the values of chi~ there (complex
    unless the grid is at Gamma).
    """
    n1, n2, n3 = grid.n
    h = grid.h
    out = []
    for c_i in range(len(chan_atom)):
        J, l = int(chan_atom[c_i]), int(chan_l[c_i])
        gamma, rc = float(chan_gamma[c_i]), float(chan_rc[c_i])
        sigma = rc / 4.0
        for m in _channel_shapes(l):
            acc = np.zeros((n3, n2, n1), dtype=np.float64 if grid.is_gamma else np.complex128)
            mask = np.zeros((n3, n2, n1), dtype=bool)
            norm2 = 0.0
            for img in _images(grid, rc):
                c = [R[J][s] + img[s] * grid.L[s] for s in range(3)]
                ii = _box_range(c[0], rc, h[0], n1)
                jj = _box_range(c[1], rc, h[1], n2)
                kk = _box_range(c[2], rc, h[2], n3)
                if len(ii) == 0 or len(jj) == 0 or len(kk) == 0:
                    continue
                dx = (ii * h[0] - c[0])[None, None, :]
                dy = (jj * h[1] - c[1])[None, :, None]
                dz = (kk * h[2] - c[2])[:, None, None]
                r2 = dx * dx + dy * dy + dz * dz
                inside = r2 <= rc * rc
                radial = np.exp(-r2 / (2.0 * sigma * sigma))
                if m is None:
                    val = radial
                else:
                    d = (dx, dy, dz)[m]
                    val = (d / sigma) * radial
                val = np.where(inside, val, 0.0)
                norm2 += float(np.sum(val * val))
                # L = img * cell lengths; the ket carries e^{i k.L}
                phase = np.exp(1j * sum(grid.k[s] * img[s] * grid.L[s] for s in range(3)))
                sub = np.ix_(kk, jj, ii)
                acc[sub] += val if grid.is_gamma else phase * val
                mask[sub] |= inside
            cnorm = 1.0 / math.sqrt(grid.dV * norm2)
            idx = np.flatnonzero(mask.reshape(-1))
            out.append({"atom": J, "l": l, "m": m, "gamma": gamma,
                        "idx": idx, "val": cnorm * acc.reshape(-1)[idx]})
    return out


def monkhorst_pack_2(L):
    """Shifted 2x2x2 Monkhorst-Pack nodes k = (2 pi / L_s)(+-1/4) and equal
    weights 1/8, no symmetry reduction (Sec. 3.3 with the grid of Sec. 4)."""
    ks, ws = [], []
    for c in (-0.25, 0.25):
        for b in (-0.25, 0.25):
            for a in (-0.25, 0.25):
                ks.append((2 * math.pi / L[0] * a, 2 * math.pi / L[1] * b, 2 * math.pi / L[2] * c))
                ws.append(1.0 / 8.0)
    return ks, ws
