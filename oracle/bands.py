"""Band structure and density of states (Sec. 4: the band structure at the electronic
ground state, obtained at every k-point of a path by repeating the CheFSI steps with
the ground-state potential fixed; the density of states
D(E) = 2 sum_n fint_BZ delta(lambda_n(k) - E) dk).

Test infrastructure (see oracle/__init__.py); never imported by the product path.

The oracle takes the converged answer the repeated CheFSI steps approach: the lowest
eigenvalues of the dense H(k) of Sec. 3.1 at each k (a library eigensolver as one
step).  The Dirac delta of the density of states is broadened to a normalised
Gaussian of width sigma (reading: the paper does not state its broadening), and the
Brillouin-zone average is the weighted sum over the given k-points.
"""
from __future__ import annotations

import math

import numpy as np

from .fd import Grid, dense_H
from .cell import projectors


def bands(n, L, kpts, veff, atoms, n_bands: int, n_o: int = 6, bc=(0, 0, 0)):
    """Lowest n_bands eigenvalues of H(k) (Sec. 2 Bloch Hamiltonian, Sec. 3.1
    discretisation) at every k of kpts (shape (n_k, 3), bohr^-1) with the
    potential veff fixed.  atoms = (R, chan_atom, chan_l, chan_gamma, chan_rc) for
    the projectors (rebuilt with the Bloch phases of each k).  Returns (n_k, n_bands)."""
    out = []
    for k in np.asarray(kpts, dtype=np.float64):
        grid = Grid(n=tuple(n), L=tuple(L), n_o=n_o, k=tuple(k), bc=tuple(bc))
        P = projectors(grid, *atoms) if atoms is not None else ()
        H = dense_H(grid, veff, P)
        out.append(np.linalg.eigvalsh(0.5 * (H + H.conj().T))[:n_bands])
    return np.array(out)


def dos(eig, wk, energies, sigma: float):
    """D(E) = 2 sum_b w_b sum_n g(E - lambda_nb) with g the normalised Gaussian of
    width sigma (the broadened delta of Sec. 4).  eig: (n_k, n_bands), wk: (n_k,)."""
    eig = np.asarray(eig, dtype=np.float64)
    wk = np.asarray(wk, dtype=np.float64)
    E = np.asarray(energies, dtype=np.float64)
    g = np.exp(-0.5 * ((E[:, None, None] - eig[None, :, :]) / sigma) ** 2) / (sigma * math.sqrt(2.0 * math.pi))
    return 2.0 * np.sum(wk[None, :, None] * g, axis=(1, 2))
