"""Shared test helpers: oracle objects for a synthetic cell, tensor conversions."""
import numpy as np

from oracle.fd import Grid
from oracle.cell import local_potential, projectors


def oracle_setup(cell, kpt=(0.0, 0.0, 0.0), n_o=6):
    grid = Grid(n=tuple(cell.n), L=tuple(cell.L), n_o=n_o, k=tuple(kpt), bc=tuple(getattr(cell, "bc", (0, 0, 0))))
    V = local_potential(grid, cell.positions, cell.depth, cell.width)
    P = projectors(grid, cell.positions, cell.chan_atom, cell.chan_l, cell.chan_gamma, cell.chan_rc)
    return grid, V, P


def colnorm_err(Y, Yref):
    """max over columns of ||Y_n - Yref_n|| / ||Yref_n||; Y, Yref as (N_d, N_s)."""
    num = np.linalg.norm(Y - Yref, axis=0)
    den = np.linalg.norm(Yref, axis=0)
    return float(np.max(num / np.maximum(den, 1e-300)))


def to_dev(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to("cuda:0")


def block_to_oracle(t):
    """(n_s, ld) device tensor -> (N_d, n_s) numpy array."""
    return t.detach().cpu().numpy().T.copy()
