"""Seeded synthetic workloads (random draws only; none of the method's arithmetic).

The paper's crystals need Troullier-Martins pseudopotentials that are not
available, so every workload is a synthetic periodic cell of Gaussian wells with
Gaussian-radial Kleinman-Bylander projectors; this module only draws the random
parameters (atom positions, well depths and widths, projector energies, the
random starting orbitals and the Lanczos start vector) from
numpy.random.default_rng([config_id, cell_id]) in a fixed order:
positions (N x 3, uniform in [0, L)), depths, widths, projector energies per
(atom, l), then the starting orbitals column by column (complex: the real block,
then the imaginary block).  Both the library and the oracle receive the same
drawn values as inputs.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# Workload definitions (sizes of the five synthetic configurations)
CONFIGS = {
    # plain FP64 CheFSI at Gamma: 12 bohr cell, 24^3, 8 atoms, s projectors
    "c1": dict(cfg_id=0, n=24, L=12.0, n_atoms=8, ls=(0,), rc=3.0, n_s=32, degree=20,
               passes=4, kpts="gamma"),
    # large Gamma cell: 96^3 at h = 0.4, 64 atoms with s + p projectors
    "c2": dict(cfg_id=1, n=96, L=38.4, n_atoms=64, ls=(0, 1), rc=3.5, n_s=512, degree=24,
               passes=6, kpts="gamma"),
    # complex Bloch cell, 8 k-points: 48^3 at h = 0.5, 16 atoms
    "c3": dict(cfg_id=2, n=48, L=24.0, n_atoms=16, ls=(0,), rc=3.0, n_s=128, degree=20,
               passes=1, kpts="mp2"),
    # SCF cells for the learned initial density: 40^3 at h = 0.5
    "c5": dict(cfg_id=4, n=40, L=20.0, n_atoms=None, ls=(0,), rc=3.0, n_s=None, degree=20,
               passes=4, kpts="gamma"),
}

# uneven batch: (grid n, atoms, states, degree) per drawn size
UNEVEN_SIZES = {32: (8, 32, 16), 48: (16, 64, 18), 64: (32, 128, 20), 80: (48, 256, 24)}


@dataclass
class Cell:
    """One synthetic periodic cell (all arrays host numpy)."""

    n: tuple
    L: tuple
    positions: np.ndarray          # (N, 3) bohr, in [0, L)
    depth: np.ndarray              # (N,) Ha
    width: np.ndarray              # (N,) bohr
    chan_atom: np.ndarray          # (n_chan,) int32
    chan_l: np.ndarray             # (n_chan,) int32
    chan_gamma: np.ndarray         # (n_chan,) Ha
    chan_rc: np.ndarray            # (n_chan,) bohr
    Z: np.ndarray                  # (N,) valence charge (2 per atom)
    n_o: int = 6
    n_s: int = 0
    degree: int = 20
    passes: int = 1
    bc: tuple = (0, 0, 0)           # per direction: 0 Bloch-periodic, 1 zero Dirichlet
    psd_rc: np.ndarray = None       # (N,) cutoff of the Coulomb-tailed local pseudopotential (bohr)
    psd_rc_ref: np.ndarray = None   # (N,) cutoff of its reference potential (bohr)
    extra: dict = field(default_factory=dict)

    @property
    def n_d(self):
        return int(self.n[0] * self.n[1] * self.n[2])

    @property
    def n_atoms(self):
        return int(self.positions.shape[0])

    @property
    def n_elec(self):
        return float(self.Z.sum())


def draw_cell(cfg_id: int, cell_id: int, n, L, n_atoms: int, ls=(0,), rc=3.0, n_s=0,
              degree=20, passes=1, rng=None):
    """Draw the random parameters of one synthetic cell; returns (Cell, rng) with
    the generator positioned for the orbital draws that follow."""
    if rng is None:
        rng = np.random.default_rng([cfg_id, cell_id])
    n = (n, n, n) if np.isscalar(n) else tuple(n)
    L = (L, L, L) if np.isscalar(L) else tuple(L)
    pos = rng.uniform(0.0, 1.0, size=(n_atoms, 3)) * np.asarray(L)[None, :]
    depth = rng.uniform(2.0, 6.0, size=n_atoms)
    width = rng.uniform(0.8, 1.5, size=n_atoms)
    gam = rng.uniform(0.5, 2.0, size=(n_atoms, len(ls)))
    chan_atom = np.repeat(np.arange(n_atoms, dtype=np.int32), len(ls))
    chan_l = np.tile(np.asarray(ls, dtype=np.int32), n_atoms)
    cell = Cell(n=n, L=L, positions=pos, depth=depth, width=width,
                chan_atom=chan_atom, chan_l=chan_l, chan_gamma=gam.reshape(-1),
                chan_rc=np.full(n_atoms * len(ls), float(rc)),
                Z=np.full(n_atoms, 2.0), n_s=n_s, degree=degree, passes=passes,
                psd_rc=2.0 * width, psd_rc_ref=1.0 * width)
    return cell, rng


def draw_orbitals(rng, n_d: int, n_s: int, complex_: bool = False, dtype=np.float64):
    """Random starting orbitals, N(0,1), column-major (N_d, N_s), returned as the
    C-contiguous (N_s, N_d) array whose row n is orbital n (so the memory is the
    column-major block).  Complex: real block first, then imaginary block."""
    re = rng.standard_normal((n_s, n_d))
    if not complex_:
        return re.astype(dtype, copy=False)
    im = rng.standard_normal((n_s, n_d))
    return (re + 1j * im).astype(np.complex128 if dtype == np.float64 else np.complex64)


def config_cell(name: str, cell_id: int = 0, with_orbitals: bool = True):
    """Cell and starting orbitals of a named configuration ("c1", "c2", "c3")."""
    c = CONFIGS[name]
    cell, rng = draw_cell(c["cfg_id"], cell_id, c["n"], c["L"], c["n_atoms"], c["ls"], c["rc"],
                          c["n_s"], c["degree"], c["passes"])
    X0 = None
    if with_orbitals:
        X0 = draw_orbitals(rng, cell.n_d, cell.n_s, complex_=(c["kpts"] != "gamma"))
    return cell, X0, rng


def scf_cell(cell_id: int, n: int = 40, L: float = 20.0, split: str = "train"):
    """A 40^3 SCF cell with 8-32 atoms; N_s = N_atoms + 24 rounded up to a
    multiple of 8 (the spectrum of these cells is dense near the Fermi level, so
    the buffer of empty states must reach ~0.07 Ha = 7 kT above it for the SCF
    to converge to 1e-6).  Seeds [4, cell_id]; the test split uses cell ids
    from 100000 on."""
    cid = cell_id if split == "train" else 100000 + cell_id
    rng = np.random.default_rng([4, cid])
    n_atoms = int(rng.integers(8, 33))
    n_s = 8 * math.ceil((n_atoms + 24) / 8)
    cell, rng = draw_cell(4, cid, n, L, n_atoms, (0,), 3.0, n_s, 20, 4, rng=rng)
    X0 = draw_orbitals(rng, cell.n_d, n_s)
    v0 = rng.standard_normal(cell.n_d)
    return cell, X0, v0


def uneven_batch(n_cells: int = 24, seed=(3, 0)):
    """Grid sizes for the batch of uneven cells, drawn from {32, 48, 64, 80}."""
    rng = np.random.default_rng(list(seed))
    return [int(x) for x in rng.choice([32, 48, 64, 80], size=n_cells)]


def mp2_kpoints(L):
    """The 8 nodes of the shifted 2x2x2 Monkhorst-Pack grid, k_s = (2 pi / L_s)(+-1/4)
    (bohr^-1, x fastest), each of weight 1/8."""
    ks = [(2 * math.pi / L[0] * a, 2 * math.pi / L[1] * b, 2 * math.pi / L[2] * c)
          for c in (-0.25, 0.25) for b in (-0.25, 0.25) for a in (-0.25, 0.25)]
    return ks, [1.0 / 8.0] * 8


def band_path(L, corners=((-0.5, 0.5, 0.5), (0.0, 0.0, 0.0), (1.0, 0.0, 0.0), (1.0, 1.0, 1.0)),
              divisions=(10, 12, 17)):
    """k-points of a piecewise-linear path through `corners` (reciprocal-lattice
    coordinates, units of 2 pi / L_s) with the given divisions per segment, corners
    included once: the L - Gamma - X - Gamma circuit with 10, 12 and 17 divisions of
    the band-structure comparison of Sec. 4 (40 points).  Returns (n_k, 3) bohr^-1."""
    c = np.asarray(corners, dtype=np.float64)
    pts = [c[0]]
    for s, nd in enumerate(divisions):
        for t in range(1, nd + 1):
            pts.append(c[s] + (c[s + 1] - c[s]) * t / nd)
    return np.asarray(pts) * (2 * math.pi / np.asarray(L, dtype=np.float64))[None, :]


def uneven_cells(n_cells: int = 24, h: float = 0.5, seed=(3, 0), with_orbitals: bool = True):
    """The batch of independent uneven cells: grid n drawn from {32, 48, 64, 80}
    (uneven_batch), spacing h, atoms / states / degree from UNEVEN_SIZES; cell i
    seeded [3, 1 + i].  Returns a list of (cell, X0, rng)."""
    out = []
    for i, n in enumerate(uneven_batch(n_cells, seed)):
        na, ns, deg = UNEVEN_SIZES[n]
        cell, rng = draw_cell(3, 1 + i, n, n * h, na, (0,), 3.0, ns, deg, 1)
        X0 = draw_orbitals(rng, cell.n_d, ns) if with_orbitals else None
        out.append((cell, X0, rng))
    return out


def lanczos_start(rng, n_d: int, complex_: bool = False):
    """Random Lanczos start vector, N(0,1)."""
    v = rng.standard_normal(n_d)
    if complex_:
        v = v + 1j * rng.standard_normal(n_d)
    return v
