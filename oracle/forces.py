"""Atomic forces (Sec. 2, "Atomic forces": f_J = -dF/dR_J; Sec. 3.6, local and
non-local components, Algorithms 2 and 3), in the reduced model of the synthetic
cell.

Test infrastructure (see oracle/__init__.py); never imported by the product path.

Local component.  The paper's local force is written with pseudocharges
(first term of the force equation of Sec. 2, discrete form of Sec. 3.6).  In
the reduced model the Gaussian wells are an external potential and the
electrostatics are jellium, so the local part of the free energy is the
trapezoidal-rule integral E_loc = h1h2h3 sum_g rho_g V_loc(x_g; R) (Sec. 3.1,
spatial integration) and its exact derivative is

    f_J,loc = -dE_loc/dR_J = h1h2h3 sum_g rho_g sum_L D_J e^{-r^2/(2 w_J^2)} (x_g - R_J - L) / w_J^2,
    r = |x_g - R_J - L|, every image L with r <= 10 w_J (the cutoff of V_loc).

There is no overlap correction f_J,c (no pseudocharges).

Non-local component (Sec. 3.6, discrete non-local force, with Y and W as
defined there; the derivative is moved from the projectors to the orbitals and
taken with the FD gradient of Sec. 3.1):

    f_J,nloc = -4 sum_n sum_b w_b g_nb sum_lm gamma_Jl Re[ Y_Jnblm W_Jnblm ],
    Y = h1h2h3 sum_g psi_n^*(g) chi~_Jlm(g),   W = h1h2h3 sum_g (grad_h psi_n)(g) chi~_Jlm^*(g),

where chi~ is the Bloch-phased image sum of the projector (the phase factors
e^{-i k.(R_J - R_J')} of the paper) and psi is normalised by h1h2h3 sum |psi|^2 = 1.
The orbitals of this code are Euclidean-orthonormal columns u = psi sqrt(h1h2h3),
so with alpha = h1h2h3 sum conj(chi~) u and beta = h1h2h3 sum conj(chi~) grad_h u:
Y W = conj(alpha) beta / (h1h2h3).

Pins (tests/test_oracle_forces.py): the gradient's symbol on Bloch plane waves;
the local force against central differences of E_loc at fixed density; the
non-local force against the same sums with the FD gradient moved back onto the
projectors (summation by parts is exact for the skew-adjoint central stencil);
the non-local force against central differences of E_nl at fixed orbitals
(agreement to the FD-gradient error of the projectors); opposite forces on an
inversion-symmetric pair; and the total force against central differences of
the SCF free energy on a small cell.
"""
from __future__ import annotations

import numpy as np

from .fd import Grid, gradient_weights, bloch_shift
from .cell import _box_range, _images, VLOC_CUTOFF_WIDTHS


def fd_gradient(f: np.ndarray, grid: Grid):
    """grad_h f of one grid function (length N_d): the central FD gradient of
    Sec. 3.1, sum_p w~_p (f^{+p} - f^{-p}) per direction, with the Bloch-periodic
    index map.  Returns an array of shape (3, N_d) (components x, y, z)."""
    n1, n2, n3 = grid.n
    f3 = f.reshape(n3, n2, n1)
    axes = (2, 1, 0)
    out = []
    for s in range(3):
        wt = gradient_weights(grid.n_o, grid.h[s])
        kL = grid.k[s] * grid.L[s]
        acc = np.zeros(f3.shape, dtype=np.complex128 if (np.iscomplexobj(f3) or kL != 0.0) else np.float64)
        for p in range(1, grid.n_o + 1):
            acc = acc + wt[p - 1] * (bloch_shift(f3, p, axes[s], grid.n[s], kL, grid.bc[s] == 1)
                                     - bloch_shift(f3, -p, axes[s], grid.n[s], kL, grid.bc[s] == 1))
        out.append(acc.reshape(-1))
    return np.stack(out)


def local_energy(grid: Grid, rho, vloc):
    """E_loc = h1h2h3 sum_g rho_g V_loc(x_g) (trapezoidal rule, Sec. 3.1)."""
    return grid.dV * float(np.dot(rho, vloc))


def local_force(grid: Grid, R, depth, width, rho):
    """f_J,loc = h1h2h3 sum_g rho_g sum_L D_J e^{-r^2/(2w^2)} (x_g - R_J - L)/w^2
    for every atom J (the exact derivative of local_energy).  Returns (N_atoms, 3)."""
    n1, n2, n3 = grid.n
    h = grid.h
    rho3 = np.asarray(rho, dtype=np.float64).reshape(n3, n2, n1)
    F = np.zeros((len(depth), 3))
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
            dx = (ii * h[0] - c[0])[None, None, :]
            dy = (jj * h[1] - c[1])[None, :, None]
            dz = (kk * h[2] - c[2])[:, None, None]
            r2 = dx * dx + dy * dy + dz * dz
            s = np.where(r2 <= rcut * rcut, D * np.exp(-r2 / (2.0 * w * w)) / (w * w), 0.0)
            s = s * rho3[np.ix_(kk, jj, ii)]
            F[J] += grid.dV * np.array([np.sum(s * dx), np.sum(s * dy), np.sum(s * dz)])
    return F


def nonlocal_energy(grid: Grid, projs, Xs, occ_w):
    """E_nl = 2 sum_b sum_n w_b g_nb sum_J gamma_J |Y_Jnb|^2 / (h1h2h3) with
    Y = h1h2h3 sum conj(chi~) u (the non-local term of the band energy,
    u^H V_nl u summed with the occupations; Sec. 2 non-local energy, Sec. 3.1)."""
    E = 0.0
    for b, X in enumerate(Xs):
        for p in projs:
            a = grid.dV * (np.conj(p["val"]) @ X[p["idx"], :])
            E += 2.0 * p["gamma"] * float(np.sum(np.asarray(occ_w[b]) * np.abs(a) ** 2)) / grid.dV
    return E


def nonlocal_force(grids, projs_k, Xs, occ_w, n_atoms: int):
    """f_J,nloc of Sec. 3.6 (discrete non-local force with Y and W), summed over
    the k-points b: grids[b], projs_k[b] (projectors at k_b), Xs[b] (N_d, N_s)
    Euclidean-orthonormal orbitals, occ_w[b] = w_b g_nb.  Returns (N_atoms, 3)."""
    F = np.zeros((n_atoms, 3))
    for b, (grid, projs, X) in enumerate(zip(grids, projs_k, Xs)):
        dV = grid.dV
        occ = np.asarray(occ_w[b], dtype=np.float64)
        # grad_h of every orbital (3, N_d, N_s)
        G = np.stack([fd_gradient(X[:, n], grid) for n in range(X.shape[1])], axis=2)
        for p in projs:
            idx, val = p["idx"], p["val"]
            Y = dV * (val @ np.conj(X[idx, :]))                        # (N_s,)  = conj(alpha)
            W = dV * np.einsum("t,dtn->dn", np.conj(val), G[:, idx, :])  # (3, N_s)
            F[p["atom"]] += -4.0 * p["gamma"] * np.real(W @ (occ * Y)) / dV
    return F


def nonlocal_force_on_projectors(grids, projs_k, Xs, occ_w, n_atoms: int):
    """The same sums with the FD gradient moved back onto the projectors:
    sum_g conj(chi~) grad_h u = -sum_g conj(grad_h chi~) u, exact for the
    skew-adjoint central stencil on the Bloch-periodic grid.  Used to pin
    nonlocal_force."""
    F = np.zeros((n_atoms, 3))
    for b, (grid, projs, X) in enumerate(zip(grids, projs_k, Xs)):
        dV = grid.dV
        occ = np.asarray(occ_w[b], dtype=np.float64)
        for p in projs:
            chi = np.zeros(grid.n_d, dtype=np.complex128)
            chi[p["idx"]] = p["val"]
            gchi = fd_gradient(chi, grid)                               # (3, N_d)
            Y = dV * (chi @ np.conj(X))                                 # (N_s,)
            W = -dV * (np.conj(gchi) @ X)                               # (3, N_s)
            F[p["atom"]] += -4.0 * p["gamma"] * np.real(W @ (occ * Y)) / dV
    return F
