"""Occupations, electron density, electrostatics, exchange, free energy and the
self-consistent field loop (Sec. 2 "Electronic ground-state" and "Free energy",
Sec. 3.3-3.5), in the reduced form of the synthetic cell.

Test infrastructure (see oracle/__init__.py); never imported by the product path.

Reduced model (readings of the paper where it does not apply as written):
  * exchange only (Slater): eps_x = -(3/4)(3/pi)^{1/3} rho^{1/3}, V_x = (4/3) eps_x;
  * jellium electrostatics: the Gaussian local potential is external, the
    Hartree potential solves -Lap_h V_H = 4 pi (rho - mean(rho)) with zero mean;
    or, with a pseudocharge b (oracle/pseudocharge.py), the paper's form: V_loc = 0,
    phi solves -Lap_h phi = 4 pi (rho + b) (mean removed), and the free energy gains
    1/2 h1h2h3 sum b phi - E_self^h + E_c^h (Sec. 3.5);
  * density mixing: linear rho_in <- rho_in + beta (rho_out - rho_in), or
    Anderson extrapolation (relaxation beta, history m) as named in Sec. 4;
  * Harris-Foulkes free energy at rho_in.
"""
from __future__ import annotations

import math

import numpy as np

from .fd import Grid, laplacian_weights, apply_H
from .chefsi import cheb_filter, rayleigh_ritz, lanczos_bounds

SLATER_EPS = -0.75 * (3.0 / math.pi) ** (1.0 / 3.0)   # eps_x / rho^{1/3}
SLATER_V = -(3.0 / math.pi) ** (1.0 / 3.0)            # V_x / rho^{1/3}


def occupations(lam, mu: float, kT: float):
    """Fermi-Dirac g = (1 + exp((lambda - mu)/kT))^{-1} (Sec. 2, Eq. for g_n),
    evaluated as (1 - tanh((lambda - mu)/(2 kT)))/2, which cannot overflow."""
    return 0.5 * (1.0 - np.tanh((np.asarray(lam) - mu) / (2.0 * kT)))


def fermi_level(lam, wk, n_elec: float, kT: float, rel_tol: float = 1e-13):
    """Fermi energy from the electron-count constraint
    2 sum_b w_b sum_n g_nb = N_e (Sec. 3.4), by bisection.
    lam has shape (N_k, N_s), wk shape (N_k,)."""
    lam = np.asarray(lam, dtype=np.float64)
    wk = np.asarray(wk, dtype=np.float64)

    def count(mu):
        return 2.0 * float(np.sum(wk[:, None] * occupations(lam, mu, kT)))

    lo = float(lam.min()) - 40.0 * kT - 1.0
    hi = float(lam.max()) + 40.0 * kT + 1.0
    if count(hi) < n_elec:
        raise ValueError("not enough states for the electron count")
    for _ in range(400):
        mid = 0.5 * (lo + hi)
        c = count(mid)
        if abs(c - n_elec) < rel_tol * n_elec:
            return mid              # the constraint holds here (inside a gap, anywhere on the plateau)
        if c < n_elec:
            lo = mid
        else:
            hi = mid
        if hi - lo < 1e-15 * max(1.0, abs(mid)):
            break
    return 0.5 * (lo + hi)


def density(Xs, occ_w, dV: float):
    """rho^{(i,j,k)} = 2 sum_b sum_n w_b g_nb |u_nb^{(i,j,k)}|^2 (Sec. 3.4) for
    Euclidean-orthonormal columns, divided by dV = h1 h2 h3 so that
    dV sum rho = N_e.  Xs: list over k of (N_d, N_s); occ_w: (N_k, N_s) = w_b g_nb."""
    rho = np.zeros(Xs[0].shape[0])
    for b, X in enumerate(Xs):
        rho += 2.0 * (np.abs(X) ** 2) @ np.asarray(occ_w[b], dtype=np.float64)
    return rho / dV


def laplacian_symbol(grid: Grid):
    """Eigenvalues sigma(G) of -Lap_h on the plane waves of the periodic grid,
    in numpy FFT order over (k, j, i): sigma = -sum_s [2 w_0 + 2 sum_p w_p cos(p G_s h_s)]."""
    h = grid.h
    sig = 0.0
    axes_n = (grid.n[2], grid.n[1], grid.n[0])
    hs = (h[2], h[1], h[0])
    for a in range(3):
        w0, w = laplacian_weights(grid.n_o, hs[a])
        G = 2.0 * math.pi * np.fft.fftfreq(axes_n[a], d=hs[a])
        term = 2.0 * w0 + 2.0 * sum(w[p - 1] * np.cos(p * G * hs[a]) for p in range(1, grid.n_o + 1))
        shape = [1, 1, 1]
        shape[a] = axes_n[a]
        sig = sig - term.reshape(shape)
    return sig


def poisson(rho, grid: Grid):
    """Hartree potential of the jellium reading: the discrete problem
    -Lap_h V_H = 4 pi (rho - mean rho) (Sec. 2, Poisson equation, with the FD
    Laplacian of Sec. 3.1), solved exactly by diagonalising the circulant
    operator with the DFT; the G = 0 component of V_H is set to zero."""
    n1, n2, n3 = grid.n
    r3 = np.asarray(rho, dtype=np.float64).reshape(n3, n2, n1)
    rhat = np.fft.fftn(r3 - r3.mean())
    sig = laplacian_symbol(grid)
    vhat = np.zeros_like(rhat)
    nz = np.abs(sig) > 1e-300
    nz[0, 0, 0] = False
    vhat[nz] = 4.0 * math.pi * rhat[nz] / sig[nz]
    return np.real(np.fft.ifftn(vhat)).reshape(-1)


def kerker(f, grid: Grid, k0: float):
    """Kerker preconditioner of a density residual (damping of the long-wavelength
    charge-sloshing modes of the mixing, a standard companion of the Anderson mixing
    of Sec. 4): P f = sigma(G) / (sigma(G) + k0^2) f-hat per plane wave, sigma the
    symbol of -Lap_h, so P removes the G = 0 component and leaves the short waves
    nearly unchanged.  Written as f - k0^2 g with (-Lap_h + k0^2) g = f, solved
    exactly by the DFT."""
    n1, n2, n3 = grid.n
    fhat = np.fft.fftn(np.asarray(f, dtype=np.float64).reshape(n3, n2, n1))
    ghat = fhat / (laplacian_symbol(grid) + k0 * k0)
    return np.asarray(f, dtype=np.float64) - k0 * k0 * np.real(np.fft.ifftn(ghat)).reshape(-1)


def slater(rho):
    """Slater exchange: returns (eps_x, V_x) per grid point (the exchange part
    of the LDA of Sec. 2)."""
    r13 = np.cbrt(np.maximum(np.asarray(rho, dtype=np.float64), 0.0))
    return SLATER_EPS * r13, SLATER_V * r13


def entropy_term(g, wk, kT: float):
    """2 kT sum_b w_b sum_n [g ln g + (1-g) ln(1-g)] (Sec. 3.5), with
    0 ln 0 = 0."""
    g = np.asarray(g, dtype=np.float64)
    with np.errstate(divide="ignore", invalid="ignore"):
        a = np.where(g > 0.0, g * np.log(np.where(g > 0.0, g, 1.0)), 0.0)
        b = np.where(g < 1.0, (1.0 - g) * np.log(np.where(g < 1.0, 1.0 - g, 1.0)), 0.0)
    return 2.0 * kT * float(np.sum(np.asarray(wk)[:, None] * (a + b)))


def harris_foulkes(lam, g, wk, rho_in, vh_in, grid: Grid, kT: float, b=None, e_const: float = 0.0):
    """Free energy of Sec. 3.5 in the reduced model, evaluated at the input
    density: F = 2 sum w g lambda + dV sum [eps_x rho - V_x rho + 1/2 (b - rho) phi]
    + entropy + e_const, where phi = vh_in.  Jellium: b = None and e_const = 0 (no
    pseudocharge, self-energy or overlap terms); with pseudocharges
    e_const = -E_self^h + E_c^h."""
    eps, vx = slater(rho_in)
    band = 2.0 * float(np.sum(np.asarray(wk)[:, None] * np.asarray(g) * np.asarray(lam)))
    half_b = 0.0 if b is None else 0.5 * np.asarray(b)
    dc = grid.dV * float(np.sum(eps * rho_in - vx * rho_in + (half_b - 0.5 * rho_in) * vh_in))
    return band + dc + entropy_term(g, wk, kT) + e_const


def sad_density(grid: Grid, R, width, Z, n_elec: float):
    """Superposition of atomic densities: rho_J proportional to
    Z_J (2 pi w_J^2)^{-3/2} exp(-r^2/(2 w_J^2)) summed over images, then
    renormalised to dV sum rho = N_e."""
    from .cell import _box_range, _images, VLOC_CUTOFF_WIDTHS
    n1, n2, n3 = grid.n
    h = grid.h
    rho = np.zeros((n3, n2, n1))
    for J in range(len(width)):
        w = float(width[J])
        rcut = VLOC_CUTOFF_WIDTHS * w
        amp = float(Z[J]) * (2.0 * math.pi * w * w) ** -1.5
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
            rho[np.ix_(kk, jj, ii)] += np.where(r2 <= rcut * rcut, amp * np.exp(-r2 / (2 * w * w)), 0.0)
    rho = rho.reshape(-1)
    return rho * (n_elec / (grid.dV * rho.sum()))


def anderson_update(x, f, hist_x, hist_f, beta: float, m: int, precond=None):
    """Anderson extrapolation of the fixed-point iteration x -> x + f (the SCF
    acceleration named in Sec. 4, relaxation beta, history m): with the
    differences dX_i = x_i - x_{i-1} and dF_i = f_i - f_{i-1} of the last m
    iterates, gamma minimises ||f - dF gamma||_2, and
    x_new = (x - dX gamma) + beta P (f - dF gamma), P the preconditioner (identity
    when precond is None).  hist_x, hist_f hold the previous iterates and residuals
    (updated in place).  m = 0 is (preconditioned) linear mixing."""
    if m > 0 and hist_x:
        dX = np.stack([x - hist_x[-1]] + [hist_x[i + 1] - hist_x[i] for i in range(len(hist_x) - 1)][::-1], axis=1)
        dF = np.stack([f - hist_f[-1]] + [hist_f[i + 1] - hist_f[i] for i in range(len(hist_f) - 1)][::-1], axis=1)
        dX, dF = dX[:, :m], dF[:, :m]
        gamma, *_ = np.linalg.lstsq(dF, f, rcond=None)
        xb = x - dX @ gamma
        fb = f - dF @ gamma
    else:
        xb, fb = x, f
    hist_x.append(x.copy())
    hist_f.append(f.copy())
    del hist_x[:-m or None]
    del hist_f[:-m or None]
    return xb + beta * (fb if precond is None else precond(fb))


def scf(grid: Grid, vloc, projs, X0, n_elec: float, degree: int, kT: float = 0.01,
        mix: float = 0.3, tol: float = 1e-6, max_iter: int = 100, n_first_passes: int = 4,
        rho_init=None, lanczos_v0=None, lanczos_steps: int = 20, callback=None, mix_history: int = 0,
        psd=None, kerker_k0: float = 0.0):
    """Minimal SCF of Sec. 2 ("fixed-point iteration ... accelerated using
    mixing") with the CheFSI policy of Sec. 3.4: the first SCF step runs
    n_first_passes filter + Rayleigh-Ritz passes from the random X0 before the
    density is formed, later steps run one pass from the rotated orbitals.
    Gamma point only (one k-point of weight 1).

    Filter bounds: lambda_max from Lanczos (once, on the first Hamiltonian);
    lambda_cut = (lambda_min + lambda_max)/2 for the first pass, then the largest
    Ritz value of the previous pass.
    Mixing: mix_history = 0 is linear density mixing rho_in + mix (rho_out - rho_in);
    mix_history > 0 is Anderson extrapolation with relaxation mix and that history;
    kerker_k0 > 0 preconditions the mixed residual with the Kerker filter of that
    wavenumber (bohr^-1).
    Electrostatics: psd = None is the jellium form; psd = the dict of
    oracle.pseudocharge.electrostatics_setup switches to pseudocharges (vloc must then
    be zero: the electrons see phi).
    Returns dict(energy, mu, iterations, converged, rho, ritz, history).
    """
    hx, hf = [], []
    rho_in = np.asarray(rho_init, dtype=np.float64).copy()
    X = np.array(X0, copy=True)
    bpsd = None if psd is None else psd["b"]
    e_const = 0.0 if psd is None else psd["ec"] - psd["eself"]

    def potential(r):
        return poisson(r if bpsd is None else r + bpsd, grid)

    vh = potential(rho_in)
    history = []
    lam = None
    lmin = lmax = None
    converged = False
    for it in range(1, max_iter + 1):
        eps, vx = slater(rho_in)
        veff = vloc + vh + vx
        if lmax is None:
            v0 = lanczos_v0 if lanczos_v0 is not None else np.ones(grid.n_d)
            lmin, lmax = lanczos_bounds(grid, veff, projs, v0, lanczos_steps)
        passes = n_first_passes if it == 1 else 1
        for _ in range(passes):
            lcut = 0.5 * (lmin + lmax) if lam is None else float(lam[-1])
            Xf = cheb_filter(X, grid, veff, projs, degree, lcut, lmax)
            lam, X = rayleigh_ritz(Xf, grid, veff, projs)
        mu = fermi_level(lam[None, :], np.array([1.0]), n_elec, kT)
        g = occupations(lam, mu, kT)
        F = harris_foulkes(lam[None, :], g[None, :], np.array([1.0]), rho_in, vh, grid, kT, bpsd, e_const)
        rho_out = density([X], g[None, :], grid.dV)
        err = float(np.linalg.norm(rho_out - rho_in) / np.linalg.norm(rho_in))
        history.append({"iter": it, "energy": F, "mu": mu, "rho_err": err})
        if callback is not None:
            callback(history[-1])
        if err < tol:
            converged = True
            break
        pre = (lambda f: kerker(f, grid, kerker_k0)) if kerker_k0 > 0 else None
        rho_in = anderson_update(rho_in, rho_out - rho_in, hx, hf, mix, mix_history, pre)
        vh = potential(rho_in)
    return {"energy": F, "mu": mu, "iterations": it, "converged": converged,
            "rho": rho_in, "ritz": lam, "history": history, "X": X, "phi": vh, "occ": g}
