"""Pseudocharge electrostatics (Sec. 2 "Electrostatic reformulation", Eqs. for b,
E_self and E_c; Sec. 3.2 pseudocharge generation, Algorithm 1 and the truncation rule
for r^b; Appendix A, discrete E_c and f_c; Sec. 3.6, discrete local force), for a
synthetic Coulomb-tailed local pseudopotential.

Test infrastructure (see oracle/__init__.py); never imported by the product path.

Sign convention (reading of the integral constraints of Sec. 2): the electron density
rho is positive, the pseudocharge b is negative with h1h2h3 sum b = -N_e, i.e. the
atom's total pseudocharge is -Z_J for valence charge Z_J > 0, and the electrostatic
potential phi (the potential energy of an electron) solves
-Lap_h phi / (4 pi) = rho + b.

Synthetic local pseudopotential (reading: the paper's Troullier-Martins tables are not
available).  The continuous pseudocharge is compactly supported in the sphere of
radius rc (as the paper states for its pseudopotentials):
    b_J(r) = -Z_J 315 / (64 pi rc^3) (1 - r^2/rc^2)^3,  r < rc;  0 beyond,
and V_J is its potential, -Lap V_J / (4 pi) = b_J:
    V_J(r) = -Z_J / r                   for r >= rc,
    V_J(r) = -(Z_J / rc) p(r / rc)      for r <  rc,
    p(s)   = (315 - 420 s^2 + 378 s^4 - 180 s^6 + 35 s^8) / 128.
The reference potential V~_J of Appendix A is the same family with its own cutoff
rc~_J (reading: the paper names its reference potential by citation only).

Discrete objects, in the order of Algorithm 1:
  * the truncation box of atom J: per direction s the half-width r^b_s = m_s h_s with
    m_s = ceil(rc/h_s) + t, where t >= 0 is the smallest step for which the charge of
    all its images inside the cell, h1h2h3 sum b_J, is within eps_b Z_J of -Z_J
    (Eq. for the choice of r^b).  A node x belongs to the box of the image at c when
    |x_s - c_s| <= m_s h_s in every direction;
  * b_J'(x) = -(1/(4 pi)) Lap_h V_J' at every node of the box, V_J' evaluated
    analytically at the node and its 6 n_o stencil neighbours (in place of the
    paper's cubic-spline interpolation of a radial table);
  * b = sum of b_J' over every image J' of every atom, and
    E_self^h = 1/2 h1h2h3 sum_J' sum_box b_J' V_J';
  * the same for the reference: b~, E~_self^h, and V_c = sum_J' (V~_J' - V_J'),
    exactly zero beyond max(rc, rc~) from every image;
  * E_c^h = 1/2 h1h2h3 sum_g [(b~ + b) V_c] + E_self^h - E~_self^h (Eq. for E_c^h).
Forces (each atom J, summed over its images J'):
  * f_J,loc = h1h2h3 sum_J' sum_{box of J'} grad_h b_J' (phi - V_J')
    (Sec. 3.6, discrete local force), with b_J' at the stencil neighbours of a box
    node computed from V_J' like inside the box (V_J' is known 2 n_o nodes out, the
    paper's extra 4 n_o points per direction);
  * f_J,c = 1/2 h1h2h3 sum_J' [ sum_{box~ of J'} (grad_h b~_J' (V_c - V~_J')
    - b~_J' grad_h V~_J') + sum_{box of J'} (grad_h b_J' (V_c + V_J')
    + b_J' grad_h V_J') + sum_g grad_h (V~_J' - V_J') (b~ + b) ] (Appendix A,
    discrete correction force); the last sum covers every node where
    grad_h (V~_J' - V_J') is non-zero.
"""
from __future__ import annotations

import math
from fractions import Fraction

import numpy as np

from .fd import Grid, laplacian_weights, gradient_weights
from .scf import poisson

P_COEF = (315.0 / 128.0, -420.0 / 128.0, 378.0 / 128.0, -180.0 / 128.0, 35.0 / 128.0)
TRUNC_MAX_STEPS = 16     # the box grows by one node per direction at most this often


def v_pseudo(r, Z: float, rc: float):
    """V(r) of the synthetic pseudopotential (header): -Z/r beyond rc, the
    polynomial -(Z/rc) p(r/rc) inside."""
    r = np.asarray(r, dtype=np.float64)
    s2 = (r / rc) ** 2
    inner = -(Z / rc) * (P_COEF[0] + s2 * (P_COEF[1] + s2 * (P_COEF[2] + s2 * (P_COEF[3] + s2 * P_COEF[4]))))
    return np.where(r < rc, inner, -Z / np.where(r < rc, 1.0, r))


def b_continuous(r, Z: float, rc: float):
    """The continuous pseudocharge -Z 315/(64 pi rc^3) (1 - r^2/rc^2)^3 inside rc."""
    r = np.asarray(r, dtype=np.float64)
    s2 = (r / rc) ** 2
    return np.where(r < rc, -Z * 315.0 / (64.0 * math.pi * rc ** 3) * (1.0 - s2) ** 3, 0.0)


def self_energy_continuous(Z: float, rc: float) -> float:
    """E_self = 1/2 int b V of one atom (Sec. 2, self energy), exactly:
    (315 Z^2 / (32 rc)) int_0^1 s^2 (1 - s^2)^3 p(s) ds, the integral done in rationals."""
    # polynomial products in s, coefficient lists by power
    one_m = [Fraction(1), Fraction(0), Fraction(-3), Fraction(0), Fraction(3), Fraction(0), Fraction(-1)]
    p = [Fraction(315, 128), 0, Fraction(-420, 128), 0, Fraction(378, 128), 0, Fraction(-180, 128), 0,
         Fraction(35, 128)]
    prod = [Fraction(0)] * (len(one_m) + len(p) - 1)
    for i, a in enumerate(one_m):
        for j, c in enumerate(p):
            prod[i + j] += a * c
    integral = sum(c / (k + 3) for k, c in enumerate(prod))        # times s^2, from 0 to 1
    return float(Fraction(315, 32) * integral) * Z * Z / rc


def background_integral(Z: float, rc: float) -> float:
    """int over R^3 of (V(r) + Z/r) = 4 pi Z rc^2 int_0^1 (s - s^2 p(s)) ds, exactly."""
    p = [Fraction(315, 128), Fraction(-420, 128), Fraction(378, 128), Fraction(-180, 128), Fraction(35, 128)]
    # int s ds = 1/2 ; int s^2 * s^{2k} ds = 1/(2k+3)
    integral = Fraction(1, 2) - sum(c / (2 * k + 3) for k, c in enumerate(p))
    return 4.0 * math.pi * Z * rc * rc * float(integral)


# ---------------------------------------------------------------- lattice helpers
def _lap_b(d, Z: float, rc: float, grid: Grid):
    """b = -(1/4pi) Lap_h V at points with offsets d = (dx, dy, dz) (broadcastable
    arrays) from the atom, V sampled analytically at the stencil points."""
    dx, dy, dz = d

    def V(ax, ay, az):
        return v_pseudo(np.sqrt(ax * ax + ay * ay + az * az), Z, rc)

    lap = 0.0
    for s in range(3):
        w0, w = laplacian_weights(grid.n_o, grid.h[s])
        lap = lap + 2.0 * w0 * V(dx, dy, dz)
        for p in range(1, grid.n_o + 1):
            e = [0.0, 0.0, 0.0]
            e[s] = p * grid.h[s]
            lap = lap + w[p - 1] * (V(dx + e[0], dy + e[1], dz + e[2]) + V(dx - e[0], dy - e[1], dz - e[2]))
    return -lap / (4.0 * math.pi)


def _grad(fun, d, grid: Grid):
    """grad_h f at points with offsets d, where fun(dx, dy, dz) evaluates f at any
    offsets (central FD gradient of Sec. 3.1).  Returns a list of 3 arrays."""
    dx, dy, dz = d
    out = []
    for s in range(3):
        wt = gradient_weights(grid.n_o, grid.h[s])
        acc = 0.0
        for p in range(1, grid.n_o + 1):
            e = [0.0, 0.0, 0.0]
            e[s] = p * grid.h[s]
            acc = acc + wt[p - 1] * (fun(dx + e[0], dy + e[1], dz + e[2]) - fun(dx - e[0], dy - e[1], dz - e[2]))
        out.append(acc)
    return out


def _image_boxes(grid: Grid, Rj, m):
    """For each image a (no images across Dirichlet directions) whose box of half-widths
    m (nodes) meets the cell: (center c, [node index arrays per direction] clipped to
    the cell).  Box nodes of the image at c = R + a L: ceil(R/h) - m <= i - a n <=
    floor(R/h) + m."""
    h = grid.h
    rng = []
    for s in range(3):
        u = Rj[s] / h[s]
        lo, hi = math.ceil(u) - m[s], math.floor(u) + m[s]
        if grid.bc[s] == 1:
            shifts = [0]
        else:
            A = (abs(lo) + abs(hi)) // grid.n[s] + 2
            shifts = range(-A, A + 1)
        opts = []
        for a in shifts:
            i0, i1 = max(0, lo + a * grid.n[s]), min(grid.n[s] - 1, hi + a * grid.n[s])
            if i0 <= i1:
                opts.append((a, np.arange(i0, i1 + 1)))
        rng.append(opts)
    for az, kk in rng[2]:
        for ay, jj in rng[1]:
            for ax, ii in rng[0]:
                c = (Rj[0] + ax * grid.L[0], Rj[1] + ay * grid.L[1], Rj[2] + az * grid.L[2])
                yield c, (ii, jj, kk)


def _offsets(grid: Grid, c, idx):
    """Broadcastable offsets (dx, dy, dz) of the nodes idx = (ii, jj, kk) from c,
    shaped for arrays indexed [k, j, i]."""
    ii, jj, kk = idx
    h = grid.h
    return ((ii * h[0] - c[0])[None, None, :], (jj * h[1] - c[1])[None, :, None],
            (kk * h[2] - c[2])[:, None, None])


# ---------------------------------------------------------------- Eq. for r^b
def truncation_box(grid: Grid, Rj, Z: float, rc: float, eps_b: float):
    """Half-widths (m1, m2, m3), in nodes, of the smallest box (steps of one node per
    direction from ceil(rc/h_s)) whose discrete pseudocharge sums to -Z within eps_b Z
    (Sec. 3.2, choice of r^b; summing one unclipped box on the infinite lattice equals
    summing all images inside the cell).  Raises ValueError after TRUNC_MAX_STEPS."""
    h = grid.h
    m0 = [math.ceil(rc / h[s]) for s in range(3)]
    js, ms = [], []
    for s in range(3):
        u = Rj[s] / h[s]
        M = m0[s] + TRUNC_MAX_STEPS
        j = np.arange(math.ceil(u) - M, math.floor(u) + M + 1)
        js.append(j)
        ms.append(np.maximum(math.ceil(u) - j, j - math.floor(u)) - m0[s])   # minimal step per node
    d = ((js[0] * h[0] - Rj[0])[None, None, :], (js[1] * h[1] - Rj[1])[None, :, None],
         (js[2] * h[2] - Rj[2])[:, None, None])
    b = _lap_b(d, Z, rc, grid)
    shell = np.maximum(0, np.maximum(np.maximum(ms[0][None, None, :], ms[1][None, :, None]), ms[2][:, None, None]))
    q = np.cumsum(np.bincount(shell.ravel(), weights=(grid.dV * b).ravel(), minlength=TRUNC_MAX_STEPS + 1))
    for t in range(TRUNC_MAX_STEPS + 1):
        if abs(q[t] + Z) < eps_b * Z:
            return (m0[0] + t, m0[1] + t, m0[2] + t)
    raise ValueError(f"no truncation box within {TRUNC_MAX_STEPS} steps meets eps_b={eps_b}")


def truncation_boxes(grid: Grid, R, Z, rc, eps_b: float):
    return [truncation_box(grid, R[J], float(Z[J]), float(rc[J]), eps_b) for J in range(len(Z))]


# ---------------------------------------------------------------- Algorithm 1 and E_c
def _pseudocharge_sum(grid: Grid, R, Z, rc, boxes):
    """Algorithm 1: b on the grid and E_self^h."""
    n1, n2, n3 = grid.n
    b = np.zeros((n3, n2, n1))
    eself = 0.0
    for J in range(len(Z)):
        Zj, rj = float(Z[J]), float(rc[J])
        for c, idx in _image_boxes(grid, R[J], boxes[J]):
            d = _offsets(grid, c, idx)
            bj = _lap_b(d, Zj, rj, grid)
            vj = v_pseudo(np.sqrt(d[0] ** 2 + d[1] ** 2 + d[2] ** 2), Zj, rj)
            b[np.ix_(idx[2], idx[1], idx[0])] += bj
            eself += 0.5 * grid.dV * float(np.sum(bj * vj))
    return b.reshape(-1), eself


def _vc(grid: Grid, R, Z, rc, rc_ref):
    """V_c = sum_J' (V~_J' - V_J') on the grid (zero beyond max(rc, rc~) of every image)."""
    n1, n2, n3 = grid.n
    vc = np.zeros((n3, n2, n1))
    for J in range(len(Z)):
        Zj = float(Z[J])
        rmax = max(float(rc[J]), float(rc_ref[J]))
        m = [math.ceil(rmax / grid.h[s]) + 1 for s in range(3)]
        for c, idx in _image_boxes(grid, R[J], m):
            d = _offsets(grid, c, idx)
            r = np.sqrt(d[0] ** 2 + d[1] ** 2 + d[2] ** 2)
            vc[np.ix_(idx[2], idx[1], idx[0])] += v_pseudo(r, Zj, float(rc_ref[J])) - v_pseudo(r, Zj, float(rc[J]))
    return vc.reshape(-1)


def electrostatics_setup(grid: Grid, R, Z, rc, rc_ref, boxes, boxes_ref):
    """Everything the pseudocharge electrostatics needs at fixed atoms: b, b~, V_c,
    E_self^h, E~_self^h and E_c^h (Algorithm 1; Appendix A, discrete E_c)."""
    b, eself = _pseudocharge_sum(grid, R, Z, rc, boxes)
    bref, eself_ref = _pseudocharge_sum(grid, R, Z, rc_ref, boxes_ref)
    vc = _vc(grid, R, Z, rc, rc_ref)
    ec = 0.5 * grid.dV * float(np.dot(bref + b, vc)) + eself - eself_ref
    return {"b": b, "bref": bref, "vc": vc, "eself": eself, "eself_ref": eself_ref, "ec": ec}


def electrostatic_potential(grid: Grid, rho, b):
    """phi from -Lap_h phi = 4 pi (rho + b) on the periodic grid (mean of the right-hand
    side removed, phi with zero mean): the Poisson equation of Sec. 2."""
    return poisson(np.asarray(rho) + np.asarray(b), grid)


def electrostatic_energy(grid: Grid, rho, st, phi=None):
    """E_el = 1/2 h1h2h3 sum (rho + b) phi - E_self^h + E_c^h (Sec. 2, electrostatic
    reformulation at its maximiser phi)."""
    if phi is None:
        phi = electrostatic_potential(grid, rho, st["b"])
    return 0.5 * grid.dV * float(np.dot(np.asarray(rho) + st["b"], phi)) - st["eself"] + st["ec"]


# ---------------------------------------------------------------- forces
def local_force(grid: Grid, R, Z, rc, boxes, phi):
    """f_J,loc = h1h2h3 sum_J' sum_box grad_h b_J' (phi - V_J') (Sec. 3.6)."""
    n1, n2, n3 = grid.n
    phi3 = np.asarray(phi, dtype=np.float64).reshape(n3, n2, n1)
    F = np.zeros((len(Z), 3))
    for J in range(len(Z)):
        Zj, rj = float(Z[J]), float(rc[J])
        for c, idx in _image_boxes(grid, R[J], boxes[J]):
            d = _offsets(grid, c, idx)
            g = _grad(lambda x, y, z: _lap_b((x, y, z), Zj, rj, grid), d, grid)
            vj = v_pseudo(np.sqrt(d[0] ** 2 + d[1] ** 2 + d[2] ** 2), Zj, rj)
            w = phi3[np.ix_(idx[2], idx[1], idx[0])] - vj
            F[J] += grid.dV * np.array([np.sum(g[s] * w) for s in range(3)])
    return F


def correction_force(grid: Grid, R, Z, rc, rc_ref, boxes, boxes_ref, st):
    """f_J,c of Appendix A (discrete correction force), summed over the images J'."""
    n1, n2, n3 = grid.n
    vc3 = st["vc"].reshape(n3, n2, n1)
    bsum3 = (st["b"] + st["bref"]).reshape(n3, n2, n1)
    F = np.zeros((len(Z), 3))
    for J in range(len(Z)):
        Zj, r1, r2 = float(Z[J]), float(rc[J]), float(rc_ref[J])
        # reference terms on the reference box, pseudocharge terms on the pseudocharge box
        for rcut, box, sign in ((r2, boxes_ref[J], -1.0), (r1, boxes[J], 1.0)):
            for c, idx in _image_boxes(grid, R[J], box):
                d = _offsets(grid, c, idx)
                gb = _grad(lambda x, y, z: _lap_b((x, y, z), Zj, rcut, grid), d, grid)
                gv = _grad(lambda x, y, z: v_pseudo(np.sqrt(x * x + y * y + z * z), Zj, rcut), d, grid)
                bj = _lap_b(d, Zj, rcut, grid)
                vj = v_pseudo(np.sqrt(d[0] ** 2 + d[1] ** 2 + d[2] ** 2), Zj, rcut)
                vcl = vc3[np.ix_(idx[2], idx[1], idx[0])]
                for s in range(3):
                    F[J, s] += 0.5 * grid.dV * float(np.sum(gb[s] * (vcl + sign * vj) + sign * bj * gv[s]))
        # grad_h (V~ - V) (b~ + b) over its support: max(rc, rc~) + n_o nodes
        rmax = max(r1, r2)
        m = [math.ceil(rmax / grid.h[s]) + grid.n_o + 1 for s in range(3)]
        for c, idx in _image_boxes(grid, R[J], m):
            d = _offsets(grid, c, idx)
            gd = _grad(lambda x, y, z: (v_pseudo(np.sqrt(x * x + y * y + z * z), Zj, r2)
                                        - v_pseudo(np.sqrt(x * x + y * y + z * z), Zj, r1)), d, grid)
            bs = bsum3[np.ix_(idx[2], idx[1], idx[0])]
            for s in range(3):
                F[J, s] += 0.5 * grid.dV * float(np.sum(gd[s] * bs))
    return F
