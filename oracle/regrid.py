"""Dynamic regridding (paper Sec. 5): refinement tags and the transfer of
solution data from one patch hierarchy to another.

TEST INFRASTRUCTURE ONLY (see the package header).

Tags (per cell of every patch, covered cells included, computed from the
synced and ghost-filled state of one problem):
* the paper's heuristic indicators (Sec. 5), with E_d and E_dd the
  centred first and second differences along axis d:
      tau^g = sum_d h_d |E_d|    / (0.1 max |E|),
      tau^c = sum_d h_d^2 |E_dd| / (0.1 max |E|),
  max |E| over the problem's composite cells; a cell is tagged when an
  indicator exceeds its user threshold;
* the relative gradient |grad E| / E > g_thr with the centred gradient in
  physical units, and material interfaces: a face neighbour whose z
  differs (a coarse-fine neighbour's z is that of the coarse cell it lies
  in, not an interpolation: materials are not interpolated).
Ghost values follow the state's ghost fill (copies at physical faces, so a
centred difference there is one-sided over half the distance).

Transfer (conservative linear refinement, Sec. 5): new level 0 copies the
old level 0; every new level l >= 1 is first filled by refining the new
level l - 1 and then overwritten with the old level-l values wherever an
old level-l patch holds the cell.  Old covered cells hold the mean of their
children, so a coarsened region receives the mean of the old fine data.
Refinement of coarse cell P to its child C:
      u_C = u_P + sum_d (+-1/4) s_d,
      s_d = minmod(u_{P+e_d} - u_P, u_P - u_{P-e_d}),
the sign + for the upper child along d; minmod(a, b) = 0 unless a and b
have the same sign, else the one of smaller magnitude.  Coarse neighbours
outside the domain copy the cell (zero difference).  The 8 children
average to u_P exactly up to rounding (conservation), and each child is at
least u_P / 4 > 0 (positivity: a same-signed slope is smaller in
magnitude than u_P).  Linear fields are reproduced exactly away from
physical faces.  The result is synced (covered cells = mean of children).

Readings (the paper names the method only): the limiter is minmod; the
refinement source is the new coarser level (so a cell two levels finer than
any old data is refined twice); z is not transferred (it is sampled on the
new hierarchy by the caller, as at creation).

Parity status: pinned by conservation of sum V E to round-off, positivity,
exactness on linear fields, the identity transfer, and a brute-force
evaluation of one refined cell from the formula above.
"""
from __future__ import annotations

import numpy as np

from .hierarchy import Hierarchy, _box_cells


# ---------------------------------------------------------------------------
# tags
# ---------------------------------------------------------------------------

def _neighbours(Eg, d):
    """(E_{i-1}, E_{i+1}) along d over the interior of a ghosted array."""
    lo = [slice(1, -1)] * 3
    up = [slice(1, -1)] * 3
    lo[d] = slice(0, -2)
    up[d] = slice(2, None)
    return Eg[tuple(lo)], Eg[tuple(up)]


def tags(H: Hierarchy, E, z, grad=0.0, z_interface=False, tau_g=0.0, tau_c=0.0):
    """Per-patch boolean tag arrays of one problem.

    E, z: per-patch interior arrays (E synced by the caller or not: it is
    synced here).  grad > 0 enables |grad E| / E > grad; z_interface enables
    the material-interface tag; tau_g, tau_c > 0 enable the paper's
    indicators with those thresholds."""
    Eg = H.from_interior(E)
    H.sync([Eg])
    H.fill_ghosts([Eg])
    zg = H.from_interior(z)
    H.fill_ghosts([zg], coarse_fine="parent")
    emax = 0.0
    for p in H.patches:
        e = Eg[p.pid][1:-1, 1:-1, 1:-1]
        emax = max(emax, float(np.max(np.abs(e[~H.covered[p.pid]]))))
    den = 0.1 * emax
    out = []
    for p in H.patches:
        h = H.h(p.level)
        e = Eg[p.pid][1:-1, 1:-1, 1:-1]
        t = np.zeros(e.shape, dtype=bool)
        if grad > 0.0:
            g2 = np.zeros(e.shape)
            for d in range(3):
                em, ep = _neighbours(Eg[p.pid], d)
                ed = (ep - em) / (2.0 * h[d])
                g2 = g2 + ed * ed
            t |= g2 > (grad * e) * (grad * e)
        if z_interface:
            zc = zg[p.pid][1:-1, 1:-1, 1:-1]
            for d in range(3):
                zm, zp = _neighbours(zg[p.pid], d)
                t |= (zm != zc) | (zp != zc)
        if tau_g > 0.0 or tau_c > 0.0:
            num_g = np.zeros(e.shape)
            num_c = np.zeros(e.shape)
            for d in range(3):
                em, ep = _neighbours(Eg[p.pid], d)
                num_g = num_g + 0.5 * np.abs(ep - em)
                num_c = num_c + np.abs((ep - e) - (e - em))
            if tau_g > 0.0:
                t |= (num_g / den) > tau_g
            if tau_c > 0.0:
                t |= (num_c / den) > tau_c
        out.append(t)
    return out


# ---------------------------------------------------------------------------
# transfer
# ---------------------------------------------------------------------------

def minmod(a, b):
    return np.where((a > 0.0) & (b > 0.0), np.minimum(a, b),
                    np.where((a < 0.0) & (b < 0.0), np.maximum(a, b), 0.0))


def _level_value(H, vals, lev, I):
    """Values of per-patch interior arrays on level lev at level indices I
    (copy rule outside the domain)."""
    I = np.clip(I, 0, H.N(lev) - 1)
    pid, loc = H.locate(lev, I)
    if np.any(pid < 0):
        raise ValueError("refinement source outside the coarser level (nesting)")
    out = np.empty(len(I))
    for q in np.unique(pid):
        m = pid == q
        l = loc[m]
        out[m] = vals[q][l[:, 0], l[:, 1], l[:, 2]]
    return out


def refine_cells(H, vals, lev, I):
    """Conservative minmod-limited linear refinement of level lev - 1 of H
    (per-patch interior arrays vals) at the level-lev indices I."""
    P = I // 2
    up = I % 2 == 1
    uP = _level_value(H, vals, lev - 1, P)
    v = uP.copy()
    for d in range(3):
        e = np.zeros(3, dtype=np.int64)
        e[d] = 1
        a = _level_value(H, vals, lev - 1, P + e) - uP
        b = uP - _level_value(H, vals, lev - 1, P - e)
        s = minmod(a, b)
        v = v + np.where(up[:, d], 0.25 * s, -0.25 * s)
    return v


def transfer(Hold: Hierarchy, old, Hnew: Hierarchy):
    """Per-patch interior arrays of one field on Hnew from those on Hold
    (which must be synced: covered cells = mean of children)."""
    new = [np.zeros(tuple(int(v) for v in p.n)) for p in Hnew.patches]
    for lev in range(Hnew.nlev):
        for p in Hnew.by_level[lev]:
            I = _box_cells(p.lo, p.hi)
            shape = tuple(int(v) for v in p.n)
            if lev == 0:
                vals = _level_value(Hold, old, 0, I)
            else:
                vals = refine_cells(Hnew, new, lev, I)
                if lev < Hold.nlev:
                    pid, loc = Hold.locate(lev, I)
                    m = pid >= 0
                    if m.any():
                        vals[m] = _level_value(Hold, old, lev, I[m])
            new[p.pid] = vals.reshape(shape, order="F")
    g = Hnew.from_interior(new)
    Hnew.sync([g])
    return Hnew.interior(g)
