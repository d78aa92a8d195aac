"""Flux-limited NRD residual, its Jacobian action and its transpose.

Definitions (paper Sec. 3.1-3.3 and 4.1):

* E_t - div(D_E grad E) =  sigma (T^4 - E),  T_t - div(D_T grad T) = -sigma (T^4 - E),
  sigma = z^3 / T^3, D_T = kappa T^(5/2)                    (eqs. E_td, T_td, sigma)
* cell balance with face fluxes D (u_b - u_a) / h          (eqs. E_int, diffusion_coeffs)
* face temperature T_f = (T_a + T_b) / 2; harmonic face coefficient of
  1/(3 sigma) at T_f; Wilson limiter with the face-normal |dE| / (h E_f)
* Marshak (Robin) boundary 1/2 n.D grad E + E/4 = R, not flux limited, with
  D = 1/(3 sigma) of the boundary cell                       (eq. robinbc)
* zero-flux faces for E elsewhere and for T everywhere       (eq. bcs)
* coarse-fine flux matching: the coarse flux through a face shared with a
  finer level is replaced by the mean of the fine fluxes (Sec. 3.2.1)
* BDF residual F(u) = c0 u - b - dt f(u)                  (eqs. bdf2, be, nonlinearsystem)

Readings (the paper is ambiguous):
* the printed face pair (D_r, then 2 D_r / (1 + D_r g)) is read as the true
  harmonic mean D_h = 2 T_f^3 / (3 (z_a^3 + z_b^3)) limited as
  D_h / (1 + lam D_h g); the default reading (System, lam = 1/2) is the
  printed pair literally, lam = 1 gives the Wilson form of Sec. 3.1 (the
  functions below take lam explicitly);
* face D_T = kappa T_f^(5/2) with the arithmetic face temperature;
* Robin ghost from the discrete boundary relation, giving the inflow flux
  q = 2 D_b (4 R - E_c) / (4 D_b + h) into the boundary cell;
* the analytic derivative of |x| at 0 is taken as 0.

Parity status: the face/residual formulas are pinned by special cases
(gradient-free limit, equilibrium, textbook Laplacian), the discrete energy
identity, mirror symmetry and second-order MMS convergence; the JVP by
brute-force finite differences; the VJP by the dot-product identity (one
level, siblings, two and three levels) and finite differences in z (one
and two levels).
"""
from __future__ import annotations

import numpy as np

from .hierarchy import Hierarchy


# ---------------------------------------------------------------------------
# slicing helpers: faces of a patch along axis d
# ---------------------------------------------------------------------------

def face_slices(d, n):
    """(lower-cell, upper-cell) ghosted slices over the n_d + 1 faces along
    d, interior in the tangential directions."""
    lo = [slice(1, -1)] * 3
    up = [slice(1, -1)] * 3
    lo[d] = slice(0, int(n[d]) + 1)
    up[d] = slice(1, int(n[d]) + 2)
    return tuple(lo), tuple(up)


def face_index(d, idx):
    s = [slice(None)] * 3
    s[d] = idx
    return tuple(s)


def cell_layer(d, idx):
    """Ghosted slice of interior layer idx (0-based interior) along d."""
    s = [slice(1, -1)] * 3
    s[d] = idx + 1
    return tuple(s)


# ---------------------------------------------------------------------------
# face formulas
# ---------------------------------------------------------------------------

def face_coeffs(Ea, Eb, Ta, Tb, z3a, z3b, h, kappa, lam=1.0):
    """Limited radiation coefficient D_E and conduction coefficient D_T on a
    face between lower cell a and upper cell b."""
    Tf = 0.5 * (Ta + Tb)
    Zf = z3a + z3b
    Dh = 2.0 * Tf**3 / (3.0 * Zf)
    g = np.abs(Eb - Ea) / (0.5 * h * (Ea + Eb))
    DE = Dh / (1.0 + lam * Dh * g)
    DT = kappa * Tf**2.5
    return DE, DT


def face_flux(Ea, Eb, Ta, Tb, z3a, z3b, h, kappa, lam=1.0):
    """Flux densities D_E dE/dx and D_T dT/dx through a face (lower a, upper b)."""
    DE, DT = face_coeffs(Ea, Eb, Ta, Tb, z3a, z3b, h, kappa, lam)
    return DE * (Eb - Ea) / h, DT * (Tb - Ta) / h


def face_flux_tangent(Ea, Eb, Ta, Tb, z3a, z3b, dEa, dEb, dTa, dTb, h, kappa,
                      lam=1.0):
    """Directional derivative of face_flux along (dE, dT)."""
    Tf = 0.5 * (Ta + Tb)
    dTf = 0.5 * (dTa + dTb)
    Zf = z3a + z3b
    Dh = 2.0 * Tf**3 / (3.0 * Zf)
    dDh = 3.0 * Dh * dTf / Tf
    dE = Eb - Ea
    ddE = dEb - dEa
    S = Ea + Eb
    dS = dEa + dEb
    g = np.abs(dE) / (0.5 * h * S)
    dg = np.sign(dE) * ddE / (0.5 * h * S) - g * dS / S
    den = 1.0 + lam * Dh * g
    DE = Dh / den
    dDE = (dDh - lam * Dh**2 * dg) / den**2
    DT = kappa * Tf**2.5
    dDT = 2.5 * DT * dTf / Tf
    dT = Tb - Ta
    ddT = dTb - dTa
    return (dDE * dE + DE * ddE) / h, (dDT * dT + DT * ddT) / h


def robin_D(Tc, z3c):
    """Unlimited boundary coefficient 1/(3 sigma) of the boundary cell."""
    return Tc**3 / (3.0 * z3c)


def robin_q(Ec, Tc, z3c, R, h):
    """Inflow flux density through a Marshak face into the boundary cell."""
    Db = robin_D(Tc, z3c)
    return 2.0 * Db * (4.0 * R - Ec) / (4.0 * Db + h)


def robin_q_tangent(Ec, Tc, z3c, dEc, dTc, R, h):
    Db = robin_D(Tc, z3c)
    dDb = 3.0 * Db * dTc / Tc
    den = 4.0 * Db + h
    return -2.0 * Db / den * dEc + 2.0 * (4.0 * R - Ec) * h / den**2 * dDb


# ---------------------------------------------------------------------------
# generic flux-form operator on the composite grid
# ---------------------------------------------------------------------------

def is_physical(H, p, d, s):
    N = H.N(p.level)
    return (p.lo[d] == 0) if s == 0 else (p.hi[d] == N[d])


def cf_faces(H, p, d):
    """Faces of patch p along d that separate a non-covered interior cell of
    p from a covered coarse cell.  Returns a list of
    (face_idx[m], tangential local (m, 2), covered_side) with covered_side 1
    when the covered cell is the upper one."""
    if p.level + 1 >= H.nlev:
        return []
    n = p.n
    cov = H.covered[p.pid]
    t1, t2 = [a for a in range(3) if a != d]
    out = []
    # covered status of the cells just outside the patch along d
    ext = []
    for s in (0, 1):
        lo = p.lo.copy()
        hi = p.hi.copy()
        if s == 0:
            lo[d], hi[d] = p.lo[d] - 1, p.lo[d]
        else:
            lo[d], hi[d] = p.hi[d], p.hi[d] + 1
        N = H.N(p.level)
        shape = [int(v) for v in n]
        shape[d] = 1
        if lo[d] < 0 or hi[d] > N[d]:
            ext.append(np.zeros(shape, dtype=bool))
        else:
            from .hierarchy import _box_cells
            I = _box_cells(lo, hi)
            ext.append(H.is_covered(p.level, I).reshape(shape, order="F"))
    full = np.concatenate([ext[0], cov, ext[1]], axis=d)   # n_d + 2 along d
    lo_sl, up_sl = [slice(None)] * 3, [slice(None)] * 3
    lo_sl[d] = slice(0, int(n[d]) + 1)
    up_sl[d] = slice(1, int(n[d]) + 2)
    cl = full[tuple(lo_sl)]
    cu = full[tuple(up_sl)]
    f_idx = np.arange(int(n[d]) + 1)
    shp = [1, 1, 1]
    shp[d] = -1
    fi = np.broadcast_to(f_idx.reshape(shp), cl.shape)
    lower_interior = fi >= 1
    upper_interior = fi <= int(n[d]) - 1
    # covered above, non-covered interior below
    mA = cu & ~cl & lower_interior
    mB = cl & ~cu & upper_interior
    for m, side in ((mA, 1), (mB, 0)):
        if m.any():
            idx = np.argwhere(m)
            out.append((idx[:, d], idx[:, [t1, t2]], side))
    return out


def _fine_face_values(H, p, d, faces, side, fine_flux):
    """Mean of the four fine fluxes on coarse faces of patch p."""
    t1, t2 = [a for a in range(3) if a != d]
    fidx, tloc, _ = faces
    m = len(fidx)
    acc = [np.zeros(m) for _ in fine_flux[p.pid][d]]
    for a in (0, 1):
        for b in (0, 1):
            Ic = np.zeros((m, 3), dtype=np.int64)
            Ic[:, d] = p.lo[d] + fidx - (0 if side == 1 else 1)   # covered cell
            Ic[:, t1] = p.lo[t1] + tloc[:, 0]
            Ic[:, t2] = p.lo[t2] + tloc[:, 1]
            If = 2 * Ic
            If[:, d] += 0 if side == 1 else 1
            If[:, t1] += a
            If[:, t2] += b
            pid, loc = H.locate(p.level + 1, If)
            assert np.all(pid >= 0)
            for q in np.unique(pid):
                mm = pid == q
                ll = loc[mm]
                fd = ll[:, d] + (0 if side == 1 else 1)   # local fine face index
                for k in range(len(acc)):
                    arr = fine_flux[q][d][k]
                    idx = [None] * 3
                    idx[d] = fd
                    idx[t1] = ll[:, t1]
                    idx[t2] = ll[:, t2]
                    acc[k][mm] += arr[idx[0], idx[1], idx[2]]
    return [a / 4.0 for a in acc]


def composite_divergence(H, nout, flux_fn, robin_fn=None):
    """Divergence of face fluxes on every patch with boundary handling and
    coarse-fine flux matching.

    flux_fn(p, d) -> list of nout flux arrays (n_d + 1 faces along d).
    robin_fn(p, d, s) -> flux of output 0 through a Marshak face (tangential
    array), or None.  Other physical faces carry zero flux.
    Returns div[pid][k] (interior arrays).
    """
    fl = {}
    for p in H.patches:
        fl[p.pid] = []
        for d in range(3):
            phis = [np.array(a, dtype=np.float64) for a in flux_fn(p, d)]
            for s in (0, 1):
                if not is_physical(H, p, d, s):
                    continue
                fs = face_index(d, 0 if s == 0 else int(p.n[d]))
                for k in range(nout):
                    phis[k][fs] = 0.0
                if robin_fn is not None and H.bc_E[2 * d + s] == 1:
                    phis[0][fs] = robin_fn(p, d, s)
            fl[p.pid].append(phis)
    # coarse-fine flux matching
    for p in H.patches:
        for d in range(3):
            for faces in cf_faces(H, p, d):
                fidx, tloc, side = faces
                vals = _fine_face_values(H, p, d, faces, side, fl)
                t1, t2 = [a for a in range(3) if a != d]
                idx = [None] * 3
                idx[d] = fidx
                idx[t1] = tloc[:, 0]
                idx[t2] = tloc[:, 1]
                for k in range(nout):
                    fl[p.pid][d][k][idx[0], idx[1], idx[2]] = vals[k]
    div = {}
    for p in H.patches:
        h = H.h(p.level)
        out = [np.zeros(tuple(int(v) for v in p.n)) for _ in range(nout)]
        for d in range(3):
            n = int(p.n[d])
            a = [slice(None)] * 3
            b = [slice(None)] * 3
            a[d] = slice(0, n)
            b[d] = slice(1, n + 1)
            for k in range(nout):
                phi = fl[p.pid][d][k]
                out[k] += (phi[tuple(b)] - phi[tuple(a)]) / h[d]
        div[p.pid] = out
    return div, fl


# ---------------------------------------------------------------------------
# state preparation
# ---------------------------------------------------------------------------

def ghosted_state(H: Hierarchy, E, T):
    """Ghosted copies of per-patch interior E, T with covered cells
    restricted and face ghosts filled."""
    Eg = H.from_interior(E)
    Tg = H.from_interior(T)
    H.sync([Eg, Tg])
    H.fill_ghosts([Eg, Tg])
    return Eg, Tg


def ghosted_z3(H: Hierarchy, z):
    """z is given on every level (covered cells included); ghosts use the
    same fill rules as the state; the cube is taken after the fill."""
    zg = H.from_interior(z)
    H.fill_ghosts([zg])
    return [a**3 for a in zg]


# ---------------------------------------------------------------------------
# residual
# ---------------------------------------------------------------------------

def residual(H, E, T, z, bE, bT, dt, c0, lam=1.0, parts=False):
    """F(u) = c0 u - b - dt f(u) on composite cells; covered cells -> 0."""
    Eg, Tg = ghosted_state(H, E, T)
    z3 = ghosted_z3(H, z)
    kappa = H.kappa

    def flux_fn(p, d):
        lo, up = face_slices(d, p.n)
        q = p.pid
        return face_flux(Eg[q][lo], Eg[q][up], Tg[q][lo], Tg[q][up],
                         z3[q][lo], z3[q][up], H.h(p.level)[d], kappa, lam)

    def robin_fn(p, d, s):
        q = p.pid
        c = cell_layer(d, 0 if s == 0 else int(p.n[d]) - 1)
        qf = robin_q(Eg[q][c], Tg[q][c], z3[q][c], H.robin_R[2 * d + s],
                     H.h(p.level)[d])
        return -qf if s == 0 else qf

    div, fl = composite_divergence(H, 2, flux_fn, robin_fn)
    FE, FT = [], []
    for p in H.patches:
        q = p.pid
        e = Eg[q][1:-1, 1:-1, 1:-1]
        t = Tg[q][1:-1, 1:-1, 1:-1]
        zz = z3[q][1:-1, 1:-1, 1:-1]
        S = zz / t**3 * (t**4 - e)
        fe = c0 * e - bE[q] - dt * (div[q][0] + S)
        ft = c0 * t - bT[q] - dt * (div[q][1] - S)
        cov = H.covered[q]
        fe[cov] = 0.0
        ft[cov] = 0.0
        FE.append(fe)
        FT.append(ft)
    if parts:
        return FE, FT, dict(Eg=Eg, Tg=Tg, z3=z3, flux=fl, div=div)
    return FE, FT


def residual_scale(H, E, T, z, bE, bT, dt, c0, lam=1.0):
    """Per-cell sum of magnitudes of the terms entering F (the scale for
    entries near the T^4 - E cancellation)."""
    Eg, Tg = ghosted_state(H, E, T)
    z3 = ghosted_z3(H, z)
    sE, sT = [], []
    for p in H.patches:
        q = p.pid
        h = H.h(p.level)
        fl = np.zeros(tuple(int(v) for v in p.n))
        flT = np.zeros_like(fl)
        for d in range(3):
            lo, up = face_slices(d, p.n)
            pe, pt = face_flux(Eg[q][lo], Eg[q][up], Tg[q][lo], Tg[q][up],
                               z3[q][lo], z3[q][up], h[d], H.kappa, lam)
            n = int(p.n[d])
            a = [slice(None)] * 3
            b = [slice(None)] * 3
            a[d] = slice(0, n)
            b[d] = slice(1, n + 1)
            fl += (np.abs(pe[tuple(a)]) + np.abs(pe[tuple(b)])) / h[d]
            flT += (np.abs(pt[tuple(a)]) + np.abs(pt[tuple(b)])) / h[d]
            # boundary inflow magnitude bound (4R + E) / h
            fl += 8.0 * max(H.robin_R) / h[d]
        e = Eg[q][1:-1, 1:-1, 1:-1]
        t = Tg[q][1:-1, 1:-1, 1:-1]
        zz = z3[q][1:-1, 1:-1, 1:-1]
        sig = zz / t**3
        cpl = sig * (t**4 + np.abs(e))
        sE.append(np.abs(c0 * e) + np.abs(bE[q]) + dt * (fl + cpl))
        sT.append(np.abs(c0 * t) + np.abs(bT[q]) + dt * (flT + cpl))
    return sE, sT


def jvp_scale(H, E, T, z, vE, vT, dt, c0, lam=1.0):
    """Per-cell sum of magnitudes of the terms entering J(u) v (the scale
    for entries whose terms cancel): every face's tangent flux split into
    its products, the Marshak tangent into its two terms, the coupling
    tangent into its E and T parts."""
    Eg, Tg = ghosted_state(H, E, T)
    dEg, dTg = ghosted_state(H, vE, vT)
    z3 = ghosted_z3(H, z)
    sE, sT = [], []
    for p in H.patches:
        q = p.pid
        h = H.h(p.level)
        fl = np.zeros(tuple(int(v) for v in p.n))
        flT = np.zeros_like(fl)
        for d in range(3):
            lo, up = face_slices(d, p.n)
            Ea, Eb, Ta, Tb = Eg[q][lo], Eg[q][up], Tg[q][lo], Tg[q][up]
            Tf = 0.5 * (Ta + Tb)
            dTf = 0.5 * (np.abs(dTg[q][lo]) + np.abs(dTg[q][up]))
            Dh = 2.0 * Tf**3 / (3.0 * (z3[q][lo] + z3[q][up]))
            S = Ea + Eb
            g = np.abs(Eb - Ea) / (0.5 * h[d] * S)
            dS = np.abs(dEg[q][lo]) + np.abs(dEg[q][up])
            dg = dS / (0.5 * h[d] * S) + g * dS / S
            den = 1.0 + lam * Dh * g
            dDE = (3.0 * Dh * dTf / Tf + lam * Dh**2 * dg) / den**2
            pe = (dDE * np.abs(Eb - Ea) + Dh / den * dS) / h[d]
            DT = H.kappa * Tf**2.5
            pt = (2.5 * DT * dTf / Tf * np.abs(Tb - Ta)
                  + DT * (np.abs(dTg[q][lo]) + np.abs(dTg[q][up]))) / h[d]
            n = int(p.n[d])
            a = [slice(None)] * 3
            b = [slice(None)] * 3
            a[d] = slice(0, n)
            b[d] = slice(1, n + 1)
            fl += (pe[tuple(a)] + pe[tuple(b)]) / h[d]
            flT += (pt[tuple(a)] + pt[tuple(b)]) / h[d]
            for s_ in (0, 1):                       # Marshak tangent terms
                if not (is_physical(H, p, d, s_) and H.bc_E[2 * d + s_] == 1):
                    continue
                c = cell_layer(d, 0 if s_ == 0 else n - 1)
                Ec, Tc, zc = Eg[q][c], Tg[q][c], z3[q][c]
                Db = robin_D(Tc, zc)
                dn = 4.0 * Db + h[d]
                m = (2.0 * Db / dn * np.abs(dEg[q][c])
                     + 2.0 * (4.0 * H.robin_R[2 * d + s_] + Ec) * h[d] / dn**2
                     * 3.0 * Db * np.abs(dTg[q][c]) / Tc) / h[d]
                fs = [slice(None)] * 3
                fs[d] = 0 if s_ == 0 else n - 1
                fl[tuple(fs)] += m
        e = Eg[q][1:-1, 1:-1, 1:-1]
        t = Tg[q][1:-1, 1:-1, 1:-1]
        de = np.abs(dEg[q][1:-1, 1:-1, 1:-1])
        dtt = np.abs(dTg[q][1:-1, 1:-1, 1:-1])
        zz = z3[q][1:-1, 1:-1, 1:-1]
        cpl = zz * ((1.0 + 3.0 * e / t**4) * dtt + de / t**3)
        sE.append(np.abs(c0) * de + dt * (fl + cpl))
        sT.append(np.abs(c0) * dtt + dt * (flT + cpl))
    return sE, sT


# ---------------------------------------------------------------------------
# analytic Jacobian action
# ---------------------------------------------------------------------------

def jvp(H, E, T, z, vE, vT, dt, c0, lam=1.0):
    """J(u) v for F above; covered entries -> 0.  Restriction, ghost fill
    and flux matching act on v exactly as on u (they are linear)."""
    Eg, Tg = ghosted_state(H, E, T)
    dEg, dTg = ghosted_state(H, vE, vT)
    z3 = ghosted_z3(H, z)
    kappa = H.kappa

    def flux_fn(p, d):
        lo, up = face_slices(d, p.n)
        q = p.pid
        return face_flux_tangent(Eg[q][lo], Eg[q][up], Tg[q][lo], Tg[q][up],
                                 z3[q][lo], z3[q][up], dEg[q][lo], dEg[q][up],
                                 dTg[q][lo], dTg[q][up], H.h(p.level)[d],
                                 kappa, lam)

    def robin_fn(p, d, s):
        q = p.pid
        c = cell_layer(d, 0 if s == 0 else int(p.n[d]) - 1)
        dq = robin_q_tangent(Eg[q][c], Tg[q][c], z3[q][c], dEg[q][c], dTg[q][c],
                             H.robin_R[2 * d + s], H.h(p.level)[d])
        return -dq if s == 0 else dq

    div, _ = composite_divergence(H, 2, flux_fn, robin_fn)
    JE, JT = [], []
    for p in H.patches:
        q = p.pid
        e = Eg[q][1:-1, 1:-1, 1:-1]
        t = Tg[q][1:-1, 1:-1, 1:-1]
        de = dEg[q][1:-1, 1:-1, 1:-1]
        dtt = dTg[q][1:-1, 1:-1, 1:-1]
        zz = z3[q][1:-1, 1:-1, 1:-1]
        dS = zz * ((1.0 + 3.0 * e / t**4) * dtt - de / t**3)
        je = c0 * de - dt * (div[q][0] + dS)
        jt = c0 * dtt - dt * (div[q][1] - dS)
        cov = H.covered[q]
        je[cov] = 0.0
        jt[cov] = 0.0
        JE.append(je)
        JT.append(jt)
    return JE, JT


# ---------------------------------------------------------------------------
# Jacobian-free (finite-difference) action, Sec. 4.1 (eq. Jac-free)
# ---------------------------------------------------------------------------

SQRT_EPS_MACH = float(np.sqrt(np.finfo(np.float64).eps))
U_MIN = 1e-6


def fd_epsilon(H, E, T, vE, vT):
    """Differencing parameter of Sec. 4.1: sqrt(eps_mach) <u,v> / ||v||^2
    when |<u,v>| > u_min ||v||_1, otherwise
    sqrt(eps_mach) u_min sign(<u,v>) ||v||_1 / ||v||^2, u_min = 1e-6.

    Readings: the sums are plain (no volume weights) over the composite
    cells of both fields; the undefined factor b is 1; the threshold is
    tested on |<u,v>|; sign(0) = +1.  v = 0 gives 1 (the difference is then
    exactly 0 whatever epsilon is)."""
    uv = l1 = v2 = 0.0
    for p in H.patches:
        q = p.pid
        keep = ~H.covered[q]
        for a, b in ((E[q], vE[q]), (T[q], vT[q])):
            a = a[keep]
            b = b[keep]
            uv += float(np.sum(a * b))
            l1 += float(np.sum(np.abs(b)))
            v2 += float(np.sum(b * b))
    if v2 == 0.0:
        return 1.0
    if abs(uv) > U_MIN * l1:
        return SQRT_EPS_MACH * uv / v2
    sign = 1.0 if uv >= 0.0 else -1.0
    return SQRT_EPS_MACH * U_MIN * sign * l1 / v2


def jvp_fd(H, E, T, z, vE, vT, bE, bT, dt, c0, lam=1.0):
    """(F(u + eps v) - F(u)) / eps with eps from fd_epsilon; covered
    entries -> 0 (F is 0 there on both sides)."""
    eps = fd_epsilon(H, E, T, vE, vT)
    F0E, F0T = residual(H, E, T, z, bE, bT, dt, c0, lam)
    E1 = [a + eps * b for a, b in zip(E, vE)]
    T1 = [a + eps * b for a, b in zip(T, vT)]
    F1E, F1T = residual(H, E1, T1, z, bE, bT, dt, c0, lam)
    return ([(f1 - f0) / eps for f1, f0 in zip(F1E, F0E)],
            [(f1 - f0) / eps for f1, f0 in zip(F1T, F0T)])


# ---------------------------------------------------------------------------
# transpose (scatter over faces, then the ghost fill and the restriction
# run backwards); hierarchies of any depth
# ---------------------------------------------------------------------------

def _face_partials(Ea, Eb, Ta, Tb, z3a, z3b, h, kappa, lam):
    """Partial derivatives of (Phi_E, Phi_T) w.r.t. the 6 face inputs."""
    Tf = 0.5 * (Ta + Tb)
    Zf = z3a + z3b
    Dh = 2.0 * Tf**3 / (3.0 * Zf)
    dE = Eb - Ea
    S = Ea + Eb
    g = np.abs(dE) / (0.5 * h * S)
    sg = np.sign(dE)
    den = 1.0 + lam * Dh * g
    DE = Dh / den
    dDh_dT = 1.5 * Dh / Tf                      # w.r.t. Ta or Tb
    dDh_dz = -Dh / Zf                           # w.r.t. z3a or z3b
    dg_dEb = sg / (0.5 * h * S) - g / S
    dg_dEa = -sg / (0.5 * h * S) - g / S
    dDE = lambda dDh, dg: (dDh - lam * Dh**2 * dg) / den**2
    P = {}
    P["E_Ea"] = dDE(0.0, dg_dEa) * dE / h - DE / h
    P["E_Eb"] = dDE(0.0, dg_dEb) * dE / h + DE / h
    P["E_T"] = dDE(dDh_dT, 0.0) * dE / h        # same for Ta and Tb
    P["E_z"] = dDE(dDh_dz, 0.0) * dE / h        # same for z3a and z3b
    DT = kappa * Tf**2.5
    dT = Tb - Ta
    c = 1.25 * DT / Tf * dT / h
    P["T_Ta"] = c - DT / h
    P["T_Tb"] = c + DT / h
    return P


def _adjoint_lambda(H, lam):
    """Ghosted copies of the per-patch multipliers for the transposed face
    fluxes: covered cells 0 (their residual is 0); a coarse-fine ghost holds
    1/8 of the multiplier of the coarse cell it lies in (that cell's
    residual takes the mean of the four fine face fluxes on the shared face,
    over the coarse mesh width: 1/4 x 1/2 of a fine cell's weight per fine
    flux); physical and sibling ghosts 0 (a face shared by two siblings is
    seen by both: each side's view carries its own cell's multiplier, and
    the two scatters add up to the face's)."""
    out = []
    for p, a in zip(H.patches, lam):
        g = np.zeros(p.gshape)
        x = np.array(a, dtype=np.float64)
        x[H.covered[p.pid]] = 0.0
        g[1:-1, 1:-1, 1:-1] = x
        out.append(g)
    inner = [a[1:-1, 1:-1, 1:-1] for a in out]
    for p in H.patches:
        for d in range(3):
            for s_ in range(2):
                G, gl, il, kind = H.ghost_kinds(p, d, s_)
                val = np.zeros(len(G))
                m = kind == 2
                if m.any():
                    pid, loc = H.locate(p.level - 1, G[m] // 2)
                    val[m] = [inner[q][tuple(l)] / 8.0 for q, l in zip(pid, loc)]
                out[p.pid][gl[:, 0], gl[:, 1], gl[:, 2]] = val
    return out


def _cf_sources(H, level, G, d):
    """The five sources of coarse-fine ghosts G on level `level` (face
    normal d) and their weights in g = 2/3 i + 1/3 f, i the 9, 3, 3, 1 / 16
    bilinear value of the coarse level (copy rule at the domain edges)."""
    t1, t2 = [a for a in range(3) if a != d]
    P = G // 2
    o1 = np.where(G[:, t1] % 2 == 1, 1, -1)
    o2 = np.where(G[:, t2] % 2 == 1, 1, -1)
    N = H.N(level - 1)
    e1 = np.zeros_like(P)
    e1[:, t1] = o1
    e2 = np.zeros_like(P)
    e2[:, t2] = o2
    return [(np.clip(Q, 0, N - 1), w) for Q, w in
            ((P, 9.0), (P + e1, 3.0), (P + e2, 3.0), (P + e1 + e2, 1.0))]


def vjp(H, E, T, z, lE, lT, dt, c0, lam=1.0, magnitude=False):
    """lambda^T dF/du (E and T parts) and lambda^T dF/dz (per cell, every
    level) on a hierarchy of any depth.  The residual's linear steps are
    transposed in reverse order: the face fluxes' partials are scattered to
    both cells of each face (ghost slots included); coarse faces taken over
    by flux matching carry no coarse flux, their fine fluxes feed the coarse
    cell's multiplier through the ghosts (see _adjoint_lambda); ghost
    sensitivities go back to their sources (sibling copies; coarse-fine
    interpolation: 2/3 x 9, 3, 3, 1 / 16 to the coarse cells, 1/3 to the
    fine cell); covered cells pass theirs to their eight children (the
    transposed restriction, coarse to fine); z has no restriction.  Covered
    entries of the E and T parts are 0.

    magnitude=True returns instead, per entry, the sum of the magnitudes of
    the terms that entry adds up (every product and difference taken in
    absolute values): the scale of its rounding error."""
    A = np.abs if magnitude else (lambda x: x)
    if magnitude:
        lE = [np.abs(a) for a in lE]
        lT = [np.abs(a) for a in lT]
    Eg, Tg = ghosted_state(H, E, T)
    zg = H.from_interior(z)
    H.fill_ghosts([zg])
    z3 = [a**3 for a in zg]
    aE = [np.zeros(p.gshape) for p in H.patches]
    aT = [np.zeros(p.gshape) for p in H.patches]
    aZ = [np.zeros(p.gshape) for p in H.patches]   # w.r.t. z^3, then z
    lEa = _adjoint_lambda(H, lE)
    lTa = _adjoint_lambda(H, lT)
    for p in H.patches:
        q = p.pid
        h = H.h(p.level)
        lEg, lTg = lEa[q], lTa[q]
        for d in range(3):
            lo, up = face_slices(d, p.n)
            P = _face_partials(Eg[q][lo], Eg[q][up], Tg[q][lo], Tg[q][up],
                               z3[q][lo], z3[q][up], h[d], H.kappa, lam)
            sgn = 1.0 if magnitude else -1.0
            muE = dt * (lEg[up] + sgn * lEg[lo]) / h[d]
            muT = dt * (lTg[up] + sgn * lTg[lo]) / h[d]
            P = {k: A(v) for k, v in P.items()}
            for s in (0, 1):                       # physical faces: no flux
                if is_physical(H, p, d, s):
                    fs = face_index(d, 0 if s == 0 else int(p.n[d]))
                    muE[fs] = 0.0
                    muT[fs] = 0.0
            t1, t2 = [a for a in range(3) if a != d]
            for fidx, tloc, _ in cf_faces(H, p, d):   # taken over by matching
                idx = [None] * 3
                idx[d] = fidx
                idx[t1] = tloc[:, 0]
                idx[t2] = tloc[:, 1]
                muE[idx[0], idx[1], idx[2]] = 0.0
                muT[idx[0], idx[1], idx[2]] = 0.0
            aE[q][lo] += muE * P["E_Ea"]
            aE[q][up] += muE * P["E_Eb"]
            aT[q][lo] += muE * P["E_T"] + muT * P["T_Ta"]
            aT[q][up] += muE * P["E_T"] + muT * P["T_Tb"]
            aZ[q][lo] += muE * P["E_z"]
            aZ[q][up] += muE * P["E_z"]
            for s in (0, 1):                       # Marshak faces
                if not (is_physical(H, p, d, s) and H.bc_E[2 * d + s] == 1):
                    continue
                c = cell_layer(d, 0 if s == 0 else int(p.n[d]) - 1)
                Ec, Tc, zc = Eg[q][c], Tg[q][c], z3[q][c]
                Db = robin_D(Tc, zc)
                den = 4.0 * Db + h[d]
                R = H.robin_R[2 * d + s]
                dq_dE = A(-2.0 * Db / den)
                dq_dDb = A(2.0 * (4.0 * R - Ec) * h[d] / den**2)
                # F_c gets -dt * q / h whichever side the face is on
                w = A(-dt * lEg[c] / h[d])
                aE[q][c] += w * dq_dE
                aT[q][c] += w * dq_dDb * 3.0 * Db / Tc
                aZ[q][c] += w * dq_dDb * A(-Db / zc)
        # cell terms
        e = Eg[q][1:-1, 1:-1, 1:-1]
        t = Tg[q][1:-1, 1:-1, 1:-1]
        zz = z3[q][1:-1, 1:-1, 1:-1]
        dS_dE = A(-zz / t**3)
        dS_dT = zz * (1.0 + 3.0 * e / t**4)
        dS_dz = (t + e / t**3) if magnitude else (t - e / t**3)
        # F_E has -dt S, F_T has +dt S (covered cells: multipliers 0)
        mE, mT = lEg[1:-1, 1:-1, 1:-1], lTg[1:-1, 1:-1, 1:-1]
        x = (mT + mE) if magnitude else (mT - mE)
        aE[q][1:-1, 1:-1, 1:-1] += c0 * mE + dt * x * dS_dE
        aT[q][1:-1, 1:-1, 1:-1] += c0 * mT + dt * x * dS_dT
        aZ[q][1:-1, 1:-1, 1:-1] += dt * x * dS_dz
    # w.r.t. z itself, ghosts included: a coarse-fine ghost interpolates z,
    # not z^3 (edge and corner ghosts hold NaN and receive nothing)
    aZ = [np.where(a != 0.0, 3.0 * np.nan_to_num(zg[p.pid])**2 * a, 0.0)
          for p, a in zip(H.patches, aZ)]
    # transpose of the ghost fill: scatter ghost sensitivities to sources
    for p in H.patches:
        for d in range(3):
            for s in range(2):
                G, gl, il, kind = H.ghost_kinds(p, d, s)
                for acc in (aE, aT, aZ):
                    g = acc[p.pid][gl[:, 0], gl[:, 1], gl[:, 2]]
                    m = kind == 0
                    np.add.at(acc[p.pid], (il[m, 0], il[m, 1], il[m, 2]), g[m])
                    m = kind == 1
                    if m.any():
                        pid, loc = H.locate(p.level, G[m])
                        for qq in np.unique(pid):
                            mm = pid == qq
                            ll = loc[mm] + 1
                            np.add.at(acc[qq], (ll[:, 0], ll[:, 1], ll[:, 2]),
                                      g[m][mm])
                    m = kind == 2
                    if m.any():
                        gm = g[m]
                        np.add.at(acc[p.pid], (il[m, 0], il[m, 1], il[m, 2]), gm / 3.0)
                        for Q, wq in _cf_sources(H, p.level, G[m], d):
                            pid, loc = H.locate(p.level - 1, Q)
                            for qq in np.unique(pid):
                                mm = pid == qq
                                ll = loc[mm] + 1
                                np.add.at(acc[qq], (ll[:, 0], ll[:, 1], ll[:, 2]),
                                          (2.0 / 3.0) * (wq / 16.0) * gm[mm])
                    acc[p.pid][gl[:, 0], gl[:, 1], gl[:, 2]] = 0.0
    # transposed restriction, coarse to fine (z is not restricted)
    H.sync_transpose([aE, aT])
    gE = [a[1:-1, 1:-1, 1:-1].copy() for a in aE]
    gT = [a[1:-1, 1:-1, 1:-1].copy() for a in aT]
    gz = [a[1:-1, 1:-1, 1:-1].copy() for a in aZ]
    return gE, gT, gz
