"""Physics-based preconditioner (paper Sec. 4.2-4.3, Alg. 1).

The Newton Jacobian is approximated by the 2x2 block operator L^k with
diffusion coefficients frozen at the Newton iterate u^k and
beta = dt (1 + alpha) / (1 + 2 alpha), split multiplicatively as
L^k ~ P1 P2 (Sec. 4.2):

* P2 = [[1 + sigma beta, -sigma beta T^3], [-sigma beta, 1 + sigma beta T^3]]
  per cell, inverted in closed form;
* P1 = diag(I - beta div D_E grad, I - beta div D_T grad), each block
  approximately inverted by one FAC V(1,0) cycle (Alg. 1) with one red-black
  Gauss-Seidel sweep per refinement level and, on the coarsest level, one
  multigrid V(1,1) cycle (Sec. 4.3 allows either a V-cycle or smoothing).

y = P^-1 w = P2^-1 (P1^-1 w).

Readings (the paper is silent or terse):
* the E block keeps the Marshak boundary, linearised with D frozen:
  the boundary cell gains 2 beta D_b / ((4 D_b + h) h) on the diagonal;
* level operators treat coarse-fine ghosts of a correction with coarse
  values 0, i.e. g = e_c / 3, folded into the diagonal; the composite
  operator uses the full linear interpolation and flux matching;
* FAC correction P^c_l adds e^l on level l and its trilinear prolongation
  (weights 3/4, 1/4 per axis; the paper's "bilinear" in 3D) on every finer
  level; the composite residual is recomputed over all levels after each
  correction and covered cells are re-synchronised;
* red cells (even i+j+k in level index space) are relaxed first; sibling
  ghosts are refreshed between the two half-sweeps;
* base multigrid on the base grid gathered from the level-0 patches (which
  tile it): coarsen by 2 while every extent is even and > 5; coarse
  face coefficient = mean of the four fine ones it covers; boundary cells
  re-discretised with the coarse h; restriction = mean of 8; bottom grid
  solved exactly (dense);
* trilinear prolongation and coarse-fine sources outside the domain use the
  copy rule.

Parity status: P2 pinned by numpy.linalg.solve; the level/MG operators by
assembled sparse matrices (symmetry, the 7-point Laplacian special case,
exact solve when the bottom grid is the whole grid) and by multigrid
contraction; the composite operator (Marshak linearisation, coarse-fine
treatment) by the analytic Jacobian's diffusion part where freezing D is
exact; red-black sweeps and FAC cycles by bitwise invariance under
splitting a level's patches into siblings; FAC by stationary convergence on
two-level problems and by a contraction that stays level independent on
2-4 nested levels (the prolongation chain to every finer level).
"""
from __future__ import annotations

import numpy as np

from .operators import (cf_faces, composite_divergence, face_coeffs,
                        face_slices, ghosted_state, ghosted_z3, is_physical,
                        robin_D)


# ---------------------------------------------------------------------------
# P2
# ---------------------------------------------------------------------------

def p2_matrix(T, z3, beta, mode="paper"):
    """Entries (a, b, c, d) of the 2x2 coupling block per cell."""
    sig = z3 / T**3
    k = 4.0 if mode == "frozen4" else 1.0
    a = 1.0 + sig * beta
    b = -k * sig * beta * T**3
    c = -sig * beta
    d = 1.0 + k * sig * beta * T**3
    return a, b, c, d


def p2_solve(T, z3, beta, eE, eT, mode="paper"):
    a, b, c, d = p2_matrix(T, z3, beta, mode)
    det = a * d - b * c
    return (d * eE - b * eT) / det, (a * eT - c * eE) / det


def p2_solve_transpose(T, z3, beta, eE, eT, mode="paper"):
    a, b, c, d = p2_matrix(T, z3, beta, mode)
    det = a * d - b * c
    return (d * eE - c * eT) / det, (a * eT - b * eE) / det


# ---------------------------------------------------------------------------
# frozen coefficients at u^k
# ---------------------------------------------------------------------------

class Snapshot:
    """Coefficients of L^k frozen at u^k.

    D[f][pid][d]: face coefficient arrays (n_d + 1 faces along d) for field
    f = 0 (E, limited D_E) and f = 1 (T, D_T).  On physical faces they hold
    D_b of the boundary cell for a Marshak face of E and 0 otherwise.
    robin[f][pid][d] = (low, high) flags of Marshak faces.
    """

    def __init__(self, H, E, T, z, beta, lam=1.0, p2_mode="paper", fac_nu=(1, 0),
                 fac_smoother="rbgs", fac_base="mg", fac_cycle="mult"):
        self.H = H
        self.fac_cycle = fac_cycle            # "mult": Alg. 1; "afacx": AFACx
        self.beta = float(beta)
        self.p2_mode = p2_mode
        self.fac_nu = tuple(fac_nu)
        self.fac_smoother = fac_smoother      # "rbgs" or "jacobi" on levels >= 1
        self.fac_base = fac_base              # "mg": V-cycle on level 0; "smooth": sweeps
        Eg, Tg = ghosted_state(H, E, T)
        z3 = ghosted_z3(H, z)
        self.T = [a[1:-1, 1:-1, 1:-1].copy() for a in Tg]
        self.z3 = [a[1:-1, 1:-1, 1:-1].copy() for a in z3]
        self.D = [{}, {}]
        self.robin = [{}, {}]
        for p in H.patches:
            q = p.pid
            h = H.h(p.level)
            self.D[0][q], self.D[1][q] = [], []
            self.robin[0][q], self.robin[1][q] = [], []
            for d in range(3):
                lo, up = face_slices(d, p.n)
                DE, DT = face_coeffs(Eg[q][lo], Eg[q][up], Tg[q][lo], Tg[q][up],
                                     z3[q][lo], z3[q][up], h[d], H.kappa, lam)
                rob = [False, False]
                for s in (0, 1):
                    if not is_physical(H, p, d, s):
                        continue
                    fi = 0 if s == 0 else int(p.n[d])
                    fs = [slice(None)] * 3
                    fs[d] = fi
                    DT[tuple(fs)] = 0.0
                    if H.bc_E[2 * d + s] == 1:
                        cs = [slice(1, -1)] * 3
                        cs[d] = 1 if s == 0 else int(p.n[d])
                        DE[tuple(fs)] = robin_D(Tg[q][tuple(cs)], z3[q][tuple(cs)])
                        rob[s] = True
                    else:
                        DE[tuple(fs)] = 0.0
                self.D[0][q].append(DE)
                self.D[1][q].append(DT)
                self.robin[0][q].append(tuple(rob))
                self.robin[1][q].append((False, False))


def robin_coef(beta, Db, h):
    return 2.0 * beta * Db / ((4.0 * Db + h) * h)


# ---------------------------------------------------------------------------
# level operator pieces: neighbour weights and diagonal
# ---------------------------------------------------------------------------

def level_weights(H, snap, f, p):
    """For patch p: neighbour weights w[d] on the n_d + 1 faces (beta D/h^2
    on faces whose far cell is read: interior and sibling faces, 0
    elsewhere) and the diagonal (1 + sum of beta D/h^2 over interior and
    sibling faces + 2/3 of it over coarse-fine faces + the Marshak term)."""
    q = p.pid
    h = H.h(p.level)
    beta = snap.beta
    n = tuple(int(v) for v in p.n)
    diag = np.ones(n)
    w = []
    for d in range(3):
        D = snap.D[f][q][d]
        a = beta * D / h[d] ** 2
        wd = a.copy()
        fold = a.copy()                          # contribution to the diagonal
        for s in (0, 1):
            fi = 0 if s == 0 else n[d]
            fs = [slice(None)] * 3
            fs[d] = fi
            fs = tuple(fs)
            if is_physical(H, p, d, s):
                wd[fs] = 0.0
                if snap.robin[f][q][d][s]:
                    fold[fs] = robin_coef(beta, D[fs], h[d])
                else:
                    fold[fs] = 0.0
            else:
                _, _, _, kind = H.ghost_kinds(p, d, s)
                shape = list(n)
                shape[d] = 1
                cf = np.take(kind.reshape(shape, order="F"), 0, axis=d) == 2
                wd[fs][cf] = 0.0                 # views: edits land in wd
                fold[fs][cf] = (2.0 / 3.0) * a[fs][cf]
        lo = [slice(None)] * 3
        hi = [slice(None)] * 3
        lo[d] = slice(0, n[d])
        hi[d] = slice(1, n[d] + 1)
        diag += fold[tuple(lo)] + fold[tuple(hi)]
        w.append(wd)
    return w, diag


def exchange_siblings(H, level, arrs):
    for p in H.by_level[level]:
        for d in range(3):
            for s in range(2):
                G, gl, il, kind = H.ghost_kinds(p, d, s)
                m = kind == 1
                if m.any():
                    arrs[p.pid][gl[m, 0], gl[m, 1], gl[m, 2]] = \
                        H.value_at(arrs, level, G[m])


def _neighbour_sum(w, e, n):
    """sum_d (w_lo e_{i-1} + w_hi e_{i+1}) over interior cells of ghosted e."""
    out = np.zeros(n)
    for d in range(3):
        lo = [slice(None)] * 3
        hi = [slice(None)] * 3
        lo[d] = slice(0, n[d])
        hi[d] = slice(1, n[d] + 1)
        em = [slice(1, -1)] * 3
        ep = [slice(1, -1)] * 3
        em[d] = slice(0, n[d])
        ep[d] = slice(2, n[d] + 2)
        out += w[d][tuple(lo)] * e[tuple(em)] + w[d][tuple(hi)] * e[tuple(ep)]
    return out


def colour_mask(lo, n, colour):
    I = [np.arange(lo[d], lo[d] + n[d]) for d in range(3)]
    X, Y, Z = np.meshgrid(*I, indexing="ij")
    return (X + Y + Z) % 2 == colour


def rbgs_level(H, snap, f, level, rhs, e, weights=None, region=None):
    """One red-black Gauss-Seidel sweep on all cells of a level (covered
    cells included) for A^l e = rhs; e ghosted per patch, updated in place.
    region (pid -> boolean interior array): only those cells are relaxed,
    every other cell keeps its value."""
    plist = H.by_level[level]
    if weights is None:
        weights = {p.pid: level_weights(H, snap, f, p) for p in plist}
    for colour in (0, 1):
        exchange_siblings(H, level, e)
        new = {}
        for p in plist:
            n = tuple(int(v) for v in p.n)
            w, diag = weights[p.pid]
            val = (rhs[p.pid] + _neighbour_sum(w, e[p.pid], n)) / diag
            m = colour_mask(p.lo, n, colour)
            if region is not None:
                m = m & region[p.pid]
            new[p.pid] = (val, m)
        for p in plist:
            val, m = new[p.pid]
            inner = e[p.pid][1:-1, 1:-1, 1:-1]
            inner[m] = val[m]


# Damping of the point Jacobi smoother: 2d / (2d + 1) in d = 3 dimensions,
# the weight that damps the upper half of the 7-point Laplacian's spectrum
# best (the paper names the smoother, not its weight).
JACOBI_OMEGA = 6.0 / 7.0


def jacobi_level(H, snap, f, level, rhs, e, omega=JACOBI_OMEGA, weights=None):
    """One damped point Jacobi sweep on all cells of a level (covered cells
    included) for A^l e = rhs: every cell from the same old values,
    e <- (1 - omega) e + omega (rhs + sum w e_nb) / diag; e ghosted per
    patch (sibling ghosts exchanged first), updated in place."""
    plist = H.by_level[level]
    if weights is None:
        weights = {p.pid: level_weights(H, snap, f, p) for p in plist}
    exchange_siblings(H, level, e)
    new = {}
    for p in plist:
        n = tuple(int(v) for v in p.n)
        w, diag = weights[p.pid]
        inner = e[p.pid][1:-1, 1:-1, 1:-1]
        new[p.pid] = (1.0 - omega) * inner + \
            omega * ((rhs[p.pid] + _neighbour_sum(w, e[p.pid], n)) / diag)
    for p in plist:
        e[p.pid][1:-1, 1:-1, 1:-1] = new[p.pid]


def line_gs_level(H, snap, f, level, rhs, e, weights=None):
    """One block Gauss-Seidel sweep on all cells of a level for A^l e = rhs
    (the third level smoother Sec. 4.3 names).  Reading: the blocks are the
    x-lines of each patch (all its cells with the same j, k); lines are
    coloured by the parity of j + k in level index space and the red lines
    go first; each line is solved exactly for its own cells (a tridiagonal
    system of the level operator along x) with every other value held: the
    y and z neighbours (lines of the other colour, or sibling and
    coarse-fine ghosts) and, at the patch's x ends, the sibling ghosts.
    Sibling ghosts are exchanged before each colour.  e ghosted per patch,
    updated in place."""
    plist = H.by_level[level]
    if weights is None:
        weights = {p.pid: level_weights(H, snap, f, p) for p in plist}
    for colour in (0, 1):
        exchange_siblings(H, level, e)
        new = {}
        for p in plist:
            n = tuple(int(v) for v in p.n)
            w, diag = weights[p.pid]
            g = e[p.pid]
            # right-hand side with the y, z neighbours and the x-end ghosts
            b = rhs[p.pid].copy()
            for d in (1, 2):
                lo = [slice(None)] * 3
                hi = [slice(None)] * 3
                lo[d] = slice(0, n[d])
                hi[d] = slice(1, n[d] + 1)
                em = [slice(1, -1)] * 3
                ep = [slice(1, -1)] * 3
                em[d] = slice(0, n[d])
                ep[d] = slice(2, n[d] + 2)
                b = b + w[d][tuple(lo)] * g[tuple(em)] + w[d][tuple(hi)] * g[tuple(ep)]
            b[0] = b[0] + w[0][0] * g[0, 1:-1, 1:-1]
            b[-1] = b[-1] + w[0][n[0]] * g[n[0] + 1, 1:-1, 1:-1]
            # tridiagonal along x: -w_lo x_{i-1} + diag x_i - w_hi x_{i+1} = b_i
            sub = -w[0][1:n[0]]                 # coupling of i and i - 1, i >= 1
            x = _thomas(sub, diag, sub, b)
            J = np.arange(p.lo[1], p.hi[1])[:, None]
            K = np.arange(p.lo[2], p.hi[2])[None, :]
            new[p.pid] = (x, ((J + K) % 2 == colour))
        for p in plist:
            x, m = new[p.pid]
            inner = e[p.pid][1:-1, 1:-1, 1:-1]
            inner[:, m] = x[:, m]


def _thomas(a, b, c, d):
    """Solves the tridiagonal systems a_i x_{i-1} + b_i x_i + c_i x_{i+1} =
    d_i along axis 0 (a, c: n - 1 entries, b, d: n) for every (j, k)."""
    n = b.shape[0]
    cp = np.zeros_like(b)
    dp = np.zeros_like(b)
    cp[0] = c[0] / b[0] if n > 1 else 0.0
    dp[0] = d[0] / b[0]
    for i in range(1, n):
        den = b[i] - a[i - 1] * cp[i - 1]
        if i < n - 1:
            cp[i] = c[i] / den
        dp[i] = (d[i] - a[i - 1] * dp[i - 1]) / den
    x = np.zeros_like(b)
    x[n - 1] = dp[n - 1]
    for i in range(n - 2, -1, -1):
        x[i] = dp[i] - cp[i] * x[i + 1]
    return x


# ---------------------------------------------------------------------------
# base-level multigrid (level 0 must be a single box)
# ---------------------------------------------------------------------------

class MGGrid:
    def __init__(self, n, h, D, robin):
        self.n = tuple(int(v) for v in n)
        self.h = np.asarray(h, dtype=np.float64)
        self.D = D              # list over d of face arrays
        self.robin = robin      # list over d of (low, high)

    def weights(self, beta):
        n = self.n
        diag = np.ones(n)
        w = []
        for d in range(3):
            a = beta * self.D[d] / self.h[d] ** 2
            wd = a.copy()
            fold = a.copy()
            for s in (0, 1):
                fs = [slice(None)] * 3
                fs[d] = 0 if s == 0 else n[d]
                fs = tuple(fs)
                wd[fs] = 0.0
                fold[fs] = (robin_coef(beta, self.D[d][fs], self.h[d])
                            if self.robin[d][s] else 0.0)
            lo = [slice(None)] * 3
            hi = [slice(None)] * 3
            lo[d] = slice(0, n[d])
            hi[d] = slice(1, n[d] + 1)
            diag += fold[tuple(lo)] + fold[tuple(hi)]
            w.append(wd)
        return w, diag

    def coarsen(self):
        nc = tuple(v // 2 for v in self.n)
        Dc = []
        for d in range(3):
            F = self.D[d]
            t1, t2 = [a for a in range(3) if a != d]
            sl = [slice(None)] * 3
            sl[d] = slice(0, None, 2)
            Fd = F[tuple(sl)]                   # coarse face positions
            acc = 0.0
            for a in (0, 1):
                for b in (0, 1):
                    s2 = [slice(None)] * 3
                    s2[t1] = slice(a, None, 2)
                    s2[t2] = slice(b, None, 2)
                    acc = acc + Fd[tuple(s2)]
            Dc.append(acc / 4.0)
        return MGGrid(nc, 2.0 * self.h, Dc, self.robin)


def can_coarsen(n):
    return all(v % 2 == 0 and v > 5 for v in n)


def gather_base(H, arrs):
    """The level-0 patches' interior arrays as one array over the base grid
    (level 0 tiles it)."""
    out = np.zeros(tuple(int(v) for v in H.base_n))
    for p in H.by_level[0]:
        out[tuple(slice(int(p.lo[d]), int(p.hi[d])) for d in range(3))] = arrs[p.pid]
    return out


def scatter_base(H, full):
    """{pid: interior array} of the level-0 patches cut from a base-grid array."""
    return {p.pid: full[tuple(slice(int(p.lo[d]), int(p.hi[d])) for d in range(3))].copy()
            for p in H.by_level[0]}


def build_mg(H, snap, f):
    """Multigrid grids below level 0: grid 0 is the base grid gathered from
    the level-0 patches (a face shared by two patches carries the same
    frozen coefficient in both), coarsened by 2 while every extent is even
    and > 5."""
    n = tuple(int(v) for v in H.base_n)
    D = []
    for d in range(3):
        shape = list(n)
        shape[d] += 1
        Dd = np.zeros(shape)
        for p in H.by_level[0]:
            sl = [slice(int(p.lo[a]), int(p.hi[a])) for a in range(3)]
            sl[d] = slice(int(p.lo[d]), int(p.hi[d]) + 1)
            Dd[tuple(sl)] = snap.D[f][p.pid][d]
        D.append(Dd)
    robin = [((H.bc_E[2 * d] == 1 and f == 0), (H.bc_E[2 * d + 1] == 1 and f == 0))
             for d in range(3)]
    g = MGGrid(n, H.h(0), D, robin)
    grids = [g]
    while can_coarsen(grids[-1].n):
        grids.append(grids[-1].coarsen())
    return grids


def _pad(e):
    out = np.zeros(tuple(v + 2 for v in e.shape))
    out[1:-1, 1:-1, 1:-1] = e
    return out


def mg_apply_op(w, diag, e):
    return diag * e - _neighbour_sum(w, _pad(e), e.shape)


def mg_rbgs(w, diag, rhs, e):
    n = e.shape
    for colour in (0, 1):
        val = (rhs + _neighbour_sum(w, _pad(e), n)) / diag
        m = colour_mask((0, 0, 0), n, colour)
        e[m] = val[m]


def restrict_mean(r):
    return 0.125 * sum(r[a::2, b::2, c::2] for a in (0, 1) for b in (0, 1)
                       for c in (0, 1))


def prolong_trilinear(ec, nf):
    """Cell-centred trilinear prolongation of ec to a grid of shape nf whose
    cells 2I, 2I+1 refine coarse cell I; copy rule beyond the edges."""
    out = np.zeros(nf)
    nc = ec.shape
    idx = [np.arange(nf[d]) for d in range(3)]
    par = [i // 2 for i in idx]
    nb = [np.clip(par[d] + np.where(idx[d] % 2 == 1, 1, -1), 0, nc[d] - 1)
          for d in range(3)]
    for a in (0, 1):
        for b in (0, 1):
            for c in (0, 1):
                ix = par[0] if a == 0 else nb[0]
                iy = par[1] if b == 0 else nb[1]
                iz = par[2] if c == 0 else nb[2]
                wgt = (0.75 if a == 0 else 0.25) * (0.75 if b == 0 else 0.25) \
                    * (0.75 if c == 0 else 0.25)
                out += wgt * ec[np.ix_(ix, iy, iz)]
    return out


def assemble_dense(w, diag):
    n = diag.shape
    N = int(np.prod(n))
    A = np.diag(diag.ravel(order="F"))
    idx = np.arange(N).reshape(n, order="F")
    for d in range(3):
        lo = [slice(None)] * 3
        lo[d] = slice(1, n[d])               # faces between cells i-1 and i
        wf = w[d][tuple(lo)]
        a = [slice(None)] * 3
        b = [slice(None)] * 3
        a[d] = slice(0, n[d] - 1)
        b[d] = slice(1, n[d])
        ia = idx[tuple(a)].ravel(order="F")
        ib = idx[tuple(b)].ravel(order="F")
        wv = wf.ravel(order="F")
        A[ia, ib] -= wv
        A[ib, ia] -= wv
    return A


def mg_vcycle(grids, beta, rhs, level=0, nu_pre=1, nu_post=1, cache=None):
    g = grids[level]
    if cache is None:
        cache = {}
    if level not in cache:
        cache[level] = g.weights(beta)
    w, diag = cache[level]
    if level == len(grids) - 1:
        A = assemble_dense(w, diag)
        x = np.linalg.solve(A, rhs.ravel(order="F"))
        return x.reshape(rhs.shape, order="F")
    e = np.zeros(rhs.shape)
    for _ in range(nu_pre):
        mg_rbgs(w, diag, rhs, e)
    r = rhs - mg_apply_op(w, diag, e)
    ec = mg_vcycle(grids, beta, restrict_mean(r), level + 1, nu_pre, nu_post,
                   cache)
    e += prolong_trilinear(ec, g.n)
    for _ in range(nu_post):
        mg_rbgs(w, diag, rhs, e)
    return e


# ---------------------------------------------------------------------------
# composite operator and FAC
# ---------------------------------------------------------------------------

def composite_apply(H, snap, f, u):
    """A^c u on composite cells (covered entries 0); u per-patch interior."""
    ug = H.from_interior(u)
    H.sync([ug])
    H.fill_ghosts([ug])
    beta = snap.beta

    def flux_fn(p, d):
        lo, up = face_slices(d, p.n)
        q = p.pid
        return [snap.D[f][q][d] * (ug[q][up] - ug[q][lo]) / H.h(p.level)[d]]

    def robin_fn(p, d, s):
        q = p.pid
        h = H.h(p.level)[d]
        fs = [slice(None)] * 3
        fs[d] = 0 if s == 0 else int(p.n[d])
        Db = snap.D[f][q][d][tuple(fs)]
        cs = [slice(1, -1)] * 3
        cs[d] = 1 if s == 0 else int(p.n[d])
        uc = ug[q][tuple(cs)]
        qlin = -2.0 * Db * uc / (4.0 * Db + h)
        return -qlin if s == 0 else qlin

    div, _ = composite_divergence(H, 1, flux_fn, robin_fn if f == 0 else None)
    out = []
    for p in H.patches:
        x = ug[p.pid][1:-1, 1:-1, 1:-1] - beta * div[p.pid][0]
        x[H.covered[p.pid]] = 0.0
        out.append(x)
    return out


def prolong_level(H, lev, e_coarse):
    """Trilinear prolongation of level lev-1 values (per patch, interior,
    all cells) onto every cell of level lev."""
    out = []
    N = H.N(lev - 1)
    for p in H.by_level[lev]:
        n = tuple(int(v) for v in p.n)
        I = [np.arange(p.lo[d], p.hi[d]) for d in range(3)]
        par = [i // 2 for i in I]
        nb = [par[d] + np.where(I[d] % 2 == 1, 1, -1) for d in range(3)]
        acc = np.zeros(n)
        for a in (0, 1):
            for b in (0, 1):
                for c in (0, 1):
                    ix = par[0] if a == 0 else nb[0]
                    iy = par[1] if b == 0 else nb[1]
                    iz = par[2] if c == 0 else nb[2]
                    X, Y, Z = np.meshgrid(ix, iy, iz, indexing="ij")
                    Q = np.stack([X.ravel(order="F"), Y.ravel(order="F"),
                                  Z.ravel(order="F")], axis=1)
                    Q = np.clip(Q, 0, N - 1)
                    v = _level_values(H, lev - 1, e_coarse, Q).reshape(n, order="F")
                    wgt = (0.75 if a == 0 else 0.25) * (0.75 if b == 0 else 0.25) \
                        * (0.75 if c == 0 else 0.25)
                    acc += wgt * v
        out.append((p.pid, acc))
    return out


def _level_values(H, lev, vals, Q):
    """vals: dict pid -> interior array on level lev."""
    pid, loc = H.locate(lev, Q)
    assert np.all(pid >= 0)
    out = np.empty(len(Q))
    for q in np.unique(pid):
        m = pid == q
        l = loc[m]
        out[m] = vals[q][l[:, 0], l[:, 1], l[:, 2]]
    return out


def fac_vcycle(H, snap, f, rhs, mg_grids=None, nu=None):
    """One FAC V(m,n) cycle for A^c u = rhs from u = 0 (Alg. 1), nu = (m, n)
    (default snap.fac_nu, else (1, 0)); the level smoother is red-black
    Gauss-Seidel or, with snap.fac_smoother == "jacobi", damped point Jacobi
    (or "line", block Gauss-Seidel on x-lines)
    (Sec. 4.3 names both); snap.fac_base == "smooth" replaces the base
    level's V-cycle by m smoothing sweeps (what the paper's runs did).

    Down-sweep, finest level to level 1: composite residual, m smoothing
    sweeps from zero on the level, correction of u on the level and (by
    trilinear prolongation) on every finer level.  Level 0: one multigrid
    V-cycle.  Up-sweep, level 1 to the finest (when n > 0): the composite
    residual refreshed with every correction so far, n sweeps from zero,
    the same correction.  rhs, result: per-patch interior arrays (result
    covered cells synced).
    """
    if nu is None:
        nu = getattr(snap, "fac_nu", (1, 0))
    smoother = getattr(snap, "fac_smoother", "rbgs")
    m_pre, n_post = int(nu[0]), int(nu[1])
    u = [np.zeros(tuple(int(v) for v in p.n)) for p in H.patches]
    L = H.nlev - 1

    def level_rhs():
        r = composite_apply(H, snap, f, u)
        r = [rhs[p.pid] - r[p.pid] for p in H.patches]
        rg = H.from_interior(r)
        for p in H.patches:                     # covered entries from finer r
            inner = rg[p.pid][1:-1, 1:-1, 1:-1]
            inner[H.covered[p.pid]] = 0.0
        H.sync([rg])
        return rg

    def smooth(lev, rg, sweeps):
        e = H.empty()
        for p in H.by_level[lev]:
            e[p.pid][...] = 0.0
        rhs_l = {p.pid: rg[p.pid][1:-1, 1:-1, 1:-1] for p in H.by_level[lev]}
        sweep = {"jacobi": jacobi_level, "line": line_gs_level}.get(smoother, rbgs_level)
        for _ in range(sweeps):
            sweep(H, snap, f, lev, rhs_l, e)
        return {p.pid: e[p.pid][1:-1, 1:-1, 1:-1].copy() for p in H.by_level[lev]}

    def correct(lev, corr):
        nonlocal u
        for q, c in corr.items():
            u[q] = u[q] + c
        for m in range(lev + 1, L + 1):
            corr = dict(prolong_level(H, m, corr))
            for q, c in corr.items():
                u[q] = u[q] + c
        ug = H.from_interior(u)
        H.sync([ug])
        u = H.interior(ug)

    base_smooth = getattr(snap, "fac_base", "mg") == "smooth"
    for lev in range(L, -1, -1):
        rg = level_rhs()
        if lev > 0 or base_smooth:
            corr = smooth(lev, rg, m_pre)
        else:
            if mg_grids is None:
                mg_grids = build_mg(H, snap, f)
            rhs0 = gather_base(H, {p.pid: rg[p.pid][1:-1, 1:-1, 1:-1]
                                   for p in H.by_level[0]})
            corr = scatter_base(H, mg_vcycle(mg_grids, snap.beta, rhs0))
        correct(lev, corr)
    if n_post > 0:
        for lev in range(1, L + 1):
            correct(lev, smooth(lev, level_rhs(), n_post))
    return u


def afacx_coarse(H, snap, f, lev, r, sweeps):
    """Coarse approximation of the pair (lev - 1, lev): red-black sweeps of
    the level-(lev - 1) operator from zero on the cells that level lev
    covers, every other cell of level lev - 1 held at 0; r: pid -> interior
    right-hand side on level lev - 1."""
    c = H.empty()
    for p in H.by_level[lev - 1]:
        c[p.pid][...] = 0.0
    region = {p.pid: H.covered[p.pid] for p in H.by_level[lev - 1]}
    for _ in range(sweeps):
        rbgs_level(H, snap, f, lev - 1, r, c, region=region)
    return {p.pid: c[p.pid][1:-1, 1:-1, 1:-1].copy() for p in H.by_level[lev - 1]}


def afacx_fine(H, snap, f, lev, r, s, sweeps):
    """Fine correction of the pair (lev - 1, lev): red-black sweeps of the
    level-lev operator (coarse-fine ghosts with coarse values 0) from the
    interpolated coarse approximation s, minus s."""
    e = H.empty()
    for p in H.by_level[lev]:
        e[p.pid][...] = 0.0
        e[p.pid][1:-1, 1:-1, 1:-1] = s[p.pid]
    for _ in range(sweeps):
        rbgs_level(H, snap, f, lev, r, e)
    return {p.pid: e[p.pid][1:-1, 1:-1, 1:-1] - s[p.pid] for p in H.by_level[lev]}


def afacx_cycle(H, snap, f, rhs, mg_grids=None, nu=None):
    """AFACx, the asynchronous fast adaptive composite-grid method the
    paper names for more asynchrony in its solver (Sec. 7, after Lee,
    McCormick, Philip and Quinlan), for A^c u = rhs from u = 0.

    r = rhs on the composite cells, covered cells the mean of their children
    (the restricted composite residual).  Level 0: one multigrid V-cycle on
    r (or m sweeps with snap.fac_base == "smooth").  Every refined level l,
    independently of the others: m red-black sweeps of the level-(l-1)
    operator from zero on the cells level l covers (the rest held at 0),
    its trilinear interpolation s onto level l, m red-black sweeps of the
    level-l operator from s, the correction e_l = result - s: the coarse
    approximation only removes from the fine correction what level l-1
    already represents.  u = the level-0 correction plus every e_l, each
    carried to every finer level by trilinear prolongation; covered cells
    synced.  m = nu[0] (default snap.fac_nu[0]).
    """
    if nu is None:
        nu = getattr(snap, "fac_nu", (1, 0))
    m = int(nu[0])
    L = H.nlev - 1
    rg = H.from_interior([np.where(H.covered[p.pid], 0.0, rhs[p.pid]) for p in H.patches])
    H.sync([rg])
    r = {p.pid: rg[p.pid][1:-1, 1:-1, 1:-1] for p in H.patches}

    def on(lev):
        return {p.pid: r[p.pid] for p in H.by_level[lev]}

    if getattr(snap, "fac_base", "mg") == "smooth":
        e = H.empty()
        for p in H.by_level[0]:
            e[p.pid][...] = 0.0
        for _ in range(m):
            rbgs_level(H, snap, f, 0, on(0), e)
        acc = {p.pid: e[p.pid][1:-1, 1:-1, 1:-1].copy() for p in H.by_level[0]}
    else:
        if mg_grids is None:
            mg_grids = build_mg(H, snap, f)
        acc = dict(scatter_base(H, mg_vcycle(mg_grids, snap.beta, gather_base(H, on(0)))))
    u = [np.zeros(tuple(int(v) for v in p.n)) for p in H.patches]
    for q, a in acc.items():
        u[q] = a
    for lev in range(1, L + 1):
        c = afacx_coarse(H, snap, f, lev, on(lev - 1), m)
        s = dict(prolong_level(H, lev, c))
        el = afacx_fine(H, snap, f, lev, on(lev), s, m)
        carried = dict(prolong_level(H, lev, acc))
        acc = {q: carried[q] + el[q] for q in el}
        for q, a in acc.items():
            u[q] = a
    ug = H.from_interior(u)
    H.sync([ug])
    return H.interior(ug)


def _p1_cycle(snap):
    return afacx_cycle if getattr(snap, "fac_cycle", "mult") == "afacx" else fac_vcycle


def precond_apply(H, snap, wE, wT, mg=None):
    """y = P2^-1 P1^-1 w (per-patch interior arrays)."""
    mgE = mg[0] if mg else None
    mgT = mg[1] if mg else None
    cycle = _p1_cycle(snap)
    eE = cycle(H, snap, 0, wE, mgE)
    eT = cycle(H, snap, 1, wT, mgT)
    yE, yT = [], []
    for p in H.patches:
        q = p.pid
        a, b = p2_solve(snap.T[q], snap.z3[q], snap.beta, eE[q], eT[q],
                        snap.p2_mode)
        yE.append(a)
        yT.append(b)
    return yE, yT


def precond_apply_transpose(H, snap, wE, wT, mg=None):
    """P^-T w = P1^-1 P2^-T w (the diffusion blocks are symmetric)."""
    xE, xT = [], []
    for p in H.patches:
        q = p.pid
        a, b = p2_solve_transpose(snap.T[q], snap.z3[q], snap.beta, wE[q],
                                  wT[q], snap.p2_mode)
        xE.append(a)
        xT.append(b)
    mgE = mg[0] if mg else None
    mgT = mg[1] if mg else None
    cycle = _p1_cycle(snap)
    return cycle(H, snap, 0, xE, mgE), cycle(H, snap, 1, xT, mgT)
