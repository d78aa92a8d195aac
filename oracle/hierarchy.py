"""Patch hierarchy of one problem (paper Sec. 3.2 and 3.2.1).

Every level l is a set of non-overlapping boxes with mesh width h0 / 2**l.
Arrays are stored per patch with one layer of ghost cells, shape
``(nx + 2, ny + 2, nz + 2)`` indexed ``[i + 1, j + 1, k + 1]``.  Only the six
face layers of ghosts are ever defined; edge and corner ghosts hold NaN so
that a stencil that reads one fails loudly.

Readings used here (the paper is silent on them):
* proper nesting: every level l >= 1 lies inside level l-1 shrunk by one
  level-(l-1) cell, except along the physical boundary;
* fine boxes are aligned to the refinement ratio 2 (even lo and hi);
* ghost values outside the domain copy the adjacent interior cell (the
  paper's first-order extrapolation);
* coarse-fine ghosts: bilinear interpolation of four coarse values to the
  point aligned with the fine interior cell, then linear interpolation along
  the face normal between that value and the fine interior cell (Sec. 3.2.1,
  Fig. "Coarse fine boundary interpolation").  Coarse values outside the
  domain use the same copy rule on the coarse level.
"""
from __future__ import annotations

import numpy as np


class Patch:
    def __init__(self, pid, level, lo, hi):
        self.pid = pid
        self.level = int(level)
        self.lo = np.asarray(lo, dtype=np.int64)
        self.hi = np.asarray(hi, dtype=np.int64)
        self.n = self.hi - self.lo

    @property
    def gshape(self):
        return tuple(int(v) + 2 for v in self.n)

    def contains(self, I):
        """I: (m, 3) level indices -> bool mask."""
        return np.all((I >= self.lo) & (I < self.hi), axis=1)


class HierarchyError(ValueError):
    pass


class Hierarchy:
    """Boxes of ONE problem.  ``boxes`` = [(level, lo, hi), ...]."""

    def __init__(self, base_n, boxes, lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0),
                 bc_E=(1, 0, 0, 0, 0, 0), robin_R=(1.0, 0, 0, 0, 0, 0),
                 kappa=0.01):
        self.base_n = np.asarray(base_n, dtype=np.int64)
        self.dom_lo = np.asarray(lo, dtype=np.float64)
        self.dom_hi = np.asarray(hi, dtype=np.float64)
        self.bc_E = tuple(int(v) for v in bc_E)
        self.robin_R = tuple(float(v) for v in robin_R)
        self.kappa = float(kappa)
        self.patches = [Patch(p, lv, l, h) for p, (lv, l, h) in enumerate(boxes)]
        self.nlev = 1 + max(p.level for p in self.patches)
        self.by_level = [[p for p in self.patches if p.level == l]
                         for l in range(self.nlev)]
        self._validate()
        self.covered = [self._covered_mask(p) for p in self.patches]

    # -- geometry ---------------------------------------------------------
    def N(self, level):
        return self.base_n * (2 ** level)

    def h(self, level):
        return (self.dom_hi - self.dom_lo) / self.N(level)

    def volume(self, level):
        return float(np.prod(self.h(level)))

    def _validate(self):
        for l, plist in enumerate(self.by_level):
            if not plist:
                raise HierarchyError(f"level {l} is empty")
            for p in plist:
                if np.any(p.n <= 0) or np.any(p.lo < 0) or np.any(p.hi > self.N(l)):
                    raise HierarchyError(f"box {p.pid} outside level {l}")
                if l > 0 and (np.any(p.lo % 2) or np.any(p.hi % 2)):
                    raise HierarchyError(f"box {p.pid} not aligned to ratio 2")
            for a in range(len(plist)):
                for b in range(a + 1, len(plist)):
                    pa, pb = plist[a], plist[b]
                    if np.all(np.maximum(pa.lo, pb.lo) < np.minimum(pa.hi, pb.hi)):
                        raise HierarchyError(f"boxes {pa.pid} and {pb.pid} overlap")
        ncell0 = sum(int(np.prod(p.n)) for p in self.by_level[0])
        if ncell0 != int(np.prod(self.base_n)):
            raise HierarchyError("level 0 must tile the base grid")
        # proper nesting: parents of every fine cell, grown by one coarse cell
        # and clipped to the domain, must lie on the coarse level.
        for l in range(1, self.nlev):
            for p in self.by_level[l]:
                clo = np.maximum(p.lo // 2 - 1, 0)
                chi = np.minimum(p.hi // 2 + 1, self.N(l - 1))
                I = _box_cells(clo, chi)
                if not np.all(self.locate(l - 1, I)[0] >= 0):
                    raise HierarchyError(f"box {p.pid} is not properly nested")

    def locate(self, level, I):
        """Owner patch id and local (interior) index of level indices I."""
        I = np.atleast_2d(np.asarray(I, dtype=np.int64))
        pid = np.full(len(I), -1, dtype=np.int64)
        loc = np.zeros_like(I)
        for p in self.by_level[level]:
            m = p.contains(I)
            pid[m] = p.pid
            loc[m] = I[m] - p.lo
        return pid, loc

    def is_covered(self, level, I):
        if level + 1 >= self.nlev:
            return np.zeros(len(I), dtype=bool)
        pid, _ = self.locate(level + 1, 2 * np.asarray(I))
        return pid >= 0

    def _covered_mask(self, p):
        I = _box_cells(p.lo, p.hi)
        return self.is_covered(p.level, I).reshape(tuple(p.n), order="F")

    # -- arrays -----------------------------------------------------------
    def empty(self):
        """Per-patch ghosted arrays, ghosts (incl. edges/corners) = NaN."""
        out = []
        for p in self.patches:
            a = np.full(p.gshape, np.nan)
            a[1:-1, 1:-1, 1:-1] = 0.0
            out.append(a)
        return out

    def from_interior(self, arrs):
        out = self.empty()
        for a, x in zip(out, arrs):
            a[1:-1, 1:-1, 1:-1] = x
        return out

    def interior(self, arrs):
        return [a[1:-1, 1:-1, 1:-1].copy() for a in arrs]

    def value_at(self, field, level, I):
        """Interior values of `field` at level indices I (must be owned)."""
        pid, loc = self.locate(level, I)
        if np.any(pid < 0):
            raise HierarchyError("value requested outside the level")
        out = np.empty(len(I))
        for q in np.unique(pid):
            m = pid == q
            l = loc[m] + 1
            out[m] = field[q][l[:, 0], l[:, 1], l[:, 2]]
        return out

    # -- restriction (covered cells <- mean of the 8 children) ------------
    def sync(self, fields):
        """In place, finest level first (Alg. 1 synchronisation step)."""
        for l in range(self.nlev - 2, -1, -1):
            for p in self.by_level[l]:
                cov = self.covered[p.pid]
                if not cov.any():
                    continue
                loc = np.argwhere(cov)
                I = loc + p.lo
                for f in fields:
                    acc = np.zeros(len(I))
                    for o in _OCT:
                        acc += self.value_at(f, l + 1, 2 * I + o)
                    f[p.pid][loc[:, 0] + 1, loc[:, 1] + 1, loc[:, 2] + 1] = acc / 8.0

    def sync_transpose(self, fields):
        """Transpose of sync, in place on ghosted arrays: coarsest level
        first, every covered cell hands 1/8 of its value to each of its
        eight children and keeps none."""
        for l in range(self.nlev - 1):
            for p in self.by_level[l]:
                cov = np.argwhere(self.covered[p.pid])
                if len(cov) == 0:
                    continue
                I = cov + p.lo
                for f in fields:
                    v = f[p.pid][cov[:, 0] + 1, cov[:, 1] + 1, cov[:, 2] + 1] / 8.0
                    for o in _OCT:
                        pid, loc = self.locate(l + 1, 2 * I + o)
                        for q in np.unique(pid):
                            m = pid == q
                            ll = loc[m] + 1
                            np.add.at(f[q], (ll[:, 0], ll[:, 1], ll[:, 2]), v[m])
                    f[p.pid][cov[:, 0] + 1, cov[:, 1] + 1, cov[:, 2] + 1] = 0.0

    # -- ghost fill -------------------------------------------------------
    def ghost_kinds(self, p, d, s):
        """Ghost layer of face (d, s) of patch p: level indices and kind.

        kind: 0 physical, 1 sibling, 2 coarse-fine.
        """
        G, ghost_loc, inner_loc = _face_layer(p, d, s)
        N = self.N(p.level)
        outside = (G[:, d] < 0) | (G[:, d] >= N[d])
        kind = np.full(len(G), 2, dtype=np.int64)
        kind[outside] = 0
        if (~outside).any():
            pid, _ = self.locate(p.level, G[~outside])
            k = kind[~outside]
            k[pid >= 0] = 1
            kind[~outside] = k
        if p.level == 0 and np.any(kind == 2):
            raise HierarchyError("level-0 ghost without an owner")
        return G, ghost_loc, inner_loc, kind

    def fill_ghosts(self, fields, coarse_fine="linear"):
        """Fill the face ghosts of every patch of every field, in place.

        coarse_fine="linear" is the inhomogeneous interpolation; "zero" uses
        coarse values 0 (the relation g = f/3 used for level corrections);
        "parent" gives a coarse-fine ghost the value of the coarse cell it
        lies in (the material of that cell, for interface tags).
        Assumes covered coarse cells already hold restricted values.
        """
        for p in self.patches:
            for d in range(3):
                for s in range(2):
                    G, gl, il, kind = self.ghost_kinds(p, d, s)
                    for f in fields:
                        arr = f[p.pid]
                        val = np.empty(len(G))
                        m = kind == 0
                        val[m] = arr[il[m, 0], il[m, 1], il[m, 2]]
                        m = kind == 1
                        if m.any():
                            val[m] = self.value_at(f, p.level, G[m])
                        m = kind == 2
                        if m.any():
                            fine_in = arr[il[m, 0], il[m, 1], il[m, 2]]
                            if coarse_fine == "zero":
                                val[m] = fine_in / 3.0
                            elif coarse_fine == "parent":
                                N = self.N(p.level - 1)
                                val[m] = self.value_at(f, p.level - 1,
                                                       np.clip(G[m] // 2, 0, N - 1))
                            else:
                                ci = self.coarse_interp(f, p.level, G[m], d)
                                val[m] = (2.0 / 3.0) * ci + (1.0 / 3.0) * fine_in
                        arr[gl[:, 0], gl[:, 1], gl[:, 2]] = val

    def coarse_interp(self, f, level, G, d):
        """Bilinear value of the coarse level at the tangential position of
        the fine ghost cells G (level indices), at the coarse cell centre
        along the normal d.  Weights 9/16, 3/16, 3/16, 1/16."""
        t1, t2 = [a for a in range(3) if a != d]
        P = G // 2
        o1 = np.where(G[:, t1] % 2 == 1, 1, -1)
        o2 = np.where(G[:, t2] % 2 == 1, 1, -1)
        N = self.N(level - 1)

        def val(I):
            I = np.clip(I, 0, N - 1)          # copy rule outside the domain
            return self.value_at(f, level - 1, I)

        e1 = np.zeros_like(P)
        e1[:, t1] = o1
        e2 = np.zeros_like(P)
        e2[:, t2] = o2
        return (9.0 * val(P) + 3.0 * val(P + e1) + 3.0 * val(P + e2)
                + val(P + e1 + e2)) / 16.0

    # -- compact <-> per patch --------------------------------------------
    def ncells(self):
        return sum(int(np.prod(p.n)) for p in self.patches)

    def pack(self, arrs):
        return np.concatenate([a[1:-1, 1:-1, 1:-1].ravel(order="F") for a in arrs])

    def unpack(self, flat):
        out, o = self.empty(), 0
        for p, a in zip(self.patches, out):
            n = int(np.prod(p.n))
            a[1:-1, 1:-1, 1:-1] = flat[o:o + n].reshape(tuple(p.n), order="F")
            o += n
        return out


_OCT = np.array([[a, b, c] for c in (0, 1) for b in (0, 1) for a in (0, 1)],
                dtype=np.int64)


def _box_cells(lo, hi):
    r = [np.arange(lo[d], hi[d]) for d in range(3)]
    g = np.meshgrid(*r, indexing="ij")
    return np.stack([x.ravel(order="F") for x in g], axis=1)


def _face_layer(p, d, s):
    """Ghost cells of face (d, s): level indices, ghosted local indices of
    the ghost and of the adjacent interior cell."""
    lo = p.lo.copy()
    hi = p.hi.copy()
    if s == 0:
        lo[d], hi[d] = p.lo[d] - 1, p.lo[d]
    else:
        lo[d], hi[d] = p.hi[d], p.hi[d] + 1
    G = _box_cells(lo, hi)
    gl = G - p.lo + 1
    il = gl.copy()
    il[:, d] += 1 if s == 0 else -1
    return G, gl, il
