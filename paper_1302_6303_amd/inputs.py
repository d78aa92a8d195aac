"""Seeded synthetic inputs for the radiation-diffusion workloads.

This module holds problem *definitions* only -- grids, patch boxes, the
material field z, initial states and time steps -- and none of the method's
arithmetic.  Both the HIP path and the CPU reference oracle consume what it
returns; neither side's computation lives here.

Conventions
-----------
* A problem lives on the box ``[lo, hi]`` (the unit cube by default) with a
  base grid of ``base_n`` cells per axis (Sec. 3.2 of the paper).
* Level ``l`` refines level 0 by ``2**l`` per axis (refinement ratio 2).
  Boxes are half-open ``[lo, hi)`` in that level's cell-index space.
* Per-box cell arrays have shape ``(nx, ny, nz)`` indexed ``[i, j, k]``; the
  compact layout flattens them with x fastest (``order='F'``), boxes in the
  given order, all E first and then all T.
* Faces are numbered ``2*d + s`` with ``d`` the axis and ``s = 0`` the low
  side, ``s = 1`` the high side.  ``bc_E[f]`` is 0 for a zero-flux (Neumann)
  face and 1 for a Marshak/Robin face with incoming value ``robin_R[f]``.

The workloads follow the paper's Marshak test problem (Sec. 6): E0 = 1e-5,
T0 = E0**0.25, kappa = 0.01, z = 10 inside axis-aligned material boxes and 1
elsewhere, Robin inflow R = 1 on the x = 0 face.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Callable, List, Sequence

import numpy as np

SEED_BASE = 13026303
E0 = 1.0e-5
T0 = E0 ** 0.25
KAPPA = 0.01


@dataclass
class Problem:
    base_n: tuple
    lo: tuple = (0.0, 0.0, 0.0)
    hi: tuple = (1.0, 1.0, 1.0)
    bc_E: tuple = (1, 0, 0, 0, 0, 0)
    robin_R: tuple = (1.0, 0.0, 0.0, 0.0, 0.0, 0.0)
    kappa: float = KAPPA

    def h(self, level: int = 0) -> np.ndarray:
        n = np.asarray(self.base_n, dtype=np.float64) * (2 ** level)
        return (np.asarray(self.hi) - np.asarray(self.lo)) / n


@dataclass
class Box:
    problem: int
    level: int
    lo: tuple
    hi: tuple

    @property
    def shape(self):
        return tuple(int(b - a) for a, b in zip(self.lo, self.hi))

    @property
    def ncells(self):
        s = self.shape
        return s[0] * s[1] * s[2]


@dataclass
class Workload:
    """Everything a run needs: problems, boxes, per-box z and initial E, T."""
    name: str
    problems: List[Problem]
    boxes: List[Box]
    z: List[np.ndarray]
    E: List[np.ndarray]
    T: List[np.ndarray]
    dt: np.ndarray                       # per problem
    nsteps: int = 1
    bdf1_only: bool = False
    extra: dict = field(default_factory=dict)

    def ncells(self) -> int:
        return sum(b.ncells for b in self.boxes)

    def compact(self, arrays: Sequence[np.ndarray]) -> np.ndarray:
        return np.concatenate([np.asarray(a, dtype=np.float64).ravel(order="F")
                               for a in arrays])

    def split(self, flat: np.ndarray) -> List[np.ndarray]:
        out, o = [], 0
        for b in self.boxes:
            n = b.ncells
            out.append(np.asarray(flat[o:o + n]).reshape(b.shape, order="F"))
            o += n
        return out


# ---------------------------------------------------------------------------
# material fields
# ---------------------------------------------------------------------------

def cell_centres(prob: Problem, box: Box):
    h = prob.h(box.level)
    ax = [prob.lo[d] + (np.arange(box.lo[d], box.hi[d]) + 0.5) * h[d]
          for d in range(3)]
    return np.meshgrid(ax[0], ax[1], ax[2], indexing="ij")


def sample_material_boxes(rng, nbox: int, zvals=None, edge=(0.2, 0.3)):
    """Axis-aligned material boxes: per axis edge ~ U[edge], lo ~ U[0, 1-edge]."""
    out = []
    for b in range(nbox):
        e = rng.uniform(edge[0], edge[1], size=3)
        lo = rng.uniform(0.0, 1.0 - e)
        zv = 10.0 if zvals is None else float(zvals[b])
        out.append((lo, lo + e, zv))
    return out


def box_field(mboxes, background: float = 1.0) -> Callable:
    """z(x, y, z) = value of the last material box containing the point."""
    def zf(X, Y, Z):
        z = np.full(X.shape, background, dtype=np.float64)
        for lo, hi, zv in mboxes:
            m = ((X >= lo[0]) & (X < hi[0]) & (Y >= lo[1]) & (Y < hi[1])
                 & (Z >= lo[2]) & (Z < hi[2]))
            z[m] = zv
        return z
    return zf


def eval_on_boxes(fun: Callable, problems, boxes):
    return [fun(*cell_centres(problems[b.problem], b)) for b in boxes]


# ---------------------------------------------------------------------------
# states
# ---------------------------------------------------------------------------

def uniform_state(boxes):
    E = [np.full(b.shape, E0) for b in boxes]
    T = [np.full(b.shape, T0) for b in boxes]
    return E, T


def front_state(problems, boxes, rng, noise=0.05, xf=None, width=None):
    """A Marshak-like front in x plus multiplicative noise.

    E ranges from about E0 behind nothing to about 4 at the heated face; T
    follows E**0.25 with an independent perturbation so that T**4 != E.
    The values are chosen once per problem so that every level of a
    hierarchy samples the same smooth profile (plus per-cell noise).
    """
    pars = []
    for _ in problems:
        xf_ = rng.uniform(0.3, 0.7) if xf is None else xf
        w_ = rng.uniform(0.05, 0.15) if width is None else width
        pars.append((xf_, w_))
    E, T = [], []
    for b in boxes:
        X, Y, Z = cell_centres(problems[b.problem], b)
        xf_, w_ = pars[b.problem]
        s = 1.0 / (1.0 + np.exp((X - xf_) / w_))
        prof = E0 + 4.0 * s * (1.0 + 0.1 * np.sin(3.0 * Y + 2.0 * Z))
        e = prof * (1.0 + noise * rng.uniform(-1.0, 1.0, size=X.shape))
        t = prof ** 0.25 * (1.0 + noise * rng.uniform(-1.0, 1.0, size=X.shape))
        E.append(e)
        T.append(t)
    return E, T


def random_vector(boxes, rng, scale_E=1.0, scale_T=1.0):
    vE = [scale_E * rng.standard_normal(b.shape) for b in boxes]
    vT = [scale_T * rng.standard_normal(b.shape) for b in boxes]
    return vE, vT


# ---------------------------------------------------------------------------
# patch tiler (stands in for clustering; produces properly nested levels)
# ---------------------------------------------------------------------------

def _dilate(mask: np.ndarray, r: int) -> np.ndarray:
    out = mask.copy()
    for d in range(3):
        acc = out.copy()
        for s in range(1, r + 1):
            acc |= _pad_shift(out, d, s)
            acc |= _pad_shift(out, d, -s)
        out = acc
    return out


def _pad_shift(m, d, s):
    """m shifted by s along axis d, filled with False."""
    out = np.zeros_like(m)
    n = m.shape[d]
    src = [slice(None)] * 3
    dst = [slice(None)] * 3
    if s > 0:
        src[d] = slice(0, n - s)
        dst[d] = slice(s, n)
    else:
        src[d] = slice(-s, n)
        dst[d] = slice(0, n + s)
    out[tuple(dst)] = m[tuple(src)]
    return out


def _erode1(mask: np.ndarray) -> np.ndarray:
    """Cells whose 26 neighbours (clipped to the domain) are all inside."""
    out = mask.copy()
    for d in range(3):
        acc = out.copy()
        for s in (1, -1):
            sh = np.ones_like(out)
            n = out.shape[d]
            src = [slice(None)] * 3
            dst = [slice(None)] * 3
            if s > 0:
                src[d] = slice(0, n - 1)
                dst[d] = slice(1, n)
            else:
                src[d] = slice(1, n)
                dst[d] = slice(0, n - 1)
            sh[tuple(dst)] = out[tuple(src)]
            acc &= sh
        out = acc
    return out


def _interface_tags(z: np.ndarray) -> np.ndarray:
    """Cells with a face neighbour of different z (the |grad z| > 0 tag)."""
    t = np.zeros(z.shape, dtype=bool)
    for d in range(3):
        a = [slice(None)] * 3
        b = [slice(None)] * 3
        a[d] = slice(0, z.shape[d] - 1)
        b[d] = slice(1, z.shape[d])
        diff = z[tuple(a)] != z[tuple(b)]
        t[tuple(a)] |= diff
        t[tuple(b)] |= diff
    return t


def _cuts(n: int, rng, gmin: int, gmax: int):
    c = [0]
    while c[-1] < n:
        c.append(min(n, c[-1] + int(rng.integers(gmin, gmax + 1))))
    return c


def _cluster(tag, nest, lo, hi, out, min_side):
    """Bounding box of the tags in [lo, hi); split until it nests."""
    sub = tag[lo[0]:hi[0], lo[1]:hi[1], lo[2]:hi[2]]
    if not sub.any():
        return
    idx = np.nonzero(sub)
    blo = [lo[d] + int(idx[d].min()) for d in range(3)]
    bhi = [lo[d] + int(idx[d].max()) + 1 for d in range(3)]
    if nest[blo[0]:bhi[0], blo[1]:bhi[1], blo[2]:bhi[2]].all():
        if min(bhi[d] - blo[d] for d in range(3)) >= min_side:
            out.append((tuple(blo), tuple(bhi)))
        return
    ext = [bhi[d] - blo[d] for d in range(3)]
    d = int(np.argmax(ext))
    if ext[d] <= 1:
        return
    mid = blo[d] + ext[d] // 2
    h1 = list(bhi)
    h1[d] = mid
    l2 = list(blo)
    l2[d] = mid
    _cluster(tag, nest, blo, h1, out, min_side)
    _cluster(tag, nest, l2, bhi, out, min_side)


def tile_levels(prob: Problem, zfun: Callable, nlevels: int, rng,
                side=(8, 32), dilate=2, pidx=0) -> List[Box]:
    """Static refinement of the material interfaces.

    Level l+1 covers the cells of level l whose z differs from a face
    neighbour, dilated by ``dilate`` cells, cut by seeded rectilinear cuts
    with even fine-side gaps in ``side`` and clipped so that every level is
    properly nested in the one below by at least one coarse cell.
    """
    n0 = np.asarray(prob.base_n, dtype=int)
    boxes = [Box(pidx, 0, (0, 0, 0), tuple(int(v) for v in n0))]
    region = np.ones(tuple(n0), dtype=bool)
    for lev in range(nlevels - 1):
        n_l = n0 * 2 ** lev
        h = prob.h(lev)
        ax = [prob.lo[d] + (np.arange(n_l[d]) + 0.5) * h[d] for d in range(3)]
        X, Y, Z = np.meshgrid(*ax, indexing="ij")
        tag = _dilate(_interface_tags(zfun(X, Y, Z)), dilate)
        nest = _erode1(region)
        tag &= nest
        found = []
        cuts = [_cuts(int(n_l[d]), rng, side[0] // 2, side[1] // 2)
                for d in range(3)]
        for a in range(len(cuts[0]) - 1):
            for b in range(len(cuts[1]) - 1):
                for c in range(len(cuts[2]) - 1):
                    lo = (cuts[0][a], cuts[1][b], cuts[2][c])
                    hi = (cuts[0][a + 1], cuts[1][b + 1], cuts[2][c + 1])
                    _cluster(tag, nest, lo, hi, found, 2)
        region = np.zeros(tuple(n_l * 2), dtype=bool)
        for lo, hi in found:
            flo = tuple(2 * v for v in lo)
            fhi = tuple(2 * v for v in hi)
            boxes.append(Box(pidx, lev + 1, flo, fhi))
            region[flo[0]:fhi[0], flo[1]:fhi[1], flo[2]:fhi[2]] = True
        if not found:
            break
    return boxes


# ---------------------------------------------------------------------------
# workloads
# ---------------------------------------------------------------------------

def uniform_workload(name, n, zfun, dt, nsteps, rng=None, state="uniform",
                     bdf1_only=False, problem_kw=None):
    prob = Problem(base_n=(n, n, n), **(problem_kw or {}))
    boxes = [Box(0, 0, (0, 0, 0), (n, n, n))]
    z = eval_on_boxes(zfun, [prob], boxes)
    if state == "uniform":
        E, T = uniform_state(boxes)
    else:
        E, T = front_state([prob], boxes, rng)
    return Workload(name, [prob], boxes, z, E, T, np.array([dt]), nsteps,
                    bdf1_only)


# The three z = 10 boxes of the paper's model problem (Sec. 6), unit cube.
PAPER_BOXES = [((0.0625, 0.375, 0.375), (0.2, 0.625, 0.625), 10.0),
               ((0.125, 0.0, 0.0), (0.375, 1.0, 0.125), 10.0),
               ((0.125, 0.0, 0.875), (0.375, 1.0, 1.0), 10.0)]


def paper_marshak(n=32, dt=1e-5, single_material=False):
    """The paper's model problem (Sec. 6) on one uniform n^3 grid: z = 10 in
    its three boxes and 1 elsewhere (z = 1 everywhere for the paper's
    single-material accuracy runs), E = E0 and T = T0 everywhere, Robin
    faces for E at x = 0 (R = 1) and x = 1 (R = 0), zero flux elsewhere;
    dt is the first step size handed to the time-step controller."""
    zf = box_field([] if single_material else PAPER_BOXES)
    return uniform_workload(f"paper{n}", n, zf, dt, 0,
                            problem_kw={"bc_E": (1, 1, 0, 0, 0, 0),
                                        "robin_R": (1.0, 0.0, 0.0, 0.0, 0.0, 0.0)})


def marshak_single(n=32, seed_k=1, state="uniform", nbox=2):
    """Single uniform patch with 2 seeded z = 10 boxes (the 32^3 workload)."""
    rng = np.random.default_rng(SEED_BASE + seed_k)
    zf = box_field(sample_material_boxes(rng, nbox))
    return uniform_workload(f"uniform{n}", n, zf, 1e-3, 5, rng, state,
                            bdf1_only=True)


def static_amr(base=64, nlevels=3, seed_k=2, side=(8, 32), state="uniform",
               nbox=2):
    """Static 3-level refinement of two material boxes (64^3 base)."""
    rng = np.random.default_rng(SEED_BASE + seed_k)
    mb = sample_material_boxes(rng, nbox)
    zf = box_field(mb)
    prob = Problem(base_n=(base, base, base))
    boxes = tile_levels(prob, zf, nlevels, rng, side=side)
    z = eval_on_boxes(zf, [prob], boxes)
    if state == "uniform":
        E, T = uniform_state(boxes)
    else:
        E, T = front_state([prob], boxes, rng)
    return Workload(f"amr{base}b{nlevels}l", [prob], boxes, z, E, T,
                    np.array([5e-4]), 20, extra={"material_boxes": mb})


def ensemble(nprob=64, seed_k=4, sizes=(32, 48, 64, 80, 96), state="uniform",
             nsteps=10):
    """Independent uniform problems of seeded sizes, z boxes and time steps."""
    rng = np.random.default_rng(SEED_BASE + seed_k)
    problems, boxes, z = [], [], []
    dts = np.empty(nprob)
    for p in range(nprob):
        n = int(rng.choice(sizes))
        nb = int(rng.integers(1, 5))
        zv = np.where(rng.uniform(size=nb) < 0.5, 1.0, 10.0)
        zf = box_field(sample_material_boxes(rng, nb, zv))
        prob = Problem(base_n=(n, n, n))
        b = Box(p, 0, (0, 0, 0), (n, n, n))
        problems.append(prob)
        boxes.append(b)
        z.append(zf(*cell_centres(prob, b)))
        dts[p] = rng.uniform(1e-4, 1e-3)
    if state == "uniform":
        E, T = uniform_state(boxes)
    else:
        E, T = front_state(problems, boxes, rng)
    return Workload(f"ensemble{nprob}", problems, boxes, z, E, T, dts, nsteps)


def smooth_random_z(n=64, seed_k=5, sigma=4.0):
    """z = 1 + 9 s with s a periodic-Gaussian-filtered noise mapped to [0, 1]."""
    rng = np.random.default_rng(SEED_BASE + seed_k)
    w = rng.standard_normal((n, n, n))
    k = np.fft.fftfreq(n) * n
    KX, KY, KZ = np.meshgrid(k, k, k, indexing="ij")
    filt = np.exp(-0.5 * (2 * np.pi * sigma / n) ** 2 * (KX**2 + KY**2 + KZ**2))
    s = np.real(np.fft.ifftn(np.fft.fftn(w) * filt))
    s = (s - s.mean()) / s.std()
    s = np.clip(0.5 + 0.35 * s, 0.0, 1.0)
    return 1.0 + 9.0 * s


def differentiation(n=64, seed_k=5, nsteps=50):
    prob = Problem(base_n=(n, n, n))
    boxes = [Box(0, 0, (0, 0, 0), (n, n, n))]
    z = [smooth_random_z(n, seed_k)]
    E, T = uniform_state(boxes)
    return Workload(f"adjoint{n}", [prob], boxes, z, E, T, np.array([1e-3]),
                    nsteps, bdf1_only=True)


def multi_patch_uniform(n=16, cuts=(6, 11), seed_k=7, state="front"):
    """One problem whose level 0 is split into several patches (siblings)."""
    rng = np.random.default_rng(SEED_BASE + seed_k)
    prob = Problem(base_n=(n, n, n))
    xs = [0, *cuts, n]
    boxes = [Box(0, 0, (xs[a], 0, 0), (xs[a + 1], n, n))
             for a in range(len(xs) - 1)]
    zf = box_field(sample_material_boxes(rng, 2))
    z = eval_on_boxes(zf, [prob], boxes)
    E, T = front_state([prob], boxes, rng) if state == "front" else uniform_state(boxes)
    return Workload(f"siblings{n}", [prob], boxes, z, E, T, np.array([1e-3]), 1)


def tiled_base(n=16, seed_k=10, state="front", refine=True):
    """One problem whose base grid is cut into four level-0 boxes at even
    planes (x = 6 and 10, and y = 8 between them), optionally with a level-1
    box that straddles the cuts."""
    rng = np.random.default_rng(SEED_BASE + seed_k)
    prob = Problem(base_n=(n, n, n))
    a, b, c = 6 * n // 16, 10 * n // 16, n // 2
    boxes = [Box(0, 0, (0, 0, 0), (a, n, n)), Box(0, 0, (a, 0, 0), (b, c, n)),
             Box(0, 0, (a, c, 0), (b, n, n)), Box(0, 0, (b, 0, 0), (n, n, n))]
    if refine:
        boxes.append(Box(0, 1, (n // 2, 3 * n // 8, 5 * n // 8),
                         (3 * n // 2, 11 * n // 8, 11 * n // 8)))
    zf = box_field(sample_material_boxes(rng, 2))
    z = eval_on_boxes(zf, [prob], boxes)
    E, T = front_state([prob], boxes, rng) if state == "front" else uniform_state(boxes)
    return Workload(f"tiled{n}", [prob], boxes, z, E, T, np.array([1e-3]), 1)


def small_amr(base=8, seed_k=8, state="front", boxes_spec=None):
    """Tiny hand-built 2- or 3-level hierarchy for oracle/GPU parity."""
    rng = np.random.default_rng(SEED_BASE + seed_k)
    prob = Problem(base_n=(base, base, base))
    spec = boxes_spec or [(1, (4, 4, 4), (12, 10, 12)),
                          (1, (4, 10, 4), (8, 14, 10))]
    boxes = [Box(0, 0, (0, 0, 0), (base, base, base))]
    boxes += [Box(0, lv, tuple(lo), tuple(hi)) for lv, lo, hi in spec]
    zf = box_field(sample_material_boxes(rng, 2))
    z = eval_on_boxes(zf, [prob], boxes)
    E, T = front_state([prob], boxes, rng) if state == "front" else uniform_state(boxes)
    return Workload(f"smallamr{base}", [prob], boxes, z, E, T, np.array([1e-3]), 1)
