"""Pins of the preconditioner readings against the residual, the Jacobian
and the paper's level-independence claim (Sec. 4.2-4.3, Sec. 6.1).

* The diffusion blocks of P1 (Sec. 4.2) are the residual's diffusion terms
  linearised with D frozen.  Where freezing D loses nothing -- no flux
  limiter for E, a uniform T for T -- the composite operator A^c must be
  exactly the analytic Jacobian's diffusion part, Marshak faces and
  coarse-fine interpolation and matching included.  The Jacobian itself is
  pinned by brute-force differences of the residual.
* Red-black Gauss-Seidel (Sec. 4.3) on a level must not depend on how the
  level is cut into patches: splitting a patch into siblings, whose shared
  faces then go through ghost exchange, gives the same sweep and the same
  FAC cycle bit for bit.
* FAC V(1,0) keeps its contraction as levels are added (the level
  independence of Sec. 6.1).
"""
import numpy as np
import pytest

from oracle import precond as pc
from oracle.hierarchy import Hierarchy
from oracle.solvers import System
from paper_1302_6303_amd import inputs as I
from tests.helpers import state, system


def _cells(H, p):
    h = H.h(p.level)
    ax = [(np.arange(p.lo[d], p.hi[d]) + 0.5) * h[d] for d in range(3)]
    return np.meshgrid(*ax, indexing="ij")


@pytest.mark.parametrize("wname", ["uniform", "amr"])
def test_composite_operator_is_the_jacobians_diffusion_part(wname):
    """A^c v = (J(u) v - coupling part) / c0 with beta = dt / c0: for the E
    block with the limiter off (D_E does not depend on E) and v = (vE, 0);
    for the T block with a uniform T (dD_T/dT multiplies grad T = 0) and
    v = (0, vT).  Covers the Marshak linearisation 2 beta D_b / ((4 D_b + h) h)
    on the diagonal and the coarse-fine treatment of A^c."""
    if wname == "uniform":
        w = I.marshak_single(6, state="front")
    else:
        w = I.small_amr(8, state="front")
    dt, c0 = 2e-3, 1.5
    beta = dt / c0
    rng = np.random.default_rng(170)
    for f in (0, 1):
        s = system(w, lam=0.0 if f == 0 else 0.5)
        H = s.H
        u = state(s, w)
        if f == 1:
            n = s.nc
            u[n:] = 0.7                       # uniform T, E stays a front
        E, T = s.split(u)
        snap = pc.Snapshot(H, E, T, s.z, beta, s.lam)
        v = rng.standard_normal(u.shape)
        if f == 0:
            v[s.nc:] = 0.0
        else:
            v[:s.nc] = 0.0
        v = s.sync(v)
        Jv = s.jvp(u, v, dt, c0)
        vE, vT = s.split(v)
        JE, JT = s.split(Jv)
        Ac = pc.composite_apply(H, snap, f, vE if f == 0 else vT)
        for p in H.patches:
            q = p.pid
            sig = snap.z3[q] / snap.T[q] ** 3
            if f == 0:
                ref = (JE[q] - dt * sig * vE[q]) / c0
            else:
                E_c = E[q]
                ref = (JT[q] - dt * snap.z3[q] * (1.0 + 3.0 * E_c / snap.T[q] ** 4)
                       * vT[q]) / c0
            keep = ~H.covered[q]
            np.testing.assert_allclose(Ac[q][keep], ref[keep], rtol=1e-12,
                                       atol=1e-12 * np.max(np.abs(ref)))


def _field_on(H, p, seed, lo, hi):
    """A smooth positive field plus per-cell noise that depends only on the
    cell's level index, so two decompositions of a level see equal values."""
    X, Y, Z = _cells(H, p)
    L = np.stack(np.meshgrid(*[np.arange(p.lo[d], p.hi[d]) for d in range(3)],
                             indexing="ij"))
    key = (L[0] * 73856093) ^ (L[1] * 19349663) ^ (L[2] * 83492791) ^ (p.level * 2654435761)
    noise = ((key * 2654435761 + seed) % 1000003) / 1000003.0
    return lo + (hi - lo) * (0.5 + 0.4 * np.sin(3 * X + 2 * Y - Z) + 0.1 * noise)


def _split_pair():
    whole = [(0, (0, 0, 0), (8, 8, 8)), (1, (4, 4, 4), (12, 12, 12))]
    split = [(0, (0, 0, 0), (8, 8, 8)), (1, (4, 4, 4), (8, 12, 12)),
             (1, (8, 4, 4), (12, 8, 12)), (1, (8, 8, 4), (12, 12, 12))]
    out = []
    for bx in (whole, split):
        H = Hierarchy((8, 8, 8), bx)
        E = [_field_on(H, p, 1, 0.05, 3.0) for p in H.patches]
        T = [_field_on(H, p, 2, 0.3, 1.2) for p in H.patches]
        z = [np.where(_field_on(H, p, 3, 0.0, 1.0) > 0.5, 10.0, 1.0) for p in H.patches]
        out.append((H, E, T, z))
    return out


def _by_index(H, arrs, level):
    """{level index: value} of per-patch interior arrays on one level."""
    d = {}
    for p in H.by_level[level]:
        a = arrs[p.pid]
        for i in range(int(p.n[0])):
            for j in range(int(p.n[1])):
                for k in range(int(p.n[2])):
                    d[(int(p.lo[0]) + i, int(p.lo[1]) + j, int(p.lo[2]) + k)] = a[i, j, k]
    return d


def test_rbgs_and_fac_are_invariant_under_splitting_level_patches():
    pair = _split_pair()
    sweeps, cycles = [], []
    for H, E, T, z in pair:
        snap = pc.Snapshot(H, E, T, z, 4e-3, 0.5)
        rhs = {p.pid: _field_on(H, p, 4, -1.0, 1.0) for p in H.by_level[1]}
        e = H.empty()
        for p in H.by_level[1]:
            e[p.pid][...] = 0.0
            e[p.pid][1:-1, 1:-1, 1:-1] = _field_on(H, p, 5, -1.0, 1.0)
        per_f = []
        for f in (0, 1):
            ef = [a.copy() for a in e]
            for _ in range(2):
                pc.rbgs_level(H, snap, f, 1, rhs, ef)
            per_f.append(_by_index(H, [a[1:-1, 1:-1, 1:-1] for a in ef], 1))
        sweeps.append(per_f)
        full = [_field_on(H, p, 6, -1.0, 1.0) for p in H.patches]
        cycles.append([(_by_index(H, c, 1), _by_index(H, c, 0))
                       for c in (pc.fac_vcycle(H, snap, f, full) for f in (0, 1))])
    for f in (0, 1):
        a, b = sweeps[0][f], sweeps[1][f]
        assert a.keys() == b.keys()
        for key in a:
            assert a[key] == b[key], (f, key, a[key], b[key])
        for lev in (0, 1):
            a, b = cycles[0][f][lev], cycles[1][f][lev]
            for key in a:
                assert a[key] == b[key], (f, lev, key, a[key], b[key])


def _nested(nlev, n=8):
    """Base n^3 and a central box of half the extent on every finer level."""
    boxes = [(0, (0, 0, 0), (n, n, n))]
    lo, hi = n // 4, 3 * n // 4
    boxes.append((1, (2 * lo,) * 3, (2 * hi,) * 3))
    for lev in range(2, nlev):
        plo, phi = boxes[-1][1][0], boxes[-1][2][0]
        c, e = plo + phi, phi - plo                 # level-lev centre and extent
        boxes.append((lev, (c - e // 2,) * 3, (c + e // 2,) * 3))
    return boxes[:nlev]


def _fac_rate_E(nlev):
    H = Hierarchy((8, 8, 8), _nested(nlev))
    E, T = [], []
    for p in H.patches:
        X, _, _ = _cells(H, p)
        prof = 1e-5 + 4.0 / (1.0 + np.exp((X - 0.5) / 0.1))
        E.append(prof)
        T.append(prof ** 0.25)
    z = [np.ones(tuple(int(v) for v in p.n)) for p in H.patches]
    snap = pc.Snapshot(H, E, T, z, 5e-2, 0.5)
    rng = np.random.default_rng(25)
    rhs = [rng.standard_normal(tuple(int(v) for v in p.n)) for p in H.patches]
    x = [np.zeros_like(r) for r in rhs]
    norms = []
    for _ in range(7):
        Ax = pc.composite_apply(H, snap, 0, x)
        r = [rhs[q] - Ax[q] for q in range(len(rhs))]
        norms.append(np.sqrt(sum(np.sum(rr[~H.covered[q]] ** 2) for q, rr in enumerate(r))))
        c = pc.fac_vcycle(H, snap, 0, r)
        x = [x[q] + c[q] for q in range(len(x))]
    return (norms[-1] / norms[2]) ** 0.25


def test_fac_contraction_is_level_independent():
    """FAC V(1,0) as a stationary iteration on the E block: adding nested
    refinement levels (2, 3, 4 levels, finest h = 1/64) leaves the
    contraction bounded and nearly unchanged, as the paper's iteration
    counts do for 2 to 5 levels (Sec. 6.1)."""
    rates = [_fac_rate_E(L) for L in (2, 3, 4)]
    assert max(rates) < 0.6, rates
    assert rates[2] - rates[1] < 0.05 and rates[1] - rates[0] < 0.12, rates


def _untiled(w):
    """The workload with its level-0 boxes merged into one (same values)."""
    from oracle import precond as pc_
    base = [b for b in w.boxes if b.level == 0]
    n = w.problems[0].base_n
    H = Hierarchy(n, [(0, b.lo, b.hi) for b in base])
    idx = [i for i, b in enumerate(w.boxes) if b.level == 0]
    rest = [i for i, b in enumerate(w.boxes) if b.level > 0]
    merge = lambda arrs: [pc_.gather_base(H, {q: arrs[i] for q, i in enumerate(idx)})] + \
        [arrs[i] for i in rest]
    boxes = [I.Box(0, 0, (0, 0, 0), tuple(n))] + [w.boxes[i] for i in rest]
    return I.Workload(w.name + "-merged", w.problems, boxes, merge(w.z), merge(w.E),
                      merge(w.T), w.dt, w.nsteps)


def test_tiled_base_level_is_the_single_base_box():
    """Level 0 cut into four boxes (siblings at even planes, a level-1 box
    across the cuts): residual, preconditioner and a BDF step equal those of
    the same hierarchy with one level-0 box (Sec. 3.2: the coarsest level is
    a union of patches)."""
    w = I.tiled_base(16)
    m = _untiled(w)
    sw, sm = system(w), system(m)
    uw, um = state(sw, w), state(sm, m)
    Ew, Tw = sw.split(uw)
    Em, Tm = sm.split(um)

    def by_cell(H, arrs):
        d = {}
        for p in H.patches:
            for lev_key, v in _by_index(H, arrs, p.level).items():
                d[(p.level,) + lev_key] = v
        return d
    for E1, H1, E2, H2 in ((Ew, sw.H, Em, sm.H),):
        a, b = by_cell(H1, E1), by_cell(H2, E2)
        assert a == b                          # same input cell by cell
    dt = 2e-3
    Fw = sw.split(sw.residual(uw, uw, dt, 1.0))
    Fm = sm.split(sm.residual(um, um, dt, 1.0))
    for f in (0, 1):
        a, b = by_cell(sw.H, Fw[f]), by_cell(sm.H, Fm[f])
        for k in a:
            assert a[k] == b[k], ("residual", f, k)
    rng = np.random.default_rng(3)
    vw = rng.standard_normal(uw.shape)
    vE, vT = sw.split(vw)
    vm = sm.join(*[_untiled_arrays(w, x) for x in (vE, vT)])
    Pw, _ = sw.precond(uw, dt)
    Pm, _ = sm.precond(um, dt)
    yw, ym = sw.split(Pw(vw)), sm.split(Pm(vm))
    for f in (0, 1):
        a, b = by_cell(sw.H, yw[f]), by_cell(sm.H, ym[f])
        for k in a:
            assert abs(a[k] - b[k]) <= 1e-13 * max(1.0, abs(b[k])), ("precond", f, k)


def _untiled_arrays(w, arrs):
    from oracle import precond as pc_
    base_i = [i for i, b in enumerate(w.boxes) if b.level == 0]
    n = w.problems[0].base_n
    H = Hierarchy(n, [(0, w.boxes[i].lo, w.boxes[i].hi) for i in base_i])
    full = pc_.gather_base(H, {q: arrs[i] for q, i in enumerate(base_i)})
    return [full] + [arrs[i] for i, b in enumerate(w.boxes) if b.level > 0]


def test_line_gauss_seidel_solves_each_line_exactly():
    """Block Gauss-Seidel on x-lines: a patch one cell thick in y and z is a
    single line, so one sweep solves A e = rhs exactly; on a general patch
    the lines of the colour swept last satisfy their equations exactly, and
    every red line is the exact solve with the black lines held."""
    from oracle import precond as pc_
    for n in ((9, 1, 1), (7, 5, 4)):
        H = Hierarchy(n, [(0, (0, 0, 0), n)])
        rng = np.random.default_rng(31)
        E = [rng.uniform(0.05, 3.0, n)]
        T = [rng.uniform(0.3, 1.2, n)]
        z = [rng.choice([1.0, 10.0], n)]
        snap = pc_.Snapshot(H, E, T, z, 3e-2, 0.5)
        p = H.patches[0]
        for f in (0, 1):
            rhs = rng.standard_normal(n)
            e = H.empty()
            e[0][...] = 0.0
            e[0][1:-1, 1:-1, 1:-1] = rng.standard_normal(n)
            pc_.line_gs_level(H, snap, f, 0, {0: rhs}, e)
            r = rhs - pc_.composite_apply(H, snap, f, [e[0][1:-1, 1:-1, 1:-1]])[0]
            J = np.arange(n[1])[:, None]
            K = np.arange(n[2])[None, :]
            black = (J + K) % 2 == 1
            scale = np.max(np.abs(rhs))
            if n[1] == 1 and n[2] == 1:
                assert np.max(np.abs(r)) <= 1e-12 * scale
            else:
                assert np.max(np.abs(r[:, black])) <= 1e-12 * scale
                assert np.max(np.abs(r[:, ~black])) > 1e-6 * scale   # red lines moved on


def test_line_smoother_beats_point_smoothing_on_stretched_cells():
    """Cells 8 times shorter in x than in y and z: the x couplings dominate
    and point Gauss-Seidel smooths them poorly; FAC with the x-line block
    Gauss-Seidel contracts much faster (the classic case for line
    relaxation)."""
    from oracle import precond as pc_
    boxes = [(0, (0, 0, 0), (16, 4, 4)), (1, (8, 2, 2), (24, 6, 6))]
    rates = {}
    for sm in ("rbgs", "line"):
        H = Hierarchy((16, 4, 4), boxes, hi=(0.5, 1.0, 1.0), bc_E=(0,) * 6)
        E, T = [], []
        for p in H.patches:
            X, _, _ = _cells(H, p)
            E.append(0.5 + 0.1 * np.sin(3 * X))
            T.append(np.full(tuple(int(v) for v in p.n), 0.8))
        z = [np.ones(tuple(int(v) for v in p.n)) for p in H.patches]
        snap = pc_.Snapshot(H, E, T, z, 5e-2, 0.5, fac_smoother=sm, fac_base="smooth")
        rng = np.random.default_rng(25)
        rhs = [rng.standard_normal(tuple(int(v) for v in p.n)) for p in H.patches]
        x = [np.zeros_like(r) for r in rhs]
        norms = []
        for _ in range(7):
            Ax = pc_.composite_apply(H, snap, 0, x)
            r = [rhs[q] - Ax[q] for q in range(len(rhs))]
            norms.append(np.sqrt(sum(np.sum(rr[~H.covered[q]] ** 2) for q, rr in enumerate(r))))
            c = pc_.fac_vcycle(H, snap, 0, r)
            x = [x[q] + c[q] for q in range(len(x))]
        rates[sm] = (norms[-1] / norms[2]) ** 0.25
    assert rates["line"] < 0.5 * rates["rbgs"] and rates["line"] < 0.5, rates


@pytest.mark.parametrize("nlev", [2, 3])
def test_sync_transpose_is_the_transpose_of_sync(nlev):
    """<S x, y> = <x, S^T y> for the restriction S that sync applies (covered
    cells take the mean of their children, finest level first) and the
    coarse-to-fine hand-down of sync_transpose, on random per-patch data."""
    H = Hierarchy((8, 8, 8), _nested(nlev))
    rng = np.random.default_rng(40 + nlev)
    x = H.from_interior([rng.standard_normal(tuple(int(v) for v in p.n)) for p in H.patches])
    y = H.from_interior([rng.standard_normal(tuple(int(v) for v in p.n)) for p in H.patches])
    Sx = [a.copy() for a in x]
    H.sync([Sx])
    Sty = [a.copy() for a in y]
    H.sync_transpose([Sty])
    inner = lambda a, b: sum(float(np.sum(u[1:-1, 1:-1, 1:-1] * v[1:-1, 1:-1, 1:-1]))
                             for u, v in zip(a, b))
    lhs, rhs = inner(Sx, y), inner(x, Sty)
    assert abs(lhs - rhs) <= 1e-13 * (abs(lhs) + abs(rhs))
