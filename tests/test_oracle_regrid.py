"""Pins of the oracle's regridding (Sec. 5): tags on fields whose
indicators are known in closed form, and the conservative linear transfer
(conservation, positivity, exactness on linear fields, identity, one cell
by hand), and the warm restart's re-solve."""
import numpy as np
import pytest

from oracle import regrid as rg
from oracle.hierarchy import Hierarchy
from oracle.solvers import Stepper, System
from paper_1302_6303_amd import inputs as I

OLD = [(0, (0, 0, 0), (8, 8, 8)), (1, (4, 4, 4), (12, 10, 12)), (1, (4, 10, 4), (8, 14, 10)),
       (2, (10, 10, 10), (18, 18, 18))]
# refines new regions (level 1 grows in x, level 2 moves), derefines others
# (the old second level-1 box is gone) and adds a third level
NEW = [(0, (0, 0, 0), (8, 8, 8)), (1, (4, 4, 4), (14, 12, 12)),
       (2, (12, 10, 10), (22, 20, 18)), (3, (28, 24, 24), (36, 32, 32))]


def _centres(H, p):
    h = H.h(p.level)
    ax = [(np.arange(p.lo[d], p.hi[d]) + 0.5) * h[d] for d in range(3)]
    return np.meshgrid(*ax, indexing="ij")


def _on(H, f):
    return [f(*_centres(H, p)) for p in H.patches]


def _synced(H, arrs):
    g = H.from_interior(arrs)
    H.sync([g])
    return H.interior(g)


def _energy(H, arrs):
    return sum(H.volume(p.level) * float(np.sum(arrs[p.pid][~H.covered[p.pid]]))
               for p in H.patches)


def _front(X, Y, Z):
    return 1e-5 + 4.0 / (1.0 + np.exp((X - 0.4) / 0.03)) * (1.0 + 0.2 * np.sin(7 * Y + 3 * Z))


def test_transfer_conserves_the_composite_integral():
    Ho, Hn = Hierarchy((8, 8, 8), OLD), Hierarchy((8, 8, 8), NEW)
    rng = np.random.default_rng(5)
    old = _synced(Ho, [_front(*_centres(Ho, p)) * rng.uniform(0.5, 1.5, tuple(int(v) for v in p.n))
                       for p in Ho.patches])
    new = rg.transfer(Ho, old, Hn)
    a, b = _energy(Ho, old), _energy(Hn, new)
    assert abs(a - b) <= 1e-13 * abs(a), (a, b)
    back = rg.transfer(Hn, new, Ho)
    assert abs(_energy(Ho, back) - a) <= 1e-13 * abs(a)


def test_transfer_keeps_values_positive():
    """Jumps over six decades (E0 next to the heated face): every refined
    value stays positive, at least a quarter of its coarse parent."""
    Ho, Hn = Hierarchy((8, 8, 8), OLD), Hierarchy((8, 8, 8), NEW)
    rng = np.random.default_rng(6)
    old = _synced(Ho, [np.exp(rng.uniform(np.log(1e-6), np.log(4.0),
                                          tuple(int(v) for v in p.n))) for p in Ho.patches])
    new = rg.transfer(Ho, old, Hn)
    assert min(float(a.min()) for a in new) > 0.0
    # a refined cell is at least u_P / 4 (each same-signed slope < u_P)
    p = Hn.by_level[3][0]
    I = np.argwhere(np.ones(tuple(int(v) for v in p.n), dtype=bool)) + p.lo
    par = rg._level_value(Hn, new, 2, I // 2)
    vals = np.array([new[p.pid][tuple(c - p.lo)] for c in I])
    assert np.all(vals >= 0.25 * par - 1e-15 * par)


def test_transfer_is_exact_for_linear_fields():
    """Cell averages of a linear field: copies, averages of children and
    minmod-limited refinement (equal one-sided differences) all reproduce
    it at every new cell centre; the new regions here stay a coarse cell
    away from the physical boundary."""
    Ho, Hn = Hierarchy((8, 8, 8), OLD), Hierarchy((8, 8, 8), NEW)
    f = lambda X, Y, Z: 2.0 + 0.7 * X - 1.3 * Y + 0.4 * Z
    old = _synced(Ho, _on(Ho, f))
    new = rg.transfer(Ho, old, Hn)
    ref = _on(Hn, f)
    for a, b in zip(new, ref):
        np.testing.assert_allclose(a, b, rtol=0, atol=1e-14)


def test_identity_transfer_is_bitwise():
    Ho = Hierarchy((8, 8, 8), OLD)
    rng = np.random.default_rng(7)
    old = _synced(Ho, [rng.uniform(0.1, 2.0, tuple(int(v) for v in p.n)) for p in Ho.patches])
    new = rg.transfer(Ho, old, Hierarchy((8, 8, 8), OLD))
    for a, b in zip(old, new):
        np.testing.assert_array_equal(a, b)


def test_one_refined_cell_by_hand():
    """Level 1 appears over a single-level 4^3 grid: the fine cell (3, 4, 5)
    (parent (1, 2, 2); the upper child in x and z, the lower in y) from the
    minmod formula written out for its parent's neighbours."""
    Ho = Hierarchy((4, 4, 4), [(0, (0, 0, 0), (4, 4, 4))])
    Hn = Hierarchy((4, 4, 4), [(0, (0, 0, 0), (4, 4, 4)), (1, (2, 2, 2), (6, 6, 6))])
    u = np.zeros((4, 4, 4))
    u[1, 2, 2] = 5.0
    u[0, 2, 2], u[2, 2, 2] = 4.0, 5.5        # x: differences 0.5 and 1 -> 0.5
    u[1, 1, 2], u[1, 3, 2] = 6.0, 3.0        # y: -2 and -1 -> -1
    u[1, 2, 1], u[1, 2, 3] = 4.0, 7.0        # z: 2 and 1 -> 1
    new = rg.transfer(Ho, [u], Hn)
    fine = new[1][3 - 2, 4 - 2, 5 - 2]
    assert fine == 5.0 + 0.25 * 0.5 - 0.25 * (-1.0) + 0.25 * 1.0
    # a local extremum (differences of opposite sign) refines to the parent
    u2 = np.full((4, 4, 4), 1.0)
    u2[1, 2, 2] = 3.0
    new2 = rg.transfer(Ho, [u2], Hn)
    np.testing.assert_array_equal(new2[1][0:2, 2:4, 2:4], 3.0)


def test_tags_of_a_linear_field_and_a_material_box():
    n = 16
    H = Hierarchy((n, n, n), [(0, (0, 0, 0), (n, n, n))])
    X, Y, Z = _centres(H, H.patches[0])
    E = [1.0 + 3.0 * X]
    z = [np.where((X > 0.25) & (X < 0.5) & (Y > 0.5) & (Z < 0.75), 10.0, 1.0)]
    # |grad E| / E = 3 / (1 + 3 x) > 1.5  <=>  x < 1/3, away from the faces
    # in x (one-sided half differences at x faces)
    t = rg.tags(H, E, z, grad=1.5)[0]
    inner = np.zeros_like(t)
    inner[1:-1] = True
    np.testing.assert_array_equal(t[inner.astype(bool)].reshape(n - 2, n, n),
                                  (3.0 / (1.0 + 3.0 * X) > 1.5)[1:-1])
    # the material tag: a face neighbour with the other z
    ti = rg.tags(H, E, z, z_interface=True)[0]
    zz = z[0]
    ref = np.zeros_like(ti)
    for d in range(3):
        a = [slice(None)] * 3
        b = [slice(None)] * 3
        a[d], b[d] = slice(0, n - 1), slice(1, n)
        diff = zz[tuple(a)] != zz[tuple(b)]
        ref[tuple(a)] |= diff
        ref[tuple(b)] |= diff
    np.testing.assert_array_equal(ti, ref)
    # tau^g = h |E_x| / (0.1 max E) = (3 h) / (0.1 max E) in the interior;
    # tau^c = 0 in the interior, h^2 |E_xx| = 3 h / 2 at the x faces
    h = 1.0 / n
    emax = float(E[0].max())
    tg = 3.0 * h / (0.1 * emax)
    assert not rg.tags(H, E, z, tau_g=1.01 * tg)[0][1:-1].any()
    assert rg.tags(H, E, z, tau_g=0.99 * tg)[0][1:-1].all()
    tc = rg.tags(H, E, z, tau_c=0.5 * (1.5 * h) / (0.1 * emax))[0]
    assert not tc[1:-1].any() and tc[0].all() and tc[-1].all()


def test_regrid_resolve_solves_the_last_step_on_the_new_grid():
    """Warm restart: after two steps on one hierarchy the history moves to
    another and the last step is solved again there.  The re-solved state
    solves the new grid's system; regridding onto the same boxes leaves the
    state where it was (it already solved that system)."""
    w = I.small_amr(8, state="uniform")
    zf = I.box_field([((0.3, 0.3, 0.3), (0.6, 0.6, 0.6), 10.0)])
    kw = dict(rtol=1e-10, atol=1e-14)
    out = {}
    for name, boxes in (("same", OLD), ("new", NEW)):
        Ho = Hierarchy((8, 8, 8), OLD)
        so = System(Ho, _on(Ho, zf))
        E0 = _on(Ho, _front)                  # the front crosses the refined boxes
        T0 = [e ** 0.25 for e in E0]
        st = Stepper(so, so.join(E0, T0), **kw)
        for dt in (1e-3, 1e-3):
            assert st.step(dt).converged
        u_before, prev_before = st.u.copy(), st.u_prev.copy()
        Hn = Hierarchy((8, 8, 8), boxes)
        sn = System(Hn, _on(Hn, zf))
        res = st.regrid(sn)
        b, c0, dt = st.last
        F = sn.residual(st.u, b, dt, c0)
        assert sn.norm(F) <= 1e-10 * res.fnorms[0] + 1e-14
        out[name] = (u_before, st.u.copy(), prev_before, st.u_prev.copy(), res.iters)
        assert st.step(1e-3).converged
    u_before, u_after, prev_before, prev_after, _ = out["same"]
    np.testing.assert_array_equal(prev_after, prev_before)
    assert np.linalg.norm(u_after - u_before) <= 1e-10 * np.linalg.norm(u_before)
    assert out["new"][4] >= 3          # interpolation left a residual to remove
