"""HIP path versus the CPU oracle through the C ABI.

Tolerances (float64 operators): residual / Jacobian action / transpose
1e-12 relative normwise per field and, per entry, 1e-12 of the sum of the
magnitudes of the terms that entry adds up (oracle residual_scale,
jvp_scale, vjp(magnitude=True)); preconditioner 1e-10 normwise (dense bottom solve and operation
order differ); implicit steps 1e-8 relative per field with both sides
converged to Newton rtol 1e-10.
"""
import numpy as np
import pytest

from oracle import operators as ops
from paper_1302_6303_amd import inputs as I
from tests.gpu_helpers import (compact_from_native, compact_state, make,
                               native_from_compact, rel_err, to_dev, to_host)
from tests.helpers import state, system

pytestmark = pytest.mark.gpu


def boxes_workload():
    """Three uniform problems of non-cubic sizes whose grids coarsen to
    different depths; Marshak faces on x-low and y-high of the first."""
    rng = np.random.default_rng(11)
    sizes = [(80, 48, 48), (40, 24, 56), (16, 16, 16)]
    problems, boxes = [], []
    for p, n in enumerate(sizes):
        kw = {}
        if p == 0:
            kw = {"bc_E": (1, 0, 0, 1, 0, 0), "robin_R": (1.0, 0.0, 0.0, 1.0, 0.0, 0.0)}
        problems.append(I.Problem(base_n=n, **kw))
        boxes.append(I.Box(p, 0, (0, 0, 0), n))
    z = []
    for prob, b in zip(problems, boxes):
        zf = I.box_field(I.sample_material_boxes(rng, 2))
        z.append(zf(*I.cell_centres(prob, b)))
    E, T = I.front_state(problems, boxes, rng)
    return I.Workload("boxes3", problems, boxes, z, E, T, np.array([2e-3, 1e-3, 5e-4]))


def odd_workload():
    """One 5 x 7 x 3 patch: odd extents, an odd block size and an odd plane
    stride (7 * 9); its coarsest multigrid grid is the patch itself."""
    rng = np.random.default_rng(17)
    prob = I.Problem(base_n=(5, 7, 3))
    box = I.Box(0, 0, (0, 0, 0), (5, 7, 3))
    zf = I.box_field(I.sample_material_boxes(rng, 2))
    z = [zf(*I.cell_centres(prob, box))]
    E, T = I.front_state([prob], [box], rng)
    return I.Workload("odd573", [prob], [box], z, E, T, np.array([1e-3]))


def tiny_workload():
    """Three small uniform problems: 4^3 and 6 x 4 x 2 are their own coarsest
    multigrid grids (bottom solve on the level-0 box), 12 x 8 x 6 coarsens
    once; all x extents even."""
    rng = np.random.default_rng(19)
    sizes = [(4, 4, 4), (6, 4, 2), (12, 8, 6)]
    problems, boxes = [], []
    for p, n in enumerate(sizes):
        problems.append(I.Problem(base_n=n))
        boxes.append(I.Box(p, 0, (0, 0, 0), n))
    z = []
    for prob, b in zip(problems, boxes):
        zf = I.box_field(I.sample_material_boxes(rng, 2))
        z.append(zf(*I.cell_centres(prob, b)))
    E, T = I.front_state(problems, boxes, rng)
    return I.Workload("tiny3", problems, boxes, z, E, T, np.array([1e-3, 2e-3, 1e-3]))


def workloads():
    return {
        "odd573": odd_workload,
        "uniform16": lambda: I.marshak_single(16, state="front"),
        "uniform10": lambda: I.uniform_workload(
            "u10", 10, I.box_field(I.sample_material_boxes(np.random.default_rng(3), 2)),
            1e-3, 1, np.random.default_rng(4), state="front"),
        "amr2": lambda: I.small_amr(8, state="front"),
        "amr3": lambda: I.static_amr(base=16, nlevels=3, side=(8, 16), state="front"),
        "amr4": lambda: I.static_amr(base=8, nlevels=4, side=(8, 16), seed_k=3,
                                     state="front"),
        # base grid cut into four level-0 boxes, without and with a level-1
        # box across the cuts
        "tiled0": lambda: I.tiled_base(16, refine=False),
        "tiled": lambda: I.tiled_base(16),
    }


WL = workloads()


def _setup(name, dt=2e-3, **opt):
    w = WL[name]()
    s = system(w)
    H = make(w, **opt)
    u_n = state(s, w)
    H.begin_step([dt])
    rng = np.random.default_rng(42)
    u = s.sync(u_n * rng.uniform(0.9, 1.1, u_n.shape))
    return w, s, H, u_n, u, dt


@pytest.mark.parametrize("stencil", [0, 1, 2, 3])
@pytest.mark.parametrize("name", list(WL))
def test_residual_parity(name, stencil):
    w, s, H, u_n, u, dt = _setup(name, stencil=stencil)
    F = H.native()
    H.residual(native_from_compact(H, u), F)
    got = compact_from_native(H, F)
    ref = s.residual(u, u_n, dt, 1.0)
    n = s.nc
    for sl in (slice(0, n), slice(n, 2 * n)):
        assert rel_err(got[sl], ref[sl]) < 1e-12
    E, T = s.split(u)
    bE, bT = s.split(u_n)
    sE, sT = ops.residual_scale(s.H, E, T, s.z, bE, bT, dt, 1.0, s.lam)
    scale = s.join(sE, sT)
    assert np.all(np.abs(got - ref) <= 1e-12 * scale + 1e-300)


@pytest.mark.parametrize("stencil", [0, 1, 2, 3])
@pytest.mark.parametrize("name", list(WL))
def test_jvp_parity(name, stencil):
    w, s, H, u_n, u, dt = _setup(name, stencil=stencil)
    rng = np.random.default_rng(7)
    v = rng.standard_normal(u.shape) * u
    Jv = H.native()
    H.jvp(native_from_compact(H, u), native_from_compact(H, v), Jv)
    got = compact_from_native(H, Jv)
    ref = s.jvp(u, v, dt, 1.0)
    n = s.nc
    for sl in (slice(0, n), slice(n, 2 * n)):
        assert rel_err(got[sl], ref[sl]) < 1e-12
    E, T = s.split(u)
    vE, vT = s.split(v)
    sE, sT = ops.jvp_scale(s.H, E, T, s.z, vE, vT, dt, 1.0, s.lam)
    scale = s.join(sE, sT)
    assert np.all(np.abs(got - ref) <= 1e-12 * scale + 1e-300)


@pytest.mark.parametrize("name", list(WL))
def test_precond_parity(name):
    w, s, H, u_n, u, dt = _setup(name)
    rng = np.random.default_rng(8)
    wv = rng.standard_normal(u.shape)
    H.precond_setup(native_from_compact(H, u))
    y = H.native()
    H.precond_apply(native_from_compact(H, wv), y)
    got = compact_from_native(H, y)
    P, _ = s.precond(u, dt)
    ref = P(wv)
    m = s.composite
    n = s.nc
    for sl in (slice(0, n), slice(n, 2 * n)):
        mm = m[sl]
        assert rel_err(got[sl][mm], ref[sl][mm]) < 1e-10


@pytest.mark.parametrize("name,nu", [("amr2", (2, 1)), ("amr2", (1, 2)), ("amr3", (2, 1)),
                                     ("amr4", (1, 2))])
def test_precond_parity_fac_vmn(name, nu):
    """FAC V(m, n) of Alg. 1 (m down-sweep sweeps, n up-sweep sweeps on the
    refreshed composite residual) against the oracle's cycle of the same
    shape, FP64, on 2-, 3- and 4-level hierarchies."""
    w = WL[name]()
    s = system(w, fac_nu=nu)
    H = make(w, fac_nu_pre=nu[0], fac_nu_post=nu[1])
    dt = 2e-3
    H.begin_step([dt])
    rng = np.random.default_rng(42)
    u = s.sync(state(s, w) * rng.uniform(0.9, 1.1, 2 * s.nc))
    wv = np.random.default_rng(8).standard_normal(u.shape)
    H.precond_setup(native_from_compact(H, u))
    y = H.native()
    H.precond_apply(native_from_compact(H, wv), y)
    got = compact_from_native(H, y)
    P, _ = s.precond(u, dt)
    ref = P(wv)
    m = s.composite
    n = s.nc
    for sl in (slice(0, n), slice(n, 2 * n)):
        mm = m[sl]
        assert rel_err(got[sl][mm], ref[sl][mm]) < 1e-10


@pytest.mark.parametrize("name,nu", [("amr2", (1, 0)), ("amr2", (3, 2)), ("amr3", (2, 1))])
def test_precond_parity_fac_jacobi(name, nu):
    """FAC with the damped point Jacobi level smoother (one, two and three
    sweeps: in place, through the second buffer and back) against the
    oracle, FP64."""
    from paper_1302_6303_amd import nrd
    w = WL[name]()
    s = system(w, fac_nu=nu, fac_smoother="jacobi")
    H = make(w, fac_nu_pre=nu[0], fac_nu_post=nu[1], fac_smoother=nrd.NRD_SMOOTH_JACOBI)
    dt = 2e-3
    H.begin_step([dt])
    rng = np.random.default_rng(42)
    u = s.sync(state(s, w) * rng.uniform(0.9, 1.1, 2 * s.nc))
    wv = np.random.default_rng(8).standard_normal(u.shape)
    H.precond_setup(native_from_compact(H, u))
    y = H.native()
    H.precond_apply(native_from_compact(H, wv), y)
    got = compact_from_native(H, y)
    P, _ = s.precond(u, dt)
    ref = P(wv)
    m = s.composite
    n = s.nc
    for sl in (slice(0, n), slice(n, 2 * n)):
        mm = m[sl]
        assert rel_err(got[sl][mm], ref[sl][mm]) < 1e-10


@pytest.mark.parametrize("name,nu,base", [("amr2", (1, 0), "mg"), ("amr3", (2, 1), "mg"),
                                          ("odd573", (1, 0), "smooth"),
                                          ("tiled", (2, 1), "smooth"),
                                          ("amr4", (1, 1), "smooth")])
def test_precond_parity_fac_line_gauss_seidel(name, nu, base):
    """FAC with the block (x-line) Gauss-Seidel level smoother against the
    oracle, FP64: on the levels above a multigrid base, and on every level
    including a tiled base when the base is only smoothed; odd line lengths
    and sibling ghosts at the lines' ends included."""
    from paper_1302_6303_amd import nrd
    w = WL[name]()
    s = system(w, fac_nu=nu, fac_smoother="line", fac_base=base)
    H = make(w, fac_nu_pre=nu[0], fac_nu_post=nu[1], fac_smoother=nrd.NRD_SMOOTH_LINE,
             fac_base=nrd.NRD_BASE_SMOOTH if base == "smooth" else nrd.NRD_BASE_MG)
    dt = 2e-3
    H.begin_step([dt])
    rng = np.random.default_rng(42)
    u = s.sync(state(s, w) * rng.uniform(0.9, 1.1, 2 * s.nc))
    wv = np.random.default_rng(8).standard_normal(u.shape)
    H.precond_setup(native_from_compact(H, u))
    y = H.native()
    for _ in range(2):                       # a second apply finds stale scratch
        H.precond_apply(native_from_compact(H, wv), y)
    got = compact_from_native(H, y)
    P, _ = s.precond(u, dt)
    ref = P(wv)
    m = s.composite
    n = s.nc
    for sl in (slice(0, n), slice(n, 2 * n)):
        mm = m[sl]
        assert rel_err(got[sl][mm], ref[sl][mm]) < 1e-10


@pytest.mark.parametrize("name,m,base", [("uniform16", 1, "mg"), ("amr2", 1, "mg"),
                                          ("amr3", 2, "mg"), ("amr4", 1, "smooth"),
                                          ("tiled", 2, "mg"), ("tiled", 1, "smooth")])
def test_precond_parity_afacx(name, m, base):
    """P1 by the AFACx cycle (every refined level's pair at once) against
    the oracle's AFACx, FP64, on 1-4 levels and a tiled base; two applies
    in a row (the second finds the first's scratch)."""
    from paper_1302_6303_amd import nrd
    w = WL[name]()
    s = system(w, fac_nu=(m, 0), fac_base=base, fac_cycle="afacx")
    H = make(w, fac_nu_pre=m, fac_cycle=nrd.NRD_FAC_AFACX,
             fac_base=nrd.NRD_BASE_SMOOTH if base == "smooth" else nrd.NRD_BASE_MG)
    dt = 2e-3
    H.begin_step([dt])
    rng = np.random.default_rng(42)
    u = s.sync(state(s, w) * rng.uniform(0.9, 1.1, 2 * s.nc))
    wv = np.random.default_rng(8).standard_normal(u.shape)
    H.precond_setup(native_from_compact(H, u))
    y = H.native()
    for _ in range(2):
        H.precond_apply(native_from_compact(H, wv), y)
    got = compact_from_native(H, y)
    P, _ = s.precond(u, dt)
    ref = P(wv)
    m_ = s.composite
    n = s.nc
    for sl in (slice(0, n), slice(n, 2 * n)):
        mm = m_[sl]
        assert rel_err(got[sl][mm], ref[sl][mm]) < 1e-10


@pytest.mark.parametrize("name", ["amr3", "tiled"])
def test_precond_parity_fac_float32_amr(name):
    """The multiplicative FAC cycle in FP32 (mixed precision) on refined
    hierarchies (three levels; a tiled base under a level-1 box) against the
    FP64 oracle."""
    from paper_1302_6303_amd import nrd
    w = WL[name]()
    s = system(w)
    H = make(w, precision=nrd.NRD_MIXED)
    dt = 2e-3
    H.begin_step([dt])
    rng = np.random.default_rng(42)
    u = s.sync(state(s, w) * rng.uniform(0.9, 1.1, 2 * s.nc))
    wv = np.random.default_rng(8).standard_normal(u.shape)
    H.precond_setup(native_from_compact(H, u))
    y = H.native()
    H.precond_apply(native_from_compact(H, wv), y)
    got = compact_from_native(H, y)
    P, _ = s.precond(u, dt)
    ref = P(wv)
    n = s.nc
    for sl in (slice(0, n), slice(n, 2 * n)):
        mm = s.composite[sl]
        assert rel_err(got[sl][mm], ref[sl][mm]) < 1e-4


def test_precond_parity_afacx_float32():
    """The AFACx cycle in FP32 (mixed precision) on three levels against
    the FP64 oracle."""
    from paper_1302_6303_amd import nrd
    w = WL["amr3"]()
    s = system(w, fac_cycle="afacx")
    H = make(w, precision=nrd.NRD_MIXED, fac_cycle=nrd.NRD_FAC_AFACX)
    dt = 2e-3
    H.begin_step([dt])
    rng = np.random.default_rng(42)
    u = s.sync(state(s, w) * rng.uniform(0.9, 1.1, 2 * s.nc))
    wv = np.random.default_rng(8).standard_normal(u.shape)
    H.precond_setup(native_from_compact(H, u))
    y = H.native()
    H.precond_apply(native_from_compact(H, wv), y)
    got = compact_from_native(H, y)
    P, _ = s.precond(u, dt)
    ref = P(wv)
    n = s.nc
    for sl in (slice(0, n), slice(n, 2 * n)):
        mm = s.composite[sl]
        assert rel_err(got[sl][mm], ref[sl][mm]) < 1e-4


@pytest.mark.parametrize("name,forcing", [("uniform16", "petsc"), ("amr2", "petsc"),
                                          ("uniform16", "kelley"), ("amr2", "kelley")])
def test_implicit_steps_parity_forcing(name, forcing):
    """Implicit steps with either choice of Eisenstat-Walker forcing terms:
    the same states and Newton iteration counts as the oracle's stepper with
    the same forcing."""
    from oracle.solvers import Stepper
    from paper_1302_6303_amd import nrd
    w = WL[name]()
    s = system(w)
    H = make(w, newton_rtol=1e-10, newton_atol=1e-16,
             newton_forcing=nrd.NRD_EW_PETSC if forcing == "petsc" else nrd.NRD_EW_KELLEY)
    st = Stepper(s, state(s, w), rtol=1e-10, atol=1e-16, forcing=forcing)
    for dt in (1e-3, 1e-3, 1.5e-3):
        rc, stats = H.implicit_step([dt])
        r = st.step(dt)
        assert r.converged and stats[0]["converged"]
        assert stats[0]["newton_iters"] == r.iters
        E, T = H.get_fields()
        got = np.concatenate([to_host(E), to_host(T)])
        n = s.nc
        for sl in (slice(0, n), slice(n, 2 * n)):
            assert rel_err(got[sl], st.u[sl]) < 1e-8


@pytest.mark.parametrize("name", ["amr2", "tiled"])
def test_implicit_steps_parity_afacx(name):
    """Implicit steps preconditioned by AFACx: same states as the oracle's
    stepper with the oracle's AFACx (both at Newton rtol 1e-10)."""
    from oracle.solvers import Stepper
    from paper_1302_6303_amd import nrd
    w = WL[name]()
    s = system(w, fac_cycle="afacx")
    H = make(w, newton_rtol=1e-10, newton_atol=1e-16, fac_cycle=nrd.NRD_FAC_AFACX)
    st = Stepper(s, state(s, w), rtol=1e-10, atol=1e-16)
    for dt in (1e-3, 1e-3, 1.5e-3):
        rc, stats = H.implicit_step([dt])
        r = st.step(dt)
        assert r.converged and stats[0]["converged"]
        E, T = H.get_fields()
        got = np.concatenate([to_host(E), to_host(T)])
        n = s.nc
        for sl in (slice(0, n), slice(n, 2 * n)):
            assert rel_err(got[sl], st.u[sl]) < 1e-8


@pytest.mark.parametrize("name,nu", [("uniform16", (1, 0)), ("uniform16", (2, 0)),
                                     ("amr2", (1, 0)), ("amr3", (2, 1))])
def test_precond_parity_fac_base_smoothing(name, nu):
    """FAC whose base level is only smoothed (fac_base = SMOOTH, as in the
    paper's runs) against the oracle's cycle of the same shape, FP64."""
    from paper_1302_6303_amd import nrd
    w = WL[name]()
    s = system(w, fac_nu=nu, fac_base="smooth")
    H = make(w, fac_nu_pre=nu[0], fac_nu_post=nu[1], fac_base=nrd.NRD_BASE_SMOOTH)
    dt = 2e-3
    H.begin_step([dt])
    rng = np.random.default_rng(42)
    u = s.sync(state(s, w) * rng.uniform(0.9, 1.1, 2 * s.nc))
    wv = np.random.default_rng(8).standard_normal(u.shape)
    H.precond_setup(native_from_compact(H, u))
    y = H.native()
    H.precond_apply(native_from_compact(H, wv), y)
    got = compact_from_native(H, y)
    P, _ = s.precond(u, dt)
    ref = P(wv)
    m = s.composite
    n = s.nc
    for sl in (slice(0, n), slice(n, 2 * n)):
        mm = m[sl]
        assert rel_err(got[sl][mm], ref[sl][mm]) < 1e-10


def _batch(parts, name):
    problems, boxes, z, E, T, dts = [], [], [], [], [], []
    for p, wp in enumerate(parts):
        problems.append(wp.problems[0])
        b = wp.boxes[0]
        boxes.append(I.Box(p, 0, b.lo, b.hi))
        z.append(wp.z[0])
        E.append(wp.E[0])
        T.append(wp.T[0])
        dts.append(float(wp.dt[0]))
    return I.Workload(name, problems, boxes, z, E, T, np.array(dts))


@pytest.mark.parametrize("precision", [1, 0])
def test_colour_split_storage_is_bitwise_native(precision):
    """The base grid's colour-split storage (single-level problems of even x
    extent) with the T-field coefficients recomputed from T gives bit for
    bit the preconditioner of the native storage: the same problem batched
    beside an odd-extent problem (which turns the colour-split storage off
    for the hierarchy) yields the same output, in float and in double."""
    from tests.gpu_helpers import problem_slices
    a = I.marshak_single(16, state="front")
    b = _batch([a, odd_workload()], "split_off")
    w_a = np.random.default_rng(14).standard_normal(2 * a.ncells())
    outs = []
    for w in (a, b):
        H = make(w, precision=precision)
        H.begin_step([float(x) for x in w.dt])
        u = compact_state(w)
        sl = problem_slices(w)[0]
        wv = np.random.default_rng(15).standard_normal(u.shape)
        wv[sl] = w_a                            # the same vector for problem 0
        H.precond_setup(native_from_compact(H, u))
        y = H.native()
        H.precond_apply(native_from_compact(H, wv), y)
        outs.append(compact_from_native(H, y)[sl])
    assert np.array_equal(outs[0], outs[1]), \
        np.abs(outs[0] - outs[1]).max() / np.abs(outs[1]).max()


@pytest.mark.parametrize("wl", [boxes_workload, tiny_workload])
def test_precond_parity_noncubic(wl):
    """Preconditioner of three non-cubic problems in one hierarchy, each
    problem against its own oracle: coarsest grids 2, 3 and 4 grids down
    (Marshak faces on two sides of the first), or two problems that are
    their own coarsest grid beside one that coarsens once."""
    from tests.gpu_helpers import problem_slices
    w = wl()
    H = make(w)
    dts = [float(x) for x in w.dt]
    H.begin_step(dts)
    rng = np.random.default_rng(12)
    u = compact_state(w) * rng.uniform(0.9, 1.1, 2 * w.ncells())
    wv = np.random.default_rng(13).standard_normal(u.shape)
    H.precond_setup(native_from_compact(H, u))
    y = H.native()
    H.precond_apply(native_from_compact(H, wv), y)
    got = compact_from_native(H, y)
    sl = problem_slices(w)
    for p in range(len(w.problems)):
        s = system(w, pidx=p)
        P, _ = s.precond(u[sl[p]], dts[p])
        ref = P(wv[sl[p]])
        g = got[sl[p]]
        n = s.nc
        for f in (slice(0, n), slice(n, 2 * n)):
            assert rel_err(g[f], ref[f]) < 1e-10


@pytest.mark.parametrize("name", ["uniform16", "uniform10", "tiled0", "amr2", "amr3", "amr4",
                                  "tiled"])
def test_vjp_parity(name):
    w, s, H, u_n, u, dt = _setup(name)
    rng = np.random.default_rng(9)
    lam = rng.standard_normal(u.shape)
    JTl = H.native()
    gz = H.compact(1)
    H.vjp(native_from_compact(H, u), native_from_compact(H, lam), JTl, gz)
    got = compact_from_native(H, JTl)
    ref, refz = s.vjp(u, lam, dt, 1.0)
    n = s.nc
    for sl in (slice(0, n), slice(n, 2 * n)):
        assert rel_err(got[sl], ref[sl]) < 1e-12
    assert rel_err(to_host(gz), refz) < 1e-12
    E, T = s.split(u)
    lE, lT = s.split(lam)
    mE, mT, mz = ops.vjp(s.H, E, T, s.z, lE, lT, dt, 1.0, s.lam, magnitude=True)
    scale = s.join(mE, mT)
    assert np.all(np.abs(got - ref) <= 1e-12 * scale + 1e-300)
    zscale = np.concatenate([a.ravel(order="F") for a in mz])
    assert np.all(np.abs(to_host(gz) - refz) <= 1e-12 * zscale + 1e-300)


@pytest.mark.parametrize("name", ["uniform16", "amr2", "tiled"])
def test_implicit_steps_parity(name):
    from oracle.solvers import Stepper
    w = WL[name]()
    s = system(w)
    H = make(w, newton_rtol=1e-10, newton_atol=1e-16)
    st = Stepper(s, state(s, w), rtol=1e-10, atol=1e-16)
    for dt in (1e-3, 1e-3, 1.5e-3):
        rc, stats = H.implicit_step([dt])
        r = st.step(dt)
        assert r.converged and stats[0]["converged"]
        E, T = H.get_fields()
        got = np.concatenate([to_host(E), to_host(T)])
        n = s.nc
        for sl in (slice(0, n), slice(n, 2 * n)):
            assert rel_err(got[sl], st.u[sl]) < 1e-8


def _far_from_equilibrium(specs):
    """6^3 problems with E = E0 exp(U(-2, 2)) and T = exp(U(-1, 1)) per cell
    (seeded): radiation far below the material temperature."""
    problems, boxes, z, E, T = [], [], [], [], []
    for p, (seed, E0) in enumerate(specs):
        w1 = I.marshak_single(6)
        rng = np.random.default_rng(seed)
        sh = w1.boxes[0].shape
        problems.append(w1.problems[0])
        boxes.append(I.Box(p, 0, (0, 0, 0), sh))
        z.append(w1.z[0])
        E.append(E0 * np.exp(rng.uniform(-2, 2, sh)))
        T.append(np.exp(rng.uniform(-1, 1, sh)))
    return I.Workload("far", problems, boxes, z, E, T, np.full(len(specs), 1e-2))


def _cut_parity(specs):
    from oracle.solvers import Stepper
    from tests.gpu_helpers import problem_slices
    w = _far_from_equilibrium(specs)
    H = make(w, newton_rtol=1e-10, newton_atol=1e-16, newton_maxit=24, bdf_max_order=1,
             newton_forcing=0)
    rc, stats = H.implicit_step([1e-2] * len(specs), raise_on_fail=False)
    E, T = H.get_fields()
    got = np.concatenate([to_host(E), to_host(T)])
    sl = problem_slices(w)
    res = []
    for p in range(len(specs)):
        s = system(w, pidx=p)
        st = Stepper(s, state(s, w, pidx=p), rtol=1e-10, atol=1e-16, maxit=24, forcing="kelley")
        r = st.step(1e-2)
        assert bool(stats[p]["converged"]) == bool(r.converged)
        assert stats[p]["newton_iters"] == r.iters
        assert stats[p]["positivity_cuts"] == r.cuts
        g = got[sl[p]]
        n = s.nc
        for f in (slice(0, n), slice(n, 2 * n)):
            assert rel_err(g[f], st.u[f]) < 1e-8
        res.append(r)
    return rc, res


def test_implicit_step_positivity_cuts_in_lock_step():
    """One BDF1 step of three problems solved together whose full Newton
    steps are accepted (seed 21) or halved (seeds 20, 25) with Kelley's
    forcing terms, each against its own oracle run: Newton iterations and
    cuts equal, states to 1e-8."""
    rc, res = _cut_parity([(20, 1e-4), (21, 1e-4), (25, 1e-2)])
    assert rc == 0
    assert res[1].cuts == 0 and res[0].cuts > 0 and res[2].cuts > 0


def test_implicit_step_positivity_stall():
    """Seed 23: every Newton step needs halving until one cannot be made
    positive at all; the oracle gives up at the same iteration with the same
    number of rejected trial steps, and the state is left unchanged."""
    rc, res = _cut_parity([(23, 1e-4)])
    assert rc == -5 and not res[0].converged


def test_adaptive_steps_match_the_oracle():
    """PC.4.7 time-step control on three problems stepped together: two
    Marshak fronts (8^3, 10^3) and a far-from-equilibrium 6^3 problem whose
    first step of 1e-2 must be halved.  Against each problem's own oracle
    adaptive run: accepted step sizes, error norms and the final state."""
    from oracle.solvers import AdaptiveStepper
    from tests.gpu_helpers import problem_slices
    parts = [I.marshak_single(8, state="front"),
             I.uniform_workload("u10", 10, I.box_field(I.sample_material_boxes(
                 np.random.default_rng(31), 2)), 5e-4, 1, np.random.default_rng(32),
                 state="front"),
             _far_from_equilibrium([(23, 1e-4)])]
    problems, boxes, z, E, T = [], [], [], [], []
    for p, wp in enumerate(parts):
        problems.append(wp.problems[0])
        b = wp.boxes[0]
        boxes.append(I.Box(p, 0, b.lo, b.hi))
        z.append(wp.z[0])
        E.append(wp.E[0])
        T.append(wp.T[0])
    w = I.Workload("adapt3", problems, boxes, z, E, T, np.array([1e-3, 5e-4, 1e-2]))
    eps, nsteps = 5e-3, 6
    kw = dict(newton_rtol=1e-10, newton_atol=1e-16, newton_maxit=24, newton_forcing=0)
    H = make(w, error_estimate=1, **kw)
    rc, dt_next, t, steps = H.adaptive_steps(nsteps, list(w.dt), eps)
    E_g, T_g = H.get_fields()
    got = np.concatenate([to_host(E_g), to_host(T_g)])
    sl = problem_slices(w)
    for p in range(3):
        s = system(w, pidx=p)
        ad = AdaptiveStepper(s, state(s, w, pidx=p), w.dt[p], eps, 1e-5, 1e-5 ** 0.25,
                             rtol=1e-10, atol=1e-16, maxit=24, forcing="kelley")
        for _ in range(nsteps):
            ad.advance()
        dts = [steps[n][p]["dt"] for n in range(nsteps)]
        errs = [steps[n][p]["err_norm"] for n in range(nsteps)]
        for n, (d_o, e_o) in enumerate(ad.log):
            assert abs(dts[n] / d_o - 1) < 1e-6, (p, n, dts[n], d_o)
            if e_o is None:
                assert errs[n] == -1.0
            else:
                assert abs(errs[n] / e_o - 1) < 1e-5, (p, n, errs[n], e_o)
        assert abs(dt_next[p] / ad.dt - 1) < 1e-6
        assert abs(t[p] - ad.t) < 1e-12
        g = got[sl[p]]
        n = s.nc
        for f in (slice(0, n), slice(n, 2 * n)):
            assert rel_err(g[f], ad.u[f]) < 1e-8
    assert steps[0][2]["dt"] < 1e-2          # the third problem's first step was halved


@pytest.mark.parametrize("stencil", [0, 1, 2, 3])
def test_per_patch_launches_match_batched_bitwise(stencil):
    """One launch per patch and one launch over the whole patch table run the
    same kernels on the same tiles: outputs are bitwise equal, run twice."""
    w = WL["amr3"]()
    s = system(w)
    u_n = state(s, w)
    rng = np.random.default_rng(5)
    u = s.sync(u_n * rng.uniform(0.9, 1.1, u_n.shape))
    v = rng.standard_normal(u.shape)
    outs = []
    for launch in (0, 1, 0):
        H = make(w, launch=launch, stencil=stencil)
        H.begin_step([2e-3])
        F = H.native()
        H.residual(native_from_compact(H, u), F)
        Jv = H.native()
        H.jvp(native_from_compact(H, u), native_from_compact(H, v), Jv)
        outs.append((compact_from_native(H, F), compact_from_native(H, Jv)))
    for a, b in outs[1:]:
        np.testing.assert_array_equal(a, outs[0][0])
        np.testing.assert_array_equal(b, outs[0][1])


@pytest.mark.parametrize("name", ["uniform16", "amr3"])
def test_fd_jvp_parity(name):
    """Jacobian-free mode (Sec. 4.1): the GPU difference quotient against the
    oracle's with the same step rule to 1e-6 (the quotient magnifies the
    round-off of the two residuals by 1/eps ~ 1e8), and against the analytic
    action to 1e-5."""
    w, s, H, u_n, u, dt = _setup(name, jvp_mode=1)
    rng = np.random.default_rng(7)
    v = s.sync(rng.standard_normal(u.shape) * u)
    v /= s.norm(v)
    Jv = H.native()
    H.jvp(native_from_compact(H, u), native_from_compact(H, v), Jv)
    got = compact_from_native(H, Jv)
    E, T = s.split(u)
    vE, vT = s.split(v)
    bE, bT = s.split(u_n)
    JE, JT = ops.jvp_fd(s.H, E, T, s.z, vE, vT, bE, bT, dt, 1.0, s.lam)
    ref = s.join(JE, JT)
    ana = s.jvp(u, v, dt, 1.0)
    n = s.nc
    for sl in (slice(0, n), slice(n, 2 * n)):
        assert rel_err(got[sl], ref[sl]) < 1e-6
        assert rel_err(got[sl], ana[sl]) < 1e-5
