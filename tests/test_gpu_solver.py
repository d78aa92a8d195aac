"""Solver-level GPU tests through the C ABI: lock-step ensembles, precision
modes, determinism, failure handling and the discrete adjoint.

Tolerances: implicit-step solutions 1e-8 relative per field (both sides at
Newton rtol 1e-10); mixed-precision preconditioning changes only the Krylov
path, so its converged solution must agree with float64 to the Newton
tolerance; gradients 1e-7 relative to the oracle's adjoint and 1e-5 to
central finite differences.
"""
import numpy as np
import pytest

from oracle.hierarchy import Hierarchy
from oracle.solvers import Stepper, System, adjoint_gradient
from paper_1302_6303_amd import inputs as I
from tests.gpu_helpers import (compact_state, make, problem_slices, rel_err, to_dev,
                               to_host)
from tests.helpers import state, system

pytestmark = pytest.mark.gpu


def small_ensemble(state_kind="front"):
    """Four independent problems of different sizes, materials and steps."""
    rng = np.random.default_rng(77)
    problems, boxes, z = [], [], []
    sizes = [8, 12, 10, 16]
    for p, n in enumerate(sizes):
        pr = I.Problem(base_n=(n, n, n))
        b = I.Box(p, 0, (0, 0, 0), (n, n, n))
        zf = I.box_field(I.sample_material_boxes(rng, 1 + p % 3,
                                                 np.where(rng.uniform(size=3) < 0.5, 1.0, 10.0)))
        problems.append(pr)
        boxes.append(b)
        z.append(zf(*I.cell_centres(pr, b)))
    if state_kind == "front":
        E, T = I.front_state(problems, boxes, rng)
    else:
        E, T = I.uniform_state(boxes)
    dts = np.array([1e-3, 5e-4, 2e-3, 8e-4])
    return I.Workload("ens4", problems, boxes, z, E, T, dts, 3)


def _fields(H):
    E, T = H.get_fields()
    return np.concatenate([to_host(E), to_host(T)])


def test_lockstep_ensemble_matches_each_problem():
    w = small_ensemble()
    H = make(w, newton_rtol=1e-10, newton_atol=1e-16)
    steppers = []
    for p in range(len(w.problems)):
        s = system(w, pidx=p)
        steppers.append((s, Stepper(s, state(s, w, pidx=p), rtol=1e-10, atol=1e-16)))
    sl = problem_slices(w)
    for step in range(3):
        dt = w.dt * (1.0 if step < 2 else 1.5)
        rc, stats = H.implicit_step(list(dt))
        got = _fields(H)
        for p, (s, st) in enumerate(steppers):
            r = st.step(float(dt[p]))
            assert r.converged and stats[p]["converged"]
            n = s.nc
            ref = st.u
            g = got[sl[p]]
            assert rel_err(g[:n], ref[:n]) < 1e-8
            assert rel_err(g[n:], ref[n:]) < 1e-8


@pytest.mark.parametrize("name", ["uniform", "amr", "amr-jacobi"])
def test_mixed_precision_preconditioner_keeps_the_solution(name):
    w = I.marshak_single(16, state="front") if name == "uniform" else \
        I.static_amr(base=16, nlevels=3, side=(8, 16), state="front")
    extra = {"fac_smoother": 1, "fac_nu_pre": 2} if name == "amr-jacobi" else {}
    Hd = make(w, precision=0, newton_rtol=1e-10, newton_atol=1e-16, **extra)
    Hm = make(w, precision=1, newton_rtol=1e-10, newton_atol=1e-16, **extra)
    kd = km = 0
    for dt in (1e-3, 1e-3, 1e-3):
        _, sd = Hd.implicit_step([dt])
        _, sm = Hm.implicit_step([dt])
        kd += sd[0]["krylov_iters"]
        km += sm[0]["krylov_iters"]
    a, b = _fields(Hd), _fields(Hm)
    n = len(a) // 2
    assert rel_err(b[:n], a[:n]) < 1e-8
    assert rel_err(b[n:], a[n:]) < 1e-8
    print(f"krylov iterations fp64 {kd} mixed {km}")


def test_reruns_are_bitwise_identical():
    w = I.static_amr(base=16, nlevels=3, side=(8, 16), state="front")
    outs = []
    for _ in range(2):
        H = make(w, precision=1)
        for dt in (1e-3, 1e-3):
            H.implicit_step([dt])
        outs.append(_fields(H))
    np.testing.assert_array_equal(outs[0], outs[1])


def test_nonpositive_fields_are_rejected_and_state_kept():
    from paper_1302_6303_amd import nrd
    w = I.marshak_single(8, state="front")
    H = make(w)
    before = _fields(H)
    u = compact_state(w)
    n = H.ncells
    bad = u.copy()
    bad[3] = -1.0
    with pytest.raises(nrd.NrdError) as e:
        H.set_fields(to_dev(bad[:n]), to_dev(bad[n:]), to_dev(w.compact(w.z)))
    assert e.value.status == nrd.NRD_ENONPOS
    nanz = w.compact(w.z).copy()
    nanz[0] = np.nan
    with pytest.raises(nrd.NrdError):
        H.set_fields(to_dev(u[:n]), to_dev(u[n:]), to_dev(nanz))
    np.testing.assert_array_equal(_fields(H), before)


def test_newton_failure_rolls_back():
    from paper_1302_6303_amd import nrd
    w = I.marshak_single(8, state="front")
    H = make(w, newton_maxit=1, newton_rtol=1e-14, newton_atol=0.0)
    before = _fields(H)
    rc, stats = H.implicit_step([1e-3], raise_on_fail=False)
    assert rc == nrd.NRD_ENOTCONV and not stats[0]["converged"]
    np.testing.assert_array_equal(_fields(H), before)


def test_calls_in_wrong_order_report_state_error():
    from paper_1302_6303_amd import nrd
    w = I.marshak_single(8, state="front")
    H = make(w)
    F = H.native()
    with pytest.raises(nrd.NrdError) as e:
        H.residual(H.native(), F)             # no begin_step yet
    assert e.value.status == nrd.NRD_ESTATE


def _smooth_z(n, seed):
    rng = np.random.default_rng(seed)
    return 1.0 + 9.0 * np.clip(0.5 + 0.35 * rng.standard_normal((n, n, n)), 0.0, 1.0)


def test_adjoint_matches_oracle_adjoint():
    n, N, every, dt = 8, 4, 2, 2e-3
    z = _smooth_z(n, 91)
    w = I.marshak_single(n)
    w.z = [z]
    H = make(w, newton_rtol=1e-11, newton_atol=1e-22, newton_maxit=24,
             adjoint_slots=N // every + every + 3, gmres_maxrestarts=20)
    gz = to_host(H.adjoint_run([dt], N, every))
    s = System(Hierarchy((n, n, n), [(0, (0, 0, 0), (n, n, n))]), [z])
    u0 = np.concatenate([w.compact(w.E), w.compact(w.T)])
    ref, _ = adjoint_gradient(s, u0, dt, N, tol=1e-13,
                              newton_kw=dict(rtol=1e-11, atol=1e-22, maxit=40))
    assert rel_err(gz, ref) < 1e-7


def _two_level(n=6):
    return I.small_amr(n, boxes_spec=[(1, (2, 2, 2), (2 * n - 2, 2 * n - 4, 2 * n - 2))])


def test_adjoint_on_two_levels_matches_oracle_adjoint():
    """Refined hierarchy: J sums E over the composite cells; dJ/dz of both
    levels (covered coarse cells included) against the oracle's adjoint."""
    from tests.helpers import state, system
    w = _two_level()
    N, every, dt = 3, 2, 2e-3
    H = make(w, newton_rtol=1e-11, newton_atol=1e-22, newton_maxit=24,
             adjoint_slots=(N + every - 1) // every + every + 3, gmres_maxrestarts=20)
    gz = to_host(H.adjoint_run([dt], N, every))
    s = system(w)
    ref, _ = adjoint_gradient(s, state(s, w), dt, N, tol=1e-13,
                              newton_kw=dict(rtol=1e-11, atol=1e-22, maxit=40))
    assert rel_err(gz, ref) < 1e-7


def test_adjoint_on_two_levels_matches_central_differences():
    """The refined hierarchy's adjoint gradient against central differences
    of the GPU forward solve, on the largest entries, a covered coarse
    cell's and a fine cell's."""
    w = _two_level(8)
    N, every, dt = 4, 2, 1e-3
    opts = dict(newton_rtol=1e-11, newton_atol=1e-22, newton_maxit=24,
                gmres_maxrestarts=30, adjoint_slots=N // every + every + 3)
    H = make(w, **opts)
    g = to_host(H.adjoint_run([dt], N, every))
    comp = system(w).composite[:H.ncells]
    n0 = w.boxes[0].ncells
    cov0 = ~comp[:n0]
    zc = w.compact(w.z)
    order = list(np.argsort(-np.abs(g))[:4])
    order.append(int(np.argmax(np.where(cov0, np.abs(g[:n0]), -1.0))))
    order.append(n0 + int(np.argmax(np.abs(g[n0:]))))
    Hf = make(w, bdf_max_order=1, **opts)

    def J(zz):
        u = compact_state(w)
        nn = Hf.ncells
        Hf.set_fields(to_dev(u[:nn]), to_dev(u[nn:]), to_dev(zz))
        for _ in range(N):
            Hf.implicit_step([dt])
        E, _ = Hf.get_fields()
        return np.sum(np.sort(to_host(E)[comp]))

    for c in order:
        hz = 1e-5 * zc[c]
        zp = zc.copy()
        zm = zc.copy()
        zp[c] += hz
        zm[c] -= hz
        fd = (J(zp) - J(zm)) / (2 * hz)
        assert abs(fd - g[c]) <= 1e-5 * abs(g[c]), (c, fd, g[c])


def test_adjoint_of_a_batch_with_a_refined_problem():
    """Two problems adjoined together, one refined (two levels) and one
    uniform with smooth random material: each problem's part of dJ/dz
    against its own oracle adjoint (J sums E over every problem's composite
    cells, so the problems' gradients are independent)."""
    a = _two_level()
    b = I.marshak_single(6)
    b.z = [_smooth_z(6, 94)]
    boxes = list(a.boxes) + [I.Box(1, bb.level, bb.lo, bb.hi) for bb in b.boxes]
    w = I.Workload("pair", a.problems + b.problems, boxes, a.z + b.z, a.E + b.E, a.T + b.T,
                   np.array([2e-3, 2e-3]))
    N, every, dt = 3, 2, 2e-3
    H = make(w, newton_rtol=1e-11, newton_atol=1e-22, newton_maxit=24,
             adjoint_slots=(N + every - 1) // every + every + 3, gmres_maxrestarts=20)
    gz = to_host(H.adjoint_run([dt, dt], N, every))
    off = 0
    for p in range(2):
        s = system(w, pidx=p)
        ref, _ = adjoint_gradient(s, state(s, w, pidx=p), dt, N, tol=1e-13,
                                  newton_kw=dict(rtol=1e-11, atol=1e-22, maxit=40))
        assert rel_err(gz[off:off + s.nc], ref) < 1e-7, p
        off += s.nc


def test_autograd_on_a_refined_hierarchy():
    """torch.autograd through RadDiffEvolve on two levels: E at the end and
    dJ/dz of J = a weighted sum of E over every cell, covered cells included
    (their E is the mean of their children's, so their weights reach the
    children), against the oracle's adjoint of the same objective."""
    import torch
    from paper_1302_6303_amd.autograd import RadDiffEvolve
    w = _two_level()
    N, every, dt = 2, 1, 2e-3
    H = make(w, newton_rtol=1e-11, newton_atol=1e-22, newton_maxit=24, bdf_max_order=1,
             adjoint_slots=N // every + every + 3, gmres_maxrestarts=20)
    u = compact_state(w)
    nc = H.ncells
    E0, T0 = to_dev(u[:nc]), to_dev(u[nc:])
    z = to_dev(w.compact(w.z)).requires_grad_(True)
    E = RadDiffEvolve.apply(z, H, E0, T0, dt, N, every)
    s = system(w)
    wts = np.random.default_rng(95).uniform(0.5, 1.5, nc)
    (E * to_dev(wts)).sum().backward()
    ref, states = adjoint_gradient(s, state(s, w), dt, N, tol=1e-13,
                                   newton_kw=dict(rtol=1e-11, atol=1e-22, maxit=40),
                                   dJdE=wts)
    assert rel_err(to_host(E), states[-1][:nc]) < 1e-8
    assert rel_err(to_host(z.grad), ref) < 1e-7


def test_adjoint_gradient_matches_central_differences():
    """dJ/dz of J = sum of E after N BDF1 steps, against central
    differences of the same GPU forward solve (h = 1e-5 z) on the cells with
    the largest sensitivity."""
    from paper_1302_6303_amd import nrd
    n, N, every, dt = 16, 6, 3, 1e-3
    z = _smooth_z(n, 92)
    w = I.marshak_single(n)
    w.z = [z]
    opts = dict(newton_rtol=1e-11, newton_atol=1e-22, newton_maxit=24,
                gmres_maxrestarts=30, adjoint_slots=N // every + every + 3)
    H = make(w, **opts)
    g = to_host(H.adjoint_run([dt], N, every))
    # the forward solve with backward Euler throughout, like the adjoint's
    zc = w.compact(w.z)
    order = np.argsort(-np.abs(g))[:6]
    Hf = make(w, bdf_max_order=1, **opts)

    def J(zz):
        u = compact_state(w)
        nn = Hf.ncells
        Hf.set_fields(to_dev(u[:nn]), to_dev(u[nn:]), to_dev(zz))
        for _ in range(N):
            Hf.implicit_step([dt])
        E, _ = Hf.get_fields()
        e = to_host(E)
        return np.sum(np.sort(e))

    for c in order:
        hz = 1e-5 * zc[c]
        zp = zc.copy()
        zm = zc.copy()
        zp[c] += hz
        zm[c] -= hz
        fd = (J(zp) - J(zm)) / (2 * hz)
        assert abs(fd - g[c]) <= 1e-5 * abs(g[c]), (c, fd, g[c])


def test_autograd_function_gives_the_adjoint_gradient():
    """torch.autograd through RadDiffEvolve equals the oracle's adjoint."""
    import torch
    from paper_1302_6303_amd.autograd import RadDiffEvolve
    n, N, every, dt = 8, 4, 2, 2e-3
    zc = _smooth_z(n, 93)
    w = I.marshak_single(n)
    w.z = [zc]
    H = make(w, newton_rtol=1e-11, newton_atol=1e-22, newton_maxit=24, bdf_max_order=1,
             adjoint_slots=N // every + every + 3, gmres_maxrestarts=20)
    u = compact_state(w)
    nc = H.ncells
    E0, T0 = to_dev(u[:nc]), to_dev(u[nc:])
    z = to_dev(w.compact(w.z)).requires_grad_(True)
    E = RadDiffEvolve.apply(z, H, E0, T0, dt, N, every)
    E.sum().backward()
    s = System(Hierarchy((n, n, n), [(0, (0, 0, 0), (n, n, n))]), [zc])
    ref, states = adjoint_gradient(s, u, dt, N, tol=1e-13,
                                   newton_kw=dict(rtol=1e-11, atol=1e-22, maxit=40))
    assert rel_err(to_host(E), states[-1][:nc]) < 1e-8
    assert rel_err(to_host(z.grad), ref) < 1e-7


def test_jacobian_free_mode_reaches_the_same_solution():
    """Newton with difference-quotient products converges to the solution of
    the analytic-Jacobian run (the products only steer the Krylov solves)."""
    w = I.static_amr(base=16, nlevels=3, side=(8, 16), state="front")
    Ha = make(w, newton_rtol=1e-10, newton_atol=1e-16)
    Hf = make(w, jvp_mode=1, newton_rtol=1e-10, newton_atol=1e-16)
    for dt in (1e-3, 1e-3):
        _, sa = Ha.implicit_step([dt])
        _, sf = Hf.implicit_step([dt])
        assert sa[0]["converged"] and sf[0]["converged"]
    a, b = _fields(Ha), _fields(Hf)
    n = len(a) // 2
    assert rel_err(b[:n], a[:n]) < 1e-8
    assert rel_err(b[n:], a[n:]) < 1e-8


@pytest.mark.parametrize("kind", ["amr", "ensemble"])
def test_graph_captured_iterations_replay_bitwise(kind):
    """FGMRES iterations captured as HIP graphs (one per Krylov index) and
    replayed across Newton iterations, restarts and steps, with eager work
    and host synchronisations in between, give bitwise the eager results."""
    w = I.static_amr(base=16, nlevels=3, side=(8, 16), state="front") if kind == "amr" \
        else small_ensemble()
    outs = []
    for g in (0, 1):
        H = make(w, precision=1, use_graph=g)
        dts = list(w.dt)
        stats = []
        for step in range(3):
            _, st = H.implicit_step([d * (1.0 if step < 2 else 1.3) for d in dts])
            stats.append([(s["newton_iters"], s["krylov_iters"]) for s in st])
            outs.append((g, step, _fields(H)))
        outs.append((g, "stats", stats))
    eager = [o for o in outs if o[0] == 0]
    graph = [o for o in outs if o[0] == 1]
    for a, b in zip(eager, graph):
        if a[1] == "stats":
            assert a[2] == b[2]
        else:
            np.testing.assert_array_equal(a[2], b[2])


@pytest.mark.parametrize("kind", ["uniform", "two_level"])
def test_graph_captured_adjoint_matches_eager(kind):
    """The transposed FGMRES iterations captured as HIP graphs give the
    eager run's gradient bit for bit (on two levels the captured iteration
    includes the transposed coarse-fine interpolation and restriction)."""
    N, every, dt = 4, 2, 2e-3
    if kind == "uniform":
        w = I.marshak_single(8)
        w.z = [_smooth_z(8, 94)]
    else:
        w = _two_level()
    g = []
    for use_graph in (0, 1):
        H = make(w, newton_rtol=1e-11, newton_atol=1e-22, newton_maxit=24,
                 adjoint_slots=N // every + every + 3, gmres_maxrestarts=20,
                 use_graph=use_graph)
        g.append(to_host(H.adjoint_run([dt], N, every)))
    np.testing.assert_array_equal(g[0], g[1])


@pytest.mark.parametrize("variant", ["afacx", "line"])
def test_adjoint_on_two_levels_with_other_preconditioners(variant):
    """The reverse sweep's transposed solves converge to the same gradient
    whatever the preconditioner: AFACx, and FAC with the block Gauss-Seidel
    smoother, against the oracle's adjoint (preconditioned by FAC)."""
    from paper_1302_6303_amd import nrd
    w = _two_level()
    N, every, dt = 3, 2, 2e-3
    extra = ({"fac_cycle": nrd.NRD_FAC_AFACX} if variant == "afacx"
             else {"fac_smoother": nrd.NRD_SMOOTH_LINE})
    H = make(w, newton_rtol=1e-11, newton_atol=1e-22, newton_maxit=24,
             adjoint_slots=(N + every - 1) // every + every + 3, gmres_maxrestarts=20, **extra)
    gz = to_host(H.adjoint_run([dt], N, every))
    s = system(w)
    ref, _ = adjoint_gradient(s, state(s, w), dt, N, tol=1e-13,
                              newton_kw=dict(rtol=1e-11, atol=1e-22, maxit=40))
    assert rel_err(gz, ref) < 1e-7


def test_paper_model_problem_step_count_matches_the_paper():
    """The paper's model problem (Sec. 6) on the uniform 32^3 grid with its
    solver settings (BDF2, PC.4.7 at eps_t = 5e-4, Newton 1e-12 / 1e-10)
    integrated to t = 1 takes the paper's number of time steps (1334 in
    its Table ndt, Levels = 1) within 5 %."""
    from paper_1302_6303_amd import nrd
    w = I.paper_marshak(32)
    H = make(w, precision=nrd.NRD_MIXED, error_estimate=1, newton_rtol=1e-12,
             newton_atol=1e-10)
    t, dt, steps = 0.0, 1e-5, 0
    while t < 1.0 - 1e-12:
        dt = min(dt, 1.0 - t)
        _, dtn, tt, _ = H.adaptive_steps(1, [dt], 5e-4, t=[t])
        t, dt = tt[0], dtn[0]
        steps += 1
        assert steps < 3000
    print(f"steps to t = 1: {steps} (paper 1334)")
    assert abs(steps - 1334) < 0.05 * 1334
