"""Parity at the full sizes of the benchmark workloads, in the launch
configuration the benchmark times (one batched launch per operator, staged
plane stencil with tuned tile shapes, float32 preconditioner inside float64
Newton-Krylov), checked against the oracle problem by problem.

Workloads: the 64-problem ensemble (32^3..96^3, 21.6 M cells) and the static
3-level AMR hierarchy on a 64^3 base (228 patches, 1.04 M cells).
Tolerances as for the small cases: 1e-12 (float64 operators), 1e-10 (float64
preconditioner), 1e-8 (implicit steps at Newton rtol 1e-10); the float32
preconditioner agrees with the float64 oracle to float32 round-off (1e-4)."""
import numpy as np
import pytest

from paper_1302_6303_amd import inputs as I
from oracle.solvers import Stepper
from tests.gpu_helpers import (compact_from_native, compact_state, make,
                               native_from_compact, problem_slices, rel_err, to_dev,
                               to_host)
from tests.helpers import state, system

pytestmark = pytest.mark.gpu

_ENS = {}


def ensemble():
    if "w" not in _ENS:
        _ENS["w"] = I.ensemble(state="front")
    return _ENS["w"]


def _perturbed(w, seed):
    rng = np.random.default_rng(seed)
    u_n = compact_state(w)            # uniform grids: no covered cells to restrict
    return u_n, u_n * rng.uniform(0.9, 1.1, u_n.shape), rng


def _per_problem(w, got, ref_fn, tol):
    sl = problem_slices(w)
    worst = 0.0
    for p in range(len(w.problems)):
        ref = ref_fn(p)
        g = got[sl[p]]
        n = len(ref) // 2
        for a, b in ((g[:n], ref[:n]), (g[n:], ref[n:])):
            worst = max(worst, rel_err(a, b))
    assert worst < tol, worst
    return worst


def test_ensemble_residual_and_jvp_every_problem():
    w = ensemble()
    H = make(w, precision=1)
    H.autotune(None)
    u_n, u, rng = _perturbed(w, 31)
    v = rng.standard_normal(u.shape) * u
    H.begin_step(list(w.dt))
    F = H.native()
    H.residual(native_from_compact(H, u), F)
    Jv = H.native()
    H.jvp(native_from_compact(H, u), native_from_compact(H, v), Jv)
    got_F, got_J = compact_from_native(H, F), compact_from_native(H, Jv)
    sl = problem_slices(w)

    def ref_F(p):
        s = system(w, pidx=p)
        return s.residual(u[sl[p]], u_n[sl[p]], float(w.dt[p]), 1.0)

    def ref_J(p):
        s = system(w, pidx=p)
        return s.jvp(u[sl[p]], v[sl[p]], float(w.dt[p]), 1.0)

    _per_problem(w, got_F, ref_F, 1e-12)
    _per_problem(w, got_J, ref_J, 1e-12)


@pytest.mark.parametrize("precision,tol", [(0, 1e-10), (1, 1e-4)])
def test_ensemble_preconditioner_every_problem(precision, tol):
    w = ensemble()
    H = make(w, precision=precision)
    u_n, u, rng = _perturbed(w, 32)
    wv = rng.standard_normal(u.shape)
    H.begin_step(list(w.dt))
    H.precond_setup(native_from_compact(H, u))
    y = H.native()
    H.precond_apply(native_from_compact(H, wv), y)
    got = compact_from_native(H, y)
    sl = problem_slices(w)

    def ref(p):
        s = system(w, pidx=p)
        P, _ = s.precond(u[sl[p]], float(w.dt[p]))
        return P(wv[sl[p]])

    _per_problem(w, got, ref, tol)


def test_ensemble_implicit_step_every_problem():
    """One lock-step BDF1 step of all 64 problems from the benchmark's
    initial state (E0, T0 = E0^(1/4) everywhere, Marshak inflow), mixed
    precision, batched; the 24 problems of 32^3 and 48^3 cells are checked
    against the oracle's own Newton-Krylov step, the 40 problems of 64^3 to
    96^3 cells by the oracle's residual of the step at the GPU's solution,
    which must be down by the Newton tolerance from its value at the initial
    guess (the oracle's own solve of those takes minutes per problem)."""
    w = I.ensemble()
    H = make(w, precision=1, newton_rtol=1e-10, newton_atol=1e-16, newton_maxit=24)
    H.autotune(None)
    rc, stats = H.implicit_step(list(w.dt), raise_on_fail=False)
    bad = [(p, st["newton_iters"], st["fnorm0"], st["fnorm"], st["krylov_iters"])
           for p, st in enumerate(stats) if not st["converged"]]
    assert not bad, bad
    E, T = H.get_fields()
    got = np.concatenate([to_host(E), to_host(T)])
    sl = problem_slices(w)
    checked = 0
    large = 0
    for p, b in enumerate(w.boxes):
        if b.shape[0] > 48:
            s = system(w, pidx=p)
            u0 = state(s, w, pidx=p)
            dt = float(w.dt[p])
            f0 = s.norm(s.residual(u0, u0, dt, 1.0))
            f1 = s.norm(s.residual(got[sl[p]], u0, dt, 1.0))
            assert f1 <= 2e-10 * f0, (p, f0, f1)
            large += 1
            continue
        s = system(w, pidx=p)
        st = Stepper(s, state(s, w, pidx=p), rtol=1e-10, atol=1e-16)
        r = st.step(float(w.dt[p]))
        assert r.converged
        g = got[sl[p]]
        n = s.nc
        assert rel_err(g[:n], st.u[:n]) < 1e-8
        assert rel_err(g[n:], st.u[n:]) < 1e-8
        checked += 1
    assert checked == 24 and large == 40


def test_static_amr_residual_full_hierarchy():
    """The 64^3-base 3-level hierarchy (228 patches): batched residual with
    coarse-fine ghosts and flux matching against the oracle."""
    w = I.static_amr(state="front")
    s = system(w)
    H = make(w)
    H.autotune(None)
    u_n = state(s, w)
    rng = np.random.default_rng(33)
    u = s.sync(u_n * rng.uniform(0.9, 1.1, u_n.shape))
    H.begin_step([5e-4])
    F = H.native()
    H.residual(native_from_compact(H, u), F)
    got = compact_from_native(H, F)
    ref = s.residual(u, u_n, 5e-4, 1.0)
    n = s.nc
    assert rel_err(got[:n], ref[:n]) < 1e-12
    assert rel_err(got[n:], ref[n:]) < 1e-12


def test_differentiation_workload_gradient_at_full_size():
    """The differentiation configuration as configured: uniform 64^3, z = 1 +
    9 s (smoothed random field), 50 backward-Euler steps of 1e-3 with state
    checkpoints every 10 steps, J = sum of E at the final time.  The adjoint
    gradient against the oracle's (a stored fixture written by
    tests/golden/make_adjoint64.py from the oracle alone) at 1e-7, and
    against central differences of the GPU's own forward solve (Newton rtol
    1e-13, h = 1e-6) on 20 seeded cells whose sensitivity is at least 1e-3
    of the largest, at 1e-5."""
    import json
    import os
    fx = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "adjoint64.json")))
    N, every, dt = fx["nsteps"], 10, fx["dt"]
    w = I.differentiation(fx["n"])
    opts = dict(newton_rtol=1e-13, newton_atol=1e-22, newton_maxit=24, gmres_maxrestarts=30,
                adjoint_slots=-(-N // every) + every + 3)
    H = make(w, **opts)
    g = to_host(H.adjoint_run([dt], N, every))
    cells = np.array(fx["fd_cells"] + fx["sample_cells"])
    ref = np.array(fx["fd_values"] + fx["sample_values"])
    scale = fx["grad_max_abs"]
    assert np.max(np.abs(g[cells] - ref)) <= 1e-7 * scale, \
        (np.max(np.abs(g[cells] - ref)), scale)
    fd_cells = np.array(fx["fd_cells"])
    assert np.all(np.abs(g[fd_cells] - ref[:20]) <= 1e-7 * np.abs(ref[:20]))
    # central differences of the forward solve, backward Euler throughout
    Hf = make(w, bdf_max_order=1, **opts)
    zc = w.compact(w.z)
    u = compact_state(w)
    nn = Hf.ncells

    def J(zz):
        Hf.set_fields(to_dev(u[:nn]), to_dev(u[nn:]), to_dev(zz))
        for _ in range(N):
            Hf.implicit_step([dt])
        E, _ = Hf.get_fields()
        return np.sum(np.sort(to_host(E)))
    h = 1e-6
    worst = 0.0
    for c in fd_cells:
        zp, zm = zc.copy(), zc.copy()
        zp[c] += h
        zm[c] -= h
        fd = (J(zp) - J(zm)) / (2 * h)
        worst = max(worst, abs(fd - g[c]) / abs(g[c]))
    assert worst <= 1e-5, worst
