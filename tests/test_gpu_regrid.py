"""Regridding on the GPU against the oracle (Sec. 5): refinement tags bit
for bit, the conservative transfer of a state to another hierarchy, and the
warm restart (re-solve of the last step on the new grid, then a BDF2 step
on the interpolated history) at the Newton tolerance."""
import numpy as np
import pytest

from oracle import regrid as rg
from oracle.hierarchy import Hierarchy
from oracle.solvers import Stepper, System
from paper_1302_6303_amd import inputs as I
from tests.gpu_helpers import compact_state, make, rel_err, to_dev, to_host
from tests.helpers import state, system

pytestmark = pytest.mark.gpu

OLD = [(0, (0, 0, 0), (8, 8, 8)), (1, (4, 4, 4), (12, 10, 12)), (1, (4, 10, 4), (8, 14, 10)),
       (2, (10, 10, 10), (18, 18, 18))]
NEW = [(0, (0, 0, 0), (8, 8, 8)), (1, (4, 4, 4), (14, 12, 12)),
       (2, (12, 10, 10), (22, 20, 18)), (3, (28, 24, 24), (36, 32, 32))]


def _workload(spec, seed=3):
    prob = I.Problem((8, 8, 8))
    boxes = [I.Box(0, lv, lo, hi) for lv, lo, hi in spec]
    zf = I.box_field([((0.3, 0.35, 0.3), (0.6, 0.65, 0.62), 10.0)])
    z = I.eval_on_boxes(zf, [prob], boxes)
    rng = np.random.default_rng(seed)
    E, T = I.front_state([prob], boxes, rng, noise=0.02, xf=0.45, width=0.08)
    return I.Workload("regrid", [prob], boxes, z, E, T, np.array([1e-3]), 1,
                      extra={"zf": zf})


@pytest.mark.parametrize("crit", [dict(grad_E=6.0), dict(tau_g=0.2), dict(tau_c=0.05),
                                  dict(z_interface=True),
                                  dict(grad_E=6.0, z_interface=True, tau_c=0.05)])
@pytest.mark.parametrize("name", ["amr3", "manual"])
def test_tags_match_the_oracle_bitwise(name, crit):
    if name == "amr3":
        w = I.static_amr(base=16, nlevels=3, side=(8, 16), state="front")
    else:
        w = _workload(OLD)
    s = system(w)
    H = make(w)
    got = to_host(H.tag(**crit).to(dtype=__import__("torch").float64)).astype(np.uint8)
    E, _ = s.split(state(s, w))
    ref = rg.tags(s.H, E, s.z, grad=crit.get("grad_E", 0.0),
                  z_interface=crit.get("z_interface", False), tau_g=crit.get("tau_g", 0.0),
                  tau_c=crit.get("tau_c", 0.0))
    ref = np.concatenate([t.ravel(order="F") for t in ref]).astype(np.uint8)
    assert ref.sum() > 0
    np.testing.assert_array_equal(got, ref)


def test_transfer_matches_the_oracle():
    wo, wn = _workload(OLD), _workload(NEW)
    Ho, Hn = make(wo), make(wn)
    zn = to_dev(wn.compact(wn.z))
    Ho.transfer_to(Hn, zn)
    E, T = Hn.get_fields()
    so, sn = system(wo), system(wn)
    Eo, To = so.split(state(so, wo))
    ref = np.concatenate([np.concatenate([a.ravel(order="F") for a in
                                          rg.transfer(so.H, Eo, sn.H)]),
                          np.concatenate([a.ravel(order="F") for a in
                                          rg.transfer(so.H, To, sn.H)])])
    got = np.concatenate([to_host(E), to_host(T)])
    np.testing.assert_allclose(got, ref, rtol=1e-15, atol=0)
    # no step was taken: the re-solve has nothing to do
    st = Hn.resolve()
    assert st[0]["newton_iters"] == 0


def test_warm_restart_matches_the_oracle():
    """Two BDF steps on one hierarchy, the history moved to another, the
    last step solved again there, then a BDF2 step on the interpolated
    history: the GPU and the oracle agree at the Newton tolerance after the
    re-solve and after the next step."""
    wo, wn = _workload(OLD), _workload(NEW)
    kw = dict(newton_rtol=1e-10, newton_atol=1e-14)
    Ho, Hn = make(wo, **kw), make(wn, **kw)
    so, sn = system(wo), system(wn)
    st = Stepper(so, state(so, wo), rtol=1e-10, atol=1e-14)
    for dt in (1e-3, 1e-3):
        Ho.implicit_step([dt])
        assert st.step(dt).converged
    Ho.transfer_to(Hn, to_dev(wn.compact(wn.z)))
    rs = Hn.resolve()
    ref = st.regrid(sn)
    assert rs[0]["converged"] and rs[0]["newton_iters"] >= 2
    E, T = Hn.get_fields()
    got = np.concatenate([to_host(E), to_host(T)])
    n = sn.nc
    assert rel_err(got[:n], st.u[:n]) < 1e-8 and rel_err(got[n:], st.u[n:]) < 1e-8
    _, s2 = Hn.implicit_step([1e-3])
    assert st.step(1e-3).converged
    E, T = Hn.get_fields()
    got = np.concatenate([to_host(E), to_host(T)])
    assert rel_err(got[:n], st.u[:n]) < 1e-8 and rel_err(got[n:], st.u[n:]) < 1e-8
    del ref


def test_transfer_conserves_the_composite_integral():
    import torch
    wo, wn = _workload(OLD), _workload(NEW)
    Ho, Hn = make(wo), make(wn)
    Ho.implicit_step([1e-3])
    Ho.transfer_to(Hn, to_dev(wn.compact(wn.z)))

    def integral(H):
        E, T = H.get_fields()
        one = torch.ones(H.ncells, dtype=torch.float64, device="cuda")
        zero = torch.zeros_like(one)
        u = H.unpack(torch.cat([E, T]))
        return H.dot(u, H.unpack(torch.cat([one, zero])))[0], \
            H.dot(u, H.unpack(torch.cat([zero, one])))[0]
    a, b = integral(Ho), integral(Hn)
    assert abs(a[0] - b[0]) <= 1e-13 * abs(a[0]) and abs(a[1] - b[1]) <= 1e-13 * abs(a[1])


def test_regrid_cycle_matches_the_oracle():
    """A whole regrid inside a run on a 3-level hierarchy: two steps, the
    tags of the state (GPU bit for bit equal to the oracle's), the boxes the
    host clustering makes of them, the history moved and re-solved, a BDF2
    step; GPU and oracle agree at the Newton tolerance."""
    from paper_1302_6303_amd import nrd
    from paper_1302_6303_amd.regrid import Regridder
    w = _workload(OLD)
    zf = w.extra["zf"]
    kw = dict(newton_rtol=1e-10, newton_atol=1e-14)
    H = make(w, **kw)
    s = system(w)
    st = Stepper(s, state(s, w), rtol=1e-10, atol=1e-14)
    for dt in (1e-3, 1e-3):
        H.implicit_step([dt])
        assert st.step(dt).converged
    crit = dict(grad_E=18.0)
    tags = to_host(H.tag(**crit).double()).astype(np.uint8)
    E, _ = s.split(st.u)
    ref = rg.tags(s.H, E, s.z, grad=18.0)
    ref = np.concatenate([t.ravel(order="F") for t in ref]).astype(np.uint8)
    # the states agree to the Newton tolerance, the tags exactly unless a
    # cell sits within that tolerance of the threshold
    assert ref.sum() > 0 and np.count_nonzero(tags != ref) == 0
    res = nrd.cluster(w.problems, w.boxes, ref, max_levels=3, buffer=1, efficiency=0.7,
                      min_side=2, max_side=8)
    boxes = [I.Box(p, lv, lo, hi) for p, lv, lo, hi in res]
    assert boxes != w.boxes and max(b.level for b in boxes) == 2

    def zfun(problems, bx):
        return to_dev(np.concatenate([a.ravel(order="F")
                                      for a in I.eval_on_boxes(zf, problems, bx)]))
    R = Regridder(nrd.default_options(**kw), crit, {}, zfun)
    Hn, _, info = R.regrid(H, boxes)
    assert info["resolve_newton"] >= 1
    pr = w.problems[0]
    Hs = Hierarchy(pr.base_n, [(b.level, b.lo, b.hi) for b in boxes])
    sn = System(Hs, I.eval_on_boxes(zf, w.problems, boxes))
    st.regrid(sn)
    Hn.implicit_step([1e-3])
    assert st.step(1e-3).converged
    E, T = Hn.get_fields()
    got = np.concatenate([to_host(E), to_host(T)])
    n = sn.nc
    assert rel_err(got[:n], st.u[:n]) < 1e-8 and rel_err(got[n:], st.u[n:]) < 1e-8
