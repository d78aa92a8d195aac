"""Time-step control of the oracle (Sec. 3.4-3.5: leapfrog predictor, BDF2 local
error estimate, scaled max norm, EPS and PC.4.7 controllers) against
properties the paper and the mathematics fix."""
import numpy as np
import pytest

from oracle import solvers as S
from paper_1302_6303_amd import inputs as I
from tests.helpers import state, system


@pytest.mark.parametrize("dtp,dt", [(0.1, 0.1), (0.1, 0.15), (0.2, 0.07), (0.05, 0.11)])
def test_bdf2_error_estimate_is_exact_for_cubics(dtp, dt):
    # u' = g(t) with u a cubic: the Taylor expansions behind the BDF2 and
    # leapfrog local errors end at the third derivative, so the estimate
    # (a + 1) / (3 a + 2) (u_{n+1} - u^p) equals the BDF2 local error
    # u_{n+1} - u(t_{n+1}) to rounding; a wrong BDF2 coefficient, predictor
    # term or estimate factor breaks the equality
    coef = np.array([[0.7, -1.3, 0.4, 2.0], [-0.2, 0.5, 1.1, -0.3], [1.5, 0.0, -2.0, 1.0]])
    u = lambda t: coef[:, 0] * t**3 + coef[:, 1] * t**2 + coef[:, 2] * t + coef[:, 3]
    du = lambda t: 3 * coef[:, 0] * t**2 + 2 * coef[:, 1] * t + coef[:, 2]
    t0 = 0.3
    t1, t2 = t0 + dtp, t0 + dtp + dt
    c0, a = S.bdf_coefficients(dt, dtp)
    b = S.bdf2_history(u(t1), u(t0), a)
    u_new = (b + dt * du(t2)) / c0               # c0 u - b = dt f, f = g(t_{n+1})
    up = S.leapfrog_predictor(u(t1), u(t0), du(t1), dt, a)
    est = S.bdf2_error_estimate(u_new, up, a)
    assert np.allclose(est, u_new - u(t2), rtol=1e-9, atol=1e-14)


def test_bdf2_local_error_is_third_order():
    # halving both steps divides the estimate of a smooth (non-polynomial)
    # solution by about 8
    u = lambda t: np.array([np.sin(3 * t), np.exp(-t)])
    du = lambda t: np.array([3 * np.cos(3 * t), -np.exp(-t)])
    errs = []
    for h in (0.01, 0.005, 0.0025):
        t0, t1, t2 = 0.4, 0.4 + h, 0.4 + 2.3 * h
        c0, a = S.bdf_coefficients(t2 - t1, h)
        b = S.bdf2_history(u(t1), u(t0), a)
        u_new = (b + (t2 - t1) * du(t2)) / c0
        errs.append(np.abs(S.bdf2_error_estimate(
            u_new, S.leapfrog_predictor(u(t1), u(t0), du(t1), t2 - t1, a), a)))
    assert np.all(np.abs(errs[0] / errs[1] / 8 - 1) < 0.06)
    assert np.all(np.abs(errs[1] / errs[2] / 8 - 1) < 0.03)


def test_controllers_fixed_points_and_exponents():
    eps = 1e-4
    assert S.eps_step_factor(eps, eps) == 1.0
    assert np.isclose(S.eps_step_factor(eps, 8 * eps), 0.5)          # k = 3
    a = 1.3
    assert np.isclose(S.pc47_ratio(eps, eps, eps, a), a)
    # integral part alone (equal successive errors): exponent 0.4 / 3
    assert np.isclose(S.pc47_ratio(eps, 2 * eps, 2 * eps, a), a * 2 ** (-0.4 / 3))
    # proportional part alone (error at the target, halved since last step)
    assert np.isclose(S.pc47_ratio(eps, eps, 2 * eps, a), a * 2 ** (0.7 / 3))


def test_scaled_max_norm_ignores_covered_cells_and_scales_per_field():
    w = I.small_amr(8)
    s = system(w)
    u = state(s, w)
    n = s.nc
    e = np.zeros_like(u)
    cov = np.where(~s.composite[:n])[0]
    comp = np.where(s.composite[:n])[0]
    assert len(cov) > 0
    e[cov[0]] = 1e6                              # covered: must not count
    e[comp[3]] = 2.0 * (u[comp[3]] + 1e-5)       # E part: ratio 2
    e[n + comp[5]] = -3.0 * (u[n + comp[5]] + 0.1)   # T part: ratio 3
    assert np.isclose(S.scaled_max_norm(s, e, u, 1e-5, 0.1), 3.0)
    e[n + comp[5]] = 0.0
    assert np.isclose(S.scaled_max_norm(s, e, u, 1e-5, 0.1), 2.0)


def test_adaptive_steps_follow_the_tolerance():
    # a tighter tolerance takes more, smaller steps and ends closer to a
    # fine fixed-step BDF2 solution (an inverted or mis-scaled controller
    # fails this)
    w = I.marshak_single(8, state="front")
    s = system(w)
    u0 = state(s, w)
    t_end = 0.02
    ref = S.Stepper(s, u0, rtol=1e-10, atol=1e-14)
    for _ in range(800):
        assert ref.step(t_end / 800).converged
    errs, steps = [], []
    for eps in (2e-2, 5e-3, 1.25e-3):
        ad = S.AdaptiveStepper(s, u0, 1e-4, eps, 1e-5, 1e-5 ** 0.25, rtol=1e-10, atol=1e-14)
        while ad.t < t_end - 1e-15:
            ad.dt = min(ad.dt, t_end - ad.t)     # land on t_end
            ad.advance()
        errs.append(s.norm(ad.u - ref.u) / s.norm(ref.u))
        steps.append(len(ad.log))
    assert steps[0] < steps[1] < steps[2]
    assert errs[0] > errs[1] > errs[2]


def test_failed_step_is_retried_with_half_the_step():
    # far from equilibrium: the Newton solve at dt = 1e-2 stalls (see the
    # positivity tests); the adaptive stepper halves until one converges
    rng = np.random.default_rng(23)
    w = I.marshak_single(6)
    sh = w.boxes[0].shape
    w.E = [1e-4 * np.exp(rng.uniform(-2, 2, sh))]
    w.T = [np.exp(rng.uniform(-1, 1, sh))]
    s = system(w)
    u0 = state(s, w)
    assert not S.Stepper(s, u0, rtol=1e-10, atol=1e-16, maxit=24).step(1e-2).converged
    ad = S.AdaptiveStepper(s, u0, 1e-2, 1e-3, 1e-5, 0.05, rtol=1e-10, atol=1e-16, maxit=24)
    ad.advance()
    assert ad.log[0][0] < 1e-2
    assert np.all(ad.u[s.composite] > 0)
