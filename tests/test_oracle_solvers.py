"""Pins of the oracle's preconditioner, Krylov, Newton, BDF and adjoint."""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import direct, precond as pc
from oracle.hierarchy import Hierarchy
from oracle.solvers import Stepper, System, adjoint_gradient, fgmres, newton
from paper_1302_6303_amd import inputs as I
from tests.helpers import hierarchy, state, system


def test_p2_closed_form_matches_dense_solve():
    rng = np.random.default_rng(20)
    T = rng.uniform(0.05, 1.5, 30)
    z3 = rng.uniform(1.0, 1000.0, 30)
    eE, eT = rng.standard_normal((2, 30))
    for mode in ("paper", "frozen4"):
        beta = 3e-4
        yE, yT = pc.p2_solve(T, z3, beta, eE, eT, mode)
        tE, tT = pc.p2_solve_transpose(T, z3, beta, eE, eT, mode)
        k = 4.0 if mode == "frozen4" else 1.0
        for c in range(30):
            sig = z3[c] / T[c] ** 3
            M = np.array([[1 + sig * beta, -k * sig * beta * T[c] ** 3],
                          [-sig * beta, 1 + k * sig * beta * T[c] ** 3]])
            np.testing.assert_allclose([yE[c], yT[c]],
                                       np.linalg.solve(M, [eE[c], eT[c]]), rtol=1e-12)
            np.testing.assert_allclose([tE[c], tT[c]],
                                       np.linalg.solve(M.T, [eE[c], eT[c]]), rtol=1e-12)


def _mg_grid_from_state(n, lam=1.0, bc=(1, 0, 0, 0, 0, 0), const=False, beta=1e-2):
    H = Hierarchy((n, n, n), [(0, (0, 0, 0), (n, n, n))], bc_E=bc)
    rng = np.random.default_rng(21)
    if const:
        E = [np.full((n, n, n), 0.5)]
        T = [np.full((n, n, n), 0.7)]
        z = [np.ones((n, n, n))]
    else:
        E = [rng.uniform(0.01, 3.0, (n, n, n))]
        T = [rng.uniform(0.2, 1.2, (n, n, n))]
        z = [rng.choice([1.0, 10.0], (n, n, n))]
    snap = pc.Snapshot(H, E, T, z, beta, lam)
    return H, snap


def _dense_from_apply(apply, shape):
    N = int(np.prod(shape))
    A = np.zeros((N, N))
    for j in range(N):
        e = np.zeros(N)
        e[j] = 1.0
        A[:, j] = apply(e.reshape(shape, order="F")).ravel(order="F")
    return A


def test_level_operator_is_symmetric_and_textbook_for_constant_D():
    n = 5
    H, snap = _mg_grid_from_state(n, lam=0.0, bc=(0,) * 6, const=True, beta=1e-2)
    for f in (0, 1):
        g = pc.build_mg(H, snap, f)[0]
        w, diag = g.weights(snap.beta)
        A = _dense_from_apply(lambda e: pc.mg_apply_op(w, diag, e), (n,) * 3)
        np.testing.assert_allclose(A, A.T, atol=1e-15)
        D = 0.7**3 / 3.0 if f == 0 else 0.01 * 0.7**2.5
        h = 1.0 / n
        L1 = sp.diags([np.ones(n - 1), -np.r_[1, 2 * np.ones(n - 2), 1], np.ones(n - 1)],
                      [-1, 0, 1]) / h**2
        Id = sp.identity(n)
        L = (sp.kron(Id, sp.kron(Id, L1)) + sp.kron(Id, sp.kron(L1, Id))
             + sp.kron(L1, sp.kron(Id, Id)))
        ref = np.eye(n**3) - snap.beta * D * L.toarray()
        np.testing.assert_allclose(A, ref, rtol=1e-12, atol=1e-14)


def test_level_operator_matches_composite_operator_on_one_level():
    """On a single-level grid the level operator and A^c coincide (Marshak
    face included)."""
    n = 6
    H, snap = _mg_grid_from_state(n)
    g = pc.build_mg(H, snap, 0)[0]
    w, diag = g.weights(snap.beta)
    rng = np.random.default_rng(22)
    e = rng.standard_normal((n, n, n))
    a = pc.mg_apply_op(w, diag, e)
    b = pc.composite_apply(H, snap, 0, [e])[0]
    np.testing.assert_allclose(a, b, rtol=1e-12, atol=1e-14)


def test_jacobi_sweep_is_the_textbook_damped_update():
    """One damped point Jacobi sweep on a single-level grid is
    e + omega D^-1 (f - A e) with A assembled column by column from the
    composite operator and D its diagonal (Marshak face included)."""
    n = 5
    H, snap = _mg_grid_from_state(n)
    p = H.by_level[0][0]
    rng = np.random.default_rng(41)
    for f in (0, 1):
        A = _dense_from_apply(lambda x: pc.composite_apply(H, snap, f, [x])[0], (n,) * 3)
        e0 = rng.standard_normal((n, n, n))
        rhs = rng.standard_normal((n, n, n))
        e = H.empty()
        e[p.pid][...] = 0.0                   # physical ghosts: weight 0
        e[p.pid][1:-1, 1:-1, 1:-1] = e0
        pc.jacobi_level(H, snap, f, 0, {p.pid: rhs}, e)
        x = e0.ravel(order="F")
        ref = x + pc.JACOBI_OMEGA * (rhs.ravel(order="F") - A @ x) / np.diag(A)
        np.testing.assert_allclose(e[p.pid][1:-1, 1:-1, 1:-1].ravel(order="F"), ref,
                                   rtol=1e-12, atol=1e-13)


def test_bottom_grid_is_an_exact_solve():
    n = 5                                     # cannot coarsen: bottom = grid
    H, snap = _mg_grid_from_state(n)
    grids = pc.build_mg(H, snap, 0)
    assert len(grids) == 1
    w, diag = grids[0].weights(snap.beta)
    f = np.random.default_rng(23).standard_normal((n, n, n))
    e = pc.mg_vcycle(grids, snap.beta, f)
    np.testing.assert_allclose(pc.mg_apply_op(w, diag, e), f, rtol=1e-11, atol=1e-12)


def _mg_contraction(n, beta):
    H, snap = _mg_grid_from_state(n, lam=0.0, bc=(0,) * 6, const=True, beta=beta)
    grids = pc.build_mg(H, snap, 1)
    w, diag = grids[0].weights(beta)
    rng = np.random.default_rng(24)
    f = rng.standard_normal((n, n, n))
    e = np.zeros_like(f)
    norms = []
    for _ in range(6):
        r = f - pc.mg_apply_op(w, diag, e)
        norms.append(np.linalg.norm(r))
        e = e + pc.mg_vcycle(grids, beta, r)
    return (norms[-1] / norms[1]) ** (1 / 4)


def test_multigrid_contraction_is_h_independent():
    # beta * D / h^2 >> 1: diffusion dominated
    rho16 = _mg_contraction(16, 50.0)
    rho32 = _mg_contraction(32, 50.0)
    assert rho16 < 0.3 and rho32 < 0.3
    assert abs(rho32 - rho16) < 0.15


def test_fac_stationary_iteration_converges_on_two_levels():
    """Smooth coefficients (one material, noise-free front): FAC V(1,0) as
    a stationary iteration on A^c u = f contracts well below 1."""
    w = I.small_amr(8, state="uniform")
    rng0 = np.random.default_rng(250)
    w.E, w.T = I.front_state(w.problems, w.boxes, rng0, noise=0.0)
    s = system(w)
    H = s.H
    s.z = [np.ones(tuple(int(v) for v in p.n)) for p in H.patches]
    u = state(s, w)
    E, T = s.split(u)
    snap = pc.Snapshot(H, E, T, s.z, 5e-2)
    rng = np.random.default_rng(25)
    for f in (0, 1):
        rhs = [rng.standard_normal(tuple(int(v) for v in p.n)) for p in H.patches]
        x = [np.zeros_like(r) for r in rhs]
        norms = []
        for _ in range(6):
            Ax = pc.composite_apply(H, snap, f, x)
            r = [rhs[q] - Ax[q] for q in range(len(rhs))]
            norms.append(np.sqrt(sum(np.sum(rr[~H.covered[q]] ** 2)
                                     for q, rr in enumerate(r))))
            c = pc.fac_vcycle(H, snap, f, r)
            x = [x[q] + c[q] for q in range(len(x))]
        rate = (norms[-1] / norms[1]) ** (1 / 4)
        assert rate < 0.5, (f, norms)


def _fac_contraction(w, nus, iters=6):
    """Per field, the contraction rate of FAC V(m, n) used as a stationary
    iteration on A^c x = rhs (smooth single-material coefficients)."""
    rng0 = np.random.default_rng(250)
    w.E, w.T = I.front_state(w.problems, w.boxes, rng0, noise=0.0)
    s = system(w)
    H = s.H
    s.z = [np.ones(tuple(int(v) for v in p.n)) for p in H.patches]
    E, T = s.split(state(s, w))
    snap = pc.Snapshot(H, E, T, s.z, 5e-2)
    out = {}
    for nu in nus:
        rng = np.random.default_rng(25)
        rates = []
        for f in (0, 1):
            rhs = [rng.standard_normal(tuple(int(v) for v in p.n)) for p in H.patches]
            x = [np.zeros_like(r) for r in rhs]
            norms = []
            for _ in range(iters):
                Ax = pc.composite_apply(H, snap, f, x)
                r = [rhs[q] - Ax[q] for q in range(len(rhs))]
                norms.append(np.sqrt(sum(np.sum(rr[~H.covered[q]] ** 2)
                                         for q, rr in enumerate(r))))
                c = pc.fac_vcycle(H, snap, f, r, nu=nu)
                x = [x[q] + c[q] for q in range(len(x))]
            rates.append((norms[-1] / norms[1]) ** (1 / (iters - 2)))
        out[nu] = rates
    return out


def test_fac_more_smoothing_contracts_faster():
    """Alg. 1 with m > 1 down-sweep sweeps or n > 0 up-sweep sweeps (on the
    refreshed composite residual) is a better stationary iteration than
    V(1,0) for both diffusion blocks.  An up-sweep that re-solves the first
    residual instead of the refreshed one diverges here (rate > 1)."""
    r = _fac_contraction(I.small_amr(8, state="uniform"), [(1, 0), (2, 0), (1, 1), (2, 1)])
    for f in (0, 1):
        for nu in ((2, 0), (1, 1), (2, 1)):
            assert r[nu][f] < 0.7 * r[(1, 0)][f], (nu, f, r)
    assert r[(2, 1)][0] < 0.25 and r[(2, 1)][1] < 0.05, r


def test_fac_with_jacobi_smoothing_converges():
    """FAC with the damped point Jacobi level smoother (Sec. 4.3) is a
    convergent stationary iteration, and more sweeps make it faster."""
    w = I.small_amr(8, state="uniform")
    orig = pc.Snapshot.__init__

    def jacobi_init(self, *a, **k):
        orig(self, *a, **k)
        self.fac_smoother = "jacobi"
    pc.Snapshot.__init__ = jacobi_init
    try:
        r = _fac_contraction(w, [(1, 0), (2, 1)])
    finally:
        pc.Snapshot.__init__ = orig
    for f in (0, 1):
        assert r[(1, 0)][f] < 0.7 and r[(2, 1)][f] < 0.7 * r[(1, 0)][f], r


def test_fac_base_smoothing_is_weaker_than_the_base_vcycle():
    """Sec. 4.3: the paper's runs only smooth on the coarsest level.  As a
    stationary iteration that still converges on two levels, but more
    slowly than with the multigrid V-cycle on the base level."""
    w = I.small_amr(8, state="uniform")
    rv = _fac_contraction(w, [(1, 0)])
    orig = pc.Snapshot.__init__

    def smooth_init(self, *a, **k):
        orig(self, *a, **k)
        self.fac_base = "smooth"
    pc.Snapshot.__init__ = smooth_init
    try:
        rs = _fac_contraction(I.small_amr(8, state="uniform"), [(1, 0)])
    finally:
        pc.Snapshot.__init__ = orig
    for f in (0, 1):
        assert rv[(1, 0)][f] < rs[(1, 0)][f] < 1.0, (rv, rs)


def test_fac_vmn_on_one_level_is_the_base_vcycle():
    """With a single level there are no levels above the base: V(m, n) of
    FAC is one base multigrid V-cycle whatever m and n."""
    w = I.marshak_single(8, state="front")
    s = system(w)
    H = s.H
    E, T = s.split(state(s, w))
    snap = pc.Snapshot(H, E, T, s.z, 3e-3)
    rng = np.random.default_rng(31)
    rhs = [rng.standard_normal(tuple(int(v) for v in p.n)) for p in H.patches]
    for f in (0, 1):
        a = pc.fac_vcycle(H, snap, f, rhs, nu=(1, 0))
        b = pc.fac_vcycle(H, snap, f, rhs, nu=(3, 2))
        for x, y in zip(a, b):
            np.testing.assert_array_equal(x, y)


def test_fgmres_newton_step_matches_sparse_direct():
    w = I.marshak_single(4, state="front")
    s = system(w)
    u = state(s, w)
    b = 0.9 * u
    dt, c0 = 1e-2, 1.0
    J = direct.assemble_jacobian(s, u, dt, c0)
    F = s.residual(u, b, dt, c0)
    ref = spla.spsolve(J.tocsc(), -F)
    P, _ = s.precond(u, dt / c0)
    x, its, est = fgmres(lambda v: s.jvp(u, v, dt, c0), P, -F, 1e-13 * s.norm(F),
                         s.dot, m=30, max_restarts=10)
    np.testing.assert_allclose(x, ref, rtol=1e-9, atol=1e-12 * np.abs(ref).max())
    # unpreconditioned with a restart length that forces restarts
    x2, its2, _ = fgmres(lambda v: s.jvp(u, v, dt, c0), lambda v: v, -F,
                         1e-12 * s.norm(F), s.dot, m=5, max_restarts=200)
    np.testing.assert_allclose(x2, ref, rtol=1e-7, atol=1e-10 * np.abs(ref).max())


def test_newton_lands_on_the_exact_discrete_solution():
    w = I.marshak_single(8, state="front")
    s = system(w)
    u0 = state(s, w)
    dt = 2e-3
    ustar = direct.solve_exact(s, u0, u0, dt, 1.0)
    res = newton(s, u0, u0, dt, 1.0, dt, rtol=1e-10, atol=1e-16)
    assert res.converged
    for a, b in zip(s.split(res.u), s.split(ustar)):
        num = np.sqrt(sum(np.sum((x - y) ** 2) for x, y in zip(a, b)))
        den = np.sqrt(sum(np.sum(y ** 2) for y in b))
        assert num / den < 1e-8


def test_converged_step_balances_energy():
    w = I.marshak_single(8)
    s = system(w)
    st = Stepper(s, state(s, w), rtol=1e-12, atol=1e-18)
    u_old = st.u.copy()
    dt = 1e-3
    r = st.step(dt)
    assert r.converged
    n = s.nc
    wgt = s.weight[:n]
    dE = np.sum(wgt * (st.u[:n] + st.u[n:] - u_old[:n] - u_old[n:]))
    # inflow through the x = 0 Marshak face at the new state
    H = s.H
    E, T = s.split(st.u)
    from oracle import operators as ops
    h = H.h(0)
    q = ops.robin_q(E[0][0], T[0][0], s.z[0][0] ** 3, 1.0, h[0])
    inflow = dt * np.sum(q) * h[1] * h[2]
    assert abs(dE - inflow) <= 1e-9 * abs(inflow)


def test_bdf2_is_second_order_in_time():
    rng = np.random.default_rng(26)
    w = I.marshak_single(6)
    E, T = I.front_state(w.problems, w.boxes, rng, noise=0.0, xf=0.4, width=0.1)
    s = system(w)
    u0 = s.sync(s.join(E, T))
    t_end = 0.016

    def run(dt):
        st = Stepper(s, u0, rtol=1e-10, atol=1e-13)
        for _ in range(int(round(t_end / dt))):
            assert st.step(dt).converged
        return st.u

    ref = run(t_end / 128)
    errs = [np.linalg.norm(run(t_end / k) - ref) for k in (4, 8, 16)]
    rates = [np.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert min(rates) > 1.7, (errs, rates)


def test_predictor_is_the_leapfrog_extrapolation():
    """For a quadratic-in-time history the generalised leapfrog predictor is
    exact (eq. leapfrog), given the BDF2 time derivative at t_n."""
    w = I.marshak_single(4)
    s = system(w)
    u0 = state(s, w)
    st = Stepper(s, u0)
    a, b2, c = 1.0, 0.3, -0.2      # u(t) = u0 * (a + b t + c t^2)
    t = [0.0, 0.1, 0.25]
    dts = [0.1, 0.15]
    u_of = lambda tt: u0 * (a + b2 * tt + c * tt * tt)
    st.u_prev = u_of(t[0])
    st.u = u_of(t[1])
    st.dt_prev = dts[0]
    # BDF2 time derivative at t_n for a quadratic is exact: (c0 u_n - b)/dt
    st.udot = u0 * (b2 + 2 * c * t[1])
    _, _, _, guess, _ = st.rhs_and_guess(dts[1])
    np.testing.assert_allclose(guess, s.sync(u_of(t[2])), rtol=1e-12)


def test_adjoint_gradient_matches_central_fd():
    n = 6
    z = 1.0 + 9.0 * np.clip(0.5 + 0.35 * np.random.default_rng(27).standard_normal((n, n, n)), 0, 1)
    H = Hierarchy((n, n, n), [(0, (0, 0, 0), (n, n, n))])
    s = System(H, [z])
    w = I.marshak_single(n)
    u0 = s.join(w.E, w.T)
    kw = dict(rtol=1e-11, atol=1e-30, maxit=40)
    dt, N = 2e-3, 3
    g, _ = adjoint_gradient(s, u0, dt, N, tol=1e-13, newton_kw=kw)

    def J(zz):
        s.z = [zz]
        st = Stepper(s, u0, bdf1_only=True, **kw)
        for _ in range(N):
            assert st.step(dt).converged
        return np.sum(st.u[:s.nc])

    order = np.argsort(-np.abs(g))
    for c in order[:4]:
        hz = 1e-3 * z.ravel(order="F")[c]
        zp = z.copy().ravel(order="F")
        zm = zp.copy()
        zp[c] += hz
        zm[c] -= hz
        fd = (J(zp.reshape(z.shape, order="F")) - J(zm.reshape(z.shape, order="F"))) / (2 * hz)
        assert abs(fd - g[c]) <= 1e-5 * abs(g[c]), (c, fd, g[c])
    s.z = [z]


def test_adjoint_gradient_on_two_levels_matches_central_fd():
    """The same on a refined hierarchy: J sums E over the composite cells;
    z of both levels is perturbed, the covered coarse cells' z included
    (it reaches the fine cells through the coarse-fine ghosts)."""
    w = I.small_amr(6, boxes_spec=[(1, (2, 2, 2), (10, 8, 10))])
    H = Hierarchy((6, 6, 6), [(b.level, b.lo, b.hi) for b in w.boxes])
    s = System(H, w.z)
    u0 = s.join(w.E, w.T)
    kw = dict(rtol=1e-11, atol=1e-30, maxit=40)
    dt, N = 2e-3, 2
    g, _ = adjoint_gradient(s, u0, dt, N, tol=1e-13, newton_kw=kw)
    z0 = [a.copy() for a in s.z]
    flat = np.concatenate([a.ravel(order="F") for a in z0])

    def J(zz):
        out, o = [], 0
        for a in z0:
            out.append(zz[o:o + a.size].reshape(a.shape, order="F"))
            o += a.size
        s.z = out
        st = Stepper(s, u0, bdf1_only=True, **kw)
        for _ in range(N):
            assert st.step(dt).converged
        return np.sum(st.u[:s.nc][s.composite[:s.nc]])

    cov0 = H.covered[0].ravel(order="F")
    order = list(np.argsort(-np.abs(g))[:1])
    order.append(int(np.argmax(np.where(cov0, np.abs(g[:cov0.size]), -1.0))))  # a covered cell
    order.append(cov0.size + int(np.argmax(np.abs(g[cov0.size:]))))           # a fine cell
    for c in order:
        hz = 1e-3 * flat[c]
        zp = flat.copy()
        zm = flat.copy()
        zp[c] += hz
        zm[c] -= hz
        fd = (J(zp) - J(zm)) / (2 * hz)
        assert abs(fd - g[c]) <= 1e-5 * abs(g[c]), (c, fd, g[c])
    s.z = z0
