"""Pins of the oracle's residual, Jacobian action and transpose.

Each test checks the oracle against something fixed by the paper or by
mathematics -- special cases, closed forms, identities, brute force -- not
against a retyped copy of its own formula.
"""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import operators as ops
from oracle.hierarchy import Hierarchy, HierarchyError
from oracle.solvers import System
from paper_1302_6303_amd import inputs as I
from tests.helpers import hierarchy, state, system


# ---------------------------------------------------------------------------
# face coefficient special cases (Sec. 3.1, 3.2)
# ---------------------------------------------------------------------------

def test_gradient_free_face_is_unlimited_diffusion():
    """dE = 0 on a face between equal materials: D_E = 1/(3 sigma(T_f))."""
    rng = np.random.default_rng(1)
    T = rng.uniform(0.05, 1.5, 50)
    z = rng.uniform(1.0, 10.0, 50)
    E = rng.uniform(1e-5, 4.0, 50)
    DE, DT = ops.face_coeffs(E, E, T, T, z**3, z**3, 0.1, 0.01)
    sigma = z**3 * T**-3
    np.testing.assert_allclose(DE, 1.0 / (3.0 * sigma), rtol=1e-14)
    np.testing.assert_allclose(DT, 0.01 * np.sqrt(T) ** 5, rtol=1e-14)


def test_wilson_form_on_uniform_material():
    """Equal z, equal T: D_E = 1/(3 sigma + |grad E| / E) with the face
    gradient |dE|/h and the face mean E (Sec. 3.1 Wilson limiter)."""
    rng = np.random.default_rng(2)
    Ea, Eb = rng.uniform(1e-5, 4.0, (2, 40))
    T = rng.uniform(0.05, 1.5, 40)
    z3 = rng.uniform(1.0, 1000.0, 40)
    h = 1.0 / 64
    DE, _ = ops.face_coeffs(Ea, Eb, T, T, z3, z3, h, 0.01, lam=1.0)
    grad_over_E = (np.abs(Eb - Ea) / h) / ((Ea + Eb) / 2)
    np.testing.assert_allclose(DE, 1.0 / (3.0 * z3 / T**3 + grad_over_E),
                               rtol=1e-13)


def test_literal_pair_with_half_limiter():
    """lam = 1/2 reproduces the printed pair D_r, 2 D_r / (1 + D_r g)."""
    rng = np.random.default_rng(3)
    Ea, Eb = rng.uniform(1e-5, 4.0, (2, 40))
    Ta, Tb = rng.uniform(0.05, 1.5, (2, 40))
    za, zb = rng.uniform(1.0, 10.0, (2, 40))
    h = 0.03
    DE, _ = ops.face_coeffs(Ea, Eb, Ta, Tb, za**3, zb**3, h, 0.01, lam=0.5)
    Tf = (Ta + Tb) / 2
    Dr = Tf**3 / (3 * (za**3 + zb**3))
    g = np.abs(Ea - Eb) / (0.5 * h * (Ea + Eb))
    np.testing.assert_allclose(DE, 2 * Dr / (1 + Dr * g), rtol=1e-13)


def test_robin_flux_solves_the_discrete_boundary_relation():
    """q is the flux D_b (E_g - E_c)/h of the ghost E_g that satisfies
    1/2 D_b (E_g - E_c)/h + (E_g + E_c)/8 = R (eq. robinbc), and q -> 2R - E/2
    as h -> 0."""
    rng = np.random.default_rng(4)
    for _ in range(20):
        Ec, R = rng.uniform(1e-5, 4.0), rng.uniform(0.0, 2.0)
        Tc, z = rng.uniform(0.05, 1.5), rng.uniform(1.0, 10.0)
        h = rng.uniform(1e-3, 0.1)
        Db = Tc**3 / (3 * z**3)
        # linear equation in E_g: (Db/(2h) + 1/8) E_g = R - Ec/8 + Db Ec/(2h)
        Eg = np.linalg.solve([[Db / (2 * h) + 0.125]], [R - Ec / 8 + Db * Ec / (2 * h)])[0]
        q = ops.robin_q(Ec, Tc, z**3, R, h)
        assert abs(q - Db * (Eg - Ec) / h) <= 1e-12 * (abs(q) + 1e-300) + 1e-15
    q0 = ops.robin_q(0.3, 1.0, 1.0, 1.0, 1e-12)
    assert abs(q0 - (2.0 - 0.15)) < 1e-9


# ---------------------------------------------------------------------------
# residual identities
# ---------------------------------------------------------------------------

def test_equilibrium_is_stationary():
    """E = T^4 uniform with u = b: F = 0; also with the Marshak face when
    E = 4R (no inflow)."""
    w = I.marshak_single(8)
    for bc, E0 in (((0,) * 6, 0.3), ((1, 0, 0, 0, 0, 0), 4.0)):
        s = system(w, bc_E=bc)
        T0 = E0 ** 0.25
        E = [np.full((8, 8, 8), E0)]
        T = [np.full((8, 8, 8), T0)]
        E[0][...] = T[0] ** 4
        u = s.join(E, T)
        F = s.residual(u, u, 1e-3, 1.0)
        assert np.max(np.abs(F)) < 1e-15


def test_textbook_laplacian_without_limiter():
    """lam = 0, z = 1, T constant: the E operator is the 7-point Neumann
    Laplacian with coefficient T^3/3 (scipy Kronecker sum)."""
    n = 6
    w = I.marshak_single(n, state="front")
    w.z = [np.ones((n, n, n))]
    s = system(w, lam=0.0, bc_E=(0,) * 6)
    rng = np.random.default_rng(5)
    E = rng.uniform(0.1, 2.0, (n, n, n))
    T = np.full((n, n, n), 0.7)
    u = s.join([E], [T])
    dt = 1e-2
    b = np.zeros_like(u)
    F = s.residual(u, b, dt, 1.0)
    h = 1.0 / n
    L1 = sp.diags([np.ones(n - 1), -np.r_[1, 2 * np.ones(n - 2), 1], np.ones(n - 1)],
                  [-1, 0, 1]) / h**2
    Id = sp.identity(n)
    L = (sp.kron(Id, sp.kron(Id, L1)) + sp.kron(Id, sp.kron(L1, Id))
         + sp.kron(L1, sp.kron(Id, Id)))
    D = 0.7**3 / 3.0
    e = E.ravel(order="F")
    S = (0.7**4 - e) / 0.7**3
    FE = e - dt * (D * (L @ e) + S)
    np.testing.assert_allclose(F[:n**3], FE, rtol=1e-12, atol=1e-14)


def energy_balance(s, u, b, dt, c0):
    """sum V (F_E + F_T) versus sum V (c0 (E+T) - b_E - b_T) - dt * boundary
    inflow: coupling cancels per cell and interior fluxes telescope."""
    F = s.residual(u, b, dt, c0)
    n = s.nc
    w = s.weight[:n]
    lhs = np.sum(w * (F[:n] + F[n:]))
    rhs = np.sum(w * (c0 * (u[:n] + u[n:]) - b[:n] - b[n:]))
    H = s.H
    E, T = s.split(u)
    inflow = 0.0
    for p in H.patches:
        h = H.h(p.level)
        for d in range(3):
            for side in (0, 1):
                if not (ops.is_physical(H, p, d, side) and H.bc_E[2 * d + side]):
                    continue
                k = 0 if side == 0 else int(p.n[d]) - 1
                q = ops.robin_q(np.take(E[p.pid], k, axis=d),
                                np.take(T[p.pid], k, axis=d),
                                np.take(s.z[p.pid], k, axis=d) ** 3,
                                H.robin_R[2 * d + side], h[d])
                cov = np.take(H.covered[p.pid], k, axis=d)
                inflow += np.sum(np.prod(h) / h[d] * q * ~cov)
    scale = np.sum(np.abs(w * F[:n])) + np.sum(np.abs(w * F[n:])) + abs(rhs)
    return lhs, rhs - dt * inflow, scale


@pytest.mark.parametrize("wname", ["uniform", "amr"])
def test_discrete_energy_identity(wname):
    if wname == "uniform":
        w = I.marshak_single(8, state="front")
    else:
        w = I.small_amr(8, state="front")
    s = system(w)
    u = state(s, w)
    rng = np.random.default_rng(6)
    b = u * rng.uniform(0.8, 1.2, u.shape)
    for dt, c0 in ((1e-3, 1.0), (5e-3, 4.0 / 3.0)):
        lhs, rhs, scale = energy_balance(s, u, b, dt, c0)
        assert abs(lhs - rhs) <= 1e-13 * max(scale, abs(rhs))


def test_energy_identity_fails_without_flux_matching(monkeypatch):
    """Planted mistake: dropping coarse-fine flux matching in the oracle
    breaks conservation on the refined hierarchy."""
    w = I.small_amr(8, state="front")
    s = system(w)
    u = state(s, w)
    b = 0.9 * u
    monkeypatch.setattr(ops, "cf_faces", lambda H, p, d: [])
    lhs, rhs, scale = energy_balance(s, u, b, 1e-3, 1.0)
    assert abs(lhs - rhs) > 1e-8 * max(scale, abs(rhs))


def test_mirror_symmetry_in_y():
    """A z field and state symmetric under y -> 1 - y give a mirrored
    residual (boundaries in y are symmetric)."""
    n = 8
    rng = np.random.default_rng(7)
    w = I.marshak_single(n, state="front")
    z = rng.choice([1.0, 10.0], size=(n, n // 2, n))
    w.z = [np.concatenate([z, z[:, ::-1, :]], axis=1)]
    E = rng.uniform(0.01, 3.0, (n, n // 2, n))
    T = rng.uniform(0.1, 1.2, (n, n // 2, n))
    E = np.concatenate([E, E[:, ::-1]], axis=1)
    T = np.concatenate([T, T[:, ::-1]], axis=1)
    s = system(w)
    u = s.join([E], [T])
    F = s.residual(u, 0.5 * u, 1e-3, 1.0)
    FE, FT = s.split(F)
    np.testing.assert_allclose(FE[0], FE[0][:, ::-1], rtol=1e-13, atol=1e-16)
    np.testing.assert_allclose(FT[0], FT[0][:, ::-1], rtol=1e-13, atol=1e-16)


def test_patch_decomposition_invariance():
    """Splitting level 0 into sibling patches changes no residual entry."""
    w = I.multi_patch_uniform(12, cuts=(4, 9))
    s = system(w)
    u = state(s, w)
    F = s.residual(u, 0.7 * u, 1e-3, 1.0)
    # same data on one patch
    E, T = s.split(u)
    Ew = np.concatenate(E, axis=0)
    Tw = np.concatenate(T, axis=0)
    zw = np.concatenate(w.z, axis=0)
    H1 = Hierarchy((12, 12, 12), [(0, (0, 0, 0), (12, 12, 12))])
    s1 = System(H1, [zw])
    u1 = s1.join([Ew], [Tw])
    F1 = s1.residual(u1, 0.7 * u1, 1e-3, 1.0)
    FE, FT = s.split(F)
    F1E, F1T = s1.split(F1)
    np.testing.assert_array_equal(np.concatenate(FE, axis=0), F1E[0])
    np.testing.assert_array_equal(np.concatenate(FT, axis=0), F1T[0])


# ---------------------------------------------------------------------------
# second-order consistency against the continuum (method of manufactured
# solutions); the discrete limiter uses the face-normal gradient, so the
# continuum flux is D_d dE/dx_d with D_d = 1/(3 sigma + |dE/dx_d| / E)
# ---------------------------------------------------------------------------

def _mms_fields(X):
    a, b, c, d = 1.0, 0.2, 0.6, 0.1
    cs = np.cos(np.pi * X[0]) + np.cos(np.pi * X[1]) + np.cos(np.pi * X[2])
    return a + b * cs, c + d * cs


def _continuum_f(X, kappa=0.01, zc=1.3):
    """f(u) of the PDE at points X, flux derivatives by a tiny central
    difference of the analytic flux (error ~1e-10, far below h^2)."""
    E, T = _mms_fields(X)
    fE = np.zeros_like(E)
    fT = np.zeros_like(E)
    dlt = 1e-5
    for d in range(3):
        def fluxes(Y):
            Ey, Ty = _mms_fields(Y)
            b, dd = 0.2, 0.1
            dEd = -b * np.pi * np.sin(np.pi * Y[d])
            dTd = -dd * np.pi * np.sin(np.pi * Y[d])
            sig = zc**3 / Ty**3
            DE = 1.0 / (3.0 * sig + np.abs(dEd) / Ey)
            return DE * dEd, kappa * Ty**2.5 * dTd
        Xp = list(X)
        Xm = list(X)
        Xp[d] = X[d] + dlt
        Xm[d] = X[d] - dlt
        p, m = fluxes(Xp), fluxes(Xm)
        fE += (p[0] - m[0]) / (2 * dlt)
        fT += (p[1] - m[1]) / (2 * dlt)
    S = zc**3 / T**3 * (T**4 - E)
    return fE + S, fT - S


def _mms_error(s, H):
    zc = 1.3
    X = []
    for p in H.patches:
        h = H.h(p.level)
        ax = [(np.arange(p.lo[d], p.hi[d]) + 0.5) * h[d] for d in range(3)]
        X.append(np.meshgrid(*ax, indexing="ij"))
    E = [_mms_fields(x)[0] for x in X]
    T = [_mms_fields(x)[1] for x in X]
    u = s.join(E, T)
    # F with c0 = 0, b = 0, dt = -1 gives f_h(u)
    F = s.residual(u, np.zeros_like(u), -1.0, 0.0)
    fx = [_continuum_f(x, zc=zc) for x in X]
    ex = s.join([f[0] for f in fx], [f[1] for f in fx])
    err = (F - ex) * s.composite
    return np.sqrt(s.dot(err, err))


def test_mms_second_order():
    errs = []
    for n in (8, 16, 32):
        H = Hierarchy((n, n, n), [(0, (0, 0, 0), (n, n, n))], bc_E=(0,) * 6)
        s = System(H, [np.full((n, n, n), 1.3)], lam=1.0)     # the continuum flux above
        errs.append(_mms_error(s, H))
    rates = [np.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert min(rates) > 1.8, (errs, rates)


def test_amr_residual_exact_for_linear_fields():
    """Limiter off, z and T constant: a linear E has constant flux density
    everywhere, so after coarse-fine interpolation and flux matching every
    composite cell away from the physical boundary has zero divergence."""
    w = I.small_amr(8, state="front")
    s = system(w, lam=0.0, bc_E=(0,) * 6)
    H = s.H
    s.z = [np.ones(tuple(int(v) for v in p.n)) for p in H.patches]
    a = np.array([0.3, -0.7, 1.1])
    E, T = [], []
    for p in H.patches:
        h = H.h(p.level)
        ax = [(np.arange(p.lo[d], p.hi[d]) + 0.5) * h[d] for d in range(3)]
        X = np.meshgrid(*ax, indexing="ij")
        E.append(5.0 + a[0] * X[0] + a[1] * X[1] + a[2] * X[2])
        T.append(np.full(X[0].shape, 0.8))
    u = s.join(E, T)
    F = s.residual(u, np.zeros_like(u), -1.0, 0.0)      # = f_h(u)
    FE, _ = s.split(F)
    S = [(0.8**4 - e) / 0.8**3 for e in E]
    checked = 0
    for p in H.patches:
        h0 = H.h(0)
        N = H.N(p.level)
        I_ = [np.arange(p.lo[d], p.hi[d]) for d in range(3)]
        X = np.meshgrid(*I_, indexing="ij")
        r = 2 ** p.level
        away = np.ones(X[0].shape, dtype=bool)
        for d in range(3):
            away &= (X[d] >= 2 * r) & (X[d] < N[d] - 2 * r)
        m = away & ~H.covered[p.pid]
        np.testing.assert_allclose(FE[p.pid][m], S[p.pid][m], rtol=1e-12,
                                   atol=1e-12)
        checked += m.sum()
    assert checked > 100


def test_mms_detects_the_literal_factor():
    """With lam = 1/2 the discrete operator converges to a different
    continuum flux, so the Wilson-form MMS stalls."""
    errs = []
    for n in (8, 16, 32):
        H = Hierarchy((n, n, n), [(0, (0, 0, 0), (n, n, n))], bc_E=(0,) * 6)
        s = System(H, [np.full((n, n, n), 1.3)], lam=0.5)
        errs.append(_mms_error(s, H))
    assert np.log2(errs[1] / errs[2]) < 1.0


# ---------------------------------------------------------------------------
# coarse-fine interpolation
# ---------------------------------------------------------------------------

def test_coarse_fine_ghosts_exact_for_linear_fields():
    w = I.small_amr(8, state="front")
    H = hierarchy(w)
    a = np.array([0.3, -0.7, 1.1])

    def lin(p):
        h = H.h(p.level)
        ax = [(np.arange(p.lo[d] - 1, p.hi[d] + 1) + 0.5) * h[d] for d in range(3)]
        X = np.meshgrid(*ax, indexing="ij")
        return 2.0 + a[0] * X[0] + a[1] * X[1] + a[2] * X[2]

    f = [lin(p)[1:-1, 1:-1, 1:-1] for p in H.patches]
    g = H.from_interior(f)
    H.sync([g])
    H.fill_ghosts([g])
    checked = 0
    for p in H.patches:
        if p.level == 0:
            continue
        ex = lin(p)
        for d in range(3):
            for side in range(2):
                G, gl, il, kind = H.ghost_kinds(p, d, side)
                # away from the domain edge the interpolation is exact
                N = H.N(p.level - 1)
                P = G // 2
                inner = np.all((P >= 1) & (P <= N - 2), axis=1)
                m = (kind == 2) & inner
                got = g[p.pid][gl[m, 0], gl[m, 1], gl[m, 2]]
                np.testing.assert_allclose(got, ex[gl[m, 0], gl[m, 1], gl[m, 2]],
                                           rtol=1e-13)
                checked += m.sum()
    assert checked > 50


def test_nesting_violations_are_rejected():
    with pytest.raises(HierarchyError):
        Hierarchy((8, 8, 8), [(0, (0, 0, 0), (8, 8, 8)), (1, (0, 0, 0), (4, 4, 4)),
                              (1, (2, 2, 2), (6, 6, 6))])          # overlap
    with pytest.raises(HierarchyError):
        Hierarchy((8, 8, 8), [(0, (0, 0, 0), (8, 8, 8)), (1, (1, 2, 2), (5, 6, 6))])  # odd
    with pytest.raises(HierarchyError):
        Hierarchy((8, 8, 8), [(0, (0, 0, 0), (8, 8, 8)), (1, (2, 2, 2), (6, 6, 6)),
                              (2, (4, 4, 4), (10, 10, 10))])       # not nested by 1


# ---------------------------------------------------------------------------
# Jacobian action and transpose
# ---------------------------------------------------------------------------

def _fd_jacobian(s, u, b, dt, c0, cols):
    out = []
    for j in cols:
        hstep = 1e-6 * max(1.0, abs(u[j]))
        e = np.zeros_like(u)
        e[j] = hstep
        out.append((s.residual(u + e, b, dt, c0) - s.residual(u - e, b, dt, c0))
                   / (2 * hstep))
    return np.array(out).T


@pytest.mark.parametrize("amr", [False, True])
def test_jvp_matches_bruteforce_fd_jacobian(amr):
    if amr:
        H = Hierarchy((4, 4, 4), [(0, (0, 0, 0), (4, 4, 4)), (1, (2, 2, 2), (6, 6, 6))])
    else:
        H = Hierarchy((4, 4, 4), [(0, (0, 0, 0), (4, 4, 4))])
    rng = np.random.default_rng(8)
    z = [rng.choice([1.0, 10.0], tuple(int(v) for v in p.n)) for p in H.patches]
    s = System(H, z)
    nc = s.nc
    u = s.sync(np.concatenate([rng.uniform(0.05, 3.0, nc), rng.uniform(0.2, 1.2, nc)]))
    b = u * 0.9
    dt, c0 = 2e-3, 1.5
    cols = np.nonzero(s.composite)[0]
    Jfd = _fd_jacobian(s, u, b, dt, c0, cols)
    Jan = np.array([s.jvp(u, np.eye(1, 2 * nc, j)[0], dt, c0) for j in cols]).T
    rows = s.composite
    err = np.abs(Jfd[rows] - Jan[rows]).max() / np.abs(Jan[rows]).max()
    assert err < 1e-6


def test_jvp_taylor_remainder_is_second_order():
    w = I.marshak_single(8, state="front")
    s = system(w)
    u = state(s, w)
    b = 0.8 * u
    rng = np.random.default_rng(9)
    v = rng.standard_normal(u.shape) * u
    F0 = s.residual(u, b, 1e-3, 1.0)
    Jv = s.jvp(u, v, 1e-3, 1.0)
    r = []
    for eps in (1e-2, 5e-3, 2.5e-3):
        r.append(np.linalg.norm(s.residual(u + eps * v, b, 1e-3, 1.0) - F0 - eps * Jv))
    assert 3.5 < r[0] / r[1] < 4.5 and 3.5 < r[1] / r[2] < 4.5


@pytest.mark.parametrize("wname", ["single", "siblings", "amr2", "amr3"])
def test_vjp_dot_product_identity(wname):
    """<l, J v> = <J^T l, v>: on refined hierarchies the transpose runs the
    coarse-fine interpolation, flux matching and restriction backwards."""
    w = {"single": lambda: I.marshak_single(8, state="front"),
         "siblings": lambda: I.multi_patch_uniform(10, cuts=(3, 7)),
         "amr2": lambda: I.small_amr(8, state="front"),
         "amr3": lambda: I.static_amr(base=8, nlevels=3, side=(8, 16), state="front")}[wname]()
    s = system(w)
    u = state(s, w)
    rng = np.random.default_rng(10)
    for _ in range(3):
        v = rng.standard_normal(u.shape)
        l = rng.standard_normal(u.shape)
        Jv = s.jvp(u, v, 1e-3, 1.0)
        JTl, _ = s.vjp(u, l, 1e-3, 1.0)
        a, b = np.dot(l, Jv), np.dot(JTl, v)
        assert abs(a - b) <= 1e-13 * (np.abs(l) @ np.abs(Jv))


@pytest.mark.parametrize("wname", ["single", "amr2"])
def test_vjp_z_derivative_matches_fd(wname):
    """l^T dF/dz against central differences of l^T F in z, every level's
    z (covered cells included: their z feeds coarse-fine ghosts)."""
    w = (I.marshak_single(6, state="front") if wname == "single"
         else I.small_amr(6, state="front", boxes_spec=[(1, (2, 2, 2), (10, 8, 10))]))
    s = system(w)
    u = state(s, w)
    b = 0.9 * u
    rng = np.random.default_rng(11)
    l = rng.standard_normal(u.shape)
    _, gz = s.vjp(u, l, 1e-3, 1.0)
    z0 = [a.copy() for a in s.z]
    flat = np.concatenate([a.ravel(order="F") for a in z0])
    for c in rng.choice(flat.size, 16, replace=False):
        hz = 1e-6 * flat[c]
        vals = []
        for sg in (1, -1):
            zz = flat.copy()
            zz[c] += sg * hz
            out, o = [], 0
            for a in z0:
                out.append(zz[o:o + a.size].reshape(a.shape, order="F"))
                o += a.size
            s.z = out
            vals.append(np.dot(l, s.residual(u, b, 1e-3, 1.0)))
        s.z = z0
        fd = (vals[0] - vals[1]) / (2 * hz)
        assert abs(fd - gz[c]) <= 1e-6 * abs(gz[c]) + 1e-8 * np.abs(gz).max(), (c, fd, gz[c])


# ---------------------------------------------------------------------------
# Jacobian-free product (Sec. 4.1)
# ---------------------------------------------------------------------------

def test_fd_epsilon_special_cases():
    """v = u gives <u,v>/||v||^2 = 1, so eps = sqrt(eps_mach); v = -u flips
    the sign; a v orthogonal to u takes the u_min branch; v = 0 gives 1."""
    w = I.static_amr(base=8, nlevels=2, side=(4, 8), state="front")
    s = system(w)
    u = state(s, w)
    E, T = s.split(u)
    root = np.sqrt(np.finfo(np.float64).eps)
    assert ops.fd_epsilon(s.H, E, T, E, T) == pytest.approx(root, rel=1e-15)
    mE, mT = s.split(-u)
    assert ops.fd_epsilon(s.H, E, T, mE, mT) == pytest.approx(-root, rel=1e-15)
    rng = np.random.default_rng(12)
    keep = s.composite
    v = rng.standard_normal(u.shape) * keep
    v -= (np.dot(u[keep], v[keep]) / np.dot(u[keep], u[keep])) * u * keep
    vE, vT = s.split(v)
    l1, v2 = np.abs(v[keep]).sum(), (v[keep] ** 2).sum()
    eps = ops.fd_epsilon(s.H, E, T, vE, vT)
    assert abs(eps) == pytest.approx(root * 1e-6 * l1 / v2, rel=1e-12)
    zE, zT = s.split(0.0 * u)
    assert ops.fd_epsilon(s.H, E, T, zE, zT) == 1.0


@pytest.mark.parametrize("amr", [False, True])
def test_fd_jvp_agrees_with_analytic(amr):
    """The Jacobian-free product approximates the analytic one (itself
    pinned by brute force) to ~sqrt(eps_mach) for normalised v."""
    w = I.static_amr(base=8, nlevels=2, side=(4, 8), state="front") if amr else \
        I.marshak_single(8, state="front")
    s = system(w)
    s_fd = system(w)
    s_fd.jvp_mode = "fd"
    u = state(s, w)
    b = 0.9 * u
    rng = np.random.default_rng(13)
    s_fd.residual(u, b, 1e-3, 1.0)
    for _ in range(3):
        v = s.sync(rng.standard_normal(u.shape) * u)
        v /= s.norm(v)
        Ja = s.jvp(u, v, 1e-3, 1.0)
        Jf = s_fd.jvp(u, v, 1e-3, 1.0)
        assert np.linalg.norm(Jf - Ja) <= 1e-6 * np.linalg.norm(Ja)
