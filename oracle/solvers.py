"""Krylov, Newton, time stepping and the discrete adjoint (paper Sec. 3.3-4.1).

* Right-preconditioned GMRES on the Newton equations (Sec. 4.1-4.2), run as
  flexible GMRES(m) -- it stores z_j = P^-1 v_j, which is the same method for
  a fixed preconditioner -- with two passes of classical Gram-Schmidt and
  Givens rotations; x0 = 0; stop when the least-squares residual estimate is
  at most eta ||F|| (eq. inexactNewtoneqns).
* Inexact Newton with Eisenstat-Walker forcing terms (Sec. 4.1).  Reading:
  the book the paper points to is not available; the forcing sequence used
  is eta_0 = 0.9, eta_k = max(min(eta_max, gamma r^2 [safeguarded by
  gamma eta_{k-1}^2 when that exceeds 0.1]), 0.5 tau / ||F_k||) with
  gamma = 0.9, eta_max = 0.9, r = ||F_k|| / ||F_{k-1}||, tau the stopping
  threshold.
* Positivity: the step length is halved until E and T stay positive
  (Sec. 4.1 remark).
* BDF1 for the first step and variable-step BDF2 afterwards (eqs. be, bdf2);
  the generalised leapfrog predictor (eq. leapfrog) with the time derivative
  taken from the previous step's BDF left-hand side (Remark 2) is the Newton
  initial guess when it is positive.
* The discrete adjoint of a BDF1 trajectory for J = sum of E over the
  composite cells.

Norms and inner products are volume weighted over composite (non-covered)
cells: <x, y> = sum_c V_c (x_E y_E + x_T y_T).
"""
from __future__ import annotations

import numpy as np

from . import operators as ops
from . import precond as pc


class System:
    """One problem: hierarchy, material field, options; compact vectors are
    [E of all patches (x fastest) | T of all patches]."""

    def __init__(self, H, z, lam=0.5, p2_mode="paper", jvp_mode="analytic", fac_nu=(1, 0),
                 fac_smoother="rbgs", fac_base="mg", fac_cycle="mult"):
        self.H = H
        self.jvp_mode = jvp_mode
        self._b = None
        self.z = [np.asarray(a, dtype=np.float64) for a in z]
        self.lam = lam
        self.p2_mode = p2_mode
        self.fac_nu = tuple(fac_nu)     # FAC V(m, n) (Alg. 1)
        self.fac_smoother = fac_smoother
        self.fac_base = fac_base
        self.fac_cycle = fac_cycle      # "mult": FAC (Alg. 1); "afacx": AFACx
        self.nc = H.ncells()
        w = []
        for p in H.patches:
            v = np.full(tuple(int(x) for x in p.n), H.volume(p.level))
            v[H.covered[p.pid]] = 0.0
            w.append(v.ravel(order="F"))
        w = np.concatenate(w)
        self.weight = np.concatenate([w, w])
        self.composite = self.weight > 0

    # -- layout -----------------------------------------------------------
    def split(self, x):
        n = self.nc
        out = []
        for part in (x[:n], x[n:]):
            lst, o = [], 0
            for p in self.H.patches:
                m = int(np.prod(p.n))
                lst.append(part[o:o + m].reshape(tuple(int(v) for v in p.n),
                                                 order="F"))
                o += m
            out.append(lst)
        return out

    def join(self, E, T):
        return np.concatenate([np.concatenate([a.ravel(order="F") for a in E]),
                               np.concatenate([a.ravel(order="F") for a in T])])

    def dot(self, x, y):
        return float(np.sum(self.weight * x * y))

    def norm(self, x):
        return float(np.sqrt(self.dot(x, x)))

    def sync(self, u):
        E, T = self.split(u)
        Eg = self.H.from_interior(E)
        Tg = self.H.from_interior(T)
        self.H.sync([Eg, Tg])
        return self.join(self.H.interior(Eg), self.H.interior(Tg))

    # -- operators --------------------------------------------------------
    def residual(self, u, b, dt, c0):
        self._b = b
        E, T = self.split(u)
        bE, bT = self.split(b)
        FE, FT = ops.residual(self.H, E, T, self.z, bE, bT, dt, c0, self.lam)
        return self.join(FE, FT)

    def jvp(self, u, v, dt, c0):
        E, T = self.split(u)
        vE, vT = self.split(v)
        if self.jvp_mode == "fd":
            # the difference quotient needs the step's b: the one of the
            # latest residual evaluation (Newton evaluates F(u^k) first)
            bE, bT = self.split(self._b)
            JE, JT = ops.jvp_fd(self.H, E, T, self.z, vE, vT, bE, bT, dt, c0, self.lam)
        else:
            JE, JT = ops.jvp(self.H, E, T, self.z, vE, vT, dt, c0, self.lam)
        return self.join(JE, JT)

    def vjp(self, u, lmb, dt, c0):
        E, T = self.split(u)
        lE, lT = self.split(lmb)
        gE, gT, gz = ops.vjp(self.H, E, T, self.z, lE, lT, dt, c0, self.lam)
        return self.join(gE, gT), np.concatenate([a.ravel(order="F") for a in gz])

    def precond(self, u, beta):
        E, T = self.split(u)
        snap = pc.Snapshot(self.H, E, T, self.z, beta, self.lam, self.p2_mode, self.fac_nu,
                           self.fac_smoother, self.fac_base, self.fac_cycle)
        mg = (pc.build_mg(self.H, snap, 0), pc.build_mg(self.H, snap, 1))

        def apply(w):
            wE, wT = self.split(w)
            yE, yT = pc.precond_apply(self.H, snap, wE, wT, mg)
            return self.join(yE, yT)

        def apply_t(w):
            wE, wT = self.split(w)
            yE, yT = pc.precond_apply_transpose(self.H, snap, wE, wT, mg)
            return self.join(yE, yT)

        return apply, apply_t


# ---------------------------------------------------------------------------
# FGMRES(m) with CGS2
# ---------------------------------------------------------------------------

def givens(a, b):
    if b == 0.0:
        return 1.0, 0.0, a
    r = np.sqrt(a * a + b * b)
    return a / r, b / r, r


def fgmres(matvec, precond, rhs, tol, dot, m=30, max_restarts=10):
    """Solve A x = rhs to ||rhs - A x|| <= tol.  Returns (x, its, est)."""
    x = np.zeros_like(rhs)
    r = rhs.copy()
    its = 0
    est = np.sqrt(dot(r, r))
    for cycle in range(max_restarts + 1):
        beta0 = np.sqrt(dot(r, r))
        est = beta0
        if beta0 <= tol:
            break
        V = [r / beta0]
        Z = []
        Hm = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta0
        k = 0
        done = False
        for j in range(m):
            z = precond(V[j])
            Z.append(z)
            w = matvec(z)
            h1 = np.array([dot(V[i], w) for i in range(j + 1)])
            w = w - sum(h1[i] * V[i] for i in range(j + 1))
            h2 = np.array([dot(V[i], w) for i in range(j + 1)])
            w = w - sum(h2[i] * V[i] for i in range(j + 1))
            col = np.zeros(m + 1)
            col[:j + 1] = h1 + h2
            hn = np.sqrt(dot(w, w))
            col[j + 1] = hn
            for i in range(j):
                t = cs[i] * col[i] + sn[i] * col[i + 1]
                col[i + 1] = -sn[i] * col[i] + cs[i] * col[i + 1]
                col[i] = t
            cs[j], sn[j], col[j] = givens(col[j], col[j + 1])
            col[j + 1] = 0.0
            Hm[:, j] = col
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            its += 1
            k = j + 1
            est = abs(g[j + 1])
            if hn == 0.0 or est <= tol:
                done = True
                break
            V.append(w / hn)
        y = np.zeros(k)
        for i in range(k - 1, -1, -1):
            y[i] = (g[i] - Hm[i, i + 1:k] @ y[i + 1:k]) / Hm[i, i]
        x = x + sum(y[i] * Z[i] for i in range(k))
        if done:
            break
        r = rhs - matvec(x)
    return x, its, est


# ---------------------------------------------------------------------------
# inexact Newton
# ---------------------------------------------------------------------------

class NewtonResult:
    def __init__(self, u, converged, iters, krylov, fnorms, cuts):
        self.u = u
        self.converged = converged
        self.iters = iters
        self.krylov = krylov
        self.fnorms = fnorms
        self.cuts = cuts


def newton(sys: System, u0, b, dt, c0, beta, rtol=1e-8, atol=1e-14, maxit=20,
           m=30, max_restarts=10, eta_max=0.9, forcing="petsc"):
    """Inexact Newton with positivity-preserving step halving.  Forcing
    terms (Eisenstat-Walker; Sec. 4.1 cites Kelley's algorithm, Sec. 6 says
    the solver is PETSc's implementation, slightly modified): "petsc"
    (PETSc's choice 2: gamma = 1, exponent (1 + 5^1/2) / 2, eta_0 = 0.3;
    the default) or "kelley" (Kelley's safeguarded choice: gamma = 0.9,
    exponent 2, eta_0 = eta_max); the same safeguard threshold 0.1, cap
    eta_max and floor 0.5 tau / ||F_k||."""
    if forcing == "petsc":
        gamma, expo, eta0 = 1.0, 0.5 * (1.0 + np.sqrt(5.0)), 0.3
    elif forcing == "kelley":
        gamma, expo, eta0 = 0.9, 2.0, eta_max
    else:
        raise ValueError(f"unknown forcing {forcing}")
    u = u0.copy()
    F = sys.residual(u, b, dt, c0)
    fn = sys.norm(F)
    stop = max(rtol * fn, atol)
    fnorms = [fn]
    krylov = []
    cuts = 0
    eta = eta0
    fn_old = fn
    k = 0
    while fn > stop and k < maxit:
        if k > 0:
            rat = fn / fn_old
            enew = gamma * rat**expo
            if gamma * eta**expo > 0.1:
                enew = max(enew, gamma * eta**expo)
            eta = min(enew, eta_max)
            eta = max(eta, 0.5 * stop / fn)
        P, _ = sys.precond(u, beta)
        s, its, _ = fgmres(lambda v: sys.jvp(u, v, dt, c0), P, -F, eta * fn,
                           sys.dot, m, max_restarts)
        krylov.append(its)
        lam = 1.0
        ok = False
        for _ in range(31):
            trial = u + lam * s
            if np.all(trial[sys.composite] > 0.0):
                ok = True
                break
            lam *= 0.5
            cuts += 1
        if not ok:
            return NewtonResult(u, False, k, krylov, fnorms, cuts)
        u = sys.sync(trial)
        fn_old = fn
        F = sys.residual(u, b, dt, c0)
        fn = sys.norm(F)
        fnorms.append(fn)
        k += 1
    return NewtonResult(u, fn <= stop, k, krylov, fnorms, cuts)


# ---------------------------------------------------------------------------
# BDF stepping
# ---------------------------------------------------------------------------

def bdf_coefficients(dt, dt_prev):
    """(c0, alpha) for BDF1 (dt_prev None) or variable-step BDF2."""
    if dt_prev is None:
        return 1.0, 0.0
    a = dt / dt_prev
    return (1.0 + 2.0 * a) / (1.0 + a), a


def bdf2_history(u, u_prev, a):
    """b of eq. bdf2 written as c0 u_{n+1} - b = dt f(u_{n+1}):
    b = (1 + a) u_n - a^2 / (1 + a) u_{n-1}, a = dt_n / dt_{n-1}."""
    return (1.0 + a) * u - (a * a / (1.0 + a)) * u_prev


def leapfrog_predictor(u, u_prev, udot, dt, a):
    """Generalised leapfrog predictor (eq. leapfrog):
    u^p_{n+1} = u_n + (1 + a) dt u'_n - a^2 (u_n - u_{n-1})."""
    return u + (1.0 + a) * dt * udot - a * a * (u - u_prev)


class Stepper:
    """Library-owned state u_n, u_{n-1}, dt_{n-1}, udot_n (eqs. be, bdf2,
    leapfrog)."""

    def __init__(self, sys: System, u0, bdf1_only=False, **newton_kw):
        self.sys = sys
        self.u = sys.sync(u0.copy())
        self.u_prev = None
        self.dt_prev = None
        self.udot = None
        self.bdf1_only = bdf1_only
        self.kw = newton_kw
        self.history = []

    def rhs_and_guess(self, dt):
        first = self.dt_prev is None or self.bdf1_only
        if first:
            c0, a = 1.0, 0.0
            b = self.u.copy()
            guess = self.u.copy()
        else:
            c0, a = bdf_coefficients(dt, self.dt_prev)
            b = bdf2_history(self.u, self.u_prev, a)
            guess = leapfrog_predictor(self.u, self.u_prev, self.udot, dt, a)
            self.predicted = guess.copy()
            if not np.all(guess[self.sys.composite] > 0.0):
                guess = self.u.copy()
            guess = self.sys.sync(guess)
        beta = dt / c0
        return c0, a, b, guess, beta

    def step(self, dt):
        """One step of size dt; on failure the state is left unchanged.
        self.predicted / self.alpha hold the step's leapfrog predictor and
        step ratio (None / 0 for a BDF1 step)."""
        self.predicted = None
        c0, a, b, guess, beta = self.rhs_and_guess(dt)
        self.alpha = a
        res = newton(self.sys, guess, b, dt, c0, beta, **self.kw)
        if not res.converged:
            return res
        self.udot = (c0 * res.u - b) / dt
        self.u_prev = self.u
        self.u = res.u
        self.dt_prev = dt
        self.last = (b, c0, dt)            # the step's system, for a re-solve
        self.history.append(res)
        return res

    def regrid(self, new_sys):
        """Move the time history to a new hierarchy and re-solve the last
        step there (Sec. 5, warm restart with a re-solve): u_n, u_{n-1} and
        the last step's history vector b are transferred by conservative
        linear refinement; the last step's system F(u) = c0 u - b - dt f(u)
        is solved again on the new grid from the transferred u_n; u'_n is
        recomputed from the re-solved state.  The next step's local error
        estimate depends on interpolated data and is not to be used
        (self.after_regrid).  Returns the Newton result of the re-solve."""
        from . import regrid as rg
        old = self.sys

        def move(x):
            E, T = old.split(x)
            return new_sys.join(rg.transfer(old.H, E, new_sys.H),
                                rg.transfer(old.H, T, new_sys.H))
        b, c0, dt = self.last
        u = move(self.u)
        self.u_prev = move(self.u_prev) if self.u_prev is not None else None
        b = move(b)
        self.sys = new_sys
        res = newton(new_sys, u, b, dt, c0, dt / c0, **self.kw)
        if not res.converged:
            raise RuntimeError("re-solve after regridding did not converge")
        self.u = res.u
        self.udot = (c0 * res.u - b) / dt
        self.last = (b, c0, dt)
        self.after_regrid = True
        return res


# ---------------------------------------------------------------------------
# time-step control (Sec. 3.4-3.5: eqs. odets, pc47, leapfrog, bdf2le)
# ---------------------------------------------------------------------------

def bdf2_error_estimate(u_new, u_pred, a):
    """Local error of a variable-step BDF2 step from the leapfrog
    predictor (eq. bdf2le): e = (a + 1) / (3 a + 2) (u_{n+1} - u^p)."""
    return (a + 1.0) / (3.0 * a + 2.0) * (u_new - u_pred)


def scaled_max_norm(sys: System, e, u, eta_E, eta_T):
    """max(max |e_E / (E + eta_E)|, max |e_T / (T + eta_T)|) over composite
    cells, u the solution the error belongs to (the scaled max norm of
    Sec. 3.5)."""
    n = sys.nc
    m = sys.composite[:n]
    eE, eT, E, T = e[:n], e[n:], u[:n], u[n:]
    return max(float(np.max(np.abs(eE[m] / (E[m] + eta_E)))),
               float(np.max(np.abs(eT[m] / (T[m] + eta_T)))))


def eps_step_factor(eps, err, k=3):
    """Elementary error-per-step controller (eq. odets): dt_{n+1} / dt_n
    = (eps / ||e_n||)^(1/k), k = 3 for BDF2."""
    return (eps / err) ** (1.0 / k)


def pc47_ratio(eps, err, err_prev, a, k=3, kI=0.4, kP=0.7):
    """PI controller PC.4.7 (eq. pc47) with k kI = 0.4, k kP = 0.7:
    a_{n+1} = (eps / ||e_n||)^kI (||e_{n-1}|| / ||e_n||)^kP a_n, the
    exponents taken as 0.4 / k and 0.7 / k."""
    return (eps / err) ** (kI / k) * (err_prev / err) ** (kP / k) * a


class AdaptiveStepper(Stepper):
    """BDF1 first step, then BDF2 with the step size chosen by PC.4.7 from
    the local error estimate (EPS for the first estimate, which has no
    predecessor).  Readings: the step ratio is kept in [ratio_min,
    ratio_max] (variable-step BDF2 is zero-stable only for ratios below
    1 + sqrt 2); a step whose Newton solve fails is retried with half the
    step (at most max_halvings times); converged steps are always accepted
    and the controller answers their error."""

    def __init__(self, sys: System, u0, dt0, eps, eta_E, eta_T, controller="pc47",
                 ratio_min=0.25, ratio_max=2.0, max_halvings=10, **newton_kw):
        super().__init__(sys, u0, **newton_kw)
        self.dt = float(dt0)
        self.eps = eps
        self.eta = (eta_E, eta_T)
        self.controller = controller
        self.ratio_min, self.ratio_max = ratio_min, ratio_max
        self.max_halvings = max_halvings
        self.err_prev = None
        self.t = 0.0
        self.log = []           # (dt, converged after halvings, err or None)

    def advance(self):
        """One accepted step (with retries); returns its Newton result."""
        dt = self.dt
        for _ in range(self.max_halvings + 1):
            res = self.step(dt)
            if res.converged:
                break
            dt *= 0.5
        else:
            raise RuntimeError("time step could not be made to converge")
        self.t += dt
        err = None
        ratio = 1.0
        if getattr(self, "after_regrid", False):
            # the first estimate after a regrid uses interpolated history: it
            # is not used (Sec. 5); the step size is kept and the next
            # estimate has no predecessor
            self.after_regrid = False
            self.err_prev = None
        elif self.predicted is not None:
            err = scaled_max_norm(self.sys, bdf2_error_estimate(self.u, self.predicted, self.alpha),
                                  self.u, *self.eta)
            if err > 0.0:
                if self.controller == "pc47" and self.err_prev is not None:
                    ratio = pc47_ratio(self.eps, err, self.err_prev, self.alpha)
                else:
                    ratio = eps_step_factor(self.eps, err)
            else:
                ratio = self.ratio_max
            self.err_prev = err
        ratio = min(max(ratio, self.ratio_min), self.ratio_max)
        self.log.append((dt, err))
        self.dt = ratio * dt
        return res


# ---------------------------------------------------------------------------
# discrete adjoint of a BDF1 trajectory, J = sum of E over cells
# ---------------------------------------------------------------------------

def adjoint_gradient(sys: System, u0, dt, nsteps, tol=1e-11, newton_kw=None,
                     m=30, max_restarts=20, dJdE=None):
    """dJ/dz for J = sum over cells of dJdE[c] E_N(c) (compact E part;
    default: 1 on every composite cell, 0 on covered cells) after nsteps
    BDF1 steps of size dt; z of every level, covered cells included.  A
    covered cell's E is the mean of its children's, so its weight passes to
    them (transposed restriction) before the reverse sweep.

    Forward: u_n solves F_n = u_n - u_{n-1} - dt f(u_n; z) = 0 on the
    composite cells, covered cells restricted from their children.  Reverse:
    A_N^T l_N = dJ/du_N, A_n^T l_n = l_{n+1}; dJ/dz = -sum_n l_n^T dF_n/dz,
    A_n^T the transpose of F_n's derivative in the composite unknowns (the
    covered entries of l carry nothing).  Every forward state is kept (the
    oracle does not checkpoint)."""
    kw = dict(newton_kw or {})
    st = Stepper(sys, u0, bdf1_only=True, **kw)
    states = [st.u.copy()]
    for _ in range(nsteps):
        r = st.step(dt)
        if not r.converged:
            raise RuntimeError("forward solve failed")
        states.append(st.u.copy())
    nc = sys.nc
    if dJdE is None:
        gE = sys.composite[:nc].astype(np.float64)
    else:
        E, _ = sys.split(np.concatenate([np.asarray(dJdE, dtype=np.float64), np.zeros(nc)]))
        Eg = sys.H.from_interior(E)
        sys.H.sync_transpose([Eg])
        gE = np.concatenate([a[1:-1, 1:-1, 1:-1].ravel(order="F") for a in Eg])
    rhs = np.concatenate([gE, np.zeros(nc)])
    grad = np.zeros(nc)
    euclid = lambda x, y: float(np.dot(x, y))
    for n in range(nsteps, 0, -1):
        u = states[n]
        _, PT = sys.precond(u, dt)
        mv = lambda v: sys.vjp(u, v, dt, 1.0)[0]
        tol_abs = tol * np.sqrt(euclid(rhs, rhs))
        lmb, _, _ = fgmres(mv, PT, rhs, tol_abs, euclid, m, max_restarts)
        _, gz = sys.vjp(u, lmb, dt, 1.0)
        grad -= gz
        rhs = lmb
    return grad, states
