"""Pins of the oracle's AFACx cycle (the asynchronous FAC variant the paper
names in Sec. 7; its steps as defined by Lee, McCormick, Philip and
Quinlan): each piece against exact solves of assembled level operators,
the whole cycle against the level operator's exact inverse where the
method must reproduce it, and as a stationary iteration.

* With one level AFACx is the base solve, as FAC is.
* Converged coarse sweeps on the region a finer level covers solve the
  principal submatrix of the coarse level operator on that region (every
  other cell held at 0).
* Converged fine sweeps from the interpolated coarse approximation s give
  A_l^-1 r - s.
* With level 1 covering the whole domain, an exact base solve and
  converged sweeps, the coarse approximation equals the base correction,
  the two cancel, and the cycle returns A_1^-1 r exactly.
"""
import numpy as np
import pytest

from oracle import precond as pc
from oracle.hierarchy import Hierarchy
from paper_1302_6303_amd import inputs as I
from tests.helpers import state, system


def _front(H, seed=250):
    E, T = [], []
    rng = np.random.default_rng(seed)
    for p in H.patches:
        h = H.h(p.level)
        ax = [(np.arange(p.lo[d], p.hi[d]) + 0.5) * h[d] for d in range(3)]
        X, Y, _ = np.meshgrid(*ax, indexing="ij")
        prof = 1e-5 + 4.0 / (1.0 + np.exp((X + 0.3 * Y - 0.6) / 0.1))
        E.append(prof * (1 + 0.05 * rng.standard_normal(prof.shape)))
        T.append(prof ** 0.25)
    z = [1.0 + 0.5 * rng.random(tuple(int(v) for v in p.n)) for p in H.patches]
    return E, T, z


def _level_matrix(H, snap, f, p):
    """Dense level operator of patch p (coarse-fine ghosts with coarse
    values 0, folded into the diagonal), x-fastest cell order."""
    w, diag = pc.level_weights(H, snap, f, p)
    n = tuple(int(v) for v in p.n)
    N = int(np.prod(n))
    A = np.diag(diag.ravel(order="F"))
    idx = np.arange(N).reshape(n, order="F")
    for d in range(3):
        lo = [slice(None)] * 3
        hi = [slice(None)] * 3
        lo[d] = slice(0, n[d] - 1)
        hi[d] = slice(1, n[d])
        a = idx[tuple(lo)].ravel()
        b = idx[tuple(hi)].ravel()
        fw = [slice(None)] * 3
        fw[d] = slice(1, n[d])
        wf = w[d][tuple(fw)].ravel()
        A[a, b] -= wf
        A[b, a] -= wf
    return A


def _snap(H, beta=5e-2):
    E, T, z = _front(H)
    return pc.Snapshot(H, E, T, z, beta, 0.5, fac_cycle="afacx")


@pytest.mark.parametrize("base", ["mg", "smooth"])
def test_afacx_on_one_level_is_the_base_solve(base):
    H = Hierarchy((8, 8, 8), [(0, (0, 0, 0), (8, 8, 8))])
    snap = _snap(H)
    snap.fac_base = base
    rng = np.random.default_rng(3)
    rhs = [rng.standard_normal((8, 8, 8))]
    for f in (0, 1):
        a = pc.afacx_cycle(H, snap, f, rhs, nu=(2, 0))
        b = pc.fac_vcycle(H, snap, f, rhs, nu=(2, 0))
        assert np.array_equal(a[0], b[0])


def test_afacx_coarse_approximation_solves_the_covered_region():
    """m -> infinity: the coarse sweeps solve A_0[R, R] c = r[R] on the
    region R level 1 covers, c = 0 elsewhere."""
    H = Hierarchy((8, 8, 8), [(0, (0, 0, 0), (8, 8, 8)), (1, (4, 2, 4), (12, 12, 10))])
    snap = _snap(H)
    p0 = H.by_level[0][0]
    rng = np.random.default_rng(5)
    r = {p0.pid: rng.standard_normal((8, 8, 8))}
    for f in (0, 1):
        c = pc.afacx_coarse(H, snap, f, 1, r, 400)[p0.pid].ravel(order="F")
        A = _level_matrix(H, snap, f, p0)
        R = H.covered[p0.pid].ravel(order="F")
        want = np.zeros(A.shape[0])
        want[R] = np.linalg.solve(A[np.ix_(R, R)], r[p0.pid].ravel(order="F")[R])
        assert np.abs(c - want).max() <= 1e-11 * np.abs(want).max()


def test_afacx_fine_correction_is_the_level_solve_minus_its_start():
    H = Hierarchy((8, 8, 8), [(0, (0, 0, 0), (8, 8, 8)), (1, (4, 2, 4), (12, 12, 10))])
    snap = _snap(H)
    p1 = H.by_level[1][0]
    n = tuple(int(v) for v in p1.n)
    rng = np.random.default_rng(6)
    r = {p1.pid: rng.standard_normal(n)}
    s = {p1.pid: rng.standard_normal(n)}
    for f in (0, 1):
        e = pc.afacx_fine(H, snap, f, 1, r, s, 400)[p1.pid].ravel(order="F")
        A = _level_matrix(H, snap, f, p1)
        want = np.linalg.solve(A, r[p1.pid].ravel(order="F")) - s[p1.pid].ravel(order="F")
        assert np.abs(e - want).max() <= 1e-11 * np.abs(want).max()


def test_afacx_with_a_whole_domain_fine_level_inverts_the_fine_operator():
    """Level 1 covers the domain, the 4^3 base is the exact bottom grid:
    base correction and coarse approximation cancel, u = A_1^-1 r."""
    H = Hierarchy((4, 4, 4), [(0, (0, 0, 0), (4, 4, 4)), (1, (0, 0, 0), (8, 8, 8))])
    snap = _snap(H, beta=2e-2)
    p1 = H.by_level[1][0]
    rng = np.random.default_rng(7)
    rhs = [rng.standard_normal((4, 4, 4)), rng.standard_normal((8, 8, 8))]
    for f in (0, 1):
        u = pc.afacx_cycle(H, snap, f, rhs, nu=(400, 0))
        A = _level_matrix(H, snap, f, p1)
        want = np.linalg.solve(A, rhs[1].ravel(order="F"))
        got = u[1].ravel(order="F")
        assert np.abs(got - want).max() <= 1e-10 * np.abs(want).max()


def test_afacx_stationary_iteration_contracts():
    """AFACx as a stationary iteration on A^c u = f (two and three levels,
    smooth coefficients) contracts below 1, and V(2) faster than V(1)."""
    for w in (I.small_amr(8, state="uniform"),
              I.static_amr(base=8, nlevels=3, side=(8, 16), state="uniform")):
        rng0 = np.random.default_rng(250)
        w.E, w.T = I.front_state(w.problems, w.boxes, rng0, noise=0.0)
        s = system(w)
        H = s.H
        s.z = [np.ones(tuple(int(v) for v in p.n)) for p in H.patches]
        E, T = s.split(state(s, w))
        snap = pc.Snapshot(H, E, T, s.z, 5e-2, fac_cycle="afacx")
        rates = {}
        for m in (1, 2):
            rng = np.random.default_rng(25)
            rhs = [rng.standard_normal(tuple(int(v) for v in p.n)) for p in H.patches]
            x = [np.zeros_like(r) for r in rhs]
            norms = []
            for _ in range(7):
                Ax = pc.composite_apply(H, snap, 0, x)
                r = [rhs[q] - Ax[q] for q in range(len(rhs))]
                norms.append(np.sqrt(sum(np.sum(rr[~H.covered[q]] ** 2)
                                         for q, rr in enumerate(r))))
                c = pc.afacx_cycle(H, snap, 0, r, nu=(m, 0))
                x = [x[q] + c[q] for q in range(len(x))]
            rates[m] = (norms[-1] / norms[2]) ** 0.25
        assert rates[1] < 0.6 and rates[2] < rates[1], rates
