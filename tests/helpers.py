"""Test helpers: build oracle objects from the seeded workloads."""
import numpy as np

from oracle.hierarchy import Hierarchy
from oracle.solvers import System


def hierarchy(w, pidx=0, **over):
    pr = w.problems[pidx]
    bx = [(b.level, b.lo, b.hi) for b in w.boxes if b.problem == pidx]
    kw = dict(lo=pr.lo, hi=pr.hi, bc_E=pr.bc_E, robin_R=pr.robin_R,
              kappa=pr.kappa)
    kw.update(over)
    return Hierarchy(pr.base_n, bx, **kw)


def system(w, pidx=0, lam=0.5, fac_nu=(1, 0), fac_smoother="rbgs", fac_base="mg",
           fac_cycle="mult", **over):
    H = hierarchy(w, pidx, **over)
    z = [zz for zz, b in zip(w.z, w.boxes) if b.problem == pidx]
    return System(H, z, lam=lam, fac_nu=fac_nu, fac_smoother=fac_smoother,
                  fac_base=fac_base, fac_cycle=fac_cycle)


def state(sys_, w, pidx=0):
    E = [e for e, b in zip(w.E, w.boxes) if b.problem == pidx]
    T = [t for t, b in zip(w.T, w.boxes) if b.problem == pidx]
    return sys_.sync(sys_.join(E, T))
