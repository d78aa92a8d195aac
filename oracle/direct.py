"""Definition layer: assembled Jacobian and the exact discrete BDF solution.

On a single-level grid every residual entry F_c depends only on cell c and
its six face neighbours (the ghost copies stay inside that star), so columns
whose cells agree in (i mod 3, j mod 3, k mod 3) never share a row: 27
colours per field recover the whole sparse Jacobian from 54 Jacobian
actions.  With it, Newton + sparse LU gives the solution u* of the discrete
BDF system F(u) = 0 (eq. nonlinearsystem) independently of GMRES and of the
preconditioner; any correct solver must land on u* within its tolerance.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .solvers import System


def _cell_index_arrays(sys: System):
    I = []
    for p in sys.H.patches:
        r = [np.arange(p.lo[d], p.hi[d]) for d in range(3)]
        g = np.meshgrid(*r, indexing="ij")
        I.append(np.stack([x.ravel(order="F") for x in g], axis=1))
    return np.concatenate(I)


def assemble_jacobian(sys: System, u, dt, c0):
    if sys.H.nlev != 1:
        raise NotImplementedError("colouring assumes a single level")
    nc = sys.nc
    I = _cell_index_arrays(sys)
    colour = (I[:, 0] % 3) + 3 * (I[:, 1] % 3) + 9 * (I[:, 2] % 3)
    # neighbour lookup: level index -> compact cell id
    key = {tuple(v): k for k, v in enumerate(I)}
    rows, cols, vals = [], [], []
    for field in (0, 1):
        for c in range(27):
            sel = np.nonzero(colour == c)[0]
            if len(sel) == 0:
                continue
            v = np.zeros(2 * nc)
            v[field * nc + sel] = 1.0
            Jv = sys.jvp(u, v, dt, c0)
            for col in sel:
                base = I[col]
                for off in ((0, 0, 0), (1, 0, 0), (-1, 0, 0), (0, 1, 0),
                            (0, -1, 0), (0, 0, 1), (0, 0, -1)):
                    k = key.get(tuple(base + np.array(off)))
                    if k is None:
                        continue
                    for rf in (0, 1):
                        val = Jv[rf * nc + k]
                        if val != 0.0:
                            rows.append(rf * nc + k)
                            cols.append(field * nc + col)
                            vals.append(val)
    return sp.csr_matrix((vals, (rows, cols)), shape=(2 * nc, 2 * nc))


def solve_exact(sys: System, u0, b, dt, c0, tol=1e-13, maxit=50):
    """Newton with the assembled Jacobian and sparse LU, damped only to keep
    E, T > 0; stops when ||F|| stagnates below tol * ||F(u0)||."""
    u = u0.copy()
    F = sys.residual(u, b, dt, c0)
    f0 = sys.norm(F)
    for _ in range(maxit):
        fn = sys.norm(F)
        if fn <= tol * f0:
            break
        J = assemble_jacobian(sys, u, dt, c0)
        s = spla.spsolve(J.tocsc(), -F)
        lam = 1.0
        while not np.all(u + lam * s > 0.0):
            lam *= 0.5
        u_new = u + lam * s
        F_new = sys.residual(u_new, b, dt, c0)
        if sys.norm(F_new) >= fn and lam == 1.0 and fn < 1e-10 * f0:
            break
        u, F = u_new, F_new
    return u
