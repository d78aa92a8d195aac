"""Writes adjoint64.json: the CPU oracle's discrete adjoint gradient for the
differentiation workload (uniform 64^3, z = 1 + 9 s with s a smoothed
random field clipped to [0, 1], 50 backward-Euler steps of 1e-3 from the
uniform initial state, J = sum of E over the cells at the final time).

Calls only the oracle and the seeded input generators.  Stored: the
gradient at 20 cells chosen (seeded) among those with |dJ/dz| >= 1e-3 of
its maximum -- the cells the GPU test also checks against central
differences -- and at 200 random cells, with the gradient's maximum and
norm and J itself.  About ten minutes on one core:

    python tests/golden/make_adjoint64.py
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle.hierarchy import Hierarchy  # noqa: E402
from oracle.solvers import System, adjoint_gradient  # noqa: E402
from paper_1302_6303_amd import inputs as I  # noqa: E402

N, DT, NSTEPS = 64, 1e-3, 50


def main():
    w = I.differentiation(N)
    pr = w.problems[0]
    H = Hierarchy(pr.base_n, [(0, (0, 0, 0), (N, N, N))], lo=pr.lo, hi=pr.hi, bc_E=pr.bc_E,
                  robin_R=pr.robin_R, kappa=pr.kappa)
    s = System(H, w.z)
    u0 = np.concatenate([w.compact(w.E), w.compact(w.T)])
    t0 = time.time()
    g, states = adjoint_gradient(s, u0, DT, NSTEPS, tol=1e-12,
                                 newton_kw=dict(rtol=1e-12, atol=1e-22, maxit=40))
    nc = s.nc
    gmax = float(np.max(np.abs(g)))
    rng = np.random.default_rng(I.SEED_BASE + 5)
    cand = np.flatnonzero(np.abs(g) >= 1e-3 * gmax)
    fd_cells = np.sort(rng.choice(cand, 20, replace=False))
    sample = np.sort(rng.choice(nc, 200, replace=False))
    out = {
        "source": "oracle.solvers.adjoint_gradient on inputs.differentiation(64): 50 "
                  "backward-Euler steps of 1e-3, J = sum of E at the final time; Newton "
                  "rtol 1e-12, atol 1e-22; transpose FGMRES tolerance 1e-12 relative",
        "n": N, "dt": DT, "nsteps": NSTEPS,
        "J": float(np.sum(np.sort(states[-1][:nc]))),
        "grad_max_abs": gmax, "grad_norm": float(np.linalg.norm(g)),
        "fd_cells": [int(c) for c in fd_cells], "fd_values": [float(g[c]) for c in fd_cells],
        "sample_cells": [int(c) for c in sample], "sample_values": [float(g[c]) for c in sample],
        "oracle_seconds": round(time.time() - t0, 1),
    }
    with open(os.path.join(HERE, "adjoint64.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps({k: v for k, v in out.items() if not isinstance(v, list)}))


if __name__ == "__main__":
    main()
