"""Benchmark of the implicit radiation-diffusion hot path on one MI355X.

One step = one BDF implicit step (inexact Newton, FGMRES, FAC/multigrid
preconditioner, flux-limited residual and Jacobian action) over every problem
of the workload.  Prints ONE JSON line:

  value        residual throughput in Gcells/s: composite cells covered by the
               residual launches of the timed implicit steps (after the first
               Newton update a launch covers only the problems still
               iterating) over their HIP-event time on the library stream
  ms_per_step  wall time per implicit step of the mixed-precision batched
               solver (float V-cycles, float64 Newton/GMRES/residual)
  fp64_plain   the same steps with a float64 preconditioner and one kernel
               launch per patch
  roofline     the residual kernel against the 8 TB/s HBM peak
  cpu_baseline the float64 CPU oracle's residual on a bounded sample

Workloads (seeded, synthetic; --workload):
  ensemble  64 independent uniform problems of 32^3..96^3 cells with random
            material boxes and time steps (21.6 M cells)
  amr       64^3 base + 2 levels of static refinement around two material
            boxes (228 patches, 1.04 M composite+covered cells), dt = 5e-4
  amr128    128^3 base + 3 levels around six material boxes (2794 patches,
            39 M cells), dt = 5e-4; run with --bdf-max-order 1 (BDF2 stalls
            at the second step without time-step control)
  dynamic   128^3 base, 4 levels regridded every 5 steps on |grad E|/E > 10
            or a material interface (Berger-Rigoutsos), 50 BDF steps of
            1e-5, warm restart after each regrid; mixed batched, replayed in
            float64 batched (solution difference, Krylov counts) and for the
            first 10 steps in float64 per patch
  uniform   one 32^3 patch, dt = 1e-3
  adjoint   64^3 smooth random material, 50 BDF1 steps: forward, checkpointed
            reverse sweep, transpose kernel
  paperN    the paper's model problem on a uniform N^3 grid integrated to
            --t-final (default 1) with PC.4.7; reports seconds, steps and
            iterations per step beside the paper's uniform-grid tables
  paperNbLl the same problem on a dynamically refined hierarchy: base N^3,
            L levels, tags tau^g or tau^c > --tau checked every 10 steps,
            regrid (transfer, warm restart with re-solve) when the boxes
            change; beside the paper's AMR columns of those tables
  paper-spatial  uniform 128^3 against a 256^3 reference with the same
            steps: L2 errors beside the paper's spatial-accuracy table
            (paper-spatial-z1: its single-material variant, z = 1)
  paper-temporal  fixed BDF2 steps 2e-4, 1e-4, 5e-5 against 2.5e-5 on
            128^3: L2 errors beside the paper's temporal-accuracy table
"""
from __future__ import annotations

import argparse
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

BYTES_PER_CELL_RESIDUAL = 56      # read E, T, z^3, b_E, b_T; write F_E, F_T (f64)
BYTES_PER_CELL_JVP = 56           # read E, T, z^3, v_E, v_T; write 2 (f64)
# red-black sweep in float: read the right-hand side (2), the frozen state
# E, T, z^3 (3) and the iterate (2), write the iterate (2); the first sweep
# of a V-cycle starts from zero and does not read the iterate
BYTES_PER_CELL_SWEEP = 36
BYTES_PER_CELL_SWEEP_ZERO = 28
HBM_PEAK_GBS = 8000.0

# HBM bytes per composite cell of the residual on the ensemble workload from
# rocprofv3 FETCH_SIZE and WRITE_SIZE runs (KiB per dispatch, FETCH scaled by
# the factor a plain 2 GiB copy reads in the same run, WRITE by its own
# factor; the 20 full launches timed after the steps), valid for the stencil
# source with this SHA-256 prefix; null otherwise.
MEASURED_TRAFFIC = {"workload": "ensemble", "stencil_sha256": "c9ec114e166c8b40",
                    "bytes_per_cell": 63.2710,
                    "fetch_bytes_per_cell": 46.6790,
                    "write_bytes_per_cell": 16.5919,
                    "fetch_scale": 2.0, "write_scale": 1.0}


def stencil_source_hash():
    import hashlib
    path = os.path.join(ROOT, "paper_1302_6303_amd", "csrc", "stencil.hip")
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def compact_state(w):
    """[E of all boxes | T of all boxes], the library's compact layout."""
    import numpy as np
    return np.concatenate([w.compact(w.E), w.compact(w.T)])


def to_dev(x):
    import numpy as np
    import torch
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).to("cuda")


def workload(name):
    from paper_1302_6303_amd import inputs as I
    if name == "ensemble":
        return I.ensemble()
    if name == "amr":
        return I.static_amr()
    if name == "uniform":
        return I.marshak_single(32)
    if name == "amr128":
        # static stand-in for the dynamically regridded 4-level hierarchy:
        # 128^3 base, 6 material boxes, patches of 12..48 cells per side
        return I.static_amr(base=128, nlevels=4, side=(24, 48), nbox=6, seed_k=3)
    raise SystemExit(f"unknown workload {name}")


def composite_cells(w):
    """Cells not covered by a finer box (host-side count)."""
    from paper_1302_6303_amd.inputs import Box
    tot = 0
    for b in w.boxes:
        n = b.ncells
        for c in w.boxes:
            if c.problem == b.problem and c.level == b.level + 1:
                ov = 1
                for d in range(3):
                    lo = max(c.lo[d] // 2, b.lo[d])
                    hi = min(c.hi[d] // 2, b.hi[d])
                    ov *= max(0, hi - lo)
                n -= ov
        tot += n
    return tot


def run_solver(w, opts, steps, warmup, time_residual, adaptive_eps=None):
    """adaptive_eps: take the steps with PC.4.7 time-step control at this
    local error tolerance (each step as long as the controller says, failed
    solves retried with half the step) instead of the workload's fixed dt."""
    import torch
    from paper_1302_6303_amd import nrd
    if adaptive_eps is not None:
        opts.error_estimate = 1
    H = nrd.Hierarchy(w.problems, w.boxes, opts)
    u = compact_state(w)
    n = H.ncells
    H.set_fields(to_dev(u[:n]), to_dev(u[n:]), to_dev(w.compact(w.z)))
    tuned = H.autotune(None)                   # tile shapes per patch-size class
    log(f"tile shapes tuned for {tuned} patch-size classes")
    dt = list(w.dt)
    newton = krylov = 0
    accepted = []
    tag = "mixed" if opts.precision == nrd.NRD_MIXED else "fp64"

    def one_step():
        nonlocal dt
        if adaptive_eps is None:
            _, st = H.implicit_step(dt)
            return st
        _, dt, _, steps_ = H.adaptive_steps(1, dt, adaptive_eps)
        accepted.append([x["dt"] for x in steps_[0]])
        return steps_[0]

    for i in range(warmup):
        st = one_step()
        log(f"{tag} warmup step {i}: newton {sum(x['newton_iters'] for x in st)} "
            f"krylov {sum(x['krylov_iters'] for x in st)}")
    torch.cuda.synchronize()
    if time_residual:
        H.timer_enable(True)
    t0 = time.perf_counter()
    for i in range(steps):
        st = one_step()
        newton += sum(s["newton_iters"] for s in st)
        krylov += sum(s["krylov_iters"] for s in st)
        log(f"{tag} step {i} done")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    res = {"s_per_step": (t1 - t0) / steps, "newton_per_step": newton / steps,
           "krylov_per_step": krylov / steps, "ws_GB": H.workspace_bytes / 1e9}
    if adaptive_eps is not None:
        res["accepted_dt_problem0"] = [round(a[0], 9) for a in accepted]
    if time_residual:
        # residual evaluations inside the timed steps always cover every
        # problem (Newton evaluates F for all of them)
        # launches after the first Newton update cover only the problems
        # still iterating: rates use the composite cells each launch covered
        ms, cnt = H.timer_read(nrd.NRD_TIMER_RESIDUAL)
        cells = H.timer_cells(nrd.NRD_TIMER_RESIDUAL)
        res["residual_ms_avg"] = ms / max(cnt, 1)
        res["residual_launches"] = cnt
        res["residual_cells_avg"] = cells / max(cnt, 1)
        H.timer_enable(False)
        # the operators again over all problems on the final state (3 warm-up
        # calls, 20 timed each): the Jacobian action and preconditioner skip
        # converged problems inside the steps, and full residual launches
        # complement the timed-region rate above
        H.begin_step(dt)
        E, T = H.get_fields()
        U = H.unpack(torch.cat([E, T]))
        V = H.unpack(torch.cat([E, T]) * 1e-3)
        Y = H.native()
        H.precond_setup(U)
        for _ in range(3):
            H.jvp(U, V, Y)
            H.precond_apply(V, Y)
        torch.cuda.synchronize()
        H.timer_enable(True)
        for _ in range(20):
            H.residual(U, Y)
        for _ in range(20):
            H.jvp(U, V, Y)
        for _ in range(20):
            H.precond_apply(V, Y)
        for key, which in (("residual_full", nrd.NRD_TIMER_RESIDUAL),
                           ("jvp", nrd.NRD_TIMER_JVP), ("precond", nrd.NRD_TIMER_PRECOND),
                           ("sweep", nrd.NRD_TIMER_SMOOTH),
                           ("sweep_zero", nrd.NRD_TIMER_SMOOTH_ZERO)):
            ms, cnt = H.timer_read(which)
            res[key + "_ms_avg"] = ms / max(cnt, 1)
            res[key + "_calls"] = cnt
        H.timer_enable(False)
        del U, V, Y
    del H
    torch.cuda.empty_cache()
    return res


def copy_calibration(nbytes=2 << 30):
    """A plain device copy of known size (for scaling HBM byte counters)."""
    import torch
    x = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    log(f"copy calibration: {nbytes} bytes read and written per copy, 3 copies")
    del x, y
    torch.cuda.empty_cache()


def cpu_baseline(w, budget_s=12.0):
    """The float64 numpy oracle's residual (one thread) over whole problems
    of the same workload, in passes over its problems until about budget_s
    seconds of CPU work have been timed."""
    from tests.helpers import system, state
    systems = []
    for p in range(len(w.problems)):
        s = system(w, pidx=p)
        systems.append((s, state(s, w, pidx=p), float(w.dt[p])))
    cells = 0
    t_used = 0.0
    evals = 0
    while t_used < budget_s:
        for s, u, dt in systems:
            t0 = time.perf_counter()
            s.residual(u, u, dt, 1.0)
            t_used += time.perf_counter() - t0
            cells += s.nc
            evals += 1
            if t_used >= budget_s:
                break
    return {"value": cells / t_used / 1e9, "unit": "Gcells/s", "cores": 1,
            "kind": "oracle",
            "sample": f"float64 numpy residual, {evals} whole-problem evaluations over the "
                      f"workload's problems ({cells} cells), {t_used:.1f} s on one core"}


# Levels = 1 column of the paper's Tables case1-li, case1-nli and ndt
# (uniform grids): average linear and nonlinear iterations per step, the
# number of steps and the final time of those runs.
PAPER_UNIFORM = {32: (7.68, 2.99, 1334, 1.0), 64: (7.15, 2.96, 3253, 1.0),
                 128: (6.43, 2.61, 8207, 1.0), 256: (6.72, 3.04, 8698, 0.5)}


def paper_bench(n, t_final, limiter=0.5, base="mg", jvp="analytic", forcing=0):
    """The paper's model problem on a uniform n^3 grid integrated to t_final
    with BDF2 and PC.4.7 at its tolerance (eps_t = 5e-4 at 32^3, halved per
    doubling), Newton tolerances 1e-12 / 1e-10, FAC V(1,0), mixed precision;
    the last step is shortened to land on t_final."""
    from paper_1302_6303_amd import inputs as I, nrd
    w = I.paper_marshak(n)
    eps = 5e-4 * 32.0 / n
    opts = nrd.default_options(precision=nrd.NRD_MIXED, error_estimate=1,
                               newton_rtol=1e-12, newton_atol=1e-10, limiter=limiter,
                               fac_base=(nrd.NRD_BASE_SMOOTH if base == "smooth"
                                         else nrd.NRD_BASE_MG),
                               jvp_mode=nrd.NRD_JVP_FD if jvp == "fd" else nrd.NRD_JVP_ANALYTIC,
                               newton_forcing=forcing)
    H = nrd.Hierarchy(w.problems, w.boxes, opts)
    u = compact_state(w)
    m = H.ncells
    H.set_fields(to_dev(u[:m]), to_dev(u[m:]), to_dev(w.compact(w.z)))
    H.autotune(None)
    t, dt = 0.0, float(w.dt[0])
    steps = newton = krylov = cuts = 0
    t0 = time.perf_counter()
    while t < t_final * (1.0 - 1e-12):
        dt = min(dt, t_final - t)
        _, dtn, tt, st = H.adaptive_steps(1, [dt], eps, t=[t])
        s = st[0][0]
        steps += 1
        newton += s["newton_iters"]
        krylov += s["krylov_iters"]
        cuts += s["positivity_cuts"]
        t, dt = tt[0], dtn[0]
        if steps % 500 == 0:
            log(f"paper{n}: step {steps}, t = {t:.4g}, dt = {dt:.3g}")
    wall = time.perf_counter() - t0
    ref = PAPER_UNIFORM.get(n)
    out = {"metric": f"seconds to t = {t_final:g}, paper model problem, uniform {n}^3",
           "value": round(wall, 3), "unit": "s", "n_gpus": 1, "higher_is_better": False,
           "dtype": "f64", "data": "synthetic",
           "config": {"workload": f"paper{n}", "cells": n ** 3, "eps_t": eps,
                      "limiter": limiter, "jvp": jvp,
                      "solver": "BDF2, PC.4.7, Newton rtol 1e-12 atol 1e-10, FGMRES(30), "
                                "FAC V(1,0) + " + ("base-level smoothing" if base == "smooth"
                                                    else "MG V(1,1)") + ", mixed precision"},
           "steps": steps, "t_final": t,
           "linear_per_step": round(krylov / steps, 3),
           "nonlinear_per_step": round(newton / steps, 3),
           "positivity_cuts": cuts, "ms_per_step": round(1e3 * wall / steps, 3),
           "paper_levels1": ({"linear_per_step": ref[0], "nonlinear_per_step": ref[1],
                              "steps": ref[2]} if ref and abs(t_final - ref[3]) < 1e-12
                             else None)}
    print(json.dumps(out), flush=True)


# The paper's efficiency tables (average linear and nonlinear iterations per
# step, steps to t = 1) for AMR runs: base n^3 and L levels -> (linear,
# nonlinear, steps).
PAPER_AMR = {(16, 2): (7.71, 2.99, 1333), (16, 3): (7.21, 2.96, 3251), (16, 4): (6.63, 2.64, 8204),
             (16, 5): (6.92, 2.71, 8697), (32, 2): (7.22, 2.96, 3251), (32, 3): (6.61, 2.63, 8204),
             (32, 4): (6.91, 2.71, 8704), (64, 2): (6.63, 2.64, 8204), (64, 3): (6.92, 2.71, 8704),
             (128, 2): (6.86, 2.72, 8734)}


def paper_amr_bench(n, nlev, t_final, every=10, tau=0.5, forcing=1, cycle=0):
    """The paper's model problem on a dynamically refined hierarchy: base
    n^3 and nlev levels, integrated to t_final with BDF2 and PC.4.7 at the
    tolerance of the finest resolution (eps_t = 5e-4 at 32^3, halved per
    doubling), Newton tolerances 1e-12 / 1e-10, mixed precision.  Every
    `every` steps the cells with tau^g or tau^c above tau are tagged (Sec. 5),
    grown by 2 cells and clustered (Berger-Rigoutsos, efficiency 0.7, sides
    4..24 tagged-level cells); a regrid (transfer, warm restart with
    re-solve) happens only when the boxes change."""
    import torch
    from paper_1302_6303_amd import inputs as I, nrd
    from paper_1302_6303_amd.regrid import Regridder
    w = I.paper_marshak(n)
    prob = w.problems[0]
    eps = 5e-4 * 32.0 / (n * 2 ** (nlev - 1))
    opts = nrd.default_options(precision=nrd.NRD_MIXED, error_estimate=1,
                               newton_rtol=1e-12, newton_atol=1e-10,
                               newton_forcing=forcing, fac_cycle=cycle)
    zfun = material_sampler(I.PAPER_BOXES)
    R = Regridder(opts, dict(tau_g=tau, tau_c=tau),
                  dict(max_levels=nlev, buffer=2, efficiency=0.7, min_side=4, max_side=24),
                  zfun)
    boxes = list(w.boxes)
    H = nrd.Hierarchy([prob], boxes, opts)
    m = H.ncells
    H.set_fields(torch.full((m,), I.E0, dtype=torch.float64, device="cuda"),
                 torch.full((m,), I.T0, dtype=torch.float64, device="cuda"),
                 zfun([prob], boxes))
    t, dt = 0.0, float(w.dt[0])
    steps = newton = krylov = cuts = 0
    regrids = rs_newton = rs_krylov = 0
    cells_sum = 0
    regrid_s = {"tag_cluster": 0.0, "create_transfer": 0.0, "resolve": 0.0}
    t0 = time.perf_counter()
    while t < t_final * (1.0 - 1e-12):
        if steps > 0 and steps % every == 0:
            ta = time.perf_counter()
            nb = R.boxes_for(H)
            regrid_s["tag_cluster"] += time.perf_counter() - ta
            key = sorted((b.level, tuple(b.lo), tuple(b.hi)) for b in nb)
            if key != sorted((b.level, tuple(b.lo), tuple(b.hi)) for b in boxes):
                Hn, boxes, info = R.regrid(H, nb)
                del H
                H = Hn
                regrids += 1
                rs_newton += info["resolve_newton"]
                rs_krylov += info["resolve_krylov"]
                regrid_s["create_transfer"] += info["create_transfer_s"]
                regrid_s["resolve"] += info["resolve_s"]
        dt = min(dt, t_final - t)
        _, dtn, tt, st = H.adaptive_steps(1, [dt], eps, t=[t])
        s = st[0][0]
        steps += 1
        newton += s["newton_iters"]
        krylov += s["krylov_iters"]
        cuts += s["positivity_cuts"]
        cells_sum += H.ncells
        t, dt = tt[0], dtn[0]
        if steps % 500 == 0:
            log(f"paper{n}b{nlev}l: step {steps}, t = {t:.4g}, dt = {dt:.3g}, "
                f"{len(boxes)} boxes, {H.ncells} cells, {regrids} regrids")
    wall = time.perf_counter() - t0
    ref = PAPER_AMR.get((n, nlev))
    out = {"metric": f"seconds to t = {t_final:g}, paper model problem, {n}^3 base, "
                     f"{nlev} levels",
           "value": round(wall, 3), "unit": "s", "n_gpus": 1, "higher_is_better": False,
           "dtype": "f64", "data": "synthetic",
           "config": {"workload": f"paper{n}b{nlev}l", "eps_t": eps, "regrid_every": every,
                      "tags": f"tau_g or tau_c > {tau}, grown by 2",
                      "solver": "BDF2, PC.4.7, Newton rtol 1e-12 atol 1e-10, FGMRES(30), "
                                + ("AFACx" if cycle else "FAC V(1,0)")
                                + " + MG V(1,1), mixed precision"},
           "steps": steps, "t_final": t,
           "linear_per_step": round(krylov / steps, 3),
           "nonlinear_per_step": round(newton / steps, 3),
           "regrids": regrids, "resolve_newton": rs_newton, "resolve_krylov": rs_krylov,
           "regrid_s": {k: round(v, 2) for k, v in regrid_s.items()},
           "positivity_cuts": cuts, "ms_per_step": round(1e3 * wall / steps, 3),
           "mean_cells": round(cells_sum / steps), "final_boxes": len(boxes),
           "paper": ({"linear_per_step": ref[0], "nonlinear_per_step": ref[1], "steps": ref[2]}
                     if ref and abs(t_final - 1.0) < 1e-12 else None)}
    print(json.dumps(out), flush=True)


# Row 128b1l of the paper's spatial-accuracy table (uniform 128^3 against
# a uniform 256^3 reference run with the same time steps): L2 errors of E
# and T at these times.
PAPER_SPATIAL_T = (0.04, 0.10, 0.19, 0.25, 0.35, 0.46)
PAPER_SPATIAL_128 = {"E": (2.38e-2, 1.39e-2, 1.17e-2, 1.11e-2, 1.44e-2, 2.29e-2),
                     "T": (5.53e-3, 4.43e-3, 5.45e-3, 7.63e-3, 1.11e-2, 1.64e-2)}
# its row 16b1l (uniform 16^3)
PAPER_SPATIAL_16 = {"E": (6.01e-2, 3.32e-1, 4.55e-1, 4.99e-1, 4.49e-1, 3.77e-1),
                    "T": (3.15e-2, 1.52e-1, 2.21e-1, 2.32e-1, 2.23e-1, 2.06e-1)}
# The same for the paper's single-material runs (z = 1 everywhere).
PAPER_SPATIAL_T_Z1 = (0.05, 0.11, 0.19, 0.27, 0.36, 0.45)
PAPER_SPATIAL_128_Z1 = {"E": (1.94e-2, 1.30e-2, 1.08e-2, 1.07e-2, 1.06e-2, 9.12e-3),
                        "T": (5.15e-3, 4.37e-3, 3.91e-3, 3.81e-3, 4.14e-3, 4.19e-3)}


def paper_spatial_bench(limiter=0.5, single_material=False):
    """Spatial error of the uniform 128^3 grid on the paper's model problem:
    a 256^3 run with PC.4.7 (steps shortened to land on the table's times)
    records its step sizes and its fields at those times, averaged onto the
    128^3 cells; the 128^3 run repeats the same steps; the error is the
    volume-weighted L2 norm of the difference (unit cube)."""
    import torch
    from paper_1302_6303_amd import inputs as I, nrd

    times = PAPER_SPATIAL_T_Z1 if single_material else PAPER_SPATIAL_T
    paper = PAPER_SPATIAL_128_Z1 if single_material else PAPER_SPATIAL_128

    def make_h(n, estimate):
        w = I.paper_marshak(n, single_material=single_material)
        o = nrd.default_options(precision=nrd.NRD_MIXED, error_estimate=estimate,
                                newton_rtol=1e-12, newton_atol=1e-10, limiter=limiter)
        H = nrd.Hierarchy(w.problems, w.boxes, o)
        u = compact_state(w)
        m = H.ncells
        H.set_fields(to_dev(u[:m]), to_dev(u[m:]), to_dev(w.compact(w.z)))
        H.autotune(None)
        return H, w

    def coarse(x, m=128):             # 256^3 compact (x fastest) -> m^3 means
        r = 256 // m
        return x.view(m, r, m, r, m, r).mean(dim=(1, 3, 5))

    t0 = time.perf_counter()
    H, w = make_h(256, 1)
    t, dt = 0.0, float(w.dt[0])
    eps = 5e-4 * 32.0 / 256
    dts, ref = [], []
    for tg in times:
        while t < tg * (1.0 - 1e-12):
            dt = min(dt, tg - t)
            _, dtn, tt, st = H.adaptive_steps(1, [dt], eps, t=[t])
            dts.append(st[0][0]["dt"])
            t, dt = tt[0], dtn[0]
            if len(dts) % 500 == 0:
                log(f"256^3 reference: step {len(dts)}, t = {t:.4g}")
        E, T = H.get_fields()
        ref.append((coarse(E).clone(), coarse(T).clone(), len(dts),
                    coarse(E, 16).clone(), coarse(T, 16).clone()))
        log(f"256^3 reference at t = {t:.4g} after {len(dts)} steps")
    del H
    torch.cuda.empty_cache()
    allerr = {}
    for m, (iE, iT) in ((128, (0, 1)), (16, (3, 4))):
        H, _ = make_h(m, 0)
        errs = {"E": [], "T": []}
        k = 0
        for i, tg in enumerate(times):
            while k < ref[i][2]:             # the reference run's steps up to tg
                H.implicit_step([dts[k]])
                k += 1
            E, T = H.get_fields()
            for name, a, b in (("E", E, ref[i][iE]), ("T", T, ref[i][iT])):
                errs[name].append(float(torch.sqrt(torch.mean((a.view(m, m, m) - b) ** 2))))
            log(f"{m}^3 at t = {tg:.4g}: E error {errs['E'][-1]:.3e}, "
                f"T error {errs['T'][-1]:.3e}")
        allerr[m] = errs
        del H
    errs = allerr[128]
    out = {"metric": "L2 error of uniform 128^3 against 256^3 with the same steps, paper "
                     "model problem",
           "value": errs["E"][-1], "unit": "L2 (E, last time)", "n_gpus": 1,
           "higher_is_better": False, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "paper-spatial" + ("-z1" if single_material else ""),
                      "times": list(times), "limiter": limiter,
                      "steps": len(dts), "eps_t_256": eps},
           "errors": {kk: [round(v, 6) for v in vv] for kk, vv in errs.items()},
           "paper_128b1l": paper,
           "errors_16": {kk: [round(v, 6) for v in vv] for kk, vv in allerr[16].items()},
           "paper_16b1l": None if single_material else PAPER_SPATIAL_16,
           "wall_s": round(time.perf_counter() - t0, 1)}
    print(json.dumps(out), flush=True)


# The paper's temporal-accuracy table (fixed BDF2 steps against a 2.5e-5
# reference, equivalent 128^3 resolution): L2 errors of E and T.
PAPER_TEMPORAL_T = (0.05, 0.15, 0.25, 0.35, 0.45)
PAPER_TEMPORAL = {2e-4: {"E": (4.53e-5, 3.93e-5, 2.87e-5, 2.47e-5, 2.36e-5),
                         "T": (2.43e-5, 2.06e-5, 1.89e-5, 1.87e-5, 1.82e-5)},
                  1e-4: {"E": (1.13e-5, 9.80e-6, 7.10e-6, 6.10e-6, 5.80e-6),
                         "T": (6.00e-6, 5.10e-6, 4.70e-6, 4.60e-6, 4.50e-6)},
                  5e-5: {"E": (2.30e-6, 2.00e-6, 1.50e-6, 1.30e-6, 1.20e-6),
                         "T": (1.20e-6, 1.00e-6, 1.00e-6, 9.00e-7, 9.00e-7)}}


def paper_temporal_bench(n=128, dt_ref=2.5e-5, limiter=0.5, ramp=False):
    """Temporal error of fixed-step BDF2 (first step BDF1) on the paper's
    model problem, uniform n^3: runs with the table's steps against a run
    with dt_ref, volume-weighted L2 norms at the table's times."""
    import torch
    from paper_1302_6303_amd import inputs as I, nrd
    w = I.paper_marshak(n)
    o = nrd.default_options(precision=nrd.NRD_MIXED, newton_rtol=1e-12, newton_atol=1e-10,
                            limiter=limiter)
    H = nrd.Hierarchy(w.problems, w.boxes, o)
    u = compact_state(w)
    m = H.ncells
    E0, T0, z = to_dev(u[:m]), to_dev(u[m:]), to_dev(w.compact(w.z))
    H.set_fields(E0, T0, z)
    H.autotune(None)
    t0 = time.perf_counter()

    def run(dt):
        H.set_fields(E0, T0, z)                # resets the history: BDF1 first
        out, k = [], 0
        if ramp and dt > dt_ref:
            # first interval as dt/4 (BDF1), dt/4, dt/2: step ratios 1 and 2
            for d in (0.25 * dt, 0.25 * dt, 0.5 * dt):
                H.implicit_step([d])
            k = 1
        for tg in PAPER_TEMPORAL_T:
            kk = int(round(tg / dt))
            while k < kk:
                H.implicit_step([dt])
                k += 1
            E, T = H.get_fields()
            out.append((E.clone(), T.clone()))
        log(f"fixed step {dt:g}: {k} steps")
        return out

    ref = run(dt_ref)
    errs = {}
    for dt in sorted(PAPER_TEMPORAL, reverse=True):
        got = run(dt)
        errs[f"{dt:g}"] = {
            "E": [round(float(torch.sqrt(torch.mean((a[0] - b[0]) ** 2))), 9)
                  for a, b in zip(got, ref)],
            "T": [round(float(torch.sqrt(torch.mean((a[1] - b[1]) ** 2))), 9)
                  for a, b in zip(got, ref)]}
    out = {"metric": f"L2 temporal error of fixed-step BDF2 against dt = {dt_ref:g}, paper "
                     f"model problem, uniform {n}^3",
           "value": errs[f"{min(PAPER_TEMPORAL):g}"]["E"][-1], "unit": "L2 (E, smallest step)",
           "n_gpus": 1, "higher_is_better": False, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "paper-temporal", "cells": n ** 3, "limiter": limiter,
                      "ramp": ramp,
                      "times": list(PAPER_TEMPORAL_T), "dt_ref": dt_ref},
           "errors": errs,
           "paper": {f"{k:g}": v for k, v in PAPER_TEMPORAL.items()},
           "wall_s": round(time.perf_counter() - t0, 1)}
    print(json.dumps(out), flush=True)


def adjoint_bench(nsteps, every, reps=20):
    """Forward BDF1 trajectory, checkpointed discrete adjoint of the sum of E
    at the final time, and the transpose kernel alone, on the 64^3 smooth
    random material field (float64 throughout)."""
    import numpy as np
    import torch
    from paper_1302_6303_amd import inputs as I, nrd
    w = I.differentiation(n=64, nsteps=nsteps)
    opts = nrd.default_options(precision=nrd.NRD_FP64, bdf_max_order=1,
                               adjoint_slots=-(-nsteps // every) + every + 3)
    H = nrd.Hierarchy(w.problems, w.boxes, opts)
    u = compact_state(w)
    n = H.ncells
    z = to_dev(w.compact(w.z))
    H.set_fields(to_dev(u[:n]), to_dev(u[n:]), z)
    H.autotune(None)
    dt = [float(w.dt[0])]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    newton = krylov = 0
    for i in range(nsteps):
        _, st = H.implicit_step(dt)
        newton += st[0]["newton_iters"]
        krylov += st[0]["krylov_iters"]
    torch.cuda.synchronize()
    fwd = time.perf_counter() - t0
    log(f"forward {nsteps} steps: {fwd:.3f} s")
    H.set_fields(to_dev(u[:n]), to_dev(u[n:]), z)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    gz = H.adjoint_run(dt, nsteps, every)
    torch.cuda.synchronize()
    adj = time.perf_counter() - t0
    log(f"forward + reverse: {adj:.3f} s")
    # transpose kernel alone
    H.begin_step(dt)
    U = H.unpack(to_dev(u))
    L = H.unpack(to_dev(np.random.default_rng(1).standard_normal(u.shape)))
    G = H.native()
    g = H.compact(1)
    for _ in range(3):
        H.vjp(U, L, G, g)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        H.vjp(U, L, G, g)
    e1.record()
    torch.cuda.synchronize()
    vjp_ms = e0.elapsed_time(e1) / reps
    out = {"metric": "adjoint s/step, 64^3 BDF1, checkpointed transpose-Jacobian FGMRES",
           "value": round((adj - fwd) / nsteps, 5), "unit": "s/step", "n_gpus": 1,
           "steps": nsteps, "higher_is_better": False, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "differentiation", "cells": n, "ckpt_every": every},
           "forward_s_per_step": round(fwd / nsteps, 5),
           "forward_plus_adjoint_s": round(adj, 4),
           "forward_newton_per_step": newton / nsteps, "forward_krylov_per_step": krylov / nsteps,
           "vjp_ms": round(vjp_ms, 4), "vjp_gcells_per_s": round(n / vjp_ms / 1e6, 2),
           "grad_norm": float(torch.linalg.norm(gz))}
    print(json.dumps(out), flush=True)


def material_sampler(mboxes):
    """zfun(problems, boxes): the compact material field of a box list on the
    device (z of the last material box holding a cell centre, 1 elsewhere;
    the same rule and arithmetic as inputs.box_field), evaluated for all
    cells at once from their flat compact index."""
    def zfun(problems, boxes):
        import torch
        dev = "cuda"
        ext = torch.tensor([[b.hi[d] - b.lo[d] for d in range(3)] for b in boxes],
                           dtype=torch.int64, device=dev)
        lo = torch.tensor([list(b.lo) for b in boxes], dtype=torch.int64, device=dev)
        h = torch.tensor([list(problems[b.problem].h(b.level)) for b in boxes],
                         dtype=torch.float64, device=dev)
        plo = torch.tensor([list(problems[b.problem].lo) for b in boxes],
                           dtype=torch.float64, device=dev)
        n = ext.prod(dim=1)
        start = torch.cumsum(n, 0) - n
        idx = torch.arange(int(n.sum()), dtype=torch.int64, device=dev)
        bid = torch.searchsorted(start, idx, right=True) - 1
        loc = idx - start[bid]
        e = ext[bid]
        ijk = torch.stack([loc % e[:, 0], (loc // e[:, 0]) % e[:, 1],
                           loc // (e[:, 0] * e[:, 1])], dim=1)
        X = [(ijk[:, d] + lo[bid, d]).to(torch.float64) for d in range(3)]
        X = [(X[d] + 0.5) * h[bid, d] + plo[bid, d] for d in range(3)]
        z = torch.ones_like(X[0])
        for blo, bhi, zv in mboxes:
            m = ((X[0] >= blo[0]) & (X[0] < bhi[0]) & (X[1] >= blo[1]) & (X[1] < bhi[1])
                 & (X[2] >= blo[2]) & (X[2] < bhi[2]))
            z[m] = zv
        return z
    return zfun


def dynamic_bench(steps, every, plain_steps, base=128, nlev=4, dt0=1e-5, adaptive_eps=None,
                  tune=True, fac_cycle=0):
    """Dynamic 4-level AMR (128^3 base, six z = 10 boxes), the paper's cold
    start (E = E0, T = T0, Marshak inflow at x = 0): steps BDF steps (BDF1
    first) of dt0 (a step whose Newton solve fails is retried with half the
    step; steps of 5e-4 stall this hierarchy's Newton solves on the cold
    front), or with adaptive_eps the paper's PC.4.7 control from a first
    step dt0; a regrid every `every` steps on |grad E| / E > 10 or a
    material interface (tags grown by 2 cells, Berger-Rigoutsos boxes of
    4..24 tagged-level cells, i.e. 8..48 cells per side), each followed by
    the warm-restart re-solve (whose step's error estimate is skipped).
    Runs the mixed-precision batched solver, replays the same boxes and the
    same step sizes with the float64 batched solver (the solution
    difference and the Krylov counts) and the first plain_steps with the
    float64 per-patch solver (its seconds per step).  fac_cycle: P1's cycle
    (NRD_FAC_MULT or NRD_FAC_AFACX) in every run."""
    import numpy as np
    import tempfile
    import torch
    from paper_1302_6303_amd import inputs as I, nrd
    from paper_1302_6303_amd.regrid import Regridder
    rng = np.random.default_rng(I.SEED_BASE + 3)
    mboxes = I.sample_material_boxes(rng, 6)
    prob = I.Problem((base, base, base))
    zfun = material_sampler(mboxes)
    crit = dict(grad_E=10.0, z_interface=True)
    clus = dict(max_levels=nlev, buffer=2, efficiency=0.7, min_side=4, max_side=24)
    cache = os.path.join(tempfile.mkdtemp(prefix="nrd_tiles_"), "tiles.txt") if tune else None

    def initial_boxes():
        """Level by level on the initial (uniform) state: only the material
        interfaces are tagged."""
        opts = nrd.default_options(precision=nrd.NRD_MIXED)
        R = Regridder(opts, crit, clus, zfun)
        boxes = [I.Box(0, 0, (0, 0, 0), (base, base, base))]
        for _ in range(nlev - 1):
            H = nrd.Hierarchy([prob], boxes, opts)
            n = H.ncells
            H.set_fields(torch.full((n,), I.E0, dtype=torch.float64, device="cuda"),
                         torch.full((n,), I.T0, dtype=torch.float64, device="cuda"),
                         zfun([prob], boxes))
            boxes = R.boxes_for(H)
            del H
        return boxes

    def run(opts, nsteps, plan=None, label="", timers=False):
        """plan: (box lists per regrid, step sizes) to replay, else recorded."""
        opts.fac_cycle = fac_cycle
        dt = dt0
        R = Regridder(opts, crit, clus, zfun, tune_cache=cache if tune else None)
        boxes = plan[0][0] if plan else initial_boxes()
        H = nrd.Hierarchy([prob], boxes, opts)
        n = H.ncells
        H.set_fields(torch.full((n,), I.E0, dtype=torch.float64, device="cuda"),
                     torch.full((n,), I.T0, dtype=torch.float64, device="cuda"),
                     zfun([prob], boxes))
        if tune:
            H.autotune(cache)
        rec_boxes, rec_dt, regrids = [boxes], [], []
        step_s = []
        newton = krylov = 0
        res_ms = res_cnt = res_cells = 0.0
        for k in range(nsteps):
            if k > 0 and k % every == 0:
                if timers:
                    ms, cnt = H.timer_read(nrd.NRD_TIMER_RESIDUAL)
                    res_ms += ms
                    res_cnt += cnt
                    res_cells += H.timer_cells(nrd.NRD_TIMER_RESIDUAL)
                nb = plan[0][len(rec_boxes)] if plan else None
                Hn, nb, info = R.regrid(H, nb)
                del H
                H = Hn
                rec_boxes.append(nb)
                regrids.append(info)
                newton += info["resolve_newton"]
                krylov += info["resolve_krylov"]
                log(f"{label} regrid at step {k}: {info['boxes']} boxes, "
                    f"{info['cells']} cells, {info['tag_cluster_s']:.2f} s tag+cluster, "
                    f"{info['create_transfer_s']:.2f} s create+transfer, "
                    f"{info['timed_classes']} classes tuned in {info['tune_s']:.2f} s, "
                    f"re-solve {info['resolve_newton']} Newton in {info['resolve_s']:.2f} s")
            if timers and (k == 0 or k % every == 0):
                H.timer_enable(True)
                torch.cuda.synchronize()
            t0 = time.perf_counter()
            if plan:
                d = plan[1][k]
                _, st = H.implicit_step([d])
            elif adaptive_eps:
                _, dtn, _, stp = H.adaptive_steps(1, [dt], adaptive_eps)
                st = stp[0]
                d, dt = st[0]["dt"], dtn[0]
            else:
                d = dt0
                for _ in range(8):
                    rc, st = H.implicit_step([d], raise_on_fail=False)
                    if rc == 0:
                        break
                    d *= 0.5
                else:
                    raise RuntimeError(f"{label}: step {k + 1} failed after 8 halvings")
            step_s.append(time.perf_counter() - t0)
            rec_dt.append(d)
            newton += st[0]["newton_iters"]
            krylov += st[0]["krylov_iters"]
            log(f"{label} step {k + 1}: dt {d:.3g}, newton {st[0]['newton_iters']}, krylov "
                f"{st[0]['krylov_iters']}, {step_s[-1] * 1e3:.1f} ms")
        out = {"s_per_step": float(np.mean(step_s)), "median_s_per_step": float(np.median(step_s)),
               "newton": newton, "krylov": krylov,
               "krylov_per_newton": krylov / max(newton, 1),
               "regrids": regrids, "final_boxes": len(rec_boxes[-1]), "final_cells": H.ncells}
        if timers:
            ms, cnt = H.timer_read(nrd.NRD_TIMER_RESIDUAL)
            res_ms += ms
            res_cnt += cnt
            res_cells += H.timer_cells(nrd.NRD_TIMER_RESIDUAL)
            H.timer_enable(False)
            out["residual_ms_avg"] = res_ms / max(res_cnt, 1)
            out["residual_cells_avg"] = res_cells / max(res_cnt, 1)
            out["residual_launches"] = int(res_cnt)
        E, T = H.get_fields()
        return H, torch.cat([E, T]), (rec_boxes, rec_dt), out

    mixed_opts = nrd.default_options(precision=nrd.NRD_MIXED,
                                     error_estimate=1 if adaptive_eps else 0)
    H, u_mixed, plan, mixed = run(mixed_opts, steps, label="mixed", timers=True)
    mixed["dt"] = [float(f"{x:.4g}") for x in plan[1]]
    mixed["t_final"] = float(sum(plan[1]))
    # operators on the final hierarchy, every launch covering every cell
    ops = operator_times(H, [plan[1][-1]])
    comp = H.ncells - covered_count(H)
    del H
    torch.cuda.empty_cache()
    H64, u64, _, fp64 = run(nrd.default_options(precision=nrd.NRD_FP64), steps, plan=plan,
                            label="fp64 batched")
    diff = {}
    for name, sl in (("E", slice(0, H64.ncells)), ("T", slice(H64.ncells, None))):
        diff[name] = float(torch.linalg.vector_norm(u_mixed[sl] - u64[sl]) /
                           torch.linalg.vector_norm(u64[sl]))
    del H64
    torch.cuda.empty_cache()
    plain = None
    if plain_steps > 0:
        Hp, _, _, plain = run(nrd.default_options(precision=nrd.NRD_FP64,
                                                  launch=nrd.NRD_PER_PATCH, stencil=1),
                              plain_steps, plan=plan, label="fp64 per-patch")
        del Hp
        torch.cuda.empty_cache()
    return mixed, fp64, plain, ops, comp, diff, plan


def covered_count(H):
    """Covered cells of a hierarchy (host count from its boxes)."""
    tot = 0
    for b in H.boxes:
        for c in H.boxes:
            if c.problem == b.problem and c.level == b.level + 1:
                ov = 1
                for d in range(3):
                    ov *= max(0, min(c.hi[d] // 2, b.hi[d]) - max(c.lo[d] // 2, b.lo[d]))
                tot += ov
    return tot


def operator_times(H, dt, reps=20):
    """Residual, Jacobian action, preconditioner and base-grid sweeps timed
    with the library's event timers over every problem (3 warm-up calls)."""
    import torch
    from paper_1302_6303_amd import nrd
    H.begin_step(dt)
    E, T = H.get_fields()
    U = H.unpack(torch.cat([E, T]))
    V = H.unpack(torch.cat([E, T]) * 1e-3)
    Y = H.native()
    H.precond_setup(U)
    for _ in range(3):
        H.residual(U, Y)
        H.jvp(U, V, Y)
        H.precond_apply(V, Y)
    torch.cuda.synchronize()
    H.timer_enable(True)
    for _ in range(reps):
        H.residual(U, Y)
    for _ in range(reps):
        H.jvp(U, V, Y)
    for _ in range(reps):
        H.precond_apply(V, Y)
    res = {}
    for key, which in (("residual", nrd.NRD_TIMER_RESIDUAL), ("jvp", nrd.NRD_TIMER_JVP),
                       ("precond", nrd.NRD_TIMER_PRECOND), ("sweep", nrd.NRD_TIMER_SMOOTH),
                       ("sweep_zero", nrd.NRD_TIMER_SMOOTH_ZERO)):
        ms, cnt = H.timer_read(which)
        res[key + "_ms_avg"] = ms / max(cnt, 1)
    H.timer_enable(False)
    return res


def dynamic_main(a):
    steps = a.steps if a.steps_given else 50
    dt0 = a.dt if a.dt else 1e-5
    from paper_1302_6303_amd import nrd
    cycle = nrd.NRD_FAC_AFACX if a.fac_cycle == "afacx" else nrd.NRD_FAC_MULT
    mixed, fp64, plain, ops, comp, diff, plan = dynamic_bench(
        steps, a.regrid_every, 0 if a.no_plain else a.plain_steps, dt0=dt0,
        adaptive_eps=a.adaptive_eps, tune=a.tune, fac_cycle=cycle)
    res_s = mixed["residual_ms_avg"] / 1e3
    cells = mixed["residual_cells_avg"]
    achieved = BYTES_PER_CELL_RESIDUAL * cells / res_s / 1e9
    def rnd(d):
        return {k: (round(v, 5) if isinstance(v, float) else v) for k, v in d.items()
                if k != "regrids"}
    out = {
        "metric": "residual Gcells/s (%HBM peak) + s/implicit step, mixed-batched vs FP64 plain",
        "value": round(cells / res_s / 1e9, 3), "unit": "Gcells/s", "n_gpus": 1,
        "steps": steps, "warmup": 0, "ms_per_step": round(mixed["s_per_step"] * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "dynamic", "base": 128, "levels": 4,
                   "regrid_every": a.regrid_every,
                   "time_control": (f"PC.4.7, eps_t {a.adaptive_eps}, first step {dt0}"
                                    if a.adaptive_eps else
                                    f"fixed steps {dt0} (halved on a failed solve)"),
                   "tags": "|grad E|/E > 10 or material interface, grown by 2",
                   "clustering": "Berger-Rigoutsos, efficiency 0.7, sides 8..48 cells",
                   "final_boxes": mixed["final_boxes"], "final_cells": mixed["final_cells"],
                   "final_composite_cells": comp,
                   "solver": "BDF1->BDF2, Newton rtol 1e-8, FGMRES(30), %s RBGS + MG V(1,1)"
                             % ("AFACx m = 1" if a.fac_cycle == "afacx" else "FAC V(1,0)")},
        "roofline": {"bound": "hbm", "kernel": "k_stencil_s<0> (residual)",
                     "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                     "bytes_per_cell": BYTES_PER_CELL_RESIDUAL,
                     "cells_per_launch": round(cells),
                     "avg_launch_ms": round(mixed["residual_ms_avg"], 4),
                     "full_launch_final_hierarchy": {
                         "cells": comp, "avg_launch_ms": round(ops["residual_ms_avg"], 4),
                         "frac": round(BYTES_PER_CELL_RESIDUAL * comp / ops["residual_ms_avg"]
                                       / 1e6 / HBM_PEAK_GBS, 4)}},
        "jvp_roofline": {"frac": round(BYTES_PER_CELL_JVP * comp / ops["jvp_ms_avg"] / 1e6
                                       / HBM_PEAK_GBS, 4),
                         "avg_launch_ms": round(ops["jvp_ms_avg"], 4)},
        "precond_ms_avg": round(ops["precond_ms_avg"], 4),
        "mixed_batched": rnd(mixed),
        "fp64_batched_replay": rnd(fp64),
        "mixed_vs_fp64_rel_diff_after_steps": diff,
        "regrids": mixed["regrids"],
        "regrid_s_total": round(sum(r["tag_cluster_s"] + r["create_transfer_s"] + r["tune_s"]
                                    for r in mixed["regrids"]), 3),
        "resolve_s_total": round(sum(r["resolve_s"] for r in mixed["regrids"]), 3),
    }
    if plain is not None:
        out["fp64_plain_first_steps"] = rnd(plain)
        out["speedup_mixed_batched_vs_fp64_plain"] = round(plain["s_per_step"] /
                                                           mixed["s_per_step"], 3)
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=4)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="ensemble")
    ap.add_argument("--no-plain", action="store_true", help="skip the FP64 per-patch run")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="end with a 2 GiB device copy (reference for HBM byte counters)")
    ap.add_argument("--graph", type=int, default=0,
                    help="1: capture FGMRES iterations as HIP graphs in the mixed run "
                         "(measured slower than direct launches on this software stack)")
    ap.add_argument("--bdf-max-order", type=int, default=2,
                    help="2: BDF1 first step then BDF2; 1: BDF1 throughout")
    ap.add_argument("--dt-scale", type=float, default=1.0,
                    help="multiplies every problem's time step")
    ap.add_argument("--adaptive-eps", type=float, default=None,
                    help="PC.4.7 time-step control with this local error tolerance "
                         "(eps_t; the paper uses 5e-4 at 32^3 resolution, halved per "
                         "doubling); default: the workload's fixed time steps")
    ap.add_argument("--ckpt-every", type=int, default=10,
                    help="adjoint workload: checkpoint interval")
    ap.add_argument("--fac-nu", type=int, nargs=2, default=(1, 0), metavar=("M", "N"),
                    help="FAC V(M, N): M down-sweep and N up-sweep red-black sweeps per "
                         "level above the base (default 1 0, the paper's V(1,0))")
    ap.add_argument("--mg-nu", type=int, nargs=2, default=(1, 1), metavar=("PRE", "POST"),
                    help="base multigrid V(PRE, POST) red-black sweeps per grid (default 1 1)")
    ap.add_argument("--fac-smoother", choices=("rbgs", "jacobi", "line"), default="rbgs",
                    help="FAC level smoother: red-black Gauss-Seidel (default), damped "
                         "point Jacobi or x-line block Gauss-Seidel")
    ap.add_argument("--forcing", choices=("petsc", "kelley"), default="petsc",
                    help="Eisenstat-Walker forcing terms of the Newton solves: PETSc's "
                         "choice 2 (default, the library's) or Kelley's choice")
    ap.add_argument("--fac-cycle", choices=("mult", "afacx"), default="mult",
                    help="P1 cycle on refined hierarchies: multiplicative FAC (default) or "
                         "AFACx (every level pair at once)")
    ap.add_argument("--limiter", type=float, default=0.5,
                    help="paper workloads: lambda of the flux limiter (0.5: the printed "
                         "pair, the library default; 1: Wilson form)")
    ap.add_argument("--fac-base", choices=("mg", "smooth"), default="mg",
                    help="paperN workloads: base level of FAC, a multigrid V-cycle (default) "
                         "or only level sweeps (the paper's runs)")
    ap.add_argument("--jvp", choices=("analytic", "fd"), default="analytic",
                    help="paperN workloads: Jacobian action, analytic (default) or the "
                         "paper's Jacobian-free difference quotient")
    ap.add_argument("--tau", type=float, default=0.5,
                    help="paperNbLl workloads: tagging threshold of tau^g and tau^c")
    ap.add_argument("--ramp", action="store_true",
                    help="paper-temporal: take each run's first interval as dt/4, dt/4, dt/2")
    ap.add_argument("--t-final", type=float, default=1.0,
                    help="paperN workloads: integrate the model problem to this time")
    ap.add_argument("--fp64-batched", action="store_true",
                    help="also time the FP64 solver with batched launches (per-patch vs "
                         "batched comparison at equal precision)")
    ap.add_argument("--dt", type=float, default=None,
                    help="dynamic workload: step size (default 1e-5; the first step with "
                         "--adaptive-eps)")
    ap.add_argument("--regrid-every", type=int, default=5,
                    help="dynamic workload: steps between regrids")
    ap.add_argument("--plain-steps", type=int, default=10,
                    help="dynamic workload: steps replayed with the FP64 per-patch solver")
    ap.add_argument("--tune", action="store_true",
                    help="dynamic workload: tune tile shapes of every new hierarchy through "
                         "one cache file (new patch-size classes only); default: the "
                         "default shapes")
    a = ap.parse_args()
    a.steps_given = "--steps" in sys.argv
    if a.gpus != 1:
        print("bench.py runs on exactly one GPU: the hot path is built and measured on a "
              "single GPU (sharding over several GPUs is a design note only)", file=sys.stderr)
        raise SystemExit(2)
    os.environ.setdefault("OMP_NUM_THREADS", "1")
    from paper_1302_6303_amd import nrd
    if a.workload == "adjoint":
        adjoint_bench(a.steps, a.ckpt_every)
        return
    if a.workload == "dynamic":
        dynamic_main(a)
        return
    if a.workload in ("paper-spatial", "paper-spatial-z1"):
        paper_spatial_bench(a.limiter, a.workload.endswith("z1"))
        return
    if a.workload == "paper-temporal":
        paper_temporal_bench(limiter=a.limiter, ramp=a.ramp)
        return
    mm = re.fullmatch(r"paper(\d+)b(\d+)l", a.workload)
    if mm:
        paper_amr_bench(int(mm.group(1)), int(mm.group(2)), a.t_final, tau=a.tau,
                        forcing=nrd.NRD_EW_PETSC if a.forcing == "petsc" else nrd.NRD_EW_KELLEY,
                        cycle=nrd.NRD_FAC_AFACX if a.fac_cycle == "afacx" else nrd.NRD_FAC_MULT)
        return
    if a.workload.startswith("paper"):
        paper_bench(int(a.workload[5:]), a.t_final, a.limiter, a.fac_base, a.jvp,
                    nrd.NRD_EW_PETSC if a.forcing == "petsc" else nrd.NRD_EW_KELLEY)
        return
    w = workload(a.workload)
    if a.dt_scale != 1.0:
        w.dt = w.dt * a.dt_scale
    ncomp = composite_cells(w)
    use_graph = a.graph
    smoother = {"rbgs": nrd.NRD_SMOOTH_RBGS, "jacobi": nrd.NRD_SMOOTH_JACOBI,
                "line": nrd.NRD_SMOOTH_LINE}[a.fac_smoother]
    cycle = nrd.NRD_FAC_AFACX if a.fac_cycle == "afacx" else nrd.NRD_FAC_MULT
    forcing = nrd.NRD_EW_PETSC if a.forcing == "petsc" else nrd.NRD_EW_KELLEY
    mixed = run_solver(w, nrd.default_options(precision=nrd.NRD_MIXED,
                                              launch=nrd.NRD_BATCHED, use_graph=use_graph,
                                              bdf_max_order=a.bdf_max_order,
                                              fac_nu_pre=a.fac_nu[0], fac_nu_post=a.fac_nu[1],
                                              fac_smoother=smoother, fac_cycle=cycle,
                                              newton_forcing=forcing, mg_nu_pre=a.mg_nu[0],
                                              mg_nu_post=a.mg_nu[1]),
                       a.steps, a.warmup, True, a.adaptive_eps)
    mixed["use_graph"] = use_graph
    plain = None
    if not a.no_plain:
        # per-patch launches need many workgroups per patch: the register
        # plane-marching stencil with short z chunks suits them best
        plain = run_solver(w, nrd.default_options(precision=nrd.NRD_FP64,
                                                  launch=nrd.NRD_PER_PATCH, stencil=1,
                                                  bdf_max_order=a.bdf_max_order,
                                                  fac_nu_pre=a.fac_nu[0], fac_nu_post=a.fac_nu[1],
                                                  fac_smoother=smoother, fac_cycle=cycle,
                                              newton_forcing=forcing, mg_nu_pre=a.mg_nu[0],
                                              mg_nu_post=a.mg_nu[1]),
                           a.steps, a.warmup, False, a.adaptive_eps)
    batched64 = None
    if a.fp64_batched:
        batched64 = run_solver(w, nrd.default_options(precision=nrd.NRD_FP64,
                                                      launch=nrd.NRD_BATCHED,
                                                      bdf_max_order=a.bdf_max_order,
                                                      fac_nu_pre=a.fac_nu[0], fac_nu_post=a.fac_nu[1],
                                                      fac_smoother=smoother, fac_cycle=cycle,
                                              newton_forcing=forcing, mg_nu_pre=a.mg_nu[0],
                                              mg_nu_post=a.mg_nu[1]),
                               a.steps, a.warmup, False, a.adaptive_eps)
    res_s = mixed["residual_ms_avg"] / 1e3
    res_cells = mixed["residual_cells_avg"]           # per launch, average
    gcells = res_cells / res_s / 1e9
    achieved = BYTES_PER_CELL_RESIDUAL * res_cells / res_s / 1e9
    traffic = None
    if (MEASURED_TRAFFIC and MEASURED_TRAFFIC["workload"] == a.workload
            and MEASURED_TRAFFIC["stencil_sha256"] == stencil_source_hash()):
        traffic = round(MEASURED_TRAFFIC["bytes_per_cell"] * res_cells)
    jvp_s = mixed["jvp_ms_avg"] / 1e3
    base_cells = sum(b.ncells for b in w.boxes if b.level == 0)
    def gbs(nbytes, ms):
        return round(nbytes / ms / 1e6, 1) if ms > 0 else None

    def frac(nbytes, ms):
        return round(nbytes / ms / 1e6 / HBM_PEAK_GBS, 4) if ms > 0 else None
    out = {
        "metric": "residual Gcells/s (%HBM peak) + s/implicit step, mixed-batched vs FP64 plain",
        "value": round(gcells, 3),
        "unit": "Gcells/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(mixed["s_per_step"] * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": a.workload, "problems": len(w.problems),
                   "boxes": len(w.boxes), "cells": w.ncells(),
                   "composite_cells": ncomp,
                   "dt_scale": a.dt_scale,
                   "time_control": (f"PC.4.7, eps_t {a.adaptive_eps}" if a.adaptive_eps
                                    else "fixed steps"),
                   "solver": ("BDF1->BDF2" if a.bdf_max_order == 2 else "BDF1") +
                             ", Newton rtol 1e-8 (%s forcing), FGMRES(30), %s V(%d,%d) %s"
                             " + MG V(%d,%d)"
                             % ("PETSc" if a.forcing == "petsc" else "Kelley",
                                "AFACx" if a.fac_cycle == "afacx" else "FAC",
                                a.fac_nu[0], a.fac_nu[1],
                                {"rbgs": "RBGS", "jacobi": "damped Jacobi",
                                 "line": "x-line block GS"}[a.fac_smoother],
                                a.mg_nu[0], a.mg_nu[1])},
        "roofline": {"bound": "hbm", "kernel": "k_stencil_s<0> (residual)",
                     "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "bytes_per_cell": BYTES_PER_CELL_RESIDUAL,
                     "cells_per_launch": round(res_cells),
                     "bytes_per_launch": round(BYTES_PER_CELL_RESIDUAL * res_cells),
                     "avg_launch_ms": round(mixed["residual_ms_avg"], 4),
                     "full_launch": {
                         "cells": ncomp,
                         "avg_launch_ms": round(mixed["residual_full_ms_avg"], 4),
                         "achieved": round(BYTES_PER_CELL_RESIDUAL * ncomp /
                                           mixed["residual_full_ms_avg"] / 1e6, 1),
                         "frac": round(BYTES_PER_CELL_RESIDUAL * ncomp /
                                       mixed["residual_full_ms_avg"] / 1e6 / HBM_PEAK_GBS, 4)}},
        "jvp_roofline": {"kernel": "k_stencil_s<1> (Jacobian action)",
                         "achieved": round(BYTES_PER_CELL_JVP * ncomp / jvp_s / 1e9, 1),
                         "unit": "GB/s",
                         "frac": round(BYTES_PER_CELL_JVP * ncomp / jvp_s / 1e9 / HBM_PEAK_GBS, 4),
                         "avg_launch_ms": round(mixed["jvp_ms_avg"], 4)},
        "smoother_roofline": {
            "kernel": "k_level<float> (red-black sweep of the base grid, one launch per colour, "
                      "colour-split iterate and right-hand side, T-field face coefficients "
                      "recomputed from T)",
            "cells": base_cells, "bytes_per_cell": BYTES_PER_CELL_SWEEP,
            "achieved": gbs(BYTES_PER_CELL_SWEEP * base_cells, mixed["sweep_ms_avg"]),
            "unit": "GB/s",
            "frac": frac(BYTES_PER_CELL_SWEEP * base_cells, mixed["sweep_ms_avg"]),
            "avg_sweep_ms": round(mixed["sweep_ms_avg"], 4),
            "zero_start": {
                "bytes_per_cell": BYTES_PER_CELL_SWEEP_ZERO,
                "achieved": gbs(BYTES_PER_CELL_SWEEP_ZERO * base_cells,
                                mixed["sweep_zero_ms_avg"]),
                "frac": frac(BYTES_PER_CELL_SWEEP_ZERO * base_cells, mixed["sweep_zero_ms_avg"]),
                "avg_sweep_ms": round(mixed["sweep_zero_ms_avg"], 4)}},
        "mixed_batched": {k: (round(v, 5) if isinstance(v, float) else v)
                          for k, v in mixed.items()},
    }
    if plain is not None:
        out["fp64_plain"] = {k: (round(v, 5) if isinstance(v, float) else v)
                             for k, v in plain.items()}
        out["speedup_mixed_batched_vs_fp64_plain"] = round(plain["s_per_step"] /
                                                           mixed["s_per_step"], 3)
    if batched64 is not None:
        out["fp64_batched"] = {k: (round(v, 5) if isinstance(v, float) else v)
                               for k, v in batched64.items()}
        if plain is not None:
            out["speedup_fp64_batched_vs_fp64_plain"] = round(plain["s_per_step"] /
                                                              batched64["s_per_step"], 3)
    if not a.no_cpu:
        out["cpu_baseline"] = cpu_baseline(w)
    if a.copy_calibration:
        copy_calibration()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
