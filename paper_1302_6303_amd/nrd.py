"""ctypes binding of libnrd.so (the C ABI in include/nrd.h).

Argument marshalling only: every step of the computation runs in the HIP
library.  PyTorch supplies device memory (the workspace and the vectors)
and the stream.  Importing this module fails loudly if the library has not
been built.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import List, Optional, Sequence

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libnrd.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with "
                      "`python -m paper_1302_6303_amd.build`")
# torch ships its own HIP runtime (soname libamdhip64.so.7); loading it first
# makes libnrd.so resolve to that same runtime instead of a second copy.
import torch  # noqa: E402,F401
_lib = C.CDLL(LIB_PATH)

NRD_OK, NRD_EINVAL, NRD_ENESTING, NRD_ESTATE = 0, -1, -2, -3
NRD_ENONPOS, NRD_ENOTCONV, NRD_EDEVICE, NRD_EUNSUPPORTED = -4, -5, -6, -7
NRD_FP64, NRD_MIXED = 0, 1
NRD_BATCHED, NRD_PER_PATCH = 0, 1
NRD_SMOOTH_RBGS, NRD_SMOOTH_JACOBI, NRD_SMOOTH_LINE = 0, 1, 2
NRD_BASE_MG, NRD_BASE_SMOOTH = 0, 1
NRD_FAC_MULT, NRD_FAC_AFACX = 0, 1
NRD_EW_KELLEY, NRD_EW_PETSC = 0, 1
NRD_JVP_ANALYTIC, NRD_JVP_FD = 0, 1
NRD_TIMER_RESIDUAL, NRD_TIMER_JVP, NRD_TIMER_PRECOND = 0, 1, 2
NRD_TIMER_SMOOTH, NRD_TIMER_SMOOTH_ZERO = 3, 4


class nrd_box(C.Structure):
    _fields_ = [("problem", C.c_int32), ("level", C.c_int32),
                ("lo", C.c_int32 * 3), ("hi", C.c_int32 * 3)]


class nrd_problem(C.Structure):
    _fields_ = [("base_n", C.c_int32 * 3), ("lo", C.c_double * 3),
                ("hi", C.c_double * 3), ("bc_E", C.c_int32 * 6),
                ("robin_R", C.c_double * 6), ("kappa", C.c_double)]


class nrd_options(C.Structure):
    _fields_ = [("precision", C.c_int32), ("launch", C.c_int32),
                ("use_graph", C.c_int32), ("jvp_mode", C.c_int32),
                ("limiter", C.c_double), ("p2_mode", C.c_int32),
                ("newton_rtol", C.c_double), ("newton_atol", C.c_double),
                ("newton_maxit", C.c_int32), ("gmres_restart", C.c_int32),
                ("gmres_maxrestarts", C.c_int32), ("mg_nu_pre", C.c_int32),
                ("mg_nu_post", C.c_int32), ("adjoint_slots", C.c_int32),
                ("stencil", C.c_int32), ("zchunk", C.c_int32),
                ("bdf_max_order", C.c_int32), ("error_estimate", C.c_int32),
                ("fac_nu_pre", C.c_int32), ("fac_nu_post", C.c_int32),
                ("fac_smoother", C.c_int32), ("err_eta_E", C.c_double),
                ("err_eta_T", C.c_double), ("fac_base", C.c_int32), ("fac_cycle", C.c_int32),
                ("newton_forcing", C.c_int32), ("pad_", C.c_int32)]


class nrd_step_stats(C.Structure):
    _fields_ = [("newton_iters", C.c_int32), ("krylov_iters", C.c_int32),
                ("positivity_cuts", C.c_int32), ("converged", C.c_int32),
                ("fnorm0", C.c_double), ("fnorm", C.c_double),
                ("krylov_per_newton", C.c_int32 * 24),
                ("dt", C.c_double), ("err_norm", C.c_double)]

    def as_dict(self):
        return {"newton_iters": self.newton_iters,
                "krylov_iters": self.krylov_iters,
                "positivity_cuts": self.positivity_cuts,
                "converged": bool(self.converged), "fnorm0": self.fnorm0,
                "fnorm": self.fnorm,
                "krylov_per_newton": list(self.krylov_per_newton[:self.newton_iters]),
                "dt": self.dt, "err_norm": self.err_norm}


NRD_CTL_PC47, NRD_CTL_EPS = 0, 1


class nrd_tagging(C.Structure):
    _fields_ = [("grad_E", C.c_double), ("tau_g", C.c_double), ("tau_c", C.c_double),
                ("z_interface", C.c_int32), ("pad_", C.c_int32)]


class nrd_cluster_opt(C.Structure):
    _fields_ = [("max_levels", C.c_int32), ("buffer", C.c_int32),
                ("efficiency", C.c_double), ("min_side", C.c_int32),
                ("max_side", C.c_int32)]


class nrd_timectl(C.Structure):
    _fields_ = [("eps", C.c_double), ("ratio_min", C.c_double),
                ("ratio_max", C.c_double), ("controller", C.c_int32),
                ("max_halvings", C.c_int32)]


_H = C.c_void_p
_P = C.c_void_p
_sigs = {
    "nrd_last_error": (C.c_char_p, []),
    "nrd_default_options": (None, [C.POINTER(nrd_options)]),
    "nrd_hierarchy_create": (C.c_int32, [C.POINTER(nrd_problem), C.c_int32,
                                         C.POINTER(nrd_box), C.c_int32,
                                         C.POINTER(nrd_options), _P, C.POINTER(_H)]),
    "nrd_hierarchy_destroy": (C.c_int32, [_H]),
    "nrd_workspace_size": (C.c_int32, [_H, C.POINTER(C.c_size_t)]),
    "nrd_bind_workspace": (C.c_int32, [_H, _P, C.c_size_t]),
    "nrd_layout": (C.c_int32, [_H, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
    "nrd_pack": (C.c_int32, [_H, _P, _P]),
    "nrd_unpack": (C.c_int32, [_H, _P, _P]),
    "nrd_set_fields": (C.c_int32, [_H, _P, _P, _P]),
    "nrd_get_fields": (C.c_int32, [_H, _P, _P]),
    "nrd_begin_step": (C.c_int32, [_H, C.POINTER(C.c_double)]),
    "nrd_residual": (C.c_int32, [_H, _P, _P]),
    "nrd_jvp": (C.c_int32, [_H, _P, _P, _P]),
    "nrd_precond_setup": (C.c_int32, [_H, _P]),
    "nrd_precond_apply": (C.c_int32, [_H, _P, _P]),
    "nrd_vjp": (C.c_int32, [_H, _P, _P, _P, _P]),
    "nrd_implicit_step": (C.c_int32, [_H, C.POINTER(C.c_double),
                                      C.POINTER(nrd_step_stats)]),
    "nrd_adaptive_steps": (C.c_int32, [_H, C.POINTER(nrd_timectl), C.c_int32,
                                       C.POINTER(C.c_double), C.POINTER(C.c_double),
                                       C.POINTER(nrd_step_stats)]),
    "nrd_adjoint_run": (C.c_int32, [_H, C.POINTER(C.c_double), C.c_int32,
                                    C.c_int32, _P, _P]),
    "nrd_tag": (C.c_int32, [_H, C.POINTER(nrd_tagging), _P]),
    "nrd_cluster": (C.c_int32, [C.POINTER(nrd_problem), C.c_int32, C.POINTER(nrd_box),
                                C.c_int32, C.POINTER(C.c_uint8), C.POINTER(nrd_cluster_opt),
                                C.POINTER(nrd_box), C.c_int32, C.POINTER(C.c_int32)]),
    "nrd_transfer": (C.c_int32, [_H, _H, _P]),
    "nrd_resolve": (C.c_int32, [_H, C.POINTER(nrd_step_stats)]),
    "nrd_dot": (C.c_int32, [_H, _P, _P, C.POINTER(C.c_double)]),
    "nrd_dot_noalloc": (C.c_int32, [_H, _P, _P, _P]),
    "nrd_autotune": (C.c_int32, [_H, C.c_char_p, C.POINTER(C.c_int32)]),
    "nrd_timer_enable": (C.c_int32, [_H, C.c_int32]),
    "nrd_timer_cells": (C.c_int32, [_H, C.c_int32, C.POINTER(C.c_int64)]),
    "nrd_timer_read": (C.c_int32, [_H, C.c_int32, C.POINTER(C.c_double),
                                   C.POINTER(C.c_int32)]),
}
EXPORTED = tuple(_sigs)
for _name, (_res, _args) in _sigs.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args
    globals()[_name] = _f


class NrdError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"nrd status {status}: {msg}")
        self.status = status


def check(status):
    if status != NRD_OK:
        raise NrdError(status, nrd_last_error().decode())
    return status


def default_options(**kw) -> nrd_options:
    o = nrd_options()
    nrd_default_options(C.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def make_problems(problems) -> C.Array:
    arr = (nrd_problem * len(problems))()
    for a, p in zip(arr, problems):
        a.base_n[:] = [int(v) for v in p.base_n]
        a.lo[:] = [float(v) for v in p.lo]
        a.hi[:] = [float(v) for v in p.hi]
        a.bc_E[:] = [int(v) for v in p.bc_E]
        a.robin_R[:] = [float(v) for v in p.robin_R]
        a.kappa = float(p.kappa)
    return arr


def make_boxes(boxes) -> C.Array:
    arr = (nrd_box * len(boxes))()
    for a, b in zip(arr, boxes):
        a.problem = int(b.problem)
        a.level = int(b.level)
        a.lo[:] = [int(v) for v in b.lo]
        a.hi[:] = [int(v) for v in b.hi]
    return arr


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else C.c_void_p(0)


def _vec(t, n, name, optional=False):
    """Device pointer of a float64 CUDA tensor of exactly n contiguous
    values.  The library reads and writes n values through the pointer, so
    a tensor of another type, device, length or stride is refused here."""
    if t is None:
        if optional:
            return C.c_void_p(0)
        raise ValueError(f"{name}: a tensor is required")
    import torch
    if t.dtype != torch.float64:
        raise ValueError(f"{name}: dtype {t.dtype}, expected torch.float64")
    if not t.is_contiguous():
        raise ValueError(f"{name}: tensor is not contiguous")
    if t.numel() != n:
        raise ValueError(f"{name}: {t.numel()} values, expected {n}")
    if not t.is_cuda:
        raise ValueError(f"{name}: tensor on {t.device}, expected a CUDA device")
    return C.c_void_p(t.data_ptr())


def _dt(values):
    return (C.c_double * len(values))(*[float(v) for v in values])


def cluster(problems, boxes, tags, max_levels, buffer=2, efficiency=0.7, min_side=4,
            max_side=24):
    """New boxes (list of (problem, level, lo, hi)) from the boxes of a
    hierarchy and its host tags (a uint8 array of ncells, compact layout)."""
    import numpy as np
    t = np.ascontiguousarray(np.asarray(tags, dtype=np.uint8))
    ncells = sum(int(np.prod([b.hi[d] - b.lo[d] for d in range(3)])) for b in boxes)
    if t.size != ncells:
        raise ValueError(f"tags: {t.size} values, expected {ncells}")
    pr = make_problems(problems)
    bx = make_boxes(boxes)
    opt = nrd_cluster_opt(int(max_levels), int(buffer), float(efficiency), int(min_side),
                          int(max_side))
    n = C.c_int32(0)
    tp = t.ctypes.data_as(C.POINTER(C.c_uint8))
    rc = nrd_cluster(pr, len(problems), bx, len(boxes), tp, C.byref(opt), None, 0, C.byref(n))
    out = (nrd_box * max(1, n.value))()
    check(nrd_cluster(pr, len(problems), bx, len(boxes), tp, C.byref(opt), out, n.value,
                      C.byref(n)))
    del rc
    return [(b.problem, b.level, tuple(b.lo), tuple(b.hi)) for b in out[:n.value]]


class Hierarchy:
    """Owns one nrd_hierarchy and its torch-allocated workspace."""

    def __init__(self, problems, boxes, options: Optional[nrd_options] = None,
                 device="cuda", stream=None, bind=True):
        import torch
        self.torch = torch
        self.problems = problems
        self.boxes = boxes
        self._probs = make_problems(problems)
        self._boxes = make_boxes(boxes)
        self.opt = options if options is not None else default_options()
        self.device = device
        h = _H()
        s = None
        if bind:
            st = stream if stream is not None else torch.cuda.current_stream()
            s = C.c_void_p(st.cuda_stream)
            self.stream = st
        check(nrd_hierarchy_create(self._probs, len(problems), self._boxes, len(boxes),
                                   C.byref(self.opt), s, C.byref(h)))
        self.h = h
        n = C.c_int64()
        nl = C.c_int64()
        check(nrd_layout(h, C.byref(n), C.byref(nl)))
        self.ncells, self.native_len = n.value, nl.value
        sz = C.c_size_t()
        check(nrd_workspace_size(h, C.byref(sz)))
        self.workspace_bytes = sz.value
        self.nprob = len(problems)
        self.ws = None
        if bind:
            self.ws = torch.empty(sz.value, dtype=torch.uint8, device=device)
            check(nrd_bind_workspace(h, _ptr(self.ws), sz.value))

    def __del__(self):
        h = getattr(self, "h", None)
        if h is None or not h.value:
            return
        self.h = None
        try:
            nrd_hierarchy_destroy(h)
        except Exception:       # interpreter shutdown: module globals may be gone
            pass

    # -- vectors ----------------------------------------------------------
    def _nat(self, t, name):
        return _vec(t, 2 * self.native_len, name)

    def _cmp(self, t, name):
        return _vec(t, 2 * self.ncells, name)

    def native(self):
        return self.torch.zeros(2 * self.native_len, dtype=self.torch.float64,
                                device=self.device)

    def compact(self, nf=2):
        return self.torch.zeros(nf * self.ncells, dtype=self.torch.float64,
                                device=self.device)

    def pack(self, native, out=None):
        out = self.compact() if out is None else out
        check(nrd_pack(self.h, self._nat(native, "native"), self._cmp(out, "out")))
        return out

    def unpack(self, compact, out=None):
        out = self.native() if out is None else out
        check(nrd_unpack(self.h, self._cmp(compact, "compact"), self._nat(out, "out")))
        return out

    # -- calls ------------------------------------------------------------
    def set_fields(self, E, T, z):
        n = self.ncells
        check(nrd_set_fields(self.h, _vec(E, n, "E"), _vec(T, n, "T"), _vec(z, n, "z")))

    def get_fields(self):
        E = self.compact(1)
        T = self.compact(1)
        check(nrd_get_fields(self.h, _vec(E, self.ncells, "E"), _vec(T, self.ncells, "T")))
        return E, T

    def begin_step(self, dt: Sequence[float]):
        check(nrd_begin_step(self.h, _dt(dt)))

    def residual(self, u, F):
        check(nrd_residual(self.h, self._nat(u, "u"), self._nat(F, "F")))
        return F

    def jvp(self, u, v, Jv):
        check(nrd_jvp(self.h, self._nat(u, "u"), self._nat(v, "v"), self._nat(Jv, "Jv")))
        return Jv

    def precond_setup(self, u):
        check(nrd_precond_setup(self.h, self._nat(u, "u")))

    def precond_apply(self, w, y):
        check(nrd_precond_apply(self.h, self._nat(w, "w"), self._nat(y, "y")))
        return y

    def vjp(self, u, lam, JTl, gz=None):
        check(nrd_vjp(self.h, self._nat(u, "u"), self._nat(lam, "lam"), self._nat(JTl, "JTl"),
                      _vec(gz, self.ncells, "gz", optional=True)))
        return JTl, gz

    def implicit_step(self, dt: Sequence[float], raise_on_fail=True):
        st = (nrd_step_stats * self.nprob)()
        rc = nrd_implicit_step(self.h, _dt(dt), st)
        if raise_on_fail:
            check(rc)
        return rc, [s.as_dict() for s in st]

    def adaptive_steps(self, nsteps, dt, eps, controller=NRD_CTL_PC47, ratio_min=0.25,
                       ratio_max=2.0, max_halvings=10, t=None, raise_on_fail=True):
        """nsteps controlled steps of every problem; returns (status, next
        step sizes, times, per-step lists of per-problem stats)."""
        ctl = nrd_timectl(float(eps), float(ratio_min), float(ratio_max), int(controller),
                          int(max_halvings))
        d = _dt(dt)
        tt = _dt(t if t is not None else [0.0] * self.nprob)
        st = (nrd_step_stats * (self.nprob * max(nsteps, 1)))()
        rc = nrd_adaptive_steps(self.h, C.byref(ctl), int(nsteps), d, tt, st)
        if raise_on_fail:
            check(rc)
        steps = [[st[n * self.nprob + p].as_dict() for p in range(self.nprob)]
                 for n in range(nsteps)]
        return rc, list(d), list(tt), steps

    def adjoint_run(self, dt, nsteps, ckpt_every, dJdE=None):
        gz = self.compact(1)
        check(nrd_adjoint_run(self.h, _dt(dt), nsteps, ckpt_every,
                              _vec(dJdE, self.ncells, "dJdE", optional=True),
                              _vec(gz, self.ncells, "gz")))
        return gz

    def autotune(self, cache_path: Optional[str] = None) -> int:
        """Pick plane-tile shapes per patch-size class; returns the number of
        classes timed (the rest came from cache_path)."""
        n = C.c_int32(0)
        path = cache_path.encode() if cache_path else None
        check(nrd_autotune(self.h, path, C.byref(n)))
        return n.value

    def dot(self, x, y) -> List[float]:
        out = (C.c_double * self.nprob)()
        check(nrd_dot(self.h, self._nat(x, "x"), self._nat(y, "y"), out))
        return list(out)

    # -- regridding (Sec. 5) ------------------------------------------------
    def tag(self, grad_E=0.0, tau_g=0.0, tau_c=0.0, z_interface=False, out=None):
        """Tags of the current state: uint8 device tensor of ncells."""
        import torch
        if out is None:
            out = torch.zeros(self.ncells, dtype=torch.uint8, device=self.device)
        if out.dtype != torch.uint8 or out.numel() != self.ncells or not out.is_contiguous() \
                or not out.is_cuda:
            raise ValueError("out: a contiguous CUDA uint8 tensor of ncells values")
        crit = nrd_tagging(float(grad_E), float(tau_g), float(tau_c), int(bool(z_interface)), 0)
        check(nrd_tag(self.h, C.byref(crit), C.c_void_p(out.data_ptr())))
        return out

    def transfer_to(self, dst, z):
        """Moves the time history to the hierarchy dst (z: its compact
        material field, a float64 CUDA tensor)."""
        check(nrd_transfer(self.h, dst.h, _vec(z, dst.ncells, "z")))

    def resolve(self):
        st = (nrd_step_stats * self.nprob)()
        check(nrd_resolve(self.h, st))
        return [x.as_dict() for x in st]

    def dot_noalloc(self, x, y, out):
        """nrd_dot into a device tensor of nprob doubles (no allocation, no
        synchronisation)."""
        check(nrd_dot_noalloc(self.h, self._nat(x, "x"), self._nat(y, "y"),
                              _vec(out, self.nprob, "out")))
        return out

    def timer_enable(self, on=True):
        check(nrd_timer_enable(self.h, 1 if on else 0))

    def timer_read(self, which):
        ms = C.c_double()
        n = C.c_int32()
        check(nrd_timer_read(self.h, which, C.byref(ms), C.byref(n)))
        return ms.value, n.value

    def timer_cells(self, which):
        cells = C.c_int64()
        check(nrd_timer_cells(self.h, which, C.byref(cells)))
        return cells.value
