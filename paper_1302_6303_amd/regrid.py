"""Dynamic regridding driver (Sec. 5) over the C ABI.

One regrid of a hierarchy: refinement tags of the current state on the
device (nrd_tag), Berger-Rigoutsos clustering of the tags into new boxes on
the host (nrd_cluster), a new hierarchy with its own workspace, its material
field sampled by the caller, the time history moved by conservative linear
refinement (nrd_transfer) and the last step solved again on the new grid
(nrd_resolve, the warm restart).  Marshalling and orchestration only: the
tags, the clustering, the transfer and the re-solve are the library's.
"""
from __future__ import annotations

import time
from typing import Callable, Optional

from . import nrd


class Regridder:
    """crit: keyword arguments of Hierarchy.tag (grad_E, tau_g, tau_c,
    z_interface); cluster: of nrd.cluster (max_levels, buffer, efficiency,
    min_side, max_side); zfun(problems, boxes) returns the compact material
    field of a box list as a float64 CUDA tensor; options: of the new
    hierarchies; tune_cache: tile-shape cache file shared by every new
    hierarchy (None: no tuning)."""

    def __init__(self, options, crit: dict, cluster: dict,
                 zfun: Callable, tune_cache: Optional[str] = None, resolve: bool = True):
        self.options = options
        self.crit = dict(crit)
        self.cluster = dict(cluster)
        self.zfun = zfun
        self.tune_cache = tune_cache
        self.resolve = resolve

    def boxes_for(self, H):
        """New box list from the current state's tags."""
        from .inputs import Box
        tags = H.tag(**self.crit).cpu().numpy()
        res = nrd.cluster(H.problems, H.boxes, tags, **self.cluster)
        return [Box(p, lv, lo, hi) for p, lv, lo, hi in res]

    def regrid(self, H, boxes=None):
        """(new hierarchy, info): the history of H moved to the boxes given,
        or to those its tags call for.  H is left intact."""
        import torch
        info = {}
        t0 = time.perf_counter()
        if boxes is None:
            boxes = self.boxes_for(H)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        Hn = nrd.Hierarchy(H.problems, boxes, self.options)
        z = self.zfun(H.problems, boxes)
        H.transfer_to(Hn, z)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        info["timed_classes"] = 0
        if self.tune_cache is not None:
            info["timed_classes"] = Hn.autotune(self.tune_cache)
        t3 = time.perf_counter()
        st = None
        info["resolved"] = False
        if self.resolve:
            st = (nrd.nrd_step_stats * Hn.nprob)()
            rc = nrd.nrd_resolve(Hn.h, st)
            if rc not in (nrd.NRD_OK, nrd.NRD_ENOTCONV):
                nrd.check(rc)
            # a re-solve that does not converge leaves the interpolated
            # state: the run continues as a plain warm restart
            info["resolved"] = rc == nrd.NRD_OK
            st = [x.as_dict() for x in st]
        torch.cuda.synchronize()
        t4 = time.perf_counter()
        info.update({"boxes": len(boxes), "cells": Hn.ncells,
                     "tag_cluster_s": t1 - t0, "create_transfer_s": t2 - t1,
                     "tune_s": t3 - t2, "resolve_s": t4 - t3,
                     "resolve_newton": sum(s["newton_iters"] for s in st) if st else 0,
                     "resolve_krylov": sum(s["krylov_iters"] for s in st) if st else 0})
        return Hn, boxes, info
