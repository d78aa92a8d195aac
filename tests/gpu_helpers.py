"""Shared plumbing of the GPU parity tests: the same seeded inputs feed the
HIP library (through the C ABI binding) and the CPU oracle."""
import numpy as np

from oracle import operators as ops
from paper_1302_6303_amd import inputs as I
from tests.helpers import system


def torch_mod():
    import torch
    return torch


def lib():
    from paper_1302_6303_amd import nrd
    return nrd


def compact_state(w):
    return np.concatenate([w.compact(w.E), w.compact(w.T)])


def to_dev(x):
    torch = torch_mod()
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).to("cuda")


def to_host(t):
    return t.detach().to("cpu").numpy().astype(np.float64)


def make(w, **opt):
    nrd = lib()
    o = nrd.default_options(**opt)
    H = nrd.Hierarchy(w.problems, w.boxes, o)
    z = to_dev(w.compact(w.z))
    u = compact_state(w)
    n = H.ncells
    H.set_fields(to_dev(u[:n]), to_dev(u[n:]), z)
    return H


def native_from_compact(H, x):
    return H.unpack(to_dev(x))


def compact_from_native(H, t):
    return to_host(H.pack(t))


def rel_err(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def problem_slices(w):
    """Per problem: indices of its cells in the compact (E | T) layout."""
    n = w.ncells()
    out = []
    off = 0
    starts = []
    for b in w.boxes:
        starts.append(off)
        off += b.ncells
    for p in range(len(w.problems)):
        idx = [np.arange(starts[i], starts[i] + b.ncells)
               for i, b in enumerate(w.boxes) if b.problem == p]
        idx = np.concatenate(idx)
        out.append(np.concatenate([idx, idx + n]))
    return out
