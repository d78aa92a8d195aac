"""C ABI on the host: the library loads, exports every declared symbol and
validates hierarchies (no device calls)."""
import os
import re

import pytest

from paper_1302_6303_amd import inputs as I

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_every_declared_symbol_is_exported():
    from paper_1302_6303_amd import nrd
    hdr = open(os.path.join(ROOT, "include", "nrd.h")).read()
    declared = set(re.findall(r"\b(nrd_[a-z_]+)\s*\(", hdr))
    assert len(declared) >= 20
    for name in declared:
        assert hasattr(nrd._lib, name), name
    assert declared == set(nrd.EXPORTED)


def _create(problems, boxes, **opt):
    from paper_1302_6303_amd import nrd
    return nrd.Hierarchy(problems, boxes, nrd.default_options(**opt), bind=False)


def test_layout_counts():
    w = I.small_amr(8)
    H = _create(w.problems, w.boxes)
    assert H.ncells == sum(b.ncells for b in w.boxes)
    assert H.native_len == sum((b.shape[0] + 2) * (b.shape[1] + 2) * (b.shape[2] + 2)
                               for b in w.boxes)
    assert H.workspace_bytes > 40 * 2 * 8 * H.native_len      # Krylov basis included


@pytest.mark.parametrize("boxes,status", [
    ([(0, (0, 0, 0), (8, 8, 8)), (1, (0, 0, 0), (4, 4, 4)), (1, (2, 2, 2), (6, 6, 6))], -2),
    ([(0, (0, 0, 0), (8, 8, 8)), (1, (1, 2, 2), (5, 6, 6))], -2),
    ([(0, (0, 0, 0), (8, 8, 8)), (1, (2, 2, 2), (6, 6, 6)), (2, (4, 4, 4), (10, 10, 10))], -2),
    ([(0, (0, 0, 0), (4, 8, 8)), (0, (4, 0, 0), (8, 8, 6))], -2),       # level 0 not tiled
    ([(0, (0, 0, 0), (4, 8, 8)), (0, (2, 0, 0), (8, 8, 8))], -2),       # level 0 overlaps
    ([(0, (0, 0, 0), (3, 8, 8)), (0, (3, 0, 0), (8, 8, 8))], -7),       # tiled at an odd plane
    ([(0, (0, 0, 0), (8, 8, 8)), (2, (4, 4, 4), (8, 8, 8))], -2),       # level gap
    ([(1, (2, 2, 2), (6, 6, 6)), (0, (0, 0, 0), (8, 8, 8))], -1),       # unordered
])
def test_invalid_hierarchies_are_rejected(boxes, status):
    from paper_1302_6303_amd import nrd
    bx = [I.Box(0, lv, lo, hi) for lv, lo, hi in boxes]
    with pytest.raises(nrd.NrdError) as e:
        _create([I.Problem((8, 8, 8))], bx)
    assert e.value.status == status


def test_tiled_base_levels_are_accepted():
    """The coarsest level is a union of patches (Sec. 3.2): level-0 boxes
    that tile the base grid at even planes, with finer boxes across the
    cuts; a base grid that cannot coarsen must stay one box."""
    from paper_1302_6303_amd import nrd
    w = I.tiled_base(16)
    H = _create(w.problems, w.boxes)
    assert H.ncells == sum(b.ncells for b in w.boxes)
    with pytest.raises(nrd.NrdError) as e:
        _create([I.Problem((5, 5, 5))], [I.Box(0, 0, (0, 0, 0), (2, 5, 5)),
                                          I.Box(0, 0, (2, 0, 0), (5, 5, 5))])
    assert e.value.status == nrd.NRD_EUNSUPPORTED


def test_bad_options_are_rejected():
    from paper_1302_6303_amd import nrd
    w = I.marshak_single(8)
    for kw in ({"gmres_restart": 0}, {"gmres_restart": 65}, {"newton_maxit": 0},
               {"jvp_mode": 2}, {"stencil": 4}, {"bdf_max_order": 3},
               {"fac_nu_pre": 0}, {"fac_nu_post": -1}, {"fac_nu_post": 9},
               {"fac_smoother": 3}, {"fac_base": 2}, {"fac_cycle": 2},
               {"fac_cycle": 1, "fac_smoother": 1}, {"fac_cycle": 1, "fac_nu_post": 1},
               {"newton_forcing": 2}):
        with pytest.raises(nrd.NrdError):
            _create(w.problems, w.boxes, **kw)


def test_unknown_timer_is_rejected():
    from paper_1302_6303_amd import nrd
    import ctypes as C
    w = I.marshak_single(8)
    H = _create(w.problems, w.boxes)
    ms, n = C.c_double(), C.c_int32()
    for which in (-1, 5):
        assert nrd.nrd_timer_read(H.h, which, C.byref(ms), C.byref(n)) == nrd.NRD_EINVAL


def test_calls_before_binding_report_state_error():
    from paper_1302_6303_amd import nrd
    import ctypes as C
    w = I.marshak_single(8)
    H = _create(w.problems, w.boxes)
    rc = nrd.nrd_residual(H.h, C.c_void_p(0), C.c_void_p(0))
    assert rc == nrd.NRD_ESTATE


def test_struct_layouts_match_the_header(tmp_path):
    # the ctypes mirrors of the public structs have the C sizes and offsets
    import ctypes as C
    import subprocess
    from paper_1302_6303_amd import nrd
    src = tmp_path / "sizes.c"
    src.write_text("""
#include <stddef.h>
#include <stdio.h>
#include "nrd.h"
int main(void) {
    printf("%zu %zu %zu %zu %zu %zu %zu\\n", sizeof(nrd_options), offsetof(nrd_options, err_eta_T),
           sizeof(nrd_step_stats), offsetof(nrd_step_stats, err_norm), sizeof(nrd_timectl),
           sizeof(nrd_problem), sizeof(nrd_box));
    return 0;
}
""")
    exe = tmp_path / "sizes"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True,
                                          check=True).stdout.split()]
    want = [C.sizeof(nrd.nrd_options), nrd.nrd_options.err_eta_T.offset,
            C.sizeof(nrd.nrd_step_stats), nrd.nrd_step_stats.err_norm.offset,
            C.sizeof(nrd.nrd_timectl), C.sizeof(nrd.nrd_problem), C.sizeof(nrd.nrd_box)]
    assert got == want


def test_wide_patch_is_accepted_with_the_default_stencil():
    """A patch whose rows do not fit the staged plane slices (the paper's
    uniform 256^3 grid) is accepted: the hierarchy falls back to the
    plane-marching variant."""
    prob = I.Problem(base_n=(256, 256, 256))
    box = I.Box(0, 0, (0, 0, 0), (256, 256, 256))
    H = _create([prob], [box])
    assert H.ncells == 256 ** 3


def test_binding_refuses_tensors_the_library_cannot_read():
    """Every device pointer the binding hands over must address exactly the
    float64 values the call reads: other dtypes, lengths, strides or a host
    tensor are refused before the library is called."""
    import torch
    from paper_1302_6303_amd import nrd
    w = I.marshak_single(8)
    H = _create(w.problems, w.boxes)
    n = H.ncells
    good = torch.zeros(n, dtype=torch.float64)
    with pytest.raises(ValueError, match="dtype"):
        H.set_fields(good.float(), good, good)
    with pytest.raises(ValueError, match="CUDA"):
        H.set_fields(good, good, good)
    with pytest.raises(ValueError, match="dtype"):
        H.residual(torch.zeros(2 * H.native_len, dtype=torch.float32),
                   torch.zeros(2 * H.native_len, dtype=torch.float32))
    with pytest.raises(ValueError, match="contiguous"):
        nrd._vec(torch.zeros(2 * n, dtype=torch.float64)[::2], n, "z")
    with pytest.raises(ValueError, match="values"):
        nrd._vec(torch.zeros(n - 1, dtype=torch.float64), n, "z")


def test_autograd_refuses_a_bdf2_hierarchy():
    """The adjoint differentiates backward-Euler steps; a hierarchy left at
    the default BDF2 order is refused instead of returning the gradient of
    another trajectory."""
    import torch
    from paper_1302_6303_amd.autograd import RadDiffEvolve
    w = I.marshak_single(8)
    H = _create(w.problems, w.boxes)
    z = torch.ones(H.ncells, dtype=torch.float64, requires_grad=True)
    with pytest.raises(ValueError, match="bdf_max_order"):
        RadDiffEvolve.apply(z, H, z.detach(), z.detach(), 1e-3, 2, 1)


def test_dot_noalloc_refuses_hierarchies_beyond_its_fixed_array():
    """The no-allocation inner product keeps one partial sum per reduction
    tile in a fixed array of 32768 doubles; a hierarchy with more tiles is
    refused with NRD_EINVAL before any device work (checked on the host)."""
    import ctypes as C
    from paper_1302_6303_amd import nrd
    n = 32
    boxes = [I.Box(0, 0, (0, 0, 0), (n, n, n))]
    for k in range(0, 2 * n, 2):
        for j in range(0, 2 * n, 2):
            for i in range(0, 2 * n, 2):
                boxes.append(I.Box(0, 1, (i, j, k), (i + 2, j + 2, k + 2)))
    H = _create([I.Problem((n, n, n))], boxes)
    rc = nrd.nrd_dot_noalloc(H.h, C.c_void_p(0), C.c_void_p(0), C.c_void_p(0))
    assert rc == nrd.NRD_EINVAL
    assert "32768" in nrd.nrd_last_error().decode()
