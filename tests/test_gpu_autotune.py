"""Tile-shape tuner: the chosen shapes change how tiles cover each patch,
never the results (bitwise), and a cache file written by one hierarchy is
reused by the next without timing."""
import numpy as np
import pytest

from paper_1302_6303_amd import inputs as I
from tests.gpu_helpers import compact_from_native, make, native_from_compact
from tests.helpers import state, system

pytestmark = pytest.mark.gpu


def _workload():
    return I.static_amr(base=16, nlevels=3, side=(8, 16), state="front")


def _outputs(H, w):
    s = system(w)
    u_n = state(s, w)
    rng = np.random.default_rng(21)
    u = s.sync(u_n * rng.uniform(0.9, 1.1, u_n.shape))
    v = rng.standard_normal(u.shape) * u
    H.begin_step([2e-3])
    F = H.native()
    H.residual(native_from_compact(H, u), F)
    Jv = H.native()
    H.jvp(native_from_compact(H, u), native_from_compact(H, v), Jv)
    return compact_from_native(H, F), compact_from_native(H, Jv)


@pytest.mark.parametrize("stencil", [1, 2, 3])
def test_tuned_shapes_keep_results_and_cache_is_reused(stencil, tmp_path):
    w = _workload()
    classes = {tuple(int(x) for x in b.shape) for b in w.boxes}
    cache = str(tmp_path / "tiles.txt")
    H = make(w, stencil=stencil)
    before = _outputs(H, w)
    timed = H.autotune(cache)
    assert timed == len(classes)
    after = _outputs(H, w)
    for a, b in zip(before, after):
        np.testing.assert_array_equal(a, b)
    lines = open(cache).read().split("\n")
    assert sum(1 for l in lines if f" v{stencil} " in l) == len(classes)
    H2 = make(w, stencil=stencil)
    assert H2.autotune(cache) == 0
    for a, b in zip(before, _outputs(H2, w)):
        np.testing.assert_array_equal(a, b)


def test_tuned_solver_steps_match_untuned():
    w = _workload()
    outs = []
    for tune in (False, True):
        H = make(w, precision=1)
        if tune:
            H.autotune(None)
        for dt in (1e-3, 1e-3):
            H.implicit_step([dt])
        E, T = H.get_fields()
        outs.append((E.cpu().numpy(), T.cpu().numpy()))
    np.testing.assert_array_equal(outs[0][0], outs[1][0])
    np.testing.assert_array_equal(outs[0][1], outs[1][1])


def test_cache_lines_with_unknown_shapes_are_ignored(tmp_path):
    """A stale or edited cache line (a plane run longer than a workgroup
    holds, an unknown plane count, another format tag) is never applied: the
    class is timed afresh and the results stay bitwise the defaults'."""
    w = _workload()
    classes = sorted({tuple(int(x) for x in b.shape) for b in w.boxes})
    H = make(w, stencil=3)
    before = _outputs(H, w)
    # learn this build's format tag and architecture from a real cache line
    good = str(tmp_path / "good.txt")
    H.autotune(good)
    arch, var, fmt = open(good).read().split("\n")[0].split()[:3]
    bad = str(tmp_path / "bad.txt")
    with open(bad, "w") as f:
        for i, c in enumerate(classes):
            dims = "x".join(str(v) for v in c)
            if i % 3 == 0:
                f.write(f"{arch} {var} {fmt} {dims} 16 1024 1.0\n")   # run > 256
            elif i % 3 == 1:
                f.write(f"{arch} {var} {fmt} {dims} 5 256 1.0\n")     # unknown planes
            else:
                f.write(f"{arch} {var} f0x0b0 {dims} 16 256 1.0\n")   # other format
    H2 = make(w, stencil=3)
    assert H2.autotune(bad) == len(classes)
    for a, b in zip(before, _outputs(H2, w)):
        np.testing.assert_array_equal(a, b)


def test_cache_is_reused_across_changing_hierarchies(tmp_path):
    """Regridding makes new hierarchies whose patch-size classes partly
    repeat: with one cache file, a new hierarchy times only the classes no
    earlier one had, and its results stay bitwise the defaults'."""
    w1 = _workload()
    w2 = I.static_amr(base=16, nlevels=3, side=(8, 16), seed_k=9, state="front")
    c1 = {tuple(int(x) for x in b.shape) for b in w1.boxes}
    c2 = {tuple(int(x) for x in b.shape) for b in w2.boxes}
    assert c1 & c2 and c2 - c1
    cache = str(tmp_path / "tiles.txt")
    assert make(w1).autotune(cache) == len(c1)
    H2 = make(w2)
    before = _outputs(H2, w2)
    assert H2.autotune(cache) == len(c2 - c1)
    for a, b in zip(before, _outputs(H2, w2)):
        np.testing.assert_array_equal(a, b)
