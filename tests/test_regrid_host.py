"""Host clustering of refinement tags (nrd_cluster, Sec. 5: Berger-Rigoutsos)
on the CPU: the boxes it returns form a valid, properly nested hierarchy,
cover every tagged cell whose neighbourhood lies on the level below, respect
the size limit, and do not depend on anything but their inputs."""
import numpy as np
import pytest

from paper_1302_6303_amd import inputs as I


def _cells(b):
    r = [np.arange(b.lo[d], b.hi[d]) for d in range(3)]
    g = np.meshgrid(*r, indexing="ij")
    return np.stack([x.ravel(order="F") for x in g], axis=1)


def _tags_of(boxes, fn, base):
    """Compact tags of fn(x, y, z) at the cell centres of every box."""
    out = []
    for b in boxes:
        h = 1.0 / (np.asarray(base) * 2 ** b.level)
        X = (_cells(b) + 0.5) * h
        out.append(fn(X[:, 0], X[:, 1], X[:, 2]))
    return np.concatenate(out).astype(np.uint8)


def _shell(x, y, z):
    r = np.sqrt((x - 0.5) ** 2 + (y - 0.45) ** 2 + (z - 0.55) ** 2)
    return (np.abs(r - 0.3) < 0.04) | ((np.abs(x - 0.2) < 0.03) & (y < 0.6))


def _as_boxes(res):
    return [I.Box(p, lv, lo, hi) for p, lv, lo, hi in res]


def _covered(boxes, level, I_):
    m = np.zeros(len(I_), dtype=bool)
    for b in boxes:
        if b.level != level:
            continue
        m |= np.all((I_ >= np.array(b.lo)) & (I_ < np.array(b.hi)), axis=1)
    return m


def test_clustered_boxes_cover_the_tags_and_nest():
    from paper_1302_6303_amd import nrd
    n = 32
    prob = I.Problem((n, n, n))
    old = [I.Box(0, 0, (0, 0, 0), (n, n, n))]
    tags = _tags_of(old, _shell, (n, n, n))
    res = nrd.cluster([prob], old, tags, max_levels=3, buffer=1, efficiency=0.7,
                      min_side=2, max_side=8)
    new = _as_boxes(res)
    assert [b.level for b in new] == sorted(b.level for b in new)
    assert {b.level for b in new} == {0, 1, 2}
    # a valid hierarchy (alignment, overlap, proper nesting checked at create)
    H = nrd.Hierarchy([prob], new, nrd.default_options(), bind=False)
    assert H.ncells == sum(b.ncells for b in new)
    # every tagged base cell lies under level 1
    T = _cells(old[0])[tags.astype(bool)]
    assert np.all(_covered(new, 1, 2 * T))
    for b in new:
        if b.level > 0:
            assert max(b.hi[d] - b.lo[d] for d in range(3)) <= 16
    # deterministic
    assert nrd.cluster([prob], old, tags, max_levels=3, buffer=1, efficiency=0.7,
                       min_side=2, max_side=8) == res


def test_reclustering_a_refined_hierarchy_uses_its_finest_tags():
    """From a 3-level hierarchy: the level-1 tags (old level 1 where it
    exists, projected base tags elsewhere) whose 26 neighbours lie on the
    new level 1 are all under the new level 2."""
    from paper_1302_6303_amd import nrd
    n = 16
    prob = I.Problem((n, n, n))
    old = _as_boxes(nrd.cluster([prob], [I.Box(0, 0, (0, 0, 0), (n, n, n))],
                                _tags_of([I.Box(0, 0, (0, 0, 0), (n, n, n))], _shell, (n,) * 3),
                                max_levels=3, buffer=1, efficiency=0.7, min_side=2,
                                max_side=8))
    moved = lambda x, y, z: _shell(x - 0.06, y, z)
    tags = _tags_of(old, moved, (n, n, n))
    new = _as_boxes(nrd.cluster([prob], old, tags, max_levels=3, buffer=0, efficiency=0.8,
                                min_side=2, max_side=12))
    nrd.Hierarchy([prob], new, nrd.default_options(), bind=False)
    # level-1 tags as the clustering sees them
    lev1 = [b for b in new if b.level == 1]
    assert lev1
    for b in lev1:
        C_ = _cells(b)
        src = np.zeros(len(C_), dtype=bool)
        done = np.zeros(len(C_), dtype=bool)
        for lv in (1, 0):                       # finest old level first
            for ob, t in zip(old, np.split(tags.astype(bool),
                                           np.cumsum([x.ncells for x in old])[:-1])):
                if ob.level != lv:
                    continue
                P = C_ >> (1 - lv)
                inb = np.all((P >= np.array(ob.lo)) & (P < np.array(ob.hi)), axis=1) & ~done
                if not inb.any():
                    continue
                sh = np.array(ob.hi) - np.array(ob.lo)
                loc = P[inb] - np.array(ob.lo)
                src[inb] = t[loc[:, 0] + sh[0] * (loc[:, 1] + sh[1] * loc[:, 2])]
                done |= inb
        # keep cells whose neighbourhood is on the new level 1
        keep = []
        for c in C_[src]:
            nb = np.stack(np.meshgrid(*[np.arange(c[d] - 1, c[d] + 2) for d in range(3)],
                                      indexing="ij"), -1).reshape(-1, 3)
            nb = np.clip(nb, 0, 2 * n - 1)
            keep.append(bool(np.all(_covered(new, 1, nb))))
        keep = np.array(keep, dtype=bool)
        if keep.any():
            assert np.all(_covered(new, 2, 2 * C_[src][keep]))


def test_no_tags_keep_only_the_base_and_bad_options_are_refused():
    from paper_1302_6303_amd import nrd
    n = 8
    prob = I.Problem((n, n, n))
    old = [I.Box(0, 0, (0, 0, 0), (n, n, n))]
    res = nrd.cluster([prob], old, np.zeros(n ** 3, np.uint8), max_levels=4)
    assert res == [(0, 0, (0, 0, 0), (n, n, n))]
    for kw in ({"efficiency": 0.0}, {"efficiency": 1.5}, {"min_side": 0},
               {"max_side": 1, "min_side": 2}, {"buffer": -1}):
        with pytest.raises(nrd.NrdError):
            nrd.cluster([prob], old, np.ones(n ** 3, np.uint8), max_levels=2, **kw)
    with pytest.raises(ValueError):
        nrd.cluster([prob], old, np.ones(7, np.uint8), max_levels=2)
