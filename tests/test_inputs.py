"""Seeded inputs: paper constants, determinism, hierarchy validity."""
import json
import os

import numpy as np

from oracle.hierarchy import Hierarchy
from paper_1302_6303_amd import inputs as I

GOLD = os.path.join(os.path.dirname(__file__), "golden", "marshak_problem.json")


def test_constants_match_the_paper_problem():
    g = json.load(open(GOLD))
    assert I.E0 == g["E0"]
    assert I.T0 == g["E0"] ** 0.25
    assert I.KAPPA == g["kappa"]
    p = I.Problem(base_n=(8, 8, 8))
    assert p.robin_R[0] == g["robin_R"]["x=0"] and p.bc_E[0] == 1
    # the paper's own three-box material layout through the box sampler's
    # field evaluator
    zf = I.box_field([(np.array(lo), np.array(hi), g["z_inside"])
                      for lo, hi in g["z_boxes"]], g["z_outside"])
    X = np.array([0.1, 0.2, 0.3, 0.9])
    Y = np.array([0.5, 0.5, 0.05, 0.5])
    Z = np.array([0.5, 0.05, 0.95, 0.5])
    np.testing.assert_array_equal(zf(X, Y, Z), [10.0, 10.0, 10.0, 1.0])


def test_workloads_are_seeded_and_nested():
    a = I.static_amr(base=16, nlevels=3, side=(8, 16))
    b = I.static_amr(base=16, nlevels=3, side=(8, 16))
    assert [(x.level, x.lo, x.hi) for x in a.boxes] == [(x.level, x.lo, x.hi) for x in b.boxes]
    assert max(x.level for x in a.boxes) == 2
    Hierarchy((16, 16, 16), [(x.level, x.lo, x.hi) for x in a.boxes])   # validates
    e = I.ensemble(nprob=8)
    assert len(e.boxes) == 8 and all(32 <= x.shape[0] <= 96 for x in e.boxes)
    assert np.all((e.dt >= 1e-4) & (e.dt <= 1e-3))


def test_paper_model_problem_layout():
    """The paper's model problem (Sec. 6): z = 10 exactly on the cells whose
    centres lie in its three boxes, Robin faces at x = 0 and x = 1 only."""
    n = 32
    w = I.paper_marshak(n)
    c = (np.arange(n) + 0.5) / n
    expect = 0
    for lo, hi, _ in I.PAPER_BOXES:
        k = 1
        for d in range(3):
            k *= int(np.sum((c >= lo[d]) & (c < hi[d])))
        expect += k
    assert int(np.sum(w.z[0] == 10.0)) == expect
    assert int(np.sum(w.z[0] == 1.0)) == n ** 3 - expect
    p = w.problems[0]
    assert tuple(p.bc_E) == (1, 1, 0, 0, 0, 0)
    assert p.robin_R[0] == 1.0 and p.robin_R[1] == 0.0
    assert np.all(w.E[0] == I.E0) and np.all(w.T[0] == I.T0)
    with open(GOLD) as f:
        gold = json.load(f)
    assert [[list(lo), list(hi)] for lo, hi, _ in I.PAPER_BOXES] == gold["z_boxes"]
    assert all(zv == gold["z_inside"] for _, _, zv in I.PAPER_BOXES)
