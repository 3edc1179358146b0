"""Pins for the oracle's lightcone removal and active-box rule (CPU only):
exact rational brute force of the removal predicate, stable partition,
volume fractions, and the paper's own shrink-schedule numbers (Table 4 and
the Fig. 5 discussion; tests/golden/paper_shrink_schedule.json)."""
import functools
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import cosmology as oc
from oracle import pm
from synth import uniform_particles

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_shrink_schedule.json")


def test_removal_predicate_against_exact_rationals():
    box, r = 100.0, 37.0
    x, _, _ = uniform_particles(4000, box, 17)
    xo = np.array([50.0, 50.0, 50.0])
    out = pm.outside_lightcone(x, xo, r)
    for row, flag in zip(x, out):
        d2 = sum((Fraction(float(v)) - Fraction(float(o))) ** 2 for v, o in zip(row, xo))
        exact_out = d2 > Fraction(r) ** 2
        # FP64 may only disagree within a few ulps of the sphere
        if abs(float(d2) - r * r) > 1e-9 * r * r:
            assert flag == exact_out


def test_removal_tie_is_kept():
    xo = np.array([0.0, 0.0, 0.0])
    x = np.array([[3.0, 4.0, 0.0], [3.0, 4.0, 1e-3]])
    assert list(pm.outside_lightcone(x, xo, 5.0)) == [False, True]


def test_shrink_is_stable_partition():
    ng, box = 16, 100.0
    x, p, ids = uniform_particles(500, box, 5)
    cfg = pm.Config(ng=ng, box=box, shrink=True, n_initial=500)
    st = pm.State(x.copy(), p.copy(), ids.copy(), 500, np.zeros((ng,) * 3), 0.5)
    removed = pm.shrink_radius(st, cfg, 45.0)
    keep = [i for i in range(500) if math.dist(x[i], (50.0, 50.0, 50.0)) <= 45.0]
    gone = [i for i in range(500) if i not in set(keep)]
    assert list(st.ids[:st.n_active]) == keep
    assert list(removed) == gone
    assert list(st.ids[st.n_active:]) == gone
    assert np.array_equal(st.x[:st.n_active], x[keep])


def test_box_rule_and_switch():
    ng, box, h = 64, 640.0, 10.0
    xo = np.array([320.0, 320.0, 320.0])
    # sphere + 2 cells still touches the mesh edge: periodic whole mesh
    dirichlet, lo, hi = pm.box_for_radius(300.0, xo, h, ng, 2)
    assert not dirichlet and list(lo) == [0, 0, 0] and list(hi) == [63, 63, 63]
    dirichlet, lo, hi = pm.box_for_radius(200.0, xo, h, ng, 2)
    assert dirichlet and list(lo) == [10, 10, 10] and list(hi) == [54, 54, 54]
    # outward rounding: planes next to the box on multiples of 8
    dirichlet, lo, hi = pm.box_for_radius(200.0, xo, h, ng, 2, 8)
    assert dirichlet and list(lo) == [9, 9, 9] and list(hi) == [55, 55, 55]
    dirichlet, lo, hi = pm.box_for_radius(211.0, xo, h, ng, 2, 8)
    assert dirichlet and list(lo) == [1, 1, 1] and list(hi) == [55, 55, 55]
    dirichlet, lo, hi = pm.box_for_radius(231.0, xo, h, ng, 2, 8)
    assert not dirichlet
    # a box that never grows
    cfg = pm.Config(ng=ng, box=box, shrink=True, n_initial=1)
    st = pm.State(np.zeros((0, 3)), np.zeros((0, 3)), np.zeros(0, np.uint32), 0,
                  np.zeros((ng,) * 3), 0.5)
    pm.shrink_radius(st, cfg, 200.0)
    pm.shrink_radius(st, cfg, 250.0)
    assert not st.periodic and list(st.lo) == [10] * 3 and list(st.hi) == [54] * 3


def _kept_fraction(box, r, n=32):
    # fraction of a uniform lattice of sample points inside the sphere
    c = (np.arange(n) + 0.5) * (box / n)
    z, y, x = np.meshgrid(c, c, c, indexing="ij")
    pts = np.stack([x.ravel(), y.ravel(), z.ravel()], 1)
    return 1.0 - pm.outside_lightcone(pts, np.full(3, box / 2), r).mean()


def test_kept_fraction_matches_sphere_volume():
    box = 1000.0
    x, _, _ = uniform_particles(200000, box, 23)
    for r in (300.0, 450.0):
        frac = 1.0 - pm.outside_lightcone(x, np.full(3, box / 2), r).mean()
        vol = 4.0 / 3.0 * math.pi * r**3 / box**3
        assert frac == pytest.approx(vol, abs=4 * math.sqrt(vol * (1 - vol) / 200000))


@functools.lru_cache(maxsize=None)
def _schedule(box, steps=1000, z_init=40.0, om=0.3, ol=0.7):
    a0 = 1.0 / (1.0 + z_init)
    edges = np.linspace(a0, 1.0, steps + 1)
    fr = []
    corner = math.sqrt(3.0) * box / 2
    for a in edges[1:]:
        r = oc.lightcone_radius(a, om, ol)
        fr.append(1.0 if r >= corner else _kept_fraction(box, r))
    return np.array(fr)


def test_paper_table4_and_fig5_geometry():
    gold = json.load(open(GOLDEN))
    for row in gold["table4"]:
        fr = _schedule(row["box"], gold["steps"], gold["z_init"])
        speedup = gold["steps"] / fr.sum()
        assert speedup == pytest.approx(row["speedup"], rel=0.15), row
    fr = _schedule(gold["fig5_largest_box"]["box"], gold["steps"], gold["z_init"])
    q = gold["fig5_largest_box"]
    assert fr[gold["steps"] // 4 - 1] == pytest.approx(q["fraction_at_quarter"], abs=0.15)
    assert fr[gold["steps"] // 2 - 1] == pytest.approx(q["fraction_at_half"], abs=0.05)
