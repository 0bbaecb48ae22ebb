"""Pins of the oracle's grid (Sec. II.A-B, eqs. 1-2)."""
import json
import math
import os

import numpy as np

import synth
from oracle import Oracle, sector_counts

GOLD = os.path.join(os.path.dirname(__file__), "golden", "paper_grid.json")


def test_paper_rule_matches_printed_counts():
    g = json.load(open(GOLD))
    n = g["N"] // 2
    ng = sector_counts("paper", 0, n)
    assert list(ng) == g["ring_cells"]
    w = synth.Workload(name="paper8", geometry="parallel2d", n_rings=n, sector_rule="paper",
                       n_views=4, span=2 * math.pi, det_u=8)
    o = Oracle(w)
    assert list(o.head[:-1]) == g["heads"]
    assert o.n_cells == g["total_cells"] == g["N"] ** 2


def test_paper_rule_equal_area():
    # eq. (1): ring n has area pi (2n-1) r^2 and 4(2n-1) cells -> every cell pi r^2 / 4
    nr = 50
    ng = sector_counts("paper", 0, nr)
    r = 1.0 / nr
    for i in range(nr):
        n = i + 1
        area = math.pi * ((n * r) ** 2 - ((n - 1) * r) ** 2)
        assert math.isclose(area / ng[i], math.pi * r * r / 4, rel_tol=1e-12)
    # total cells of N/2 rings equals N^2 (one-to-one with the Cartesian grid)
    assert ng.sum() == (2 * nr) ** 2


def test_multiple_rule_properties():
    # every count is the smallest multiple of m that is >= the ring's area / r^2
    for m, nr in [(8, 32), (16, 32), (16, 128), (32, 256), (64, 100)]:
        ng = sector_counts("multiple", m, nr)
        for i in range(nr):
            target = 2 * math.pi * (i + 0.5)      # ring area / r^2
            assert ng[i] % m == 0
            assert ng[i] >= target
            assert ng[i] - m < target


def test_workload_cell_counts():
    # cells per slice for the three single-problem workloads, recounted from
    # the sector rule (independent sum; the values were also derived by hand)
    expect = {"par2d-32r-8v": 3472, "cone-128r-16v": 52512, "cone-256r-32v-hc": 210016}
    for name, c2d in expect.items():
        w = synth.get(name)
        ng = sector_counts(w.sector_rule, w.sector_multiple, w.n_rings)
        assert int(ng.sum()) == c2d
        total = sum(w.sector_multiple * math.ceil(2 * math.pi * (i + 0.5) / w.sector_multiple)
                    for i in range(w.n_rings))
        assert total == c2d


def test_literal_sector_rule_breaks_the_shift():
    # with sector counts multiples of 8 but 8 views over a half turn (22.5 degree
    # steps = 1/16 of a turn) the rotation is not a whole number of sectors
    w = synth.get("par2d-32r-8v").with_(sector_multiple=8)
    o = Oracle(w)
    assert not o.shift_ok()
    assert Oracle(synth.get("par2d-32r-8v")).shift_ok()
