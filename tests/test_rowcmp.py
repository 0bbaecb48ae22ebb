"""The tie-ray rule of the row comparison: a ray running along a sector
boundary may take either side of it, but no other sector (Sec. III.B: a piece
lies in the cell containing its midpoint; a midpoint on the boundary has two
correct cells)."""
import numpy as np
import pytest

import synth
from oracle import Oracle
from rowcmp import compare_rows, on_axis


def _tie_case():
    w = synth.small_cone("cone-odd", n_rings=13, n_views=4, det=27, m=4, n_slices=9)
    o = Oracle(w)
    ties = [r for r in range(o.n_rays) if on_axis(o, r)]
    assert ties, "the odd detector has a centre column on the x axis"
    r = ties[len(ties) // 2]
    c, l = o.trace_line(*o.ray(0, r))
    return o, r, c, l


def _split(o, cell):
    c2d = o.head[-1]
    k, rem = divmod(int(cell), int(c2d))
    i = int(np.searchsorted(o.head, rem, side="right") - 1)
    return k, i, rem - int(o.head[i])


def test_other_side_of_the_boundary_is_accepted():
    o, r, c, l = _tie_case()
    # move one piece across the boundary it lies on: sector 0 <-> n_g - 1,
    # or n_g / 2 - 1 <-> n_g / 2
    k, i, s = _split(o, c[0])
    ng = int(o.ng[i])
    other = {0: ng - 1, ng - 1: 0, ng // 2 - 1: ng // 2, ng // 2: ng // 2 - 1}[s]
    c2 = c.copy()
    c2[0] = k * o.head[-1] + o.head[i] + other
    if len(set(c2.tolist())) == len(c2):
        compare_rows(o, r, c2, l, c, l)


def test_wrong_sector_with_the_right_ring_is_rejected():
    o, r, c, l = _tie_case()
    k, i, s = _split(o, c[0])
    ng = int(o.ng[i])
    c2 = c.copy()
    c2[0] = k * o.head[-1] + o.head[i] + (s + 2) % ng   # same slice and ring, wrong sector
    with pytest.raises(AssertionError):
        compare_rows(o, r, c2, l, c, l)
