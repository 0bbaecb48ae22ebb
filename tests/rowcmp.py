"""Row comparison helpers shared by the CPU walk tests and the GPU tests."""
import numpy as np

LEN_RTOL, LEN_ATOL = 1e-9, 1e-10


def on_axis(o, r):
    """A view-0 ray through the axis lies on the x axis, which is a sector
    boundary of every ring: either side is a correct cell (a tie)."""
    S, D = o.ray(0, r)
    e = D - S
    return abs(S[0] * e[1] - S[1] * e[0]) < 1e-12


def ring_keys(o, cells):
    c2d = o.head[-1]
    rem = cells % c2d
    return (cells // c2d) * 100000 + np.searchsorted(o.head, rem, side="right") - 1


def beside_line(o, view, r, cells):
    """For a tie ray (its in-plane line runs through the axis along a sector
    boundary of every ring), whether every cell lies on one of the two sides
    of that boundary: the sector's lower or upper edge is the line's azimuth
    (beyond the axis) or that azimuth plus pi (before the axis)."""
    S, D = o.ray(view, r)
    e = D - S
    phi = np.arctan2(e[1], e[0]) % (2 * np.pi)
    c2d = o.head[-1]
    rem = np.asarray(cells) % c2d
    i = np.searchsorted(o.head, rem, side="right") - 1
    s = rem - o.head[i]
    width = 2 * np.pi / o.ng[i]
    ok = np.zeros(len(rem), dtype=bool)
    for edge in (s * width, (s + 1) * width):
        for a in (phi, phi + np.pi):
            d = np.abs((edge - a + np.pi) % (2 * np.pi) - np.pi)
            ok |= d < 1e-9
    return ok


def compare_rows(o, r, c1, l1, c2, l2, rtol=LEN_RTOL, atol=LEN_ATOL, view=0):
    """Same cells and lengths.  A tie ray has two correct assignments: its
    (slice, ring) length sums must agree, and every cell of either row must
    lie on one of the two sides of the sector boundary the ray runs along."""
    assert len(c1) == len(set(np.asarray(c1).tolist())), r
    if on_axis(o, r):
        k1, k2 = ring_keys(o, c1), ring_keys(o, c2)
        for k in set(k1.tolist()) | set(k2.tolist()):
            a, b = l1[k1 == k].sum(), l2[k2 == k].sum()
            assert abs(a - b) <= atol + rtol * abs(b), r
        assert beside_line(o, view, r, c1).all() and beside_line(o, view, r, c2).all(), r
        return
    ia, ib = np.argsort(c1), np.argsort(c2)
    assert np.array_equal(c1[ia], c2[ib]), r
    assert np.allclose(l1[ia], l2[ib], rtol=rtol, atol=atol), r
