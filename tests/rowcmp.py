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


def compare_rows(o, r, c1, l1, c2, l2, rtol=LEN_RTOL, atol=LEN_ATOL):
    """Same cells and lengths; tie rays only per (slice, ring) length sums."""
    assert len(c1) == len(set(np.asarray(c1).tolist())), r
    if on_axis(o, r):
        k1, k2 = ring_keys(o, c1), ring_keys(o, c2)
        for k in set(k1.tolist()) | set(k2.tolist()):
            a, b = l1[k1 == k].sum(), l2[k2 == k].sum()
            assert abs(a - b) <= atol + rtol * abs(b), r
        return
    ia, ib = np.argsort(c1), np.argsort(c2)
    assert np.array_equal(c1[ia], c2[ib]), r
    assert np.allclose(l1[ia], l2[ib], rtol=rtol, atol=atol), r
