"""Pins of the oracle's coefficient rows (Sec. III.A-C, eqs. 3-16, Alg. 1).

* row sums equal the chord length through the disk / cylinder (textbook
  quadratic, written here independently of eqs. 3-4);
* brute force by dense sampling of the cell definition on tiny grids;
* rotated reference rows equal rows traced directly in every view;
* mirror symmetries of the reference view (Sec. III.C, quarter symmetry).
"""
import math

import numpy as np
import pytest

import synth
from oracle import Oracle

# Lengths of the same piece computed from a rotated ray differ by rounding
# only; near tangency the distance formula of eq. 3 (|S|^2 - t^2 |S-D'|^2)
# cancels, and the circle crossings inherit ~1e-15 / sqrt(rho^2 - d^2).
LEN_RTOL, LEN_ATOL = 1e-9, 1e-10


def chord_length(S, D, R, zlim=None):
    """Length of the segment of the line S + t (D - S) inside the disk / cylinder."""
    S = np.asarray(S, float)
    e = np.asarray(D, float) - S
    a = e[0] ** 2 + e[1] ** 2
    b = 2 * (S[0] * e[0] + S[1] * e[1])
    c = S[0] ** 2 + S[1] ** 2 - R * R
    disc = b * b - 4 * a * c
    if disc <= 0:
        return 0.0
    t1 = (-b - math.sqrt(disc)) / (2 * a)
    t2 = (-b + math.sqrt(disc)) / (2 * a)
    if zlim is not None:
        if e[2] != 0:
            za, zb = (zlim[0] - S[2]) / e[2], (zlim[1] - S[2]) / e[2]
            t1, t2 = max(t1, min(za, zb)), min(t2, max(za, zb))
        elif not (zlim[0] <= S[2] <= zlim[1]):
            return 0.0
    if t2 <= t1:
        return 0.0
    return (t2 - t1) * math.sqrt(e @ e if zlim is not None else a)


def cell_of_points(o: Oracle, P):
    """Cell id of points [n, 3] from the cell definition (half-open ring,
    sector and slice intervals; azimuth in [0, 2 pi))."""
    w = o.w
    r = w.radius / w.n_rings
    rho = np.hypot(P[:, 0], P[:, 1])
    ring = np.minimum((rho / r).astype(np.int64), w.n_rings - 1)
    phi = np.mod(np.arctan2(P[:, 1], P[:, 0]), 2 * np.pi)
    ng = o.ng[ring]
    sec = np.minimum(np.floor(phi * ng / (2 * np.pi)).astype(np.int64), ng - 1)
    cell = o.head[ring] + sec
    if w.is3d:
        h = w.height / w.n_slices
        k = np.clip(np.floor((P[:, 2] + w.height / 2) / h).astype(np.int64), 0, w.n_slices - 1)
        cell = cell + k * o.head[-1]
    return cell


def dense_row(o: Oracle, S, D, M=2_000_000):
    """Cell lengths of one ray by midpoint sampling of M points on its chord."""
    w = o.w
    S = np.asarray(S, float)
    e = np.asarray(D, float) - S
    if not w.is3d:
        e[2] = 0.0
    # sample the chord through the disk; in 3D points outside the slab are discarded
    a = e[0] ** 2 + e[1] ** 2
    b = 2 * (S[0] * e[0] + S[1] * e[1])
    c = S[0] ** 2 + S[1] ** 2 - w.radius ** 2
    disc = b * b - 4 * a * c
    if disc <= 0:
        return {}
    t1 = (-b - math.sqrt(disc)) / (2 * a)
    t2 = (-b + math.sqrt(disc)) / (2 * a)
    dt = (t2 - t1) / M
    t = t1 + (np.arange(M) + 0.5) * dt
    P = S[None, :] + t[:, None] * e[None, :]
    keep = np.hypot(P[:, 0], P[:, 1]) < w.radius
    if w.is3d:
        keep &= np.abs(P[:, 2]) < w.height / 2
    cells = cell_of_points(o, P[keep])
    L = np.linalg.norm(e)
    u, cnt = np.unique(cells, return_counts=True)
    return {int(k): float(v) * dt * L for k, v in zip(u, cnt)}


def test_row_sums_equal_chords_2d():
    w = synth.get("par2d-32r-8v")
    o = Oracle(w)
    for v in range(w.n_views):
        csr = o.trace_view(v)
        for r in range(o.n_rays):
            S, D = o.ray(v, r)
            _, lens = csr.row(r)
            assert math.isclose(lens.sum(), chord_length(S, D, w.radius), rel_tol=1e-12, abs_tol=1e-14)


def test_row_sums_equal_chords_cone():
    w = synth.small_cone(n_rings=24, n_views=8, det=40, m=8)
    o = Oracle(w)
    for v in (0, 3):
        csr = o.trace_view(v)
        for r in range(o.n_rays):
            S, D = o.ray(v, r)
            _, lens = csr.row(r)
            ch = chord_length(S, D, w.radius, (-w.height / 2, w.height / 2))
            assert math.isclose(lens.sum(), ch, rel_tol=1e-12, abs_tol=1e-13)


def test_row_sums_equal_chords_fan():
    # fan beam (Table 1 scans) with intersection lengths: each row sums to the
    # ray's chord through the disk, in the reference view and a rotated one
    w = synth.small_cone(n_rings=20, n_views=6, det=30, m=6).with_(
        geometry="fan2d", n_slices=1, height=0.0, det_v=1)
    o = Oracle(w)
    hit = 0
    for v in (0, 2):
        csr = o.trace_view(v)
        for r in range(o.n_rays):
            S, D = o.ray(v, r)
            _, lens = csr.row(r)
            ch = chord_length(S, D, w.radius)
            assert math.isclose(lens.sum(), ch, rel_tol=1e-12, abs_tol=1e-14)
            hit += ch > 0
    assert hit > o.n_rays   # most rays of both views cross the disk


def test_tangent_and_missing_rays_are_empty():
    w = synth.get("par2d-32r-8v")
    o = Oracle(w)
    cells, _ = o.trace_line([-2.0, 1.0, 0], [2.0, 1.0, 0])      # tangent to the disk
    assert len(cells) == 0
    cells, _ = o.trace_line([-2.0, 1.5, 0], [2.0, 1.2, 0])      # misses
    assert len(cells) == 0


def _near_tangent_rays(o, rng, n):
    """Rays that dip just below a ring circle in the middle of a sector of
    the ring outside it: they enter one annular sector twice."""
    w = o.w
    r = w.radius / w.n_rings
    out = []
    for _ in range(n):
        j = int(rng.integers(1, w.n_rings))
        ngj = o.ng[j]
        s = int(rng.integers(0, ngj))
        az = (s + 0.5) * 2 * math.pi / ngj              # closest point azimuth
        d = j * r * (1 - 10 ** rng.uniform(-6, -2.5))
        cpt = d * np.array([math.cos(az), math.sin(az)])
        dirn = np.array([-math.sin(az), math.cos(az)])
        z0, z1 = (rng.uniform(-0.9, 0.9, 2) if w.is3d else (0.0, 0.0))
        S = np.array([*(cpt - 3 * dirn), z0])
        D = np.array([*(cpt + 3 * dirn), z1])
        out.append((S, D))
    return out


@pytest.mark.parametrize("kind", ["paper2d", "multiple2d", "cone"])
def test_dense_sampling_brute_force(kind):
    rng = np.random.default_rng(11)
    if kind == "paper2d":
        w = synth.Workload(name="t", geometry="parallel2d", n_rings=3, sector_rule="paper",
                           n_views=4, span=2 * math.pi, det_u=8)
    elif kind == "multiple2d":
        w = synth.Workload(name="t", geometry="parallel2d", n_rings=3, sector_multiple=8,
                           n_views=4, span=math.pi, det_u=8)
    else:
        w = synth.small_cone(n_rings=3, n_views=8, det=8, m=8, n_slices=2)
    o = Oracle(w)
    rays = []
    for _ in range(12):
        S = np.array([*rng.uniform(-3, 3, 2), rng.uniform(-0.8, 0.8) if w.is3d else 0.0])
        D = np.array([*rng.uniform(-3, 3, 2), rng.uniform(-0.8, 0.8) if w.is3d else 0.0])
        rays.append((S, D))
    rays += _near_tangent_rays(o, rng, 6)
    for S, D in rays:
        cells, lens = o.trace_line(S, D)
        assert len(set(cells.tolist())) == len(cells)        # one entry per cell
        ref = dense_row(o, S, D)
        got = dict(zip(cells.tolist(), lens.tolist()))
        for c in set(ref) | set(got):
            assert abs(ref.get(c, 0.0) - got.get(c, 0.0)) < 2e-5, (kind, c)


def test_duplicate_cells_are_merged():
    # ring 1 of the paper grid has 12 sectors of 30 degrees; a ray whose closest
    # point (azimuth 105 deg, distance 0.99 r) dips into ring 0 enters sector 3
    # of ring 1 twice.  The row has one entry for it with the summed length.
    w = synth.Workload(name="t", geometry="parallel2d", n_rings=3, sector_rule="paper",
                       n_views=4, span=2 * math.pi, det_u=8)
    o = Oracle(w)
    r = 1 / 3
    az = math.radians(105)
    cpt = 0.99 * r * np.array([math.cos(az), math.sin(az)])
    dirn = np.array([-math.sin(az), math.cos(az)])
    S = np.array([*(cpt - 2 * dirn), 0.0])
    D = np.array([*(cpt + 2 * dirn), 0.0])
    cells, lens = o.trace_line(S, D)
    target = o.head[1] + 3
    assert list(cells).count(target) == 1
    ref = dense_row(o, S, D, M=4_000_000)
    assert abs(ref[target] - lens[list(cells).index(target)]) < 1e-5
    # the two visits are separated by ring-0 cells in the ray's order
    pos = list(cells).index(target)
    assert any(c < o.head[1] for c in cells[pos + 1:])


@pytest.mark.parametrize("name", ["par2d-32r-8v", "cone-small", "par2d-literal"])
def test_rotation_equals_direct_trace(name):
    if name == "cone-small":
        w = synth.small_cone(n_rings=16, n_views=8, det=32, m=8)
    elif name == "par2d-literal":
        w = synth.get("par2d-32r-8v").with_(sector_multiple=8)
    else:
        w = synth.get(name)
    o = Oracle(w)
    csr0 = o.trace_view(0)
    if name == "par2d-literal":
        # not shift-invariant: the method must refuse, direct tracing still works
        with pytest.raises(ValueError):
            o.rotate(csr0, 1)
        for v in range(w.n_views):
            csr = o.trace_view(v)
            for r in range(o.n_rays):
                S, D = o.ray(v, r)
                assert math.isclose(csr.row(r)[1].sum(), chord_length(S, D, w.radius), rel_tol=1e-12)
        return
    for v in range(w.n_views):
        rot = o.rotate(csr0, v)
        direct = o.trace_view(v)
        assert np.array_equal(rot.rowptr, direct.rowptr)
        for r in range(o.n_rays):
            a_c, a_l = rot.row(r)
            b_c, b_l = direct.row(r)
            ia, ib = np.argsort(a_c), np.argsort(b_c)
            assert np.array_equal(a_c[ia], b_c[ib])
            assert np.allclose(a_l[ia], b_l[ib], rtol=LEN_RTOL, atol=LEN_ATOL)


def test_rotation_equals_direct_trace_cone128_sampled():
    w = synth.get("cone-128r-16v")
    o = Oracle(w)
    rays = list(range(0, o.n_rays, 997))
    for v in (1, 5, 15):
        for r in rays:
            S0, D0 = o.ray(0, r)
            c0, l0 = o.trace_line(S0, D0)
            S, D = o.ray(v, r)
            c1, l1 = o.trace_line(S, D)
            from oracle.oracle import CSR
            rot = o.rotate(CSR(np.array([0, len(c0)]), c0, l0), v)
            ia, ib = np.argsort(rot.cells), np.argsort(c1)
            assert np.array_equal(rot.cells[ia], c1[ib])
            assert np.allclose(l0[ia], l1[ib], rtol=LEN_RTOL, atol=LEN_ATOL)


def _split(o, cells):
    c2d = o.head[-1]
    k = cells // c2d
    rem = cells % c2d
    i = np.searchsorted(o.head, rem, side="right") - 1
    s = rem - o.head[i]
    return k, i, s


def test_mirror_symmetry_reference_view():
    # the reference view is symmetric under y -> -y (detector column u ->
    # U-1-u, sector s -> n_g-1-s) and, in 3D, under z -> -z (row w -> V-1-w,
    # slice k -> Nz-1-k): tracing a quarter of the rays suffices (Sec. III.C)
    for w in (synth.get("par2d-32r-8v"), synth.small_cone(n_rings=16, n_views=8, det=32, m=8)):
        o = Oracle(w)
        csr = o.trace_view(0)
        U, V = w.det_u, w.det_v
        c2d = o.head[-1]
        for r in range(o.n_rays):
            u, wv = r % U, r // U
            c, l = csr.row(r)
            k, i, s = _split(o, c)
            mu = csr.row(wv * U + (U - 1 - u))
            km, im, sm = _split(o, mu[0])
            exp = {(kk, ii, o.ng[ii] - 1 - ss): ll for kk, ii, ss, ll in zip(k, i, s, l)}
            got = {(kk, ii, ss): ll for kk, ii, ss, ll in zip(km, im, sm, mu[1])}
            assert exp.keys() == got.keys()
            assert all(abs(exp[x] - got[x]) < 1e-12 for x in exp)
            if w.is3d:
                mz = csr.row((V - 1 - wv) * U + u)
                kz, iz, sz = _split(o, mz[0])
                exp = {(w.n_slices - 1 - kk, ii, ss): ll for kk, ii, ss, ll in zip(k, i, s, l)}
                got = {(kk, ii, ss): ll for kk, ii, ss, ll in zip(kz, iz, sz, mz[1])}
                assert exp.keys() == got.keys()
                assert all(abs(exp[x] - got[x]) < 1e-12 for x in exp)
        assert c2d > 0


def test_binary_mode_rows_are_indicators():
    w = synth.get("par2d-32r-8v")
    o = Oracle(w)
    ob = Oracle(w.with_(binary=True))
    a, b = o.trace_view(2), ob.trace_view(2)
    assert np.array_equal(a.rowptr, b.rowptr) and np.array_equal(a.cells, b.cells)
    assert np.all(b.lens == 1.0)
