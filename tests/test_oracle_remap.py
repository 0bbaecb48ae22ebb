"""Pins of the oracle's USPG -> Cartesian remap (Sec. II.B) and of the
synthetic projection generator's line integrals."""
import math

import numpy as np

import synth
from oracle import Oracle


def test_point_remap_constant_and_brute_force():
    w = synth.get("par2d-32r-8v")
    o = Oracle(w)
    nc = 64
    cart = o.remap(np.full(o.n_cells, 3.0), nc)
    X = 2 * np.arange(nc) + 1 - nc
    x = X / nc
    rho = np.hypot(x[None, :], x[:, None])
    assert np.all(cart[0][rho < 1] == 3.0) and np.all(cart[0][rho >= 1] == 0.0)
    # brute force: the pixel value is the value of the cell containing its centre
    f = np.arange(o.n_cells, dtype=float) + 1.0
    cart = o.remap(f, nc)[0]
    for iy in range(nc):
        for ix in range(nc):
            px, py = x[ix], x[iy]
            rr = math.hypot(px, py)
            if rr >= 1:
                assert cart[iy, ix] == 0
                continue
            ring = int(rr * w.n_rings)
            # sector from exact rational geometry: count sector boundaries below the angle
            ang = math.atan2(py, px) % (2 * math.pi)
            s = int(ang / (2 * math.pi / o.ng[ring]))
            if abs(px) == abs(py):           # exact diagonal: odd multiple of pi/4
                octant = {(1, 1): 1, (-1, 1): 3, (-1, -1): 5, (1, -1): 7}[(int(np.sign(px)), int(np.sign(py)))]
                s = octant * o.ng[ring] // 8
            assert cart[iy, ix] == f[o.head[ring] + s]


def test_bijection_remap_paper_grid():
    nr = 8
    w = synth.Workload(name="p", geometry="parallel2d", n_rings=nr, sector_rule="paper",
                       n_views=4, span=2 * math.pi, det_u=16)
    o = Oracle(w)
    nc = 2 * nr
    f = np.arange(o.n_cells, dtype=float) + 1.0
    cart = o.remap(f, nc, mode="bijection")[0]
    # one to one: every cell appears exactly once
    assert sorted(cart.ravel().tolist()) == f.tolist()
    X = 2 * np.arange(nc) + 1 - nc
    sq = np.maximum(np.abs(X)[None, :], np.abs(X)[:, None])       # 2n - 1
    for n in range(1, nr + 1):
        vals = cart[sq == 2 * n - 1]
        assert len(vals) == 4 * (2 * n - 1)                            # eq. (1), Fig. 2
        assert set((vals - 1).astype(int)) == set(range(o.head[n - 1], o.head[n]))
    # numbering starts at the +x axis and runs anticlockwise (Sec. II.B)
    n = 3
    iy0, ix = nc // 2, nc // 2 + n - 1        # pixel (X = 2n-1, Y = 1)
    assert cart[iy0, ix] == f[o.head[n - 1]]
    assert cart[iy0 - 1, ix] == f[o.head[n] - 1]                     # (2n-1, -1) is last


def test_analytic_projection_matches_quadrature():
    # a single ellipse / ellipsoid line integral against numerical quadrature
    rng = np.random.default_rng(0)
    for two_d in (True, False):
        cen = np.array([0.1, -0.2, 0.05])
        ax = np.array([0.3, 0.2, 0.25])
        objs = [(cen, ax, 0.7, 1.5)]
        for _ in range(5):
            S = np.array([-3.0, rng.uniform(-0.3, 0.1), rng.uniform(-0.2, 0.2)])
            D = np.array([3.0, rng.uniform(-0.4, 0.0), rng.uniform(-0.2, 0.2)])
            if two_d:
                S[2] = D[2] = 0.0
            val = synth.project(objs, S[None], D[None], two_d)[0]
            t = (np.arange(400000) + 0.5) / 400000
            P = S[None] + t[:, None] * (D - S)[None]
            c, s = math.cos(0.7), math.sin(0.7)
            x = P - cen
            xr = np.stack([c * x[:, 0] + s * x[:, 1], -s * x[:, 0] + c * x[:, 1], x[:, 2]], 1)
            dims = 2 if two_d else 3
            inside = np.sum((xr[:, :dims] / ax[:dims]) ** 2, 1) <= 1
            L = np.linalg.norm((D - S)[:dims])
            assert abs(val - 1.5 * inside.mean() * L) < 1e-4


def test_generator_rays_match_oracle_rays():
    # a value-1 object covering the whole domain projects to the chord lengths:
    # ties the generator's scan geometry to the oracle's rays
    w = synth.small_cone(n_rings=8, n_views=4, det=16, m=4)
    o = Oracle(w)
    csr = o.trace_view(0)
    S, D = synth.scan_rays(w, 0)
    for r in range(0, o.n_rays, 7):
        So, Do = o.ray(0, r)
        assert np.allclose(S[r], So, atol=1e-14) and np.allclose(D[r], Do, atol=1e-14)
    # and for a rotated view of the 2D workload
    w2 = synth.get("par2d-32r-8v")
    o2 = Oracle(w2)
    S, D = synth.scan_rays(w2, 3)
    for r in range(o2.n_rays):
        So, Do = o2.ray(3, r)
        assert np.allclose(S[r], So, atol=1e-14) and np.allclose(D[r], Do, atol=1e-14)
    assert csr.nnz > 0
