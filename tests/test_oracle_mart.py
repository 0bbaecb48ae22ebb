"""Pins of the oracle's MART (Sec. III.D, eqs. 17-19) and of its ray order."""
import math

import numpy as np
import pytest

import synth
from oracle import Oracle


def dense_matrix(o, csr0):
    """All views' rows stacked into a dense matrix [views * rays, cells]."""
    w = o.w
    A = np.zeros((w.n_views * o.n_rays, o.n_cells))
    for v in range(w.n_views):
        rv = o.rotate(csr0, v)
        for r in range(o.n_rays):
            c, l = rv.row(r)
            A[v * o.n_rays + r, c] = l
    return A


def tiny2d(**kw):
    # 2 rings, sector multiple 8 -> 8 + 16 = 24 cells; 4 views over a half turn
    # (q = 8 divides every ring); 16 bins
    return synth.Workload(name="tiny2d", geometry="parallel2d", n_rings=2, sector_multiple=8,
                          n_views=4, span=math.pi, det_u=16, **kw)


def tiny_fan2d():
    # fan beam, 2 rings (24 cells), 8 views over a full turn, 16 bins: full
    # rank (a parallel-beam scan of this symmetric grid leaves a null space)
    return synth.Workload(name="tinyfan", geometry="fan2d", n_rings=2, sector_multiple=8,
                          n_views=8, span=2 * math.pi, det_u=16,
                          det_half_u=8 / math.sqrt(15), src_axis=4.0, src_det=8.0)


def tiny3d():
    return synth.small_cone("tiny3d", n_rings=2, n_views=8, det=8, m=8, n_slices=2)


def test_binary_update_identity():
    # binary coefficients: after ray r's own update its new sum is exactly
    # (1 - beta) Pbar + beta P; with beta = 1 its equation holds exactly
    w = synth.get("par2d-32r-8v").with_(binary=True)
    o = Oracle(w)
    csr = o.trace_view(0)
    rng = np.random.default_rng(3)
    for r in (5, 20, 31, 40):
        ids, a = csr.row(r)
        for beta in (0.3, 1.0):
            f = rng.uniform(0.5, 2.0, o.n_cells)
            pbar = f[ids].sum()
            P = rng.uniform(0.2, 3.0) * pbar
            o.mart_ray(ids, a, P, f, beta)
            assert math.isclose(f[ids].sum(), (1 - beta) * pbar + beta * P, rel_tol=1e-13)


def test_length_update_matches_row_normalised_form():
    # with lengths the correction of each cell scales with a_j / a_max; the
    # cell with the largest share gets exactly eq. 18's factor
    w = synth.get("par2d-32r-8v")
    o = Oracle(w)
    csr = o.trace_view(0)
    ids, a = csr.row(33)
    f = np.full(o.n_cells, 1.5)
    f0 = f.copy()
    pbar = (a * f[ids]).sum()
    P, beta = 0.8 * pbar, 0.4
    o.mart_ray(ids, a, P, f, beta)
    j = int(np.argmax(a))
    assert math.isclose(f[ids[j]] / f0[ids[j]], 1 - beta * (1 - P / pbar), rel_tol=1e-14)
    untouched = np.setdiff1d(np.arange(o.n_cells), ids)
    assert np.array_equal(f[untouched], f0[untouched])


def test_positivity_every_sweep():
    w = synth.get("par2d-32r-8v")
    o = Oracle(w)
    csr = o.trace_view(0)
    lat = o.colour(csr)
    P = synth.make_projections(w)
    f = np.ones(o.n_cells)
    for _ in range(w.sweeps):
        f = o.mart(csr, lat, P, f, 1, w.beta)
        assert np.all(f > 0)
    # also with zero data (P = 0 allowed: factor 1 - beta w > 0)
    f = o.mart(csr, lat, np.zeros_like(P), np.ones(o.n_cells), 3, 0.9)
    assert np.all(f > 0)


def test_fixed_point_and_zero_relaxation():
    for w in (tiny2d(), synth.get("par2d-32r-8v"), tiny3d()):
        o = Oracle(w)
        csr = o.trace_view(0)
        lat = o.colour(csr)
        A = dense_matrix(o, csr)
        rng = np.random.default_rng(5)
        ftrue = rng.uniform(0.5, 2.0, o.n_cells)
        P = A @ ftrue
        f = o.mart(csr, lat, P, ftrue, 3, 0.7)
        assert np.allclose(f, ftrue, rtol=1e-12, atol=0)
        f = o.mart(csr, lat, P * 1.3, ftrue, 2, 0.0)
        assert np.array_equal(f, ftrue)


@pytest.mark.parametrize("dim", [2, 3])
def test_converges_on_tiny_consistent_case(dim):
    w = tiny_fan2d() if dim == 2 else tiny3d()
    o = Oracle(w)
    csr = o.trace_view(0)
    A = dense_matrix(o, csr)
    assert np.linalg.matrix_rank(A) == o.n_cells
    # piecewise-constant image: ring 0 at 0.5, ring 1 alternating 1.0 / 2.0
    ftrue = np.zeros(o.n_cells)
    for k in range(w.n_slices):
        base = k * o.head[-1]
        ftrue[base:base + o.ng[0]] = 0.5 + 0.25 * k
        ftrue[base + o.head[1]:base + o.head[2]] = np.where(np.arange(o.ng[1]) % 2 == 0, 1.0, 2.0)
    P = A @ ftrue
    lat = o.colour(csr)
    f = o.mart(csr, lat, P, np.ones(o.n_cells), 5000 if dim == 2 else 3000, 0.5)
    assert np.max(np.abs(f - ftrue)) <= 1e-8 * np.max(np.abs(ftrue))


def test_stopping_rule():
    w = tiny2d()
    o = Oracle(w)
    csr = o.trace_view(0)
    A = dense_matrix(o, csr)
    ftrue = np.linspace(0.5, 1.5, o.n_cells)
    lat = o.colour(csr)
    f = o.mart(csr, lat, A @ ftrue, np.ones(o.n_cells), 10000, 0.5, tol=1e-6)
    done = o.sweeps_done
    assert 1 < done < 10000
    # the stop is the first sweep whose relative change is <= tol (eq. 19)
    g_prev = o.mart(csr, lat, A @ ftrue, np.ones(o.n_cells), done - 1, 0.5)
    g = o.mart(csr, lat, A @ ftrue, g_prev, 1, 0.5)
    assert np.array_equal(g, f)
    assert np.max(np.abs((g - g_prev) / g_prev)) <= 1e-6
    g_pp = o.mart(csr, lat, A @ ftrue, np.ones(o.n_cells), done - 2, 0.5)
    assert np.max(np.abs((g_prev - g_pp) / g_pp)) > 1e-6


def _classes_disjoint(o, csr, ku, kv):
    U = o.w.det_u
    owner = {}
    for r in range(o.n_rays):
        cls = ((r // U) % kv) * ku + (r % U) % ku
        for c in csr.row(r)[0]:
            key = (int(c), cls)
            if key in owner and owner[key] != r:
                return False
            owner[key] = r
    return True


@pytest.mark.parametrize("which", ["par2d", "cone"])
def test_colouring_valid_and_minimal(which):
    w = synth.get("par2d-32r-8v") if which == "par2d" else synth.small_cone(n_rings=12, n_views=8, det=24, m=8)
    o = Oracle(w)
    csr = o.trace_view(0)
    ku, kv = o.colour(csr)
    assert _classes_disjoint(o, csr, ku, kv)
    # every lattice earlier in the search order has a conflict
    K = ku * kv
    for P in range(1, K + 1):
        for a in range(1, P + 1):
            if P % a:
                continue
            b = P // a
            if (P, a) >= (K, ku) or a > w.det_u or b > w.det_v:
                continue
            assert not _classes_disjoint(o, csr, a, b), (a, b)
    # a disjoint class update is order independent: threads give the same bits
    P = synth.make_projections(w)
    f1 = o.mart(csr, (ku, kv), P, np.ones(o.n_cells), 2, 0.1, nthreads=1)
    f4 = o.mart(csr, (ku, kv), P, np.ones(o.n_cells), 2, 0.1, nthreads=4)
    assert np.array_equal(f1, f4)
    # forcing an invalid lattice is refused, a coarser valid one accepted
    with pytest.raises(ValueError):
        o.colour(csr, force=(1, 1))
    assert o.colour(csr, force=(ku * 2, kv)) == (ku * 2, kv)


def test_colour_order_changes_result_only_slightly():
    # every ray order is a legitimate MART; the class order is the contract
    w = synth.get("par2d-32r-8v")
    o = Oracle(w)
    csr = o.trace_view(0)
    P = synth.make_projections(w)
    ku, kv = o.colour(csr)
    a = o.mart(csr, (ku, kv), P, np.ones(o.n_cells), 10, 0.1)
    b = o.mart(csr, (w.det_u, 1), P, np.ones(o.n_cells), 10, 0.1)   # detector order
    rel = np.max(np.abs(a - b)) / np.max(np.abs(a))
    assert 0 < rel < 0.2


def test_class_order_contract_non_square_detector():
    # the MART order: views ascending, classes c = (w mod Kv) Ku + (u mod Ku)
    # ascending, rays of a class by ascending index r = w U + u.  Replayed here
    # ray by ray with the oracle's single-ray update on a U != V detector.
    w = synth.small_cone("rect", n_rings=6, n_views=4, det=10, m=4, n_slices=4).with_(det_v=6)
    o = Oracle(w)
    csr = o.trace_view(0)
    ku, kv = o.colour(csr, force=(3, 2))
    P = synth.make_projections(w)
    f_ref = np.ones(o.n_cells)
    U, V = w.det_u, w.det_v
    for _ in range(2):
        for v in range(w.n_views):
            rv = o.rotate(csr, v)
            for c in range(ku * kv):
                for r in range(U * V):
                    if ((r // U) % kv) * ku + (r % U) % ku != c:
                        continue
                    ids, a = rv.row(r)
                    o.mart_ray(ids, a, P[v].ravel()[r], f_ref, 0.3)
    f = o.mart(csr, (ku, kv), P, np.ones(o.n_cells), 2, 0.3)
    assert np.array_equal(f, f_ref)
    # the rays of a class share no cell: spreading them over threads keeps the bits
    f4 = o.mart(csr, (ku, kv), P, np.ones(o.n_cells), 2, 0.3, nthreads=4)
    assert np.array_equal(f4, f_ref)


@pytest.mark.parametrize("seed", [0, 1])
def test_rays_of_a_class_commute(seed):
    """Rays of one class share no cell, so applying them in any order gives
    the same image bit for bit (Sec. III.D applies rays one after another;
    the class structure is what lets the GPU apply them together).  Replayed
    ray by ray with every class's rays in a random order, then compared with
    the oracle's ascending order."""
    w = synth.small_cone("perm", n_rings=6, n_views=4, det=12, m=4, n_slices=4).with_(det_v=8)
    o = Oracle(w)
    csr = o.trace_view(0)
    ku, kv = o.colour(csr)
    assert ku * kv > 1
    P = synth.make_projections(w)
    rng = np.random.default_rng(seed)
    f = np.ones(o.n_cells)
    U, V = w.det_u, w.det_v
    for _ in range(2):
        for v in range(w.n_views):
            rv = o.rotate(csr, v)
            for c in range(ku * kv):
                rays = [r for r in range(U * V) if ((r // U) % kv) * ku + (r % U) % ku == c]
                for r in rng.permutation(rays):
                    ids, a = rv.row(int(r))
                    o.mart_ray(ids, a, P[v].ravel()[int(r)], f, 0.3)
    f_ref = o.mart(csr, (ku, kv), P, np.ones(o.n_cells), 2, 0.3)
    assert np.array_equal(f, f_ref)
    # a permutation across classes is another MART order and changes the bits
    g = np.ones(o.n_cells)
    for _ in range(2):
        for v in range(w.n_views):
            rv = o.rotate(csr, v)
            for r in rng.permutation(U * V):
                ids, a = rv.row(int(r))
                o.mart_ray(ids, a, P[v].ravel()[int(r)], g, 0.3)
    assert not np.array_equal(g, f_ref)
