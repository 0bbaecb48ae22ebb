"""Degenerate and edge cases of the GPU path against the FP64 oracle: zero
sweeps, one ring, one view, one detector pixel, rays that miss the grid,
all-zero projections, a stopping rule met after the first sweep, and the
literal scheme on a half-turn scan with three views; maximum sizes and
short buffers are refused."""
import math
import os

import numpy as np
import pytest
import torch

import synth
from oracle import Oracle

pytestmark = pytest.mark.gpu
NTHREADS = min(16, os.cpu_count() or 1)


@pytest.fixture(scope="module")
def U():
    assert torch.cuda.is_available()
    import paper_2208_12964_amd as U
    U.lib()
    return U


def dev():
    return torch.device("cuda:0")


def check(U, w, P=None, dtype=torch.float64, tol=1e-10, rebin=False):
    P = synth.make_projections(w) if P is None else P
    img, _, g, co = U.reconstruct(w, torch.as_tensor(P, device=dev()), dtype=dtype)
    o = Oracle(w, nthreads=NTHREADS)
    f_ref, _, lat = o.reconstruct_rebin(P) if rebin else o.reconstruct(P)
    assert co.lattice == lat
    f = img.cpu().numpy().astype(np.float64)
    scale = max(np.max(np.abs(f_ref)), 1e-300)
    assert np.max(np.abs(f - f_ref)) / scale <= tol, w.name
    return f, f_ref


def test_zero_sweeps_leave_the_image(U):
    w = synth.small_cone("e-zero", n_rings=6, n_views=4, det=8, m=4)
    g = U.Grid.from_workload(w)
    co = U.Coeffs.from_workload(g, w)
    img = torch.rand(g.n_cells, device=dev()) + 0.5
    keep = img.clone()
    assert U.mart(co, torch.ones(w.n_views * w.n_rays, device=dev()), img, 0, 0.1) == 0
    torch.cuda.synchronize()
    assert torch.equal(img, keep)


@pytest.mark.parametrize("w", [
    synth.parallel("e-1ring", 1, 4, 6, 8, phantom="ellipses", sweeps=3),
    synth.parallel("e-1view", 8, 1, 16, 8, phantom="ellipses", sweeps=3).with_(span=2 * math.pi),
    synth.parallel("e-1ray", 8, 4, 1, 8, phantom="ellipses", sweeps=3),
    synth.small_cone("e-cone-1ring", n_rings=1, n_views=4, det=4, m=4, n_slices=3, sweeps=2),
    synth.small_cone("e-cone-1px", n_rings=5, n_views=4, det=1, m=4, n_slices=4, sweeps=2),
], ids=lambda w: w.name)
def test_tiny_grids_and_scans(U, w):
    check(U, w)
    check(U, w, dtype=torch.float32, tol=1e-4)


def test_rays_missing_the_grid_and_zero_data(U):
    # a fan twice as wide as the disk: the outer half of the rays miss it
    w = synth.small_cone("e-wide", n_rings=8, n_views=4, det=20, m=4).with_(
        geometry="fan2d", n_slices=1, height=0.0, det_v=1)
    w = w.with_(det_half_u=2 * w.det_half_u)
    check(U, w)
    # all-zero data: every ray multiplies its cells by 1 - beta
    Z = np.zeros((w.n_views, 1, w.det_u))
    f, f_ref = check(U, w, P=Z)
    assert np.all(f < 1.0) and np.all(f > 0.0)


def test_stop_after_first_sweep(U):
    w = synth.small_cone("e-stop", n_rings=6, n_views=4, det=8, m=4)
    g = U.Grid.from_workload(w)
    co = U.Coeffs.from_workload(g, w, torch.float64)
    P = torch.as_tensor(synth.make_projections(w), device=dev())
    img = torch.ones(g.n_cells, dtype=torch.float64, device=dev())
    assert U.mart(co, P, img, 10, 0.1, tol=1e9) == 1
    ref = torch.ones(g.n_cells, dtype=torch.float64, device=dev())
    U.mart(co, P, ref, 1, 0.1)
    torch.cuda.synchronize()
    assert torch.equal(img, ref)


def test_literal_scheme_half_turn_three_views(U):
    w = synth.parallel("e-lit-half", 10, 3, 24, 1, phantom="ellipses", sweeps=4).with_(
        sector_rule="paper", rebin=True, binary=True)
    check(U, w, rebin=True)
    check(U, w, dtype=torch.float32, tol=1e-4, rebin=True)


def test_size_limits(U):
    """Maximum sizes are refused before any device work: more than 2^31
    cells, 2^31 rays, 65,536 slices for segment records, a Cartesian grid of
    2^31 pixels, and a bijection remap off the paper's grid."""
    with pytest.raises(U.USPGError) as e:
        U.Grid(30000, 1, 1.0, 0.0, "multiple", 8)           # about 2.8e9 cells
    assert e.value.code == -1
    g3 = U.Grid(4, 4, 1.0, 2.0, "multiple", 8)
    with pytest.raises(U.USPGError) as e:
        U.Coeffs(g3, "cone3d", 8, 2 * math.pi, 1 << 16, 1 << 15, 1.0, 1.0, 4.0, 8.0)   # 2^31 rays
    assert e.value.code == -1
    g = U.Grid(4, 1, 1.0, 0.0, "multiple", 8)
    gz = U.Grid(1, 1 << 16, 1.0, 2.0, "multiple", 4)
    with pytest.raises(U.USPGError) as e:
        U.Coeffs(gz, "cone3d", 4, 2 * math.pi, 4, 4, 1.0, 1.0, 4.0, 8.0, weights="segments")
    assert e.value.code == -1
    img = torch.ones(g.n_cells, device=dev())
    out = torch.empty(1, device=dev())
    with pytest.raises(U.USPGError) as e:       # 46,341^2 > 2^31 pixels (refused before any write)
        U._check(U.lib().uspg_to_cartesian(g.handle, 0, img.data_ptr(), out.data_ptr(), 46341, 0, None))
    assert e.value.code == -1
    with pytest.raises(U.USPGError) as e:
        U.to_cartesian(g, img, 2 * 4, mode="bijection")     # not the paper's sector rule
    assert e.value.code == -1


def test_binding_refuses_short_buffers(U):
    """The binding checks tensor sizes and dtypes against the problem before
    handing raw pointers to the library."""
    w = synth.get("par2d-32r-8v")
    g = U.Grid.from_workload(w)
    co = U.Coeffs.from_workload(g, w)
    proj = torch.ones(w.n_views * w.det_u, device=dev())
    img = torch.ones(g.n_cells, device=dev())
    for p, im in ((proj[:-1], img), (proj, img[:-1]), (proj.double(), img)):
        with pytest.raises(ValueError):
            U.mart(co, p, im, 1, 0.1)
    with pytest.raises(ValueError):
        U.to_cartesian(g, img, 16, out=torch.empty(16 * 16 - 1, device=dev()))
    eng = U.Engine(1, torch.float64)
    with pytest.raises(ValueError):
        eng.admit(co, proj, img, 1, 0.1)                     # float32 buffers, float64 engine
    eng.close()
    with pytest.raises(ValueError):
        U.Slabs(co, 1).run(proj[:-1], img, 1, 0.1)


def test_timing_is_per_stream(U):
    # batch timing is kept per stream: a solve on another stream neither adds
    # to it nor turns it off
    w = synth.small_cone("t-cone", n_rings=8, n_views=4, det=12, m=4, sweeps=2)
    g = U.Grid.from_workload(w)
    co = U.Coeffs.from_workload(g, w)
    P = torch.as_tensor(synth.make_projections(w), dtype=torch.float32, device=dev()).contiguous()
    a, b = torch.cuda.Stream(), torch.cuda.Stream()
    U.mart_timing(True, stream=a)
    img_b = torch.ones(g.n_cells, device=dev())
    with torch.cuda.stream(b):
        U.mart(co, P, img_b, w.sweeps, w.beta, stream=b)
    b.synchronize()
    assert U.mart_timing(True, stream=a)[1] == 0         # nothing on a yet (and reset)
    img_a = torch.ones(g.n_cells, device=dev())
    with torch.cuda.stream(a):
        U.mart(co, P, img_a, w.sweeps, w.beta, stream=a)
    a.synchronize()
    ms, n = U.mart_timing(False, stream=a)
    assert n == w.sweeps * w.n_views * co.lattice[0] * co.lattice[1] and ms > 0
    assert torch.equal(img_a, img_b)
