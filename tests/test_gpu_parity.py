"""Parity of the HIP library (through the C ABI) with the FP64 CPU oracle.

Tolerances (err = max_j |f_gpu - f_oracle| / max_j |f_oracle|):
  * FP64 arithmetic with FP64 coefficients: 1e-10 (only the summation order
    differs: per-ray tree reductions instead of sequential sums);
  * FP32 arithmetic with FP32 coefficients: 1e-4 after the workload's sweeps.
Coefficient rows: identical cell sets; lengths equal to rounding of the
stored type.  Integer results (lattice, conflict map, remap of an image) are
compared exactly.
"""
import math
import os

import numpy as np
import pytest
import torch

import synth
from oracle import Oracle
from rowcmp import compare_rows

pytestmark = pytest.mark.gpu

NTHREADS = min(16, os.cpu_count() or 1)
TOL32, TOL64 = 1e-4, 1e-10


def rel_inf(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


@pytest.fixture(scope="module")
def U():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2208_12964_amd as U
    U.lib()
    return U


def dev():
    return torch.device("cuda:0")


def gpu_solve(U, w, P, dtype, coeff_dtype=None, sweeps=None, beta=None, colour=(0, 0), f0=None):
    grid = U.Grid.from_workload(w)
    co = U.Coeffs.from_workload(grid, w, coeff_dtype or dtype, colour)
    img = (torch.ones(grid.n_cells, dtype=dtype, device=dev()) if f0 is None
           else torch.as_tensor(f0, dtype=dtype).to(dev()).contiguous())
    proj = torch.as_tensor(np.ascontiguousarray(P)).to(dev(), dtype).contiguous()
    done = U.mart(co, proj, img, w.sweeps if sweeps is None else sweeps, w.beta if beta is None else beta)
    torch.cuda.synchronize()
    return img.cpu().numpy().astype(np.float64), grid, co, done


def cone_cases():
    return [synth.small_cone(n_rings=16, n_views=8, det=32, m=8),
            synth.small_cone("cone-odd", n_rings=13, n_views=4, det=27, m=4, n_slices=9),
            synth.small_cone("cone-wide", n_rings=24, n_views=16, det=40, m=16, n_slices=17).with_(det_v=21)]


def _cmp_rows(co, o, views, rays, tol_rel):
    for v in views:
        for r in rays:
            c1, l1 = co.row(v, int(r))
            S, D = o.ray(v, int(r))
            c2, l2 = o.trace_line(S, D)
            compare_rows(o, int(r), c1, l1, c2, l2, rtol=tol_rel, atol=1e-10 if tol_rel < 1e-8 else 1e-7,
                         view=v)


def test_rows_equal_oracle_2d(U):
    w = synth.get("par2d-32r-8v")
    o = Oracle(w)
    grid = U.Grid.from_workload(w)
    co = U.Coeffs.from_workload(grid, w, torch.float64)
    assert co.nnz == o.trace_view(0).nnz
    _cmp_rows(co, o, range(w.n_views), range(o.n_rays), 1e-9)
    co32 = U.Coeffs.from_workload(grid, w, torch.float32)
    _cmp_rows(co32, o, (0, 5), range(o.n_rays), 2e-7)


@pytest.mark.parametrize("k", range(3))
def test_rows_lattice_conflicts_small_cones(U, k):
    w = cone_cases()[k]
    o = Oracle(w, nthreads=NTHREADS)
    csr0 = o.trace_view(0)
    grid = U.Grid.from_workload(w)
    co = U.Coeffs.from_workload(grid, w, torch.float64)
    assert co.nnz == csr0.nnz
    assert np.array_equal(co.conflicts(), o.conflict_offsets(csr0))
    assert co.lattice == o.colour(csr0)
    _cmp_rows(co, o, range(w.n_views), range(0, o.n_rays, 7), 1e-9)


def test_mart_par2d_fp64_and_fp32(U):
    w = synth.get("par2d-32r-8v")
    P = synth.make_projections(w)
    o = Oracle(w)
    f_ref, csr0, lat = o.reconstruct(P)
    f64, _, co, done = gpu_solve(U, w, P, torch.float64)
    assert co.lattice == lat and done == w.sweeps
    assert rel_inf(f64, f_ref) <= TOL64
    f32, _, _, _ = gpu_solve(U, w, P, torch.float32)
    assert rel_inf(f32, f_ref) <= TOL32
    assert np.all(f32 > 0)


@pytest.mark.parametrize("k", range(3))
def test_mart_small_cones(U, k):
    w = cone_cases()[k]
    P = synth.make_projections(w)
    o = Oracle(w, nthreads=NTHREADS)
    f_ref, _, lat = o.reconstruct(P)
    f64, _, co, _ = gpu_solve(U, w, P, torch.float64)
    assert co.lattice == lat
    assert rel_inf(f64, f_ref) <= TOL64
    f32, _, _, _ = gpu_solve(U, w, P, torch.float32)
    assert rel_inf(f32, f_ref) <= TOL32


def test_binary_weights(U):
    w = synth.small_cone(n_rings=12, n_views=8, det=24, m=8).with_(binary=True)
    P = synth.make_projections(w)
    o = Oracle(w, nthreads=NTHREADS)
    f_ref, _, _ = o.reconstruct(P)
    f64, _, _, _ = gpu_solve(U, w, P, torch.float64)
    assert rel_inf(f64, f_ref) <= TOL64


def test_mart_cone128_full_size_fp32(U):
    w = synth.get("cone-128r-16v")
    P = synth.make_projections(w)
    f32, grid, co, _ = gpu_solve(U, w, P, torch.float32)
    o = Oracle(w, nthreads=NTHREADS)
    csr0 = o.trace_view(0)
    assert co.nnz == csr0.nnz
    lat = o.colour(csr0)
    assert co.lattice == lat
    f_ref = o.mart(csr0, lat, P, np.ones(o.n_cells), w.sweeps, w.beta)
    err = rel_inf(f32, f_ref)
    print(f"cone-128r-16v fp32 err_inf={err:.3e}")
    assert err <= TOL32
    # beta <= 1, P >= 0, f0 > 0: every factor of eq. 18 is positive (cells
    # seen only by P = 0 rays shrink geometrically, so after 20 sweeps FP32 may
    # underflow there; one sweep of the 256-ring cone below must stay > 0)
    assert f32.min() >= 0


def test_cone256_full_size_rows_and_one_sweep(U):
    # full-size high-contrast workload: sampled rows exactly, the lattice and
    # conflict map exactly, and one full FP32 sweep (3.5e9 updates) element by
    # element against the oracle
    w = synth.get("cone-256r-32v-hc")
    o = Oracle(w, nthreads=NTHREADS)
    grid = U.Grid.from_workload(w)
    co = U.Coeffs.from_workload(grid, w, torch.float32)
    rng = np.random.default_rng(5)
    _cmp_rows(co, o, (0, 17), rng.integers(0, o.n_rays, 60), 2e-7)
    csr0 = o.trace_view(0)
    assert co.nnz == csr0.nnz
    assert np.array_equal(co.conflicts(), o.conflict_offsets(csr0))
    lat = o.colour(csr0)
    assert co.lattice == lat
    P = synth.make_projections(w)
    img = torch.ones(grid.n_cells, dtype=torch.float32, device=dev())
    U.mart(co, torch.as_tensor(P).to(dev(), torch.float32).contiguous(), img, 1, w.beta)
    f_ref = o.mart(csr0, lat, P, np.ones(o.n_cells), 1, w.beta)
    err = rel_inf(img.cpu().numpy().astype(np.float64), f_ref)
    print(f"cone-256r-32v-hc one sweep fp32 err_inf={err:.3e}")
    assert err <= TOL32
    assert img.min().item() > 0


def test_remap_point_and_bijection(U):
    w = synth.get("par2d-32r-8v")
    o = Oracle(w)
    grid = U.Grid.from_workload(w)
    rng = np.random.default_rng(2)
    f = rng.uniform(0.1, 2.0, grid.n_cells)
    for nc in (64, 97, 128):
        cart = U.to_cartesian(grid, torch.as_tensor(f, device=dev()), nc).cpu().numpy()
        assert np.array_equal(cart, o.remap(f, nc))
    wc = synth.small_cone(n_rings=10, n_views=4, det=16, m=4, n_slices=5)
    oc = Oracle(wc)
    gc = U.Grid.from_workload(wc)
    fc = rng.uniform(0.1, 2.0, gc.n_cells).astype(np.float32)
    cart = U.to_cartesian(gc, torch.as_tensor(fc, device=dev()), 40).cpu().numpy()
    assert np.array_equal(cart.astype(np.float64), oc.remap(fc.astype(np.float64), 40))
    wp = synth.Workload(name="paper", geometry="parallel2d", n_rings=16, sector_rule="paper",
                        n_views=2, span=math.pi, det_u=32)
    op = Oracle(wp)
    gp = U.Grid.from_workload(wp)
    fp = rng.uniform(0.1, 2.0, gp.n_cells)
    cart = U.to_cartesian(gp, torch.as_tensor(fp, device=dev()), 32, mode="bijection").cpu().numpy()
    assert np.array_equal(cart, op.remap(fp, 32, mode="bijection"))


def test_stopping_rule_matches_oracle(U):
    # consistent data (P = A f_true from the oracle's rows) so that MART
    # converges and eq. 19's relative change falls below tol
    w = synth.Workload(name="tinyfan", geometry="fan2d", n_rings=3, sector_multiple=8, n_views=8,
                       span=2 * math.pi, det_u=24, det_half_u=8 / math.sqrt(15), src_axis=4.0,
                       src_det=8.0)
    o = Oracle(w)
    csr0 = o.trace_view(0)
    lat = o.colour(csr0)
    ftrue = np.random.default_rng(4).uniform(0.5, 1.5, o.n_cells)
    P = np.zeros((w.n_views, o.n_rays))
    for v in range(w.n_views):
        rv = o.rotate(csr0, v)
        for r in range(o.n_rays):
            c, l = rv.row(r)
            P[v, r] = l @ ftrue[c]
    f_ref = o.mart(csr0, lat, P, np.ones(o.n_cells), 5000, 0.5, tol=1e-6)
    assert 2 < o.sweeps_done < 5000
    grid = U.Grid.from_workload(w)
    co = U.Coeffs.from_workload(grid, w, torch.float64)
    img = torch.ones(grid.n_cells, dtype=torch.float64, device=dev())
    done = U.mart(co, torch.as_tensor(P, device=dev()), img, 5000, 0.5, tol=1e-6)
    assert done == o.sweeps_done
    assert rel_inf(img.cpu().numpy(), f_ref) <= TOL64


def test_resume_and_determinism(U):
    w = cone_cases()[0]
    P = synth.make_projections(w)
    a, _, _, _ = gpu_solve(U, w, P, torch.float32, sweeps=8)
    b, _, _, _ = gpu_solve(U, w, P, torch.float32, sweeps=8)
    assert np.array_equal(a, b)                                 # no atomics, fixed reduction order
    c, _, _, _ = gpu_solve(U, w, P, torch.float32, sweeps=5)
    d, _, _, _ = gpu_solve(U, w, P, torch.float32, sweeps=3, f0=c.astype(np.float32))
    assert np.array_equal(a, d)                                 # 5 + 3 sweeps == 8 sweeps


def test_error_paths(U):
    w = synth.get("par2d-32r-8v").with_(sector_multiple=8)      # views are half sectors
    grid = U.Grid.from_workload(w)
    with pytest.raises(U.USPGError) as e:
        U.Coeffs.from_workload(grid, w)
    assert e.value.code == -2
    w = synth.get("par2d-32r-8v")
    grid = U.Grid.from_workload(w)
    with pytest.raises(U.USPGError) as e:
        U.Coeffs.from_workload(grid, w, colour=(1, 1))            # neighbours share cells
    assert e.value.code == -1
    co = U.Coeffs.from_workload(grid, w)
    img = torch.ones(grid.n_cells, device=dev())
    proj = torch.ones(w.n_views * w.det_u, device=dev())
    with pytest.raises(U.USPGError):
        U.mart(co, proj, img, 1, -0.5)
    with pytest.raises(U.USPGError):
        U.mart(co, proj, img, 1, 0.1, work=torch.empty(16, dtype=torch.uint8, device=dev()))


def test_cone256_full_size_20_sweeps_against_golden(U):
    # the high-contrast 256-ring workload after its full 20 FP32 sweeps
    # (Sec. III.D, eqs. 17-18) against the FP64 oracle's image of the same
    # inputs, stored by tests/golden/make_cone256_golden.py (oracle and input
    # generators only): every cell around the three dense inclusions, every
    # 997th cell, and max |f| over all cells
    gold = np.load(os.path.join(os.path.dirname(__file__), "golden", "cone256_sweeps20.npz"))
    w = synth.get(str(gold["workload"]))
    assert w.sweeps == int(gold["sweeps"]) and w.beta == float(gold["beta"])
    P = synth.make_projections(w)
    f32, grid, co, done = gpu_solve(U, w, P, torch.float32)
    assert done == w.sweeps
    assert grid.n_cells == int(gold["n_cells"]) and co.nnz == int(gold["nnz"])
    assert tuple(co.lattice) == tuple(int(x) for x in gold["lattice"])
    cells, ref, max_ref = gold["cells"], gold["values"], float(gold["max_abs"])
    d = np.abs(f32[cells] - ref)
    err = float(d.max()) / max_ref
    err_local = float(d.max()) / float(np.abs(ref).max())
    err_max = abs(float(np.abs(f32).max()) - max_ref) / max_ref
    print(f"cone-256r-32v-hc 20 sweeps fp32: err_inf={err:.3e} over {len(cells)} cells "
          f"(against the sampled max {err_local:.3e}), max|f| rel diff {err_max:.3e}, min f {f32.min():.3e}")
    assert err <= TOL32
    assert err_max <= TOL32
    assert f32.min() > 0
