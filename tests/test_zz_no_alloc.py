"""The allocation-free entry point mart_run_noalloc (through the C ABI) gives
the same image as mart_run with a caller work buffer, on two calls in a row
(the second on a smaller problem, so it starts from the first call's
leftovers in the shared work space), and against the FP64 oracle
(Sec. III.D, eqs. 17-19).  Problems whose work space exceeds the fixed array
are refused before anything is enqueued."""
import math

import numpy as np
import pytest
import torch

import synth
from oracle import Oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def U():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2208_12964_amd as U
    U.lib()
    return U


def dev():
    return torch.device("cuda:0")


def _both(U, w, dtype, tol=0.0, sweeps=None):
    P = synth.make_projections(w)
    g = U.Grid.from_workload(w)
    co = U.Coeffs.from_workload(g, w, dtype)
    proj = torch.as_tensor(P).to(dev(), dtype).contiguous()
    n = w.sweeps if sweeps is None else sweeps
    ref = torch.ones(g.n_cells, dtype=dtype, device=dev())
    d_ref = U.mart(co, proj, ref, n, w.beta, tol=tol)
    img = torch.ones(g.n_cells, dtype=dtype, device=dev())
    d_na = U.mart_run_noalloc(co, proj, img, n, w.beta, tol=tol)
    torch.cuda.synchronize()
    return P, co, ref.cpu().numpy(), img.cpu().numpy(), d_ref, d_na


def _oracle_err(w, P, f, sweeps=None, tol=0.0):
    o = Oracle(w)
    csr0 = o.trace_view(0)
    lat = o.colour(csr0)
    f_ref = o.mart(csr0, lat, P, np.ones(o.n_cells), w.sweeps if sweeps is None else sweeps, w.beta, tol=tol)
    return float(np.max(np.abs(f.astype(np.float64) - f_ref)) / np.max(np.abs(f_ref))), o


def test_two_calls_equal_mart_run_and_oracle(U):
    # first call: a 24-ring cone, FP32, fixed sweeps
    w1 = synth.small_cone("na-cone", n_rings=24, n_views=16, det=40, m=16, n_slices=17, sweeps=6)
    P1, co1, ref1, img1, _, _ = _both(U, w1, torch.float32)
    assert co1.workspace_bytes(torch.float32) <= U.NOALLOC_SCRATCH_BYTES
    assert np.array_equal(img1, ref1)
    err1, _ = _oracle_err(w1, P1, img1)
    assert err1 <= 1e-4
    # second call: a smaller fan-beam problem in FP64 with the stopping rule
    # (eq. 19) on consistent data P = A f_true, so that MART converges; its
    # work space is a prefix of the first call's, which it must rewrite
    w2 = synth.Workload(name="na-fan", geometry="fan2d", n_rings=3, sector_multiple=8, n_views=8,
                        span=2 * math.pi, det_u=24, det_half_u=8 / math.sqrt(15), src_axis=4.0,
                        src_det=8.0)
    o2 = Oracle(w2)
    csr0 = o2.trace_view(0)
    lat = o2.colour(csr0)
    ftrue = np.random.default_rng(4).uniform(0.5, 1.5, o2.n_cells)
    P2 = np.zeros((w2.n_views, o2.n_rays))
    for v in range(w2.n_views):
        rv = o2.rotate(csr0, v)
        for r in range(o2.n_rays):
            c, l = rv.row(r)
            P2[v, r] = l @ ftrue[c]
    g2 = U.Grid.from_workload(w2)
    co2 = U.Coeffs.from_workload(g2, w2, torch.float64)
    assert co2.workspace_bytes(torch.float64, 1e-6) < co1.workspace_bytes(torch.float32)
    proj2 = torch.as_tensor(P2, device=dev())
    ref2 = torch.ones(g2.n_cells, dtype=torch.float64, device=dev())
    d_ref = U.mart(co2, proj2, ref2, 5000, 0.5, tol=1e-6)
    img2 = torch.ones_like(ref2)
    d_na = U.mart_run_noalloc(co2, proj2, img2, 5000, 0.5, tol=1e-6)
    torch.cuda.synchronize()
    f_ref = o2.mart(csr0, lat, P2, np.ones(o2.n_cells), 5000, 0.5, tol=1e-6)
    assert d_na == d_ref == o2.sweeps_done and 2 < d_na < 5000
    assert torch.equal(img2, ref2)
    f2 = img2.cpu().numpy()
    assert np.max(np.abs(f2 - f_ref)) / np.max(np.abs(f_ref)) <= 1e-10


def test_oversized_problem_is_refused(U):
    # a 128-ring, 128-slice cylinder: 54 MB of FP64 device-layout image, so
    # with the stopping rule (two images) the work space exceeds 64 MiB
    w = synth.small_cone("na-big", n_rings=128, n_views=16, det=8, m=16, n_slices=128)
    g = U.Grid.from_workload(w)
    co = U.Coeffs.from_workload(g, w, torch.float64)
    assert co.workspace_bytes(torch.float64, 1e-3) > U.NOALLOC_SCRATCH_BYTES
    proj = torch.ones(w.n_views * co.n_rays, dtype=torch.float64, device=dev())
    img = torch.ones(g.n_cells, dtype=torch.float64, device=dev())
    with pytest.raises(U.USPGError) as e:
        U.mart_run_noalloc(co, proj, img, 2, 0.1, tol=1e-3)
    assert e.value.code == -3 and "work space" in str(e.value)
    torch.cuda.synchronize()
    assert torch.all(img == 1)
    # the same problem without the stopping rule fits and matches mart_run
    ref = torch.ones_like(img)
    U.mart(co, proj, ref, 2, 0.1)
    U.mart_run_noalloc(co, proj, img, 2, 0.1)
    torch.cuda.synchronize()
    assert torch.equal(img, ref)
