"""z-slab decomposition of one solve (uspg_build_slabs / mart_run_slabs), the
layout several devices would share a cone-beam volume in, run on one GPU:
one slab gives mart_run's image bit for bit; several slabs (uneven, and one
slice each) stay within 1e-4 (FP32) / 1e-10 (FP64) of the FP64 oracle; the
slab rows partition the reference rows; bad arguments are refused."""
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


def cases():
    return [
        synth.small_cone("sl-cone9", n_rings=10, n_views=8, det=20, m=8, n_slices=9, sweeps=3),
        synth.serve_request(21, 12, 4, 4),
    ]


def rel_err(f, ref):
    return np.max(np.abs(f - ref)) / np.max(np.abs(ref))


def setup(U, w, dtype):
    dev = torch.device("cuda:0")
    g = U.Grid.from_workload(w)
    co = U.Coeffs.from_workload(g, w, dtype)
    P = synth.make_projections(w)
    proj = torch.as_tensor(P, device=dev).to(dtype).contiguous()
    return g, co, P, proj


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
@pytest.mark.parametrize("w", cases(), ids=lambda w: w.name)
def test_one_slab_equals_mart_run(U, w, dtype):
    g, co, _, proj = setup(U, w, dtype)
    a = torch.ones(g.n_cells, dtype=dtype, device=proj.device)
    U.mart(co, proj, a, w.sweeps, w.beta)
    sl = U.Slabs(co, 1)
    b = torch.ones_like(a)
    sl.run(proj, b, w.sweeps, w.beta)
    torch.cuda.synchronize()
    assert torch.equal(a, b)


@pytest.mark.parametrize("dtype,tol", [(torch.float32, 1e-4), (torch.float64, 1e-10)])
@pytest.mark.parametrize("w", cases(), ids=lambda w: w.name)
def test_slabs_equal_oracle(U, w, dtype, tol):
    g, co, P, proj = setup(U, w, dtype)
    f_ref, _, _ = Oracle(w, nthreads=NTHREADS).reconstruct(P)
    for n in sorted({2, 4, w.n_slices}):
        sl = U.Slabs(co, n)
        info = [sl.info(k) for k in range(n)]
        # the slabs tile the slices and split the reference entries
        assert info[0]["slices"][0] == 0 and info[-1]["slices"][1] == w.n_slices
        assert all(info[k]["slices"][1] == info[k + 1]["slices"][0] for k in range(n - 1))
        assert sum(i["nnz"] for i in info) == co.nnz
        img = torch.ones(g.n_cells, dtype=dtype, device=proj.device)
        sl.run(proj, img, w.sweeps, w.beta)
        torch.cuda.synchronize()
        assert rel_err(img.cpu().numpy().astype(np.float64), f_ref) <= tol, (w.name, n)


def test_full_size_eight_slabs_one_sweep(U):
    """cone-128r-16v (6.7 M cells, 65,536 rays) in 8 slabs of 16 slices: one
    FP32 sweep within 1e-4 of mart_run's, whose own parity with the oracle is
    tested at this size elsewhere (the slabs only re-associate ray sums)."""
    w = synth.get("cone-128r-16v").with_(sweeps=1)
    print("case cone-128r-16v 8 slabs", flush=True)
    dev = torch.device("cuda:0")
    g = U.Grid.from_workload(w)
    co = U.Coeffs.from_workload(g, w)
    proj = synth.make_projections_torch(w, dev, torch.float32).reshape(-1).contiguous()
    a = torch.ones(g.n_cells, device=dev)
    U.mart(co, proj, a, 1, w.beta)
    sl = U.Slabs(co, 8)
    b = torch.ones_like(a)
    sl.run(proj, b, 1, w.beta)
    torch.cuda.synchronize()
    assert [sl.info(k)["slices"] for k in range(8)] == [(16 * k, 16 * k + 16) for k in range(8)]
    assert not torch.equal(a, b)        # the sums really were split
    assert ((a - b).abs().max() / a.abs().max()).item() <= 1e-4


def test_errors(U):
    w = cases()[0]
    g, co, _, proj = setup(U, w, torch.float32)
    for n in (0, w.n_slices + 1, 65):
        with pytest.raises(U.USPGError) as e:
            U.Slabs(co, n)
        assert e.value.code == -1
    sl = U.Slabs(co, 3)
    img = torch.ones(g.n_cells, device=proj.device)
    small = torch.empty(sl.workspace_bytes() - 1, dtype=torch.uint8, device=proj.device)
    with pytest.raises(U.USPGError) as e:
        sl.run(proj, img, 1, 0.1, work=small)
    assert e.value.code == -3
    with pytest.raises(U.USPGError) as e:
        sl.run(proj, img, 1, 0.0)
    assert e.value.code == -1
    wl = synth.small_cone("sl-lit", n_rings=7, n_views=7, det=10, m=7, sweeps=1).with_(
        sector_rule="paper", n_slices=5, rebin=True, binary=True)
    gl = U.Grid.from_workload(wl)
    cl = U.Coeffs.from_workload(gl, wl)
    with pytest.raises(U.USPGError) as e:
        U.Slabs(cl, 2)
    assert e.value.code == -1
