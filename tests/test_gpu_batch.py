"""Many problems in one persistent launch: every problem's image equals the
one mart_run gives for it alone (bit for bit: same per-ray arithmetic and
order), and matches the FP64 oracle within 1e-4 (FP32) / 1e-10 (FP64);
autotuning changes speed only."""
import math
import os

import numpy as np
import pytest
import torch

import synth
from oracle import Oracle

pytestmark = pytest.mark.gpu
NTHREADS = min(16, os.cpu_count() or 1)


def problems(n=10, seed=11):
    """2D parallel-beam slices of uneven ring and view counts (2 Nr bins,
    sector multiple 2p, half-turn scans) plus two small cone-beam volumes."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(n):
        nr = int(rng.choice([8, 16, 24, 32, 48]))
        p = int(rng.choice([4, 8, 16]))
        out.append(synth.parallel(f"b{k}", nr, p, 2 * nr, 2 * p, phantom="ellipses", n_objects=6,
                                  seed=4000 + k, sweeps=int(rng.integers(3, 8)), beta=0.1, dtype="f32"))
    out.append(synth.small_cone("bc0", n_rings=10, n_views=8, det=20, m=8, n_slices=6, sweeps=4))
    out.append(synth.small_cone("bc1", n_rings=16, n_views=4, det=24, m=4, n_slices=10, sweeps=3))
    return out


@pytest.fixture(scope="module")
def U():
    assert torch.cuda.is_available()
    import paper_2208_12964_amd as U
    U.lib()
    return U


@pytest.mark.parametrize("dtype,tol", [(torch.float32, 1e-4), (torch.float64, 1e-10)])
def test_batch_equals_alone_and_oracle(U, dtype, tol):
    dev = torch.device("cuda:0")
    ws = problems()
    grids = [U.Grid.from_workload(w) for w in ws]
    cos = [U.Coeffs.from_workload(g, w, dtype) for g, w in zip(grids, ws)]
    Ps = [synth.make_projections(w) for w in ws]
    projs = [torch.as_tensor(P, device=dev).to(dtype).contiguous() for P in Ps]
    alone = []
    for co, proj, w, g in zip(cos, projs, ws, grids):
        img = torch.ones(g.n_cells, dtype=dtype, device=dev)
        U.mart(co, proj, img, w.sweeps, w.beta)
        alone.append(img)
    b = U.Batch(cos, dtype)
    for mode, block, lds in (("lockstep", 256, False), ("lockstep", 128, False),
                             ("persistent", 256, True), ("persistent", 1024, True),
                             ("persistent", 512, False)):
        b.set(mode, block, lds)
        if mode == "persistent":
            assert (b.info()["n_lds"] > 0) == lds    # small images fit the LDS
        imgs = [torch.ones(g.n_cells, dtype=dtype, device=dev) for g in grids]
        b.run(projs, imgs, [w.sweeps for w in ws], [w.beta for w in ws])
        torch.cuda.synchronize()
        for a, m in zip(alone, imgs):
            assert torch.equal(a, m), (mode, block, lds)
    for w, P, img in zip(ws, Ps, alone):
        o = Oracle(w, nthreads=NTHREADS)
        f_ref, _, _ = o.reconstruct(P)
        f = img.cpu().numpy().astype(np.float64)
        assert np.max(np.abs(f - f_ref)) / np.max(np.abs(f_ref)) <= tol, w.name


def test_autotune_keeps_results(U):
    dev = torch.device("cuda:0")
    ws = problems(6, seed=5)
    grids = [U.Grid.from_workload(w) for w in ws]
    cos = [U.Coeffs.from_workload(g, w) for g, w in zip(grids, ws)]
    projs = [torch.as_tensor(synth.make_projections(w), dtype=torch.float32, device=dev) for w in ws]
    b = U.Batch(cos)
    imgs0 = [torch.ones(g.n_cells, device=dev) for g in grids]
    ms = b.autotune(projs, imgs0, [w.beta for w in ws], probe_sweeps=1)
    assert ms > 0
    assert all(torch.all(i == 1) for i in imgs0)          # the caller's images are untouched
    imgs = [torch.ones(g.n_cells, device=dev) for g in grids]
    b.run(projs, imgs, [w.sweeps for w in ws], [w.beta for w in ws])
    for co, proj, w, g, m in zip(cos, projs, ws, grids, imgs):
        img = torch.ones(g.n_cells, device=dev)
        U.mart(co, proj, img, w.sweeps, w.beta)
        assert torch.equal(img, m)


def test_graph_replays_match_eager(U):
    # the lockstep sequence is one captured graph: replay it several times with
    # the program's own eager work and synchronisations in between, and check
    # every replay against the problems solved alone
    dev = torch.device("cuda:0")
    ws = problems(8, seed=3)
    grids = [U.Grid.from_workload(w) for w in ws]
    cos = [U.Coeffs.from_workload(g, w) for g, w in zip(grids, ws)]
    projs = [torch.as_tensor(synth.make_projections(w), dtype=torch.float32, device=dev) for w in ws]
    b = U.Batch(cos)
    b.set("lockstep", 256)
    works = b.work_buffers(dev)
    for rep in range(4):
        sweeps = [w.sweeps + (rep % 2) for w in ws]          # step count changes -> re-capture
        imgs = [torch.ones(g.n_cells, device=dev) for g in grids]
        b.run(projs, imgs, sweeps, [w.beta for w in ws], works=works)
        junk = torch.randn(1 << 20, device=dev).sum()        # eager work between replays
        torch.cuda.synchronize()
        for co, proj, g, w, s_, m in zip(cos, projs, grids, ws, sweeps, imgs):
            img = torch.ones(g.n_cells, device=dev)
            U.mart(co, proj, img, s_, w.beta)
            assert torch.equal(img, m), rep
        assert torch.isfinite(junk)


def test_batch_configuration_sizes_equal_oracle(U):
    # slices of the batched workload's largest sizes (Nr 128 and 256, 32 views
    # over a half turn, 2 Nr bins, sector multiple 2p, 15 sweeps): their rows
    # run past 8 chunks of 64 entries, so the lockstep and persistent kernels
    # take their 16-chunk register bodies; every image equals the problem
    # alone and the FP64 oracle within 1e-4
    dev = torch.device("cuda:0")
    ws = [synth.parallel(f"bs{k}", nr, 32, 2 * nr, 64, phantom="ellipses", n_objects=6, seed=4100 + k,
                         sweeps=15, beta=0.1, dtype="f32")
          for k, nr in enumerate((256, 128, 256, 64))]
    print("case batch configuration sizes", [w.name for w in ws], flush=True)
    grids = [U.Grid.from_workload(w) for w in ws]
    cos = [U.Coeffs.from_workload(g, w) for g, w in zip(grids, ws)]
    assert max(co.max_row for co in cos) > 8 * 64            # the 16-chunk bodies
    Ps = [synth.make_projections(w) for w in ws]
    projs = [torch.as_tensor(P, dtype=torch.float32, device=dev).contiguous() for P in Ps]
    alone = []
    for co, proj, w, g in zip(cos, projs, ws, grids):
        img = torch.ones(g.n_cells, device=dev)
        U.mart(co, proj, img, w.sweeps, w.beta)
        alone.append(img)
    b = U.Batch(cos)
    for mode, block, lds in (("lockstep", 256, False), ("persistent", 1024, True)):
        b.set(mode, block, lds)
        imgs = [torch.ones(g.n_cells, device=dev) for g in grids]
        b.run(projs, imgs, [w.sweeps for w in ws], [w.beta for w in ws])
        torch.cuda.synchronize()
        for a, m in zip(alone, imgs):
            assert torch.equal(a, m), mode
    for w, P, img in zip(ws, Ps, alone):
        f_ref, _, _ = Oracle(w, nthreads=NTHREADS).reconstruct(P)
        f = img.cpu().numpy().astype(np.float64)
        err = np.max(np.abs(f - f_ref)) / np.max(np.abs(f_ref))
        print(f"{w.name} (Nr {w.n_rings}): err_inf {err:.2e}")
        assert err <= 1e-4, w.name


def test_cone_batch_in_cache_sized_groups_equal_alone(U):
    # ten 128-ring, 32-view cone requests: the image lines one step touches
    # (about 21 MB per request) outgrow the last-level cache together, so the
    # lockstep batch runs them in two groups, the second from the step the
    # first ends; every result equals the request alone bit for bit
    dev = torch.device("cuda:0")
    ws = [synth.serve_request(40 + k, 128, 32, 2) for k in range(10)]
    print("case grouped cone batch", len(ws), flush=True)
    g = U.Grid.from_workload(ws[0])
    co = U.Coeffs.from_workload(g, ws[0])
    projs = [synth.make_projections_torch(w, dev, torch.float32).reshape(-1).contiguous() for w in ws]
    alone = []
    for proj, w in zip(projs, ws):
        img = torch.ones(g.n_cells, device=dev)
        U.mart(co, proj, img, w.sweeps, w.beta)
        alone.append(img)
    b = U.Batch([co] * len(ws))
    b.set("lockstep", 256)
    imgs = [torch.ones(g.n_cells, device=dev) for _ in ws]
    b.run(projs, imgs, [w.sweeps for w in ws], [w.beta for w in ws])
    torch.cuda.synchronize()
    for k, (a, m) in enumerate(zip(alone, imgs)):
        assert torch.equal(a, m), k
    b.close()
