"""The paper's literal variant on the GPU (weights = SEGMENTS): segment
records re-binned per view for view counts that are not whole sector shifts.
Rows, conflict map and lattice equal the FP64 oracle's; MART is within 1e-4
(FP32) / 1e-10 (FP64) of the oracle's, with every view's rows kept or
re-binned on the fly; with kept rows the problems join batches and engines
bit for bit."""
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
        synth.small_cone("gr-cone7", n_rings=7, n_views=7, det=10, m=7, sweeps=4).with_(
            sector_rule="paper", n_slices=5, rebin=True, binary=True),
        synth.small_cone("gr-cone50", n_rings=12, n_views=50, det=18, m=1, sweeps=3).with_(
            sector_rule="paper", n_slices=9, rebin=True, binary=True),
        synth.small_cone("gr-fan", n_rings=24, n_views=50, det=40, m=5, sweeps=5).with_(
            geometry="fan2d", n_slices=1, height=0.0, det_v=1, sector_rule="paper", rebin=True, binary=True,
            phantom="ellipses", n_objects=6),
        synth.parallel("gr-par70", 31, 70, 60, 1, phantom="ellipses", n_objects=6, seed=12, sweeps=5).with_(
            sector_rule="paper", rebin=True, binary=True),
        # most rays miss the disk: empty rows next to rows of up to 47 records
        # in one wavefront's class
        synth.parallel("gr-wide", 24, 50, 121, 1, phantom="ellipses", n_objects=6, seed=14, sweeps=4).with_(
            sector_rule="paper", rebin=True, binary=True, det_half_u=3.7),
        # 30 rays of up to 155 records: one ray per workgroup of 256 lanes
        synth.small_cone("gr-fanlong", n_rings=80, n_views=20, det=30, m=5, sweeps=3).with_(
            geometry="fan2d", n_slices=1, height=0.0, det_v=1, sector_rule="paper", rebin=True, binary=True,
            phantom="ellipses", n_objects=6),
    ]


def rel_err(f, ref):
    return np.max(np.abs(f - ref)) / np.max(np.abs(ref))


@pytest.mark.parametrize("w", cases(), ids=lambda w: w.name)
def test_rows_conflicts_lattice_equal_oracle(U, w):
    g = U.Grid.from_workload(w)
    co = U.Coeffs.from_workload(g, w)
    o = Oracle(w, nthreads=NTHREADS)
    seg = o.segments_view()
    assert co.nnz == seg.count and co.n_rays == o.n_rays
    assert np.array_equal(co.conflicts(), o.rebin_conflicts(seg))
    assert co.lattice == o.colour_rebin(seg)
    rng = np.random.default_rng(3)
    for v in sorted(set([0, 1, w.n_views - 1] + rng.integers(0, w.n_views, 4).tolist())):
        rows = o.rebin_view(seg, v)
        for r in range(o.n_rays):
            cells, lens = co.row(v, r)
            assert np.array_equal(cells, rows.row(r)[0]), (v, r)
            assert np.all(lens == 1.0)


@pytest.mark.parametrize("view_rows", ["keep", "rebin"])
@pytest.mark.parametrize("dtype,tol", [(torch.float32, 1e-4), (torch.float64, 1e-10)])
@pytest.mark.parametrize("w", cases(), ids=lambda w: w.name)
def test_mart_equals_oracle(U, w, dtype, tol, view_rows):
    """Both solvers: every view's rows kept from the colouring pass, and
    rows re-binned from the records on the fly during MART."""
    dev = torch.device("cuda:0")
    P = synth.make_projections(w)
    img, _, g, co = U.reconstruct(w, torch.as_tensor(P, device=dev), dtype=dtype, view_rows=view_rows)
    f_ref, _, lat = Oracle(w, nthreads=NTHREADS).reconstruct_rebin(P)
    assert co.lattice == lat
    assert rel_err(img.cpu().numpy().astype(np.float64), f_ref) <= tol


def test_stopping_rule_and_resume(U):
    dev = torch.device("cuda:0")
    w = cases()[0]
    o = Oracle(w, nthreads=NTHREADS)
    seg = o.segments_view()
    # consistent positive data (P = A f_true for the re-binned rows), so that
    # the relative change of eq. 19 falls below tol
    f_true = 1.0 + np.random.default_rng(1).random(o.n_cells)
    Pn = np.zeros((w.n_views, o.n_rays))
    for v in range(w.n_views):
        rows = o.rebin_view(seg, v)
        for r in range(o.n_rays):
            Pn[v, r] = f_true[rows.row(r)[0]].sum()
    P = torch.as_tensor(Pn, device=dev)
    g = U.Grid.from_workload(w)
    co = U.Coeffs.from_workload(g, w, torch.float64)
    a = torch.ones(g.n_cells, dtype=torch.float64, device=dev)
    U.mart(co, P, a, 5, 0.5)
    b = torch.ones(g.n_cells, dtype=torch.float64, device=dev)
    U.mart(co, P, b, 2, 0.5)
    U.mart(co, P, b, 3, 0.5)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    c = torch.ones(g.n_cells, dtype=torch.float64, device=dev)
    tol = 1e-2
    done = U.mart(co, P, c, 200, 0.5, tol=tol)
    assert 2 < done < 200
    # eq. 19 decides only when to stop: the image is the plain run of `done`
    # sweeps, whose last sweep changed every cell by at most tol while the
    # sweep before changed some cell by more
    f = []
    for k in (done - 2, done - 1, done):
        x = torch.ones(g.n_cells, dtype=torch.float64, device=dev)
        U.mart(co, P, x, k, 0.5)
        f.append(x)
    torch.cuda.synchronize()
    assert torch.equal(c, f[2])
    assert ((f[2] - f[1]) / f[1]).abs().max().item() <= tol
    assert ((f[1] - f[0]) / f[0]).abs().max().item() > tol
    ref = o.mart_rebin(seg, o.colour_rebin(seg), Pn, np.ones(o.n_cells), done, 0.5)
    assert rel_err(c.cpu().numpy(), ref) <= 1e-10


def _alone(U, co, g, proj, w):
    img = torch.ones(g.n_cells, device=proj.device)
    U.mart(co, proj, img, w.sweeps, w.beta)
    return img


def test_kept_rows_join_batches_and_engines(U):
    """Literal-scheme problems whose view rows are kept run in batches
    (lockstep and persistent) and in the serving engine beside stored-row
    problems, each ending bit for bit as mart_run alone; with rows re-binned
    on the fly they are refused."""
    dev = torch.device("cuda:0")
    ws = [cases()[0], synth.parallel("b-par", 16, 8, 32, 16, phantom="ellipses", n_objects=5, seed=31, sweeps=3),
          cases()[2], synth.small_cone("b-cone", n_rings=8, n_views=4, det=16, m=4, n_slices=5, sweeps=3)]
    grids = [U.Grid.from_workload(w) for w in ws]
    cos = [U.Coeffs.from_workload(g, w) for g, w in zip(grids, ws)]
    projs = [torch.as_tensor(synth.make_projections(w), dtype=torch.float32, device=dev).reshape(-1).contiguous()
             for w in ws]
    alone = [_alone(U, co, g, p, w) for co, g, p, w in zip(cos, grids, projs, ws)]
    b = U.Batch(cos)
    for mode, lds in (("lockstep", False), ("persistent", True), ("persistent", False)):
        b.set(mode, 256, lds)
        imgs = [torch.ones(g.n_cells, device=dev) for g in grids]
        b.run(projs, imgs, [w.sweeps for w in ws], [w.beta for w in ws])
        torch.cuda.synchronize()
        for i, (a, m) in enumerate(zip(alone, imgs)):
            assert torch.equal(a, m), (mode, lds, ws[i].name)
    eng = U.Engine(2)
    imgs = [torch.ones(g.n_cells, device=dev) for g in grids]
    todo, slot_of = list(range(len(ws))), {}
    while todo or slot_of:
        while todo and len(slot_of) < 2:
            i = todo.pop(0)
            slot_of[eng.admit(cos[i], projs[i], imgs[i], ws[i].sweeps, ws[i].beta)] = i
        for sl in eng.step(5):
            slot_of.pop(sl)
    torch.cuda.synchronize()
    for i, (a, m) in enumerate(zip(alone, imgs)):
        assert torch.equal(a, m), ("engine", ws[i].name)
    eng.close()
    # the literal problems against the oracle as well
    for i in (0, 2):
        f_ref, _, _ = Oracle(ws[i], nthreads=NTHREADS).reconstruct_rebin(synth.make_projections(ws[i]))
        assert rel_err(alone[i].cpu().numpy().astype(np.float64), f_ref) <= 1e-4
    # rows re-binned on the fly: refused
    co_r = U.Coeffs.from_workload(grids[0], ws[0], view_rows="rebin")
    with pytest.raises(U.USPGError) as e:
        U.Batch([co_r])
    assert e.value.code == -1
    eng = U.Engine(2)
    with pytest.raises(U.USPGError) as e:
        eng.admit(co_r, projs[0], torch.ones(grids[0].n_cells, device=dev), 1, 0.1)
    assert e.value.code == -1
    eng.close()


@pytest.mark.parametrize("w", [cases()[0], cases()[2], cases()[3]], ids=lambda w: w.name)
def test_quarter_tracing_equals_full_and_oracle(U, w):
    """Sec. III.C: tracing one detector quadrant and mirroring its records
    gives the same rows (tie-free scans), so the same colouring, per-view
    work and MART bits as tracing every ray."""
    dev = torch.device("cuda:0")
    g = U.Grid.from_workload(w)
    full = U.Coeffs.from_workload(g, w)
    quart = U.Coeffs.from_workload(g, w.with_(quarter=True))
    assert full.nnz == quart.nnz and full.lattice == quart.lattice
    assert np.array_equal(full.conflicts(), quart.conflicts())
    o = Oracle(w, nthreads=NTHREADS)
    seg = o.segments_view()
    want = np.array([o.rebin_view(seg, v).nnz for v in range(w.n_views)])
    assert np.array_equal(full.view_nnz(), want) and np.array_equal(quart.view_nnz(), want)
    for v in (0, w.n_views // 3, w.n_views - 1):
        rows = o.rebin_view(seg, v)
        for r in range(o.n_rays):
            assert np.array_equal(quart.row(v, r)[0], rows.row(r)[0]), (v, r)
    P = torch.as_tensor(synth.make_projections(w), dtype=torch.float32, device=dev)
    a = torch.ones(g.n_cells, device=dev)
    b = torch.ones(g.n_cells, device=dev)
    U.mart(full, P, a, 3, w.beta)
    U.mart(quart, P, b, 3, w.beta)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
