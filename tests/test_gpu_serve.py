"""Continuous batching: problems admitted into the engine at different
steps, and requests served through the server's lanes, each end bit for
bit equal to mart_run on the problem alone, and within 1e-4 (FP32) /
1e-10 (FP64) of the FP64 oracle."""
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


def problems(seed=21):
    rng = np.random.default_rng(seed)
    out = []
    for k in range(6):
        nr = int(rng.choice([8, 16, 24, 32]))
        p = int(rng.choice([4, 8, 16]))
        out.append(synth.parallel(f"e{k}", nr, p, 2 * nr, 2 * p, phantom="ellipses", n_objects=6,
                                  seed=6000 + k, sweeps=int(rng.integers(2, 7)), beta=0.1))
    out.append(synth.small_cone("ec0", n_rings=10, n_views=8, det=20, m=8, n_slices=6, sweeps=3))
    out.append(synth.serve_request(1, 12, 4, 4))
    return out


def rel_err(f, ref):
    return np.max(np.abs(f - ref)) / np.max(np.abs(ref))


@pytest.mark.parametrize("dtype,tol", [(torch.float32, 1e-4), (torch.float64, 1e-10)])
def test_engine_staggered_admission_equals_alone(U, dtype, tol):
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
    eng = U.Engine(3, dtype)
    imgs = [torch.ones(g.n_cells, dtype=dtype, device=dev) for g in grids]
    rng = np.random.default_rng(3)
    todo = list(range(len(ws)))
    slot_of, finished = {}, []
    while todo or slot_of:
        while todo and len(slot_of) < 3 and (not slot_of or rng.random() < 0.6):
            i = todo.pop(0)
            s = eng.admit(cos[i], projs[i], imgs[i], ws[i].sweeps, ws[i].beta)
            assert s not in slot_of
            slot_of[s] = i
        if len(slot_of) == 3 and todo:
            with pytest.raises(U.USPGError) as e:
                eng.admit(cos[todo[0]], projs[todo[0]], imgs[todo[0]], 1, 0.1)
            assert e.value.code == -3
        for s in eng.step(int(rng.integers(1, 9))):
            finished.append(slot_of.pop(s))
    torch.cuda.synchronize()
    assert sorted(finished) == list(range(len(ws)))
    assert eng.info()["active"] == 0
    for i, (a, m) in enumerate(zip(alone, imgs)):
        assert torch.equal(a, m), ws[i].name
    for i in (0, len(ws) - 2, len(ws) - 1):
        f_ref, _, _ = Oracle(ws[i], nthreads=NTHREADS).reconstruct(Ps[i])
        assert rel_err(imgs[i].cpu().numpy().astype(np.float64), f_ref) <= tol, ws[i].name
    eng.close()


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_engine_wide_problems_equal_alone(U, dtype):
    """Problems whose classes fill the chip alone (256-ring serving requests,
    43,776 rays per class) run each step with the single-problem kernel, the
    others share the lockstep launch; every result is still bit for bit the
    one mart_run gives alone."""
    dev = torch.device("cuda:0")
    ws = [synth.serve_request(11, 256, 8, 1), synth.serve_request(12, 32, 8, 3),
          synth.serve_request(13, 256, 8, 1).with_(seed=5017)]
    print("case wide engine", dtype, [w.name for w in ws], flush=True)
    grids = [U.Grid.from_workload(w) for w in ws]
    cos = [U.Coeffs.from_workload(g, w, dtype) for g, w in zip(grids, ws)]
    projs = [synth.make_projections_torch(w, dev, dtype).reshape(-1).contiguous() for w in ws]
    alone = []
    for co, proj, w, g in zip(cos, projs, ws, grids):
        img = torch.ones(g.n_cells, dtype=dtype, device=dev)
        U.mart(co, proj, img, w.sweeps, w.beta)
        alone.append(img)
    eng = U.Engine(3, dtype)
    imgs = [torch.ones(g.n_cells, dtype=dtype, device=dev) for g in grids]
    slot_of = {eng.admit(cos[0], projs[0], imgs[0], ws[0].sweeps, ws[0].beta): 0}
    finished = []
    for s in eng.step(5):
        finished.append(slot_of.pop(s))
    for i in (1, 2):
        slot_of[eng.admit(cos[i], projs[i], imgs[i], ws[i].sweeps, ws[i].beta)] = i
    while slot_of:
        for s in eng.step(7):
            finished.append(slot_of.pop(s))
    torch.cuda.synchronize()
    assert sorted(finished) == [0, 1, 2]
    for i, (a, m) in enumerate(zip(alone, imgs)):
        assert torch.equal(a, m), ws[i].name


def test_engine_128_ring_cone_requests_equal_oracle(U):
    # two 128-ring cone requests (fewer rays per class than fill the chip, so
    # they share the lockstep launch, whose rows of up to 8 chunks take its
    # 8-chunk body) admitted at different steps beside a small one: each
    # result equals the request alone and the FP64 oracle within 1e-4
    dev = torch.device("cuda:0")
    ws = [synth.serve_request(21, 128, 8, 3), synth.serve_request(22, 128, 16, 2),
          synth.serve_request(23, 16, 8, 3)]
    print("case 128-ring engine", [w.name for w in ws], flush=True)
    grids = [U.Grid.from_workload(w) for w in ws]
    cos = [U.Coeffs.from_workload(g, w) for g, w in zip(grids, ws)]
    assert 5 * 64 < max(co.max_row for co in cos[:2]) <= 8 * 64
    Ps = [synth.make_projections(w) for w in ws]
    projs = [torch.as_tensor(P, dtype=torch.float32, device=dev).reshape(-1).contiguous() for P in Ps]
    alone = []
    for co, proj, w, g in zip(cos, projs, ws, grids):
        img = torch.ones(g.n_cells, device=dev)
        U.mart(co, proj, img, w.sweeps, w.beta)
        alone.append(img)
    eng = U.Engine(4)
    imgs = [torch.ones(g.n_cells, device=dev) for g in grids]
    slot_of = {eng.admit(cos[0], projs[0], imgs[0], ws[0].sweeps, ws[0].beta): 0}
    finished = []
    for s in eng.step(11):
        finished.append(slot_of.pop(s))
    for i in (1, 2):
        slot_of[eng.admit(cos[i], projs[i], imgs[i], ws[i].sweeps, ws[i].beta)] = i
    while slot_of:
        for s in eng.step(13):
            finished.append(slot_of.pop(s))
    torch.cuda.synchronize()
    assert sorted(finished) == [0, 1, 2]
    for i, (a, m) in enumerate(zip(alone, imgs)):
        assert torch.equal(a, m), ws[i].name
        f_ref, _, _ = Oracle(ws[i], nthreads=NTHREADS).reconstruct(Ps[i])
        err = rel_err(m.cpu().numpy().astype(np.float64), f_ref)
        print(f"{ws[i].name}: err_inf {err:.2e}")
        assert err <= 1e-4, ws[i].name
    eng.close()


def test_engine_errors(U):
    dev = torch.device("cuda:0")
    w = problems()[0]
    g = U.Grid.from_workload(w)
    co64 = U.Coeffs.from_workload(g, w, torch.float64)
    co32 = U.Coeffs.from_workload(g, w, torch.float32)
    proj = torch.as_tensor(synth.make_projections(w), dtype=torch.float32, device=dev)
    img = torch.ones(g.n_cells, device=dev)
    eng = U.Engine(2, torch.float32)
    for co, sw, beta in ((co64, 2, 0.1), (co32, 0, 0.1), (co32, 2, 0.0)):
        with pytest.raises(U.USPGError) as e:
            eng.admit(co, proj, img, sw, beta)
        assert e.value.code == -1
    small = torch.empty(16, dtype=torch.uint8, device=dev)
    with pytest.raises(U.USPGError) as e:
        eng.admit(co32, proj, img, 2, 0.1, work=small)
    assert e.value.code == -3
    assert eng.step(4) == [] and eng.info() == {"active": 0, "global_step": 0}
    with pytest.raises(U.USPGError):
        U.Engine(0)
    eng.close()


def _serve_requests(dev, n=14, seed=8):
    rng = np.random.default_rng(seed)
    items = []
    for k in range(n):
        nr = int(rng.choice([8, 12, 16]))
        p = int(rng.choice([4, 8]))
        items.append(synth.ServeItem(k, 0.02 * k, nr, p, int(rng.integers(2, 6))))
    return items


@pytest.mark.parametrize("shared_stream", [False, True], ids=["lane-streams", "shared-stream"])
def test_server_results_equal_alone_and_oracle(U, shared_stream):
    from paper_2208_12964_amd.serve import Request, Server, serve_fifo

    dev = torch.device("cuda:0")
    items = _serve_requests(dev)
    geo = {}

    def geometry(key):
        w = synth.serve_request(0, key[0], key[1], 1)
        g = U.Grid.from_workload(w)
        geo[key] = (g, U.Coeffs.from_workload(g, w))
        return geo[key]

    projs = [synth.make_projections_torch(it.workload(), dev, torch.float32).reshape(-1) for it in items]
    reqs = [Request(it.k, it.arrival, it.key, pr, it.sweeps, 0.1) for it, pr in zip(items, projs)]
    # budget: the resident coefficient sets (charged as their geometries are
    # built) plus about three of the largest requests at once, so admission waits
    srv = Server(geometry, budget=1, steps_per_call=5, shared_stream=shared_stream)
    for r in reqs:
        srv.prepare(r)
    assert srv.admission.resident == sum(co.device_bytes for _, co in geo.values()) > 0
    srv.admission.budget = srv.admission.resident + 3 * max(r.footprint for r in reqs)
    cancelled = reqs[5]
    assert srv.cancel(cancelled)
    stats = srv.run(reqs)
    srv.close()
    assert stats["completed"] == len(reqs) - 1 and stats["rejected"] == 0
    assert stats["p99_s"] >= stats["p50_s"] > 0 and srv.admission.in_use == srv.admission.resident
    assert cancelled.image is None and cancelled.t_done is None
    fifo_reqs = [Request(r.k, r.arrival, r.key, r.proj, r.sweeps, r.beta) for r in reqs]
    fifo = serve_fifo(geometry, fifo_reqs)
    assert fifo["completed"] == len(reqs)
    for r, q in zip(reqs, fifo_reqs):
        if r is cancelled:
            continue
        assert torch.equal(r.image, q.image), r.k
    for it, r in list(zip(items, reqs))[:3]:
        w = it.workload()
        f_ref, _, _ = Oracle(w, nthreads=NTHREADS).reconstruct(
            r.proj.reshape(w.n_views, w.det_v, w.det_u).cpu().numpy().astype(np.float64))
        assert rel_err(r.image.cpu().numpy().astype(np.float64), f_ref) <= 1e-4, it
