"""Host logic of the serving layer, on the CPU: the seeded request stream,
admission by device-memory footprint, latency percentiles and the
device-side projection generator (run here on the CPU device)."""
import math
from collections import Counter, deque

import numpy as np
import pytest
import torch

import synth
from paper_2208_12964_amd.serve import Admission, Request, percentile


def test_trace_is_seeded_and_poisson():
    a, b = synth.serve_trace(), synth.serve_trace()
    assert [(r.k, r.arrival, r.key, r.sweeps) for r in a] == [(r.k, r.arrival, r.key, r.sweeps) for r in b]
    n = len(a)
    # 20/s over 120 s: count within 4 standard deviations of 2400
    assert abs(n - 2400) < 4 * math.sqrt(2400)
    assert all(0 < x.arrival < 120 for x in a)
    assert all(a[i].arrival < a[i + 1].arrival for i in range(n - 1))
    gaps = np.diff([0.0] + [r.arrival for r in a])
    assert abs(gaps.mean() - 0.05) < 0.005
    keys = Counter(r.key for r in a)
    assert set(keys) == {(nr, p) for nr in (64, 128, 256) for p in (8, 16, 32)}
    assert min(keys.values()) > n / 9 * 0.8
    sw = Counter(r.sweeps for r in a)
    assert set(sw) == set(range(10, 21))
    w = a[0].workload()
    assert (w.n_rings, w.n_slices, w.det_u, w.det_v, w.n_views, w.sector_multiple) == \
        (a[0].n_rings, a[0].n_rings, 2 * a[0].n_rings, 2 * a[0].n_rings, a[0].n_views, a[0].n_views)
    assert w.seed == 5000 and w.span == pytest.approx(2 * math.pi)


def _req(k, t, fp, lane=0):
    r = Request(k, t, (0, 0), torch.empty(0), 1, 0.1)
    r.footprint, r.lane = fp, lane
    return r


def test_admission_fifo_budget_and_slots():
    adm = Admission(100, skip_ahead=False)
    q = deque([_req(0, 0.0, 40), _req(1, 0.1, 40), _req(2, 0.2, 40), _req(3, 0.3, 10)])
    got, rej = adm.pick(q, 0.5, {0: 8})
    assert [r.k for r in got] == [0, 1] and not rej
    assert [r.k for r in q] == [2, 3] and adm.in_use == 80   # FIFO: 3 waits behind 2
    adm.release(got[0])
    got, _ = adm.pick(q, 0.6, {0: 8})
    assert [r.k for r in got] == [2, 3] and adm.in_use == 90 and not q
    # slot limit per lane: FIFO within the lane, other lanes unaffected
    adm2 = Admission(1000, skip_ahead=False)
    q = deque([_req(0, 0, 1, lane=1), _req(1, 0, 1, lane=1), _req(2, 0, 1, lane=2), _req(3, 0, 1, lane=1)])
    free = {1: 1, 2: 4}
    got, _ = adm2.pick(q, 0.0, free)
    assert [r.k for r in got] == [0, 2] and free == {1: 0, 2: 3}
    assert [r.k for r in q] == [1, 3]


def test_admission_skip_ahead_and_starvation_guard():
    adm = Admission(100, skip_ahead=True, max_wait=1.0)
    adm.in_use = 50
    q = deque([_req(0, 0.0, 60, lane=0), _req(1, 0.1, 20, lane=1), _req(2, 0.2, 20, lane=2),
               _req(3, 0.2, 5, lane=0)])
    got, _ = adm.pick(q, 0.5, {0: 8, 1: 8, 2: 8})
    # other lanes pass the request that waits for memory; its own lane does not
    assert [r.k for r in got] == [1, 2] and [r.k for r in q] == [0, 3]
    # once it has waited longer than max_wait nothing passes it
    q = deque([_req(4, 0.0, 60, lane=0), _req(5, 0.1, 5, lane=1)])
    adm.in_use = 50
    got, _ = adm.pick(q, 2.0, {0: 8, 1: 8})
    assert got == [] and [r.k for r in q] == [4, 5]
    # without skip-ahead a memory wait blocks at once
    adm3 = Admission(100, skip_ahead=False)
    adm3.in_use = 50
    q = deque([_req(6, 0.0, 60, lane=0), _req(7, 0.0, 5, lane=1)])
    got, _ = adm3.pick(q, 0.0, {0: 8, 1: 8})
    assert got == [] and len(q) == 2


def test_admission_rejects_oversized():
    adm = Admission(100)
    q = deque([_req(0, 0.0, 101), _req(1, 0.0, 100)])
    got, rej = adm.pick(q, 0.0, {0: 2})
    assert [r.k for r in rej] == [0] and [r.k for r in got] == [1] and not q


def test_admission_counts_resident_coefficients():
    # resident coefficient sets take their share of the budget for good
    adm = Admission(100, skip_ahead=False)
    adm.reserve(30)
    q = deque([_req(0, 0.0, 71), _req(1, 0.0, 40), _req(2, 0.0, 40)])
    got, rej = adm.pick(q, 0.0, {0: 8})
    assert [r.k for r in rej] == [0]                   # more than the 70 left after the resident sets
    assert [r.k for r in got] == [1] and [r.k for r in q] == [2] and adm.in_use == 70
    adm.release(got[0])
    assert adm.in_use == 30                            # the resident share stays


def test_percentile_nearest_rank():
    xs = list(range(1, 201))
    assert percentile(xs, 50) == 100 and percentile(xs, 99) == 198 and percentile(xs, 100) == 200
    assert percentile([3.0], 50) == 3.0
    assert percentile([4, 1, 3, 2], 50) == 2


@pytest.mark.parametrize("w", [synth.small_cone(n_rings=12, n_views=8, det=24, seed=9),
                               synth.parallel("p", 16, 8, 32, 16, phantom="ellipses", seed=3),
                               synth.serve_request(3, 16, 8, 10)])
def test_torch_projections_match_numpy(w):
    a = synth.make_projections(w, noise=False)
    b = synth.make_projections_torch(w, "cpu", noise=False).numpy()
    assert b.shape == a.shape
    assert np.max(np.abs(a - b)) <= 1e-11 * np.max(np.abs(a))
    n = synth.make_projections_torch(w, "cpu")
    assert torch.equal(n, synth.make_projections_torch(w, "cpu"))     # seeded
    assert (n >= 0).all() and not torch.equal(n, torch.as_tensor(b))
