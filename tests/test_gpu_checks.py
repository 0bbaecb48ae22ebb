"""Debug checks: the lattice race check (uspg_check_lattice) counts, for
every view tried, the same collisions as the FP64 oracle's rotated rows -
none for the chosen lattice, the oracle's count for smaller lattices - and
the projection check (uspg_check_projections) counts NaN, infinite and
negative entries exactly."""
import numpy as np
import pytest
import torch

import synth
from oracle import Oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def U():
    assert torch.cuda.is_available()
    import paper_2208_12964_amd as U
    U.lib()
    return U


def cases():
    return [synth.get("par2d-32r-8v"),
            synth.small_cone(n_rings=16, n_views=8, det=32, m=8),
            synth.small_cone("cone-wide", n_rings=24, n_views=16, det=40, m=16, n_slices=17).with_(det_v=21)]


def oracle_collisions(o, csr, w, ku, kv):
    """Entries minus distinct cells, summed over the classes of (ku, kv)."""
    total = 0
    for cl in range(ku * kv):
        cu, cw = cl % ku, cl // ku
        parts = [csr.row(wv * w.det_u + u)[0] for wv in range(cw, w.det_v, kv) for u in range(cu, w.det_u, ku)]
        cells = np.concatenate(parts) if parts else np.zeros(0, dtype=np.int64)
        total += len(cells) - len(np.unique(cells))
    return total


@pytest.mark.parametrize("w", cases(), ids=lambda w: w.name)
def test_lattice_check_equals_oracle(U, w):
    g = U.Grid.from_workload(w)
    co = U.Coeffs.from_workload(g, w)
    o = Oracle(w)
    csr0 = o.trace_view(0)
    ku, kv = co.lattice
    smaller = {(1, 1), (max(ku - 1, 1), kv), (ku, max(kv - 1, 1))} - {(ku, kv)}
    for v in sorted({0, 1, w.n_views - 1}):
        csr = o.rotate(csr0, v)
        assert co.check_lattice(v) == 0 == oracle_collisions(o, csr, w, ku, kv), (w.name, v)
        for lat in sorted(smaller):
            got = co.check_lattice(v, lat)
            assert got == oracle_collisions(o, csr, w, *lat), (w.name, v, lat)
            assert got > 0, (w.name, v, lat)     # the chosen lattice is the smallest valid one


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_projection_check(U, dtype):
    w = cases()[1]
    g = U.Grid.from_workload(w)
    co = U.Coeffs.from_workload(g, w)
    proj = torch.as_tensor(synth.make_projections(w), dtype=dtype, device="cuda:0").reshape(-1).contiguous()
    assert co.check_projections(proj) == 0
    bad = proj.clone()
    bad[3] = float("nan")
    bad[100] = -1e-30
    bad[-1] = float("inf")
    bad[-2] = float("-inf")
    assert co.check_projections(bad) == 4
    with pytest.raises(ValueError):
        co.check_projections(proj[:-1])


def test_check_errors(U):
    w = cases()[1]
    g = U.Grid.from_workload(w)
    co = U.Coeffs.from_workload(g, w)
    for view, lat in ((-1, (1, 1)), (w.n_views, (1, 1)), (0, (0, 1)), (0, (w.det_u + 1, 1))):
        with pytest.raises(U.USPGError) as e:
            co.check_lattice(view, lat)
        assert e.value.code == -1
    wl = synth.small_cone("ck-lit", n_rings=7, n_views=7, det=10, m=7, sweeps=1).with_(
        sector_rule="paper", n_slices=5, rebin=True, binary=True)
    cl = U.Coeffs.from_workload(U.Grid.from_workload(wl), wl)
    with pytest.raises(U.USPGError) as e:
        cl.check_lattice(0)
    assert e.value.code == -1


def test_lattice_check_full_size(U):
    """The 256-ring cone (262,144 rays, 109 M entries): no two rays of a class
    of the chosen 2 x 3 lattice share a cell in any view tried, while the
    smaller 2 x 2 lattice has collisions."""
    w = synth.get("cone-256r-32v-hc")
    print("case cone-256r-32v-hc lattice check", flush=True)
    co = U.Coeffs.from_workload(U.Grid.from_workload(w), w)
    assert co.lattice == (2, 3)
    for v in (0, 13, 31):
        assert co.check_lattice(v) == 0, v
    assert co.check_lattice(7, (2, 2)) > 0
