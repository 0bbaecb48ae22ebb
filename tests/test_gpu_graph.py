"""mart_run (tol = 0) and the Cartesian remap recorded into a HIP graph by
stream capture: every replay, with eager work and synchronisations between
replays, equals the eager calls bit for bit, for stored reference rows, kept
literal-scheme view rows and rows re-binned on the fly.  tol > 0 on a
capturing stream is refused before anything is enqueued, and captured calls
are not timed."""
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def U():
    assert torch.cuda.is_available()
    import paper_2208_12964_amd as U
    U.lib()
    return U


def workload(kind):
    if kind == "stored":
        return synth.small_cone("gg-cone", n_rings=12, n_views=8, det=24, m=8, sweeps=4), "keep"
    w = synth.small_cone("gg-literal", n_rings=7, n_views=7, det=10, m=7, sweeps=3).with_(
        sector_rule="paper", n_slices=5, rebin=True, binary=True, quarter=True)
    return w, ("keep" if kind == "kept" else "rebin")


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
@pytest.mark.parametrize("kind", ["stored", "kept", "rebin"])
def test_captured_mart_run_replays_equal_eager(U, kind, dtype):
    dev = torch.device("cuda:0")
    w, view_rows = workload(kind)
    grid = U.Grid.from_workload(w)
    co = U.Coeffs.from_workload(grid, w, view_rows=view_rows)
    proj = torch.as_tensor(synth.make_projections(w), dtype=dtype, device=dev).contiguous()
    eager = torch.ones(grid.n_cells, dtype=dtype, device=dev)
    U.mart(co, proj, eager, w.sweeps, w.beta)
    nc = 2 * w.n_rings
    cart_eager = U.to_cartesian(grid, eager, nc)
    torch.cuda.synchronize()

    img = torch.ones(grid.n_cells, dtype=dtype, device=dev)
    work = torch.empty(co.workspace_bytes(dtype), dtype=torch.uint8, device=dev)
    g = torch.cuda.CUDAGraph()
    cart = torch.empty_like(cart_eager)
    with torch.cuda.graph(g):
        cs = torch.cuda.current_stream()                 # the capturing stream
        U.mart_timing(True, stream=cs)
        U.mart(co, proj, img, w.sweeps, w.beta, work=work)
        U.to_cartesian(grid, img, nc, out=cart)
    torch.cuda.synchronize()
    for rep in range(4):
        img.fill_(1.0)                                   # a fill kernel, not a memset node
        cart.fill_(-1.0)
        g.replay()
        junk = torch.randn(1 << 18, device=dev).sum()    # eager work between replays
        torch.cuda.synchronize()
        assert torch.equal(img, eager), (kind, rep)
        assert torch.equal(cart, cart_eager), (kind, rep)
        assert torch.isfinite(junk)
    _, launches = U.mart_timing(False, stream=cs)
    assert launches == 0                                 # the captured call was not timed
    del g


def test_stopping_rule_refused_under_capture(U):
    dev = torch.device("cuda:0")
    w, _ = workload("stored")
    grid = U.Grid.from_workload(w)
    co = U.Coeffs.from_workload(grid, w)
    proj = torch.as_tensor(synth.make_projections(w), dtype=torch.float32, device=dev).contiguous()
    img = torch.ones(grid.n_cells, device=dev)
    work = torch.empty(co.workspace_bytes(torch.float32, 1e-3), dtype=torch.uint8, device=dev)
    dummy = torch.ones(64, device=dev)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    err = None
    with torch.cuda.stream(s):
        g.capture_begin()
        try:
            dummy.mul_(2.0)      # keeps the captured graph non-empty
            U.mart(co, proj, img, 5, w.beta, tol=1e-3, work=work)
        except Exception as e:   # the library refuses before enqueuing anything
            err = e
        finally:
            g.capture_end()
    torch.cuda.synchronize()
    assert err is not None and "captur" in str(err)
    # nothing was enqueued: the image is untouched and the stream still works
    assert torch.equal(img, torch.ones_like(img))
    U.mart(co, proj, img, 2, w.beta, tol=1e-3, work=work)
    torch.cuda.synchronize()
    assert torch.isfinite(img).all()
    del g
