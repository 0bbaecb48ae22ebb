"""The two-call coefficient build through the C ABI (size query, then a fill
into the caller's work space), its refusals, and allocation failures forced
from the host: every failed build returns USPG_E_NOMEM and leaves no library
allocation behind."""
import ctypes as C

import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu

E_ARG, E_NOMEM = -1, -3


@pytest.fixture(scope="module")
def U():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2208_12964_amd as U
    U.lib()
    return U


def dev():
    return torch.device("cuda:0")


def desc(U, w, rows="coded"):
    weights = "segments" if w.rebin else ("binary" if w.binary else "length")
    return U._ScanDesc(U.GEOMETRY[w.geometry], w.n_views, w.span, w.det_u, w.det_v, w.det_half_u, w.det_half_v,
                       w.src_axis, w.src_det, U.WEIGHTS[weights], 0, 0, 0, 1 if w.quarter else 0, 0,
                       {"coded": 0, "stored": 1}[rows])


def query(U, grid, d):
    L = U.lib()
    h, need = C.c_void_p(), C.c_size_t()
    rc = L.uspg_build_coeffs(grid.handle, C.byref(d), None, 0, C.byref(need), None, C.byref(h))
    return rc, h, need.value


def fill(U, grid, d, ws, nbytes, h):
    need = C.c_size_t()
    rc = U.lib().uspg_build_coeffs(grid.handle, C.byref(d), C.c_void_p(ws.data_ptr()), nbytes, C.byref(need),
                                   None, C.byref(h))
    return rc, need.value


CASES = [synth.small_cone("b-cone", n_rings=12, n_views=8, det=24, m=8),
         synth.get("par2d-32r-8v"),
         synth.small_cone("b-lit", n_rings=7, n_views=7, det=10, m=7, sweeps=3).with_(
             sector_rule="paper", n_slices=5, rebin=True, binary=True)]


@pytest.mark.parametrize("w", CASES, ids=lambda w: w.name)
def test_query_then_fill(U, w):
    L = U.lib()
    grid = U.Grid.from_workload(w)
    d = desc(U, w)
    live0 = U.debug_alloc()
    rc, h, need = query(U, grid, d)
    assert rc == 0 and need > 0 and h.value
    # a pending handle is refused by the solver and the row reader
    img = torch.ones(grid.n_cells, device=dev())
    proj = torch.ones(w.n_views * w.det_u * w.det_v, device=dev())
    work = torch.empty(1 << 24, dtype=torch.uint8, device=dev())
    assert L.mart_run(h, 0, C.c_void_p(proj.data_ptr()), C.c_void_p(img.data_ptr()),
                      C.c_void_p(work.data_ptr()), work.numel(), 1, 0.1, 0.0, None, None) == E_ARG
    # a short work space: E_NOMEM, nothing written, the handle stays pending
    ws = torch.full((need,), 0xAB, dtype=torch.uint8, device=dev())
    rc, need2 = fill(U, grid, d, ws, need - 1, h)
    assert rc == E_NOMEM and need2 == need and h.value
    torch.cuda.synchronize()
    assert bool((ws == 0xAB).all())
    # another scan with this pending handle is refused
    d_other = desc(U, w)
    d_other.n_views += 1
    assert fill(U, grid, d_other, ws, need, h)[0] == E_ARG
    # the fill: every array inside the work space, same solve as the binding's build
    rc, _ = fill(U, grid, d, ws, need, h)
    assert rc == 0
    db = C.c_int64()
    assert L.uspg_coeffs_info(h, None, None, None, None, None, C.byref(db)) == 0 and db.value == need
    P = torch.as_tensor(synth.make_projections(w), dtype=torch.float32, device=dev()).contiguous()
    a = torch.ones(grid.n_cells, device=dev())
    work = torch.empty(L.uspg_mart_workspace_bytes(h, 0, 0.0), dtype=torch.uint8, device=dev())
    assert L.mart_run(h, 0, C.c_void_p(P.data_ptr()), C.c_void_p(a.data_ptr()), C.c_void_p(work.data_ptr()),
                      work.numel(), w.sweeps, w.beta, 0.0, None, None) == 0
    co = U.Coeffs.from_workload(grid, w)
    b = torch.ones(grid.n_cells, device=dev())
    U.mart(co, P, b, w.sweeps, w.beta)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    L.uspg_free_coeffs(h)
    co.close()
    assert U.debug_alloc() == live0


def test_fill_without_query_and_free_pending(U):
    L = U.lib()
    w = CASES[0]
    grid = U.Grid.from_workload(w)
    d = desc(U, w)
    live0 = U.debug_alloc()
    rc, h, need = query(U, grid, d)
    assert rc == 0
    assert U.debug_alloc() > live0            # the pending handle keeps its counts
    L.uspg_free_coeffs(h)
    assert U.debug_alloc() == live0
    ws = torch.empty(need, dtype=torch.uint8, device=dev())
    h = C.c_void_p()
    assert fill(U, grid, d, ws, need, h)[0] == 0 and h.value   # counts run in the fill call
    nnz = C.c_int64()
    assert L.uspg_coeffs_info(h, C.byref(nnz), None, None, None, None, None) == 0 and nnz.value > 0
    L.uspg_free_coeffs(h)
    assert U.debug_alloc() == live0


@pytest.mark.parametrize("w", CASES, ids=lambda w: w.name)
def test_forced_allocation_failures_leak_nothing(U, w):
    # the k-th library allocation of a build fails: E_NOMEM, and every
    # allocation the build had made is freed again
    grid = U.Grid.from_workload(w)
    live0 = U.debug_alloc()
    failed = 0
    for k in range(1, 64):
        U.debug_alloc(k)
        try:
            co = U.Coeffs.from_workload(grid, w)
        except U.USPGError as e:
            assert e.code == E_NOMEM, (k, str(e))
            failed += 1
        else:
            co.close()
            U.debug_alloc(0)
            break
        finally:
            torch.cuda.synchronize()
        assert U.debug_alloc() == live0, k
    else:
        pytest.fail("the build kept failing")
    U.debug_alloc(0)
    assert failed >= 3 and U.debug_alloc() == live0
    print(f"{w.name}: {failed} forced failures, none leaked")
