"""Python binding of libuspg (MART on a uniformly sampled polar / cylindrical
grid, HIP on gfx950).

Thin ctypes marshalling over the C ABI in ``include/uspg.h``: every step of
the computation runs in the library's kernels.  Torch tensors are used only as
device memory and for the current stream.  Loading fails loudly if the
library has not been built (``python paper_2208_12964_amd/build.py``).
"""
from __future__ import annotations

import ctypes as C
import math
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libuspg.so")

# enumerations (mirror include/uspg.h)
SECTORS = {"paper": 0, "multiple": 1, "explicit": 2}
GEOMETRY = {"parallel2d": 0, "fan2d": 1, "cone3d": 2}
WEIGHTS = {"length": 0, "binary": 1, "segments": 2}
DTYPE = {torch.float32: 0, torch.float64: 1}
REMAP = {"point": 0, "bijection": 1}


class USPGError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"uspg error {code}: {msg}")
        self.code = code


class _GridDesc(C.Structure):
    _fields_ = [("n_rings", C.c_int32), ("n_slices", C.c_int32), ("radius", C.c_double),
                ("height", C.c_double), ("sector_rule", C.c_int32), ("sector_multiple", C.c_int32),
                ("sectors", C.POINTER(C.c_int32))]


class _ScanDesc(C.Structure):
    _fields_ = [("geometry", C.c_int32), ("n_views", C.c_int32), ("span", C.c_double),
                ("det_u", C.c_int32), ("det_v", C.c_int32), ("det_half_u", C.c_double),
                ("det_half_v", C.c_double), ("src_axis", C.c_double), ("src_det", C.c_double),
                ("weights", C.c_int32), ("coeff_dtype", C.c_int32), ("colour_u", C.c_int32),
                ("colour_v", C.c_int32), ("quarter", C.c_int32), ("view_rows", C.c_int32),
                ("row_codes", C.c_int32)]


_lib = None


def lib():
    """The loaded library (raises if it is missing)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"libuspg.so is not built ({LIB_PATH}); run paper_2208_12964_amd/build.py")
    L = C.CDLL(LIB_PATH)
    P, I32, I64, D, SZ = C.c_void_p, C.c_int32, C.c_int64, C.c_double, C.c_size_t
    L.uspg_build_grid.argtypes = [C.POINTER(_GridDesc), C.POINTER(P)]
    L.uspg_grid_info.argtypes = [P, P, P, P, P]
    L.uspg_grid_tables.argtypes = [P, P, P]
    L.uspg_free_grid.argtypes = [P]
    L.uspg_free_grid.restype = None
    L.uspg_build_coeffs.argtypes = [P, C.POINTER(_ScanDesc), P, SZ, P, P, C.POINTER(P)]
    L.uspg_debug_alloc.argtypes = [I32, P]
    L.uspg_coeffs_info.argtypes = [P, P, P, P, P, P, P]
    L.uspg_coeffs_row.argtypes = [P, I32, I64, P, P, I32, P]
    L.uspg_coeffs_conflicts.argtypes = [P, P]
    L.uspg_coeffs_view_nnz.argtypes = [P, P]
    L.uspg_coeffs_code_info.argtypes = [P, P, P, P, P]
    L.uspg_free_coeffs.argtypes = [P]
    L.uspg_free_coeffs.restype = None
    L.uspg_mart_workspace_bytes.argtypes = [P, I32, D]
    L.uspg_mart_workspace_bytes.restype = SZ
    L.mart_run.argtypes = [P, I32, P, P, P, SZ, I32, D, D, P, P]
    L.mart_run_noalloc.argtypes = [P, I32, P, P, I32, D, D, P, P]
    L.uspg_to_cartesian.argtypes = [P, I32, P, P, I32, I32, P]
    L.uspg_mart_timing.argtypes = [I32, P, P, P]
    L.uspg_build_batch.argtypes = [I32, P, I32, C.POINTER(P)]
    L.uspg_batch_set.argtypes = [P, I32, I32, I32]
    L.uspg_batch_info.argtypes = [P, P, P, P, P, P]
    L.mart_run_batch.argtypes = [P, P, P, P, P, P, P, P]
    L.uspg_batch_autotune.argtypes = [P, P, P, P, P, I32, P, P, P]
    L.uspg_free_batch.argtypes = [P]
    L.uspg_free_batch.restype = None
    L.uspg_engine_create.argtypes = [I32, I32, I32, C.POINTER(P)]
    L.uspg_engine_admit.argtypes = [P, P, P, P, P, SZ, I32, D, P, P]
    L.uspg_engine_step.argtypes = [P, I32, P, P, I32, P]
    L.uspg_engine_info.argtypes = [P, P, P]
    L.uspg_engine_destroy.argtypes = [P]
    L.uspg_engine_destroy.restype = None
    L.uspg_build_slabs.argtypes = [P, I32, P, C.POINTER(P)]
    L.uspg_slabs_info.argtypes = [P, I32, P, P, P]
    L.uspg_slabs_workspace_bytes.argtypes = [P, I32]
    L.uspg_slabs_workspace_bytes.restype = SZ
    L.mart_run_slabs.argtypes = [P, I32, P, P, P, SZ, I32, D, P]
    L.uspg_free_slabs.argtypes = [P]
    L.uspg_free_slabs.restype = None
    L.uspg_check_lattice.argtypes = [P, I32, I32, I32, P, P]
    L.uspg_check_projections.argtypes = [P, I32, P, P, P]
    L.uspg_last_error.restype = C.c_char_p
    for name in ("uspg_build_grid", "uspg_grid_info", "uspg_grid_tables", "uspg_build_coeffs",
                 "uspg_coeffs_info", "uspg_coeffs_row", "uspg_coeffs_conflicts", "uspg_coeffs_view_nnz", "uspg_coeffs_code_info", "mart_run", "mart_run_noalloc",
                 "uspg_to_cartesian", "uspg_mart_timing", "uspg_build_batch", "uspg_batch_set",
                 "uspg_batch_info", "mart_run_batch", "uspg_batch_autotune", "uspg_engine_create",
                 "uspg_engine_admit", "uspg_engine_step", "uspg_engine_info", "uspg_build_slabs",
                 "uspg_slabs_info", "mart_run_slabs", "uspg_check_lattice", "uspg_check_projections",
                 "uspg_debug_alloc"):
        getattr(L, name).restype = C.c_int
    _lib = L
    return L


def _check(rc: int):
    if rc != 0:
        raise USPGError(rc, lib().uspg_last_error().decode())


def _stream(stream=None) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


class Grid:
    """USPG / USCG grid (Sec. II.A): ``uspg_build_grid``."""

    def __init__(self, n_rings: int, n_slices: int = 1, radius: float = 1.0, height: float = 0.0,
                 sector_rule: str = "multiple", sector_multiple: int = 8, sectors=None):
        L = lib()
        self._keep = None
        ptr = None
        if sectors is not None:
            arr = (C.c_int32 * len(sectors))(*[int(x) for x in sectors])
            self._keep = arr
            ptr = C.cast(arr, C.POINTER(C.c_int32))
        d = _GridDesc(n_rings, n_slices, radius, height, SECTORS[sector_rule], sector_multiple, ptr)
        h = C.c_void_p()
        _check(L.uspg_build_grid(C.byref(d), C.byref(h)))
        self.handle = h
        n_cells, c2d = C.c_int64(), C.c_int64()
        _check(L.uspg_grid_info(h, C.byref(n_cells), C.byref(c2d), None, None))
        self.n_cells, self.cells_per_slice = n_cells.value, c2d.value
        self.n_rings, self.n_slices = n_rings, n_slices

    @classmethod
    def from_workload(cls, w) -> "Grid":
        return cls(w.n_rings, w.n_slices, w.radius, w.height, w.sector_rule, w.sector_multiple)

    def tables(self):
        import numpy as np
        ng = np.zeros(self.n_rings, dtype=np.int32)
        head = np.zeros(self.n_rings + 1, dtype=np.int64)
        _check(lib().uspg_grid_tables(self.handle, ng.ctypes.data_as(C.c_void_p),
                                      head.ctypes.data_as(C.c_void_p)))
        return ng, head

    def close(self):
        if getattr(self, "handle", None):
            lib().uspg_free_grid(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Coeffs:
    """Reference-view coefficients and colouring (Sec. III.A-C):
    ``uspg_build_coeffs``.  Keeps its grid alive."""

    def __init__(self, grid: Grid, geometry: str, n_views: int, span: float, det_u: int, det_v: int = 1,
                 det_half_u: float = 1.0, det_half_v: float = 0.0, src_axis: float = 0.0,
                 src_det: float = 0.0, weights: str = "length", coeff_dtype=torch.float32,
                 colour=(0, 0), stream=None, quarter: bool = False, view_rows: str = "keep",
                 rows: str = "coded"):
        L = lib()
        self.grid = grid
        d = _ScanDesc(GEOMETRY[geometry], n_views, span, det_u, det_v, det_half_u, det_half_v,
                      src_axis, src_det, WEIGHTS[weights], DTYPE[coeff_dtype], colour[0], colour[1],
                      1 if quarter else 0, {"keep": 0, "rebin": 1}[view_rows], {"coded": 0, "stored": 1}[rows])
        # two calls: the size query leaves a pending handle with the counts,
        # the fill carves the coefficients out of a torch work space
        h = C.c_void_p()
        need = C.c_size_t()
        st = C.c_void_p(_stream(stream))
        _check(L.uspg_build_coeffs(grid.handle, C.byref(d), None, 0, C.byref(need), st, C.byref(h)))
        self.handle = h
        dev = torch.device("cuda", torch.cuda.current_device())
        self.workspace = torch.empty(max(need.value, 1), dtype=torch.uint8, device=dev)
        _check(L.uspg_build_coeffs(grid.handle, C.byref(d), C.c_void_p(self.workspace.data_ptr()),
                                   self.workspace.numel(), C.byref(need), st, C.byref(h)))
        self.n_views, self.det_u, self.det_v = n_views, det_u, det_v
        nnz, nr, ku, kv, mr, db = (C.c_int64(), C.c_int64(), C.c_int32(), C.c_int32(), C.c_int32(),
                                   C.c_int64())
        _check(L.uspg_coeffs_info(h, C.byref(nnz), C.byref(nr), C.byref(ku), C.byref(kv), C.byref(mr),
                                  C.byref(db)))
        self.nnz, self.n_rays = nnz.value, nr.value
        self.lattice = (ku.value, kv.value)
        self.max_row, self.device_bytes = mr.value, db.value
        cd, ncr, nxr, cb = C.c_int32(), C.c_int64(), C.c_int64(), C.c_int64()
        _check(L.uspg_coeffs_code_info(h, C.byref(cd), C.byref(ncr), C.byref(nxr), C.byref(cb)))
        self.coded, self.coded_rays, self.explicit_rays, self.code_bytes = bool(cd.value), ncr.value, nxr.value, cb.value

    @classmethod
    def from_workload(cls, grid: Grid, w, coeff_dtype=torch.float32, colour=(0, 0), stream=None,
                      view_rows: str = "keep", rows: str = "coded"):
        weights = "segments" if w.rebin else ("binary" if w.binary else "length")
        return cls(grid, w.geometry, w.n_views, w.span, w.det_u, w.det_v, w.det_half_u, w.det_half_v,
                   w.src_axis, w.src_det, weights, coeff_dtype, colour, stream, quarter=w.quarter,
                   view_rows=view_rows, rows=rows)

    def row(self, view: int, ray: int):
        import numpy as np
        cap = max(self.max_row, 1)
        while True:
            cells = np.zeros(cap, dtype=np.int64)
            lens = np.zeros(cap)
            n = C.c_int32()
            rc = lib().uspg_coeffs_row(self.handle, view, ray, cells.ctypes.data_as(C.c_void_p),
                                       lens.ctypes.data_as(C.c_void_p), cap, C.byref(n))
            if rc == -3 and n.value > cap:    # re-binned rows can outgrow max_row
                cap = n.value
                continue
            _check(rc)
            return cells[:n.value].copy(), lens[:n.value].copy()

    def view_nnz(self):
        """Row entries of every view (the MART work per view)."""
        import numpy as np
        out = np.zeros(self.n_views, dtype=np.int64)
        _check(lib().uspg_coeffs_view_nnz(self.handle, out.ctypes.data_as(C.c_void_p)))
        return out

    def conflicts(self):
        import numpy as np
        mark = np.zeros(self.n_rays, dtype=np.uint8)
        _check(lib().uspg_coeffs_conflicts(self.handle, mark.ctypes.data_as(C.c_void_p)))
        return mark.reshape(self.det_v, self.det_u)

    def workspace_bytes(self, dtype=torch.float32, tol: float = 0.0) -> int:
        return int(lib().uspg_mart_workspace_bytes(self.handle, DTYPE[dtype], tol))

    def check_lattice(self, view: int, lattice=None, stream=None) -> int:
        """``uspg_check_lattice``: hits on cells already hit by another ray of
        the same class in `view` (0 for a valid lattice; default: the chosen one)."""
        ku, kv = lattice if lattice is not None else self.lattice
        n = C.c_int64()
        _check(lib().uspg_check_lattice(self.handle, int(view), int(ku), int(kv), C.c_void_p(_stream(stream)),
                                        C.byref(n)))
        return n.value

    def check_projections(self, proj: torch.Tensor, stream=None) -> int:
        """``uspg_check_projections``: entries of proj that are NaN, infinite or negative."""
        _dev_check(proj, "proj")
        if proj.numel() < self.n_views * self.n_rays:
            raise ValueError("proj holds fewer than n_views x n_rays values")
        n = C.c_int64()
        _check(lib().uspg_check_projections(self.handle, DTYPE[proj.dtype], C.c_void_p(proj.data_ptr()),
                                            C.c_void_p(_stream(stream)), C.byref(n)))
        return n.value

    def close(self):
        if getattr(self, "handle", None):
            lib().uspg_free_coeffs(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _dev_check(t: torch.Tensor, name: str):
    if not (t.is_cuda and t.is_contiguous()):
        raise ValueError(f"{name} must be a contiguous device tensor")


def _problem_check(coeffs, proj: torch.Tensor, image: torch.Tensor, dtype=None):
    """The library reads n_views x rays projections and writes n_cells image
    values through raw pointers: refuse tensors that are too small or of
    another dtype than the image's before any device work."""
    _dev_check(proj, "proj")
    _dev_check(image, "image")
    if image.dtype not in DTYPE or proj.dtype != image.dtype or (dtype is not None and image.dtype != dtype):
        raise ValueError("proj and image must share dtype float32 or float64 (and the caller's dtype)")
    if proj.numel() < coeffs.n_views * coeffs.n_rays:
        raise ValueError(f"proj holds {proj.numel()} values, fewer than n_views x rays = "
                         f"{coeffs.n_views * coeffs.n_rays}")
    if image.numel() < coeffs.grid.n_cells:
        raise ValueError(f"image holds {image.numel()} values, fewer than the grid's {coeffs.grid.n_cells} cells")


def _used_on(stream, *tensors):
    """Tell torch's caching allocator that the library's work on `stream`
    (None: the current stream) uses these tensors, so memory freed on the
    host is not handed out again before that work has run."""
    s = stream if stream is not None else torch.cuda.current_stream()
    for t in tensors:
        if t is not None:
            t.record_stream(s)


def mart(coeffs: Coeffs, proj: torch.Tensor, image: torch.Tensor, n_sweeps: int, beta: float,
         tol: float = 0.0, work: torch.Tensor | None = None, stream=None) -> int:
    """Sp-MART in place on ``image`` (paper numbering): ``mart_run``.
    Returns the number of sweeps run (exact only after a stream sync when tol == 0)."""
    _problem_check(coeffs, proj, image)
    need = coeffs.workspace_bytes(image.dtype, tol)
    if work is None:
        work = torch.empty(need, dtype=torch.uint8, device=image.device)
    _dev_check(work, "work")
    done = C.c_int32()
    _check(lib().mart_run(coeffs.handle, DTYPE[image.dtype], C.c_void_p(proj.data_ptr()),
                          C.c_void_p(image.data_ptr()), C.c_void_p(work.data_ptr()),
                          work.numel() * work.element_size(), n_sweeps, beta, tol, C.byref(done),
                          C.c_void_p(_stream(stream))))
    if stream is not None:
        _used_on(stream, proj, image, work)
    return done.value


NOALLOC_SCRATCH_BYTES = 64 << 20   # USPG_NOALLOC_SCRATCH_BYTES


def mart_run_noalloc(coeffs: Coeffs, proj: torch.Tensor, image: torch.Tensor, n_sweeps: int, beta: float,
                     tol: float = 0.0, stream=None) -> int:
    """Sp-MART in place on ``image`` with the library's fixed work space
    (``mart_run_noalloc``: no device allocation; calls on one device must not
    overlap).  Returns the number of sweeps run."""
    _problem_check(coeffs, proj, image)
    done = C.c_int32()
    _check(lib().mart_run_noalloc(coeffs.handle, DTYPE[image.dtype], C.c_void_p(proj.data_ptr()),
                                  C.c_void_p(image.data_ptr()), n_sweeps, beta, tol, C.byref(done),
                                  C.c_void_p(_stream(stream))))
    if stream is not None:
        _used_on(stream, proj, image)
    return done.value


def to_cartesian(grid: Grid, image: torch.Tensor, nc: int, mode: str = "point",
                 out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """USPG -> Cartesian remap (Sec. II.B): ``uspg_to_cartesian``."""
    _dev_check(image, "image")
    if image.dtype not in DTYPE or image.numel() < grid.n_cells:
        raise ValueError("image must be float32 / float64 with at least the grid's cells")
    if out is None:
        out = torch.empty((grid.n_slices, max(nc, 0), max(nc, 0)), dtype=image.dtype, device=image.device)
    _dev_check(out, "out")
    if out.dtype != image.dtype or out.numel() < grid.n_slices * max(nc, 0) ** 2:
        raise ValueError("out must have the image's dtype and hold n_slices x nc x nc values")
    _check(lib().uspg_to_cartesian(grid.handle, DTYPE[image.dtype], C.c_void_p(image.data_ptr()),
                                   C.c_void_p(out.data_ptr()), nc, REMAP[mode], C.c_void_p(_stream(stream))))
    return out


def mart_timing(enable: bool, stream=None):
    """Turn batch-kernel timing of mart_run on `stream` (None: the current
    stream) on (resets) or off; returns (batch_ms, batch_launches) of that
    stream so far."""
    ms, n = C.c_double(), C.c_int64()
    _check(lib().uspg_mart_timing(1 if enable else 0, C.c_void_p(_stream(stream)), C.byref(ms), C.byref(n)))
    return ms.value, n.value


def debug_alloc(fail_after: int = -1) -> int:
    """``uspg_debug_alloc``: live library device allocations; fail_after > 0
    makes that library allocation from now fail (0 cancels)."""
    live = C.c_int64()
    _check(lib().uspg_debug_alloc(int(fail_after), C.byref(live)))
    return live.value


def _ptr_array(ptrs):
    arr = (C.c_void_p * len(ptrs))(*[C.c_void_p(int(p)) for p in ptrs])
    return arr


class Batch:
    """Many independent problems in one persistent launch: ``uspg_build_batch``,
    ``mart_run_batch``, ``uspg_batch_autotune``.  Keeps its coefficients alive."""

    def __init__(self, coeffs: list, dtype=torch.float32):
        self.coeffs = list(coeffs)
        self.dtype = dtype
        arr = _ptr_array([c.handle.value for c in self.coeffs])
        h = C.c_void_p()
        _check(lib().uspg_build_batch(len(self.coeffs), arr, DTYPE[dtype], C.byref(h)))
        self.handle = h

    def work_buffers(self, device):
        return [torch.empty(c.workspace_bytes(self.dtype), dtype=torch.uint8, device=device)
                for c in self.coeffs]

    MODES = {"persistent": 0, "lockstep": 1}

    def set(self, mode: str = "lockstep", block_threads: int = 256, use_lds: bool = True):
        _check(lib().uspg_batch_set(self.handle, self.MODES[mode], block_threads, 1 if use_lds else 0))

    def info(self):
        md, bt, ul, nl, lb = C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32(), C.c_int64()
        _check(lib().uspg_batch_info(self.handle, C.byref(md), C.byref(bt), C.byref(ul), C.byref(nl),
                                     C.byref(lb)))
        return {"mode": "lockstep" if md.value == 1 else "persistent", "block_threads": bt.value,
                "use_lds": bool(ul.value), "n_lds": nl.value, "lds_bytes": lb.value}

    def _args(self, projs, images, works, sweeps, betas):
        n = len(self.coeffs)
        if not (len(projs) == len(images) == len(works) == len(sweeps) == len(betas) == n):
            raise ValueError("one projection set, image, work buffer, sweep count and beta per problem")
        for co, p, im in zip(self.coeffs, projs, images):
            _problem_check(co, p, im, self.dtype)
        for t in works:
            _dev_check(t, "work")
        wb = (C.c_size_t * n)(*[w.numel() * w.element_size() for w in works])
        sw = (C.c_int32 * n)(*[int(x) for x in sweeps])
        be = (C.c_double * n)(*[float(x) for x in betas])
        return (_ptr_array([p.data_ptr() for p in projs]), _ptr_array([i.data_ptr() for i in images]),
                _ptr_array([w.data_ptr() for w in works]), wb, sw, be)

    def run(self, projs, images, sweeps, betas, works=None, stream=None):
        works = works if works is not None else self.work_buffers(images[0].device)
        P, I, W, wb, sw, be = self._args(projs, images, works, sweeps, betas)
        _check(lib().mart_run_batch(self.handle, P, I, W, wb, sw, be, C.c_void_p(_stream(stream))))
        if stream is not None:
            _used_on(stream, *projs, *images, *works)
        self._keep = (works,)
        return works

    def autotune(self, projs, images, betas, probe_sweeps: int = 1, works=None, stream=None) -> float:
        works = works if works is not None else self.work_buffers(images[0].device)
        P, I, W, wb, sw, be = self._args(projs, images, works, [probe_sweeps] * len(self.coeffs), betas)
        ms = C.c_double()
        _check(lib().uspg_batch_autotune(self.handle, P, I, W, wb, probe_sweeps, be,
                                         C.c_void_p(_stream(stream)), C.byref(ms)))
        return ms.value

    def close(self):
        if getattr(self, "handle", None):
            lib().uspg_free_batch(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Engine:
    """Continuous batching: ``uspg_engine_create`` / ``_admit`` / ``_step`` /
    ``_info`` / ``_destroy``.  Problems enter free slots between step calls
    and leave when their sweeps are done; each result equals ``mart`` run
    alone.  Holds references to every admitted problem's tensors and
    coefficients until its slot is reported finished."""

    def __init__(self, max_slots: int, dtype=torch.float32, coeff_dtype=None):
        self.dtype = dtype
        self.max_slots = max_slots
        h = C.c_void_p()
        _check(lib().uspg_engine_create(max_slots, DTYPE[dtype], DTYPE[coeff_dtype or dtype], C.byref(h)))
        self.handle = h
        self._held = {}
        self._fin = (C.c_int32 * max_slots)()

    def admit(self, coeffs: Coeffs, proj: torch.Tensor, image: torch.Tensor, n_sweeps: int, beta: float,
              work: torch.Tensor | None = None, stream=None) -> int:
        _problem_check(coeffs, proj, image, self.dtype)
        if work is None:
            work = torch.empty(coeffs.workspace_bytes(self.dtype), dtype=torch.uint8, device=image.device)
        _dev_check(work, "work")
        slot = C.c_int32()
        _check(lib().uspg_engine_admit(self.handle, coeffs.handle, C.c_void_p(proj.data_ptr()),
                                       C.c_void_p(image.data_ptr()), C.c_void_p(work.data_ptr()),
                                       work.numel() * work.element_size(), int(n_sweeps), float(beta),
                                       C.c_void_p(_stream(stream)), C.byref(slot)))
        # the engine's later step calls use these buffers on `stream`
        _used_on(stream, proj, image, work)
        self._held[slot.value] = (coeffs, proj, image, work)
        return slot.value

    def step(self, n_steps: int, stream=None) -> list:
        """Advances every admitted problem; returns the slots that finished
        (their images are final once the stream reaches this point)."""
        nf = C.c_int32()
        _check(lib().uspg_engine_step(self.handle, int(n_steps), C.c_void_p(_stream(stream)), self._fin,
                                      self.max_slots, C.byref(nf)))
        done = [self._fin[i] for i in range(nf.value)]
        for sl in done:
            self._held.pop(sl, None)
        return done

    def info(self):
        a, g = C.c_int32(), C.c_int64()
        _check(lib().uspg_engine_info(self.handle, C.byref(a), C.byref(g)))
        return {"active": a.value, "global_step": g.value}

    def close(self):
        if getattr(self, "handle", None):
            lib().uspg_engine_destroy(self.handle)
            self.handle = None
            self._held.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Slabs:
    """z-slab decomposition of one solve: ``uspg_build_slabs`` /
    ``_slabs_info`` / ``_slabs_workspace_bytes`` / ``mart_run_slabs`` /
    ``uspg_free_slabs``.  Keeps its coefficient set alive."""

    def __init__(self, coeffs: Coeffs, n_slabs: int, stream=None):
        self.coeffs = coeffs
        self.n_slabs = n_slabs
        h = C.c_void_p()
        _check(lib().uspg_build_slabs(coeffs.handle, int(n_slabs), C.c_void_p(_stream(stream)), C.byref(h)))
        self.handle = h

    def info(self, slab: int) -> dict:
        b, e, n = C.c_int32(), C.c_int32(), C.c_int64()
        _check(lib().uspg_slabs_info(self.handle, int(slab), C.byref(b), C.byref(e), C.byref(n)))
        return {"slices": (b.value, e.value), "nnz": n.value}

    def workspace_bytes(self, dtype=torch.float32) -> int:
        return lib().uspg_slabs_workspace_bytes(self.handle, DTYPE[dtype])

    def run(self, proj: torch.Tensor, image: torch.Tensor, n_sweeps: int, beta: float,
            work: torch.Tensor | None = None, stream=None):
        """``mart_run_slabs`` in place on ``image`` (paper numbering)."""
        _problem_check(self.coeffs, proj, image)
        if work is None:
            work = torch.empty(self.workspace_bytes(image.dtype), dtype=torch.uint8, device=image.device)
        _dev_check(work, "work")
        _check(lib().mart_run_slabs(self.handle, DTYPE[image.dtype], C.c_void_p(proj.data_ptr()),
                                    C.c_void_p(image.data_ptr()), C.c_void_p(work.data_ptr()),
                                    work.numel() * work.element_size(), int(n_sweeps), float(beta),
                                    C.c_void_p(_stream(stream))))
        _used_on(stream, proj, image, work)

    def close(self):
        if getattr(self, "handle", None):
            lib().uspg_free_slabs(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


EXPORTED = ("uspg_build_grid", "uspg_grid_info", "uspg_grid_tables", "uspg_free_grid",
            "uspg_build_coeffs", "uspg_coeffs_info", "uspg_coeffs_row", "uspg_coeffs_conflicts",
            "uspg_free_coeffs", "uspg_mart_workspace_bytes", "mart_run", "mart_run_noalloc", "uspg_to_cartesian",
            "uspg_coeffs_view_nnz", "uspg_coeffs_code_info",
            "uspg_last_error", "uspg_mart_timing", "uspg_build_batch", "uspg_batch_set",
            "uspg_batch_info", "mart_run_batch", "uspg_batch_autotune", "uspg_free_batch",
            "uspg_engine_create", "uspg_engine_admit", "uspg_engine_step", "uspg_engine_info",
            "uspg_engine_destroy", "uspg_build_slabs", "uspg_slabs_info", "uspg_slabs_workspace_bytes",
            "mart_run_slabs", "uspg_free_slabs", "uspg_check_lattice", "uspg_check_projections",
            "uspg_debug_alloc")


def reconstruct(w, proj: torch.Tensor, dtype=torch.float32, coeff_dtype=None, colour=(0, 0),
                sweeps=None, beta=None, remap_nc: int = 0, view_rows: str = "keep"):
    """Whole path for one workload record: grid, coefficients, MART from a
    ones image, optional Cartesian remap.  Returns (image, cart, grid, coeffs)."""
    grid = Grid.from_workload(w)
    coeffs = Coeffs.from_workload(grid, w, coeff_dtype or dtype, colour, view_rows=view_rows)
    image = torch.ones(grid.n_cells, dtype=dtype, device=proj.device)
    mart(coeffs, proj.to(dtype).contiguous(), image, w.sweeps if sweeps is None else sweeps,
         w.beta if beta is None else beta)
    cart = to_cartesian(grid, image, remap_nc) if remap_nc else None
    return image, cart, grid, coeffs


__all__ = ["Grid", "Coeffs", "Batch", "Engine", "Slabs", "mart", "mart_run_noalloc", "mart_timing", "to_cartesian", "reconstruct", "USPGError", "lib", "LIB_PATH",
           "EXPORTED", "math"]
