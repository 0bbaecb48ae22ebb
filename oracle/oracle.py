"""ctypes binding of the FP64 CPU oracle (test infrastructure only).

The compiled library is ``oracle/liboracle.so`` built from ``uspg_oracle.c``
with gcc.  ``build_oracle()`` compiles it; loading never builds implicitly.
"""

from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "uspg_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

GEOM = {"parallel2d": 0, "fan2d": 1, "cone3d": 2}
RULE = {"paper": 0, "multiple": 1, "explicit": 2}

_lib = None


# gcc flags of a build with AddressSanitizer and UndefinedBehaviorSanitizer
# (host code only; the tests load such a build with the ASan runtime preloaded)
SANITIZE = ["-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
            "-fno-omit-frame-pointer"]


def build_oracle(force: bool = True, out: str | None = None, sanitize: bool = False) -> str:
    """Compile the oracle shared library with gcc (OpenMP, -O2, IEEE math);
    `sanitize` builds it with the sanitizers into `out` instead."""
    out = out or _LIB
    if force or not os.path.exists(out):
        opt = SANITIZE if sanitize else ["-O2"]
        cmd = ["gcc", *opt, "-std=c11", "-fopenmp", "-fPIC", "-shared", "-Wall",
               "-Wno-unused-function", _SRC, "-o", out + ".tmp", "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(out + ".tmp", out)
    return out


def _load():
    global _lib
    if _lib is not None:
        return _lib
    # USPG_ORACLE_LIB points the tests at another oracle build: a deliberately
    # broken one (mutation checks of the pins) or a sanitized one; never set
    # in normal runs.
    path = os.environ.get("USPG_ORACLE_LIB", _LIB)
    if not os.path.exists(path):
        raise RuntimeError(f"oracle library missing: {path} (run __graft_entry__.build())")
    lib = C.CDLL(path)
    P, I, I64, D = C.c_void_p, C.c_int, C.c_int64, C.c_double
    lib.orc_sector_counts.argtypes = [I, I, I, P, P]
    lib.orc_create.restype = P
    lib.orc_create.argtypes = [I, I, D, D, P, I, I, D, I, I, D, D, D, D, I]
    lib.orc_destroy.argtypes = [P]
    lib.orc_ncells.restype = I64
    lib.orc_ncells.argtypes = [P]
    lib.orc_nrays.restype = I64
    lib.orc_nrays.argtypes = [P]
    lib.orc_grid_tables.argtypes = [P, P, P]
    lib.orc_ray.argtypes = [P, I, I64, P, P]
    lib.orc_trace_line.argtypes = [P, P, P, P, P, I, P]
    lib.orc_trace_view.restype = I64
    lib.orc_trace_view.argtypes = [P, I, P, P, P, I64, I]
    lib.orc_shift_ok.argtypes = [P]
    lib.orc_rotate_cells.argtypes = [P, I, P, I64, P]
    lib.orc_conflict_offsets.argtypes = [P, P, P, P]
    lib.orc_colour.argtypes = [P, P, P, P]
    lib.orc_mart_ray.argtypes = [P, P, I64, D, P, D]
    lib.orc_mart.argtypes = [P, P, P, P, I, I, P, P, I, D, D, P, I]
    lib.orc_remap.argtypes = [P, P, P, I, I]
    lib.orc_segments_line.argtypes = [P, P, P, P, P, P, P, I, P]
    lib.orc_segments_view.restype = I64
    lib.orc_segments_view.argtypes = [P, P, P, P, P, P, I64, I]
    lib.orc_rebin_view.restype = I64
    lib.orc_rebin_view.argtypes = [P, I, P, P, P, P, P, P, P, I64, I]
    lib.orc_rebin_conflicts.argtypes = [P, P, P, P, P, P, P, I]
    lib.orc_mart_rebin.argtypes = [P, P, P, P, P, P, I, I, P, P, I, D, I]
    _lib = lib
    return lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def sector_counts(rule: str, m: int, nr: int, table=None) -> np.ndarray:
    lib = _load()
    ng = np.zeros(nr, dtype=np.int32)
    tab = None if table is None else np.ascontiguousarray(table, dtype=np.int32)
    rc = lib.orc_sector_counts(RULE[rule], int(m), int(nr), None if tab is None else _ptr(tab), _ptr(ng))
    if rc != 0:
        raise ValueError(f"orc_sector_counts failed ({rc})")
    return ng


class CSR:
    """Coefficient rows: rowptr [rays+1], cells [nnz] (paper numbering), lens [nnz]."""

    def __init__(self, rowptr, cells, lens):
        self.rowptr, self.cells, self.lens = rowptr, cells, lens

    @property
    def nnz(self) -> int:
        return int(self.rowptr[-1])

    def row(self, r: int):
        b, e = int(self.rowptr[r]), int(self.rowptr[r + 1])
        return self.cells[b:e], self.lens[b:e]


class Segments:
    """Segment records of the reference view (Alg. 1, tracing of the reference view): per ray a
    run of (slice, ring, azimuth at entry, azimuth at exit)."""

    def __init__(self, segptr, slice_, ring, phia, phib):
        self.segptr, self.slice, self.ring, self.phia, self.phib = segptr, slice_, ring, phia, phib

    @property
    def count(self) -> int:
        return int(self.segptr[-1])

    def ray(self, r: int):
        b, e = int(self.segptr[r]), int(self.segptr[r + 1])
        return self.slice[b:e], self.ring[b:e], self.phia[b:e], self.phib[b:e]

    def args(self):
        return (_ptr(self.segptr), _ptr(self.slice), _ptr(self.ring), _ptr(self.phia), _ptr(self.phib))


class Oracle:
    """One (grid, scan) problem in the oracle."""

    def __init__(self, w, sectors=None, nthreads: int = 1):
        lib = _load()
        self.w = w
        if sectors is None:
            sectors = sector_counts(w.sector_rule, w.sector_multiple, w.n_rings)
        self.ng = np.ascontiguousarray(sectors, dtype=np.int32)
        self.nthreads = nthreads
        h = lib.orc_create(w.n_rings, w.n_slices, w.radius, w.height, _ptr(self.ng),
                           GEOM[w.geometry], w.n_views, w.span, w.det_u, w.det_v,
                           w.det_half_u, w.det_half_v, w.src_axis, w.src_det, int(w.binary))
        if not h:
            raise ValueError("orc_create rejected the problem")
        self._h = h
        self.lib = lib
        self.n_cells = int(lib.orc_ncells(h))
        self.n_rays = int(lib.orc_nrays(h))
        self.head = np.zeros(w.n_rings + 1, dtype=np.int64)
        lib.orc_grid_tables(h, _ptr(self.ng), _ptr(self.head))

    def __del__(self):
        if getattr(self, "_h", None):
            self.lib.orc_destroy(self._h)
            self._h = None

    # -- rays and tracing -------------------------------------------------
    def ray(self, view: int, r: int):
        S = np.zeros(3)
        D = np.zeros(3)
        self.lib.orc_ray(self._h, view, r, _ptr(S), _ptr(D))
        return S, D

    def trace_line(self, S, D):
        S = np.ascontiguousarray(S, dtype=np.float64)
        D = np.ascontiguousarray(D, dtype=np.float64)
        cap = 4096
        while True:
            cells = np.zeros(cap, dtype=np.int64)
            lens = np.zeros(cap)
            need = C.c_int(0)
            n = self.lib.orc_trace_line(self._h, _ptr(S), _ptr(D), _ptr(cells), _ptr(lens), cap,
                                        C.byref(need))
            if n >= 0:
                return cells[:n].copy(), lens[:n].copy()
            cap = need.value

    def trace_view(self, view: int = 0) -> CSR:
        rowptr = np.zeros(self.n_rays + 1, dtype=np.int64)
        nnz = self.lib.orc_trace_view(self._h, view, _ptr(rowptr), None, None, 0, self.nthreads)
        cells = np.zeros(max(nnz, 1), dtype=np.int64)
        lens = np.zeros(max(nnz, 1))
        got = self.lib.orc_trace_view(self._h, view, _ptr(rowptr), _ptr(cells), _ptr(lens), nnz,
                                      self.nthreads)
        if got != nnz:
            raise RuntimeError("orc_trace_view inconsistent")
        return CSR(rowptr, cells[:nnz], lens[:nnz])

    def shift_ok(self) -> bool:
        return self.lib.orc_shift_ok(self._h) == 0

    def rotate(self, csr0: CSR, view: int) -> CSR:
        out = np.zeros(max(csr0.nnz, 1), dtype=np.int64)
        cells = np.ascontiguousarray(csr0.cells)
        rc = self.lib.orc_rotate_cells(self._h, view, _ptr(cells), csr0.nnz, _ptr(out))
        if rc != 0:
            raise ValueError(f"rotation not exact for this grid ({rc})")
        return CSR(csr0.rowptr, out[:csr0.nnz], csr0.lens)

    # -- colouring ----------------------------------------------------------
    def conflict_offsets(self, csr0: CSR) -> np.ndarray:
        mark = np.zeros(self.n_rays, dtype=np.uint8)
        self.lib.orc_conflict_offsets(self._h, _ptr(csr0.rowptr), _ptr(np.ascontiguousarray(csr0.cells)),
                                      _ptr(mark))
        return mark.reshape(self.w.det_v, self.w.det_u)

    def colour(self, csr0: CSR, force=None):
        mark = np.ascontiguousarray(self.conflict_offsets(csr0).ravel())
        ku = C.c_int(force[0] if force else 0)
        kv = C.c_int(force[1] if force else 0)
        rc = self.lib.orc_colour(self._h, _ptr(mark), C.byref(ku), C.byref(kv))
        if rc != 0:
            raise ValueError("lattice rejected")
        return ku.value, kv.value

    # -- MART -----------------------------------------------------------------
    def mart(self, csr0: CSR, lattice, P, f0, sweeps, beta, tol=0.0, nthreads=None):
        """MART in the order views > lattice classes > rays of the class
        (ascending ray index), from the reference rows rotated to each view."""
        P = np.ascontiguousarray(P, dtype=np.float64).ravel()
        f = np.array(f0, dtype=np.float64, copy=True).ravel()
        done = C.c_int(0)
        rc = self.lib.orc_mart(self._h, _ptr(csr0.rowptr), _ptr(np.ascontiguousarray(csr0.cells)),
                               _ptr(np.ascontiguousarray(csr0.lens)), int(lattice[0]), int(lattice[1]),
                               _ptr(P), _ptr(f), int(sweeps), float(beta), float(tol),
                               C.byref(done), int(nthreads if nthreads is not None else self.nthreads))
        if rc != 0:
            raise ValueError(f"orc_mart failed ({rc})")
        self.sweeps_done = done.value
        return f

    def mart_ray(self, ids, a, P, f, beta):
        ids = np.ascontiguousarray(ids, dtype=np.int64)
        a = np.ascontiguousarray(a, dtype=np.float64)
        self.lib.orc_mart_ray(_ptr(ids), _ptr(a), len(ids), float(P), _ptr(f), float(beta))

    # -- remap ------------------------------------------------------------
    def remap(self, f, nc: int, mode: str = "point") -> np.ndarray:
        f = np.ascontiguousarray(f, dtype=np.float64)
        cart = np.zeros((self.w.n_slices, nc, nc))
        rc = self.lib.orc_remap(self._h, _ptr(f), _ptr(cart), nc, {"point": 0, "bijection": 1}[mode])
        if rc != 0:
            raise ValueError(f"orc_remap failed ({rc})")
        return cart

    # -- the paper's literal variant: re-binned segment records -----------
    def segments_line(self, S, D):
        S = np.ascontiguousarray(S, dtype=np.float64)
        D = np.ascontiguousarray(D, dtype=np.float64)
        cap = 4096
        while True:
            sl = np.zeros(cap, dtype=np.int32)
            rg = np.zeros(cap, dtype=np.int32)
            pa = np.zeros(cap)
            pb = np.zeros(cap)
            need = C.c_int(0)
            n = self.lib.orc_segments_line(self._h, _ptr(S), _ptr(D), _ptr(sl), _ptr(rg), _ptr(pa), _ptr(pb),
                                           cap, C.byref(need))
            if n >= 0:
                return sl[:n].copy(), rg[:n].copy(), pa[:n].copy(), pb[:n].copy()
            cap = need.value

    def segments_view(self) -> Segments:
        segptr = np.zeros(self.n_rays + 1, dtype=np.int64)
        ns = self.lib.orc_segments_view(self._h, _ptr(segptr), None, None, None, None, 0, self.nthreads)
        sl = np.zeros(max(ns, 1), dtype=np.int32)
        rg = np.zeros(max(ns, 1), dtype=np.int32)
        pa = np.zeros(max(ns, 1))
        pb = np.zeros(max(ns, 1))
        got = self.lib.orc_segments_view(self._h, _ptr(segptr), _ptr(sl), _ptr(rg), _ptr(pa), _ptr(pb), ns,
                                         self.nthreads)
        if got != ns:
            raise RuntimeError("orc_segments_view inconsistent")
        return Segments(segptr, sl, rg, pa, pb)

    def rebin_view(self, seg: Segments, view: int) -> CSR:
        rowptr = np.zeros(self.n_rays + 1, dtype=np.int64)
        nnz = self.lib.orc_rebin_view(self._h, view, *seg.args(), _ptr(rowptr), None, 0, self.nthreads)
        cells = np.zeros(max(nnz, 1), dtype=np.int64)
        got = self.lib.orc_rebin_view(self._h, view, *seg.args(), _ptr(rowptr), _ptr(cells), nnz, self.nthreads)
        if got != nnz:
            raise RuntimeError("orc_rebin_view inconsistent")
        return CSR(rowptr, cells[:nnz], np.ones(nnz))

    def rebin_conflicts(self, seg: Segments) -> np.ndarray:
        mark = np.zeros(self.n_rays, dtype=np.uint8)
        self.lib.orc_rebin_conflicts(self._h, *seg.args(), _ptr(mark), self.nthreads)
        return mark.reshape(self.w.det_v, self.w.det_u)

    def colour_rebin(self, seg: Segments, force=None):
        mark = np.ascontiguousarray(self.rebin_conflicts(seg).ravel())
        ku = C.c_int(force[0] if force else 0)
        kv = C.c_int(force[1] if force else 0)
        if self.lib.orc_colour(self._h, _ptr(mark), C.byref(ku), C.byref(kv)) != 0:
            raise ValueError("lattice rejected")
        return ku.value, kv.value

    def mart_rebin(self, seg: Segments, lattice, P, f0, sweeps, beta, nthreads=None):
        P = np.ascontiguousarray(P, dtype=np.float64).ravel()
        f = np.array(f0, dtype=np.float64, copy=True).ravel()
        rc = self.lib.orc_mart_rebin(self._h, *seg.args(), int(lattice[0]), int(lattice[1]), _ptr(P), _ptr(f),
                                     int(sweeps), float(beta),
                                     int(nthreads if nthreads is not None else self.nthreads))
        if rc != 0:
            raise ValueError(f"orc_mart_rebin failed ({rc})")
        return f

    def reconstruct_rebin(self, P, sweeps=None, beta=None, f0=None, lattice=None):
        """The literal variant end to end: segment records, union colouring,
        binary MART re-binned per view."""
        w = self.w
        seg = self.segments_view()
        lat = lattice or self.colour_rebin(seg)
        f0 = np.ones(self.n_cells) if f0 is None else f0
        f = self.mart_rebin(seg, lat, P, f0, w.sweeps if sweeps is None else sweeps,
                            w.beta if beta is None else beta)
        return f, seg, lat

    # -- whole pipeline -----------------------------------------------------
    def reconstruct(self, P, sweeps=None, beta=None, f0=None, lattice=None):
        w = self.w
        csr0 = self.trace_view(0)
        lat = lattice or self.colour(csr0)
        f0 = np.ones(self.n_cells) if f0 is None else f0
        f = self.mart(csr0, lat, P, f0, w.sweeps if sweeps is None else sweeps,
                      w.beta if beta is None else beta)
        return f, csr0, lat
