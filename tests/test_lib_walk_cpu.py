"""The library's reference-ray walk (host build of trace_walk.hpp) against the
oracle's direct trace, on the CPU: same cells, lengths equal up to rounding,
and the wedge-major index shift reproduces every view's rows."""
import ctypes as C
import math
import os
import subprocess

import numpy as np
import pytest

import synth
from oracle import Oracle
from oracle.oracle import SANITIZE
from rowcmp import LEN_ATOL, LEN_RTOL, compare_rows, on_axis

HERE = os.path.dirname(os.path.abspath(__file__))
BUILD = os.path.join(HERE, "_build")
GEOM = {"parallel2d": 0, "fan2d": 1, "cone3d": 2}


@pytest.fixture(scope="module")
def hw():
    os.makedirs(BUILD, exist_ok=True)
    # USPG_HOST_SANITIZE=1: the build with the sanitizers (test_sanitizers.py)
    san = os.environ.get("USPG_HOST_SANITIZE") == "1"
    so = os.path.join(BUILD, "host_walk" + ("_asan" if san else "") + ".so")
    opt = SANITIZE if san else ["-O2"]
    subprocess.run(["g++", *opt, "-std=c++17", "-fPIC", "-shared", "-ffp-contract=off",
                    "-Wno-unknown-pragmas", os.path.join(HERE, "host_walk.cpp"), "-o", so], check=True)
    L = C.CDLL(so)
    L.hw_setup.argtypes = [C.c_int, C.c_int, C.c_double, C.c_double, C.c_void_p, C.c_int, C.c_int,
                           C.c_int, C.c_int, C.c_int, C.c_double, C.c_double, C.c_double, C.c_double,
                           C.c_int]
    L.hw_trace.argtypes = [C.c_int64, C.c_void_p, C.c_void_p, C.c_int]
    L.hw_tables.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
    L.hw_tables.restype = C.c_int64
    L.hw_columns.restype = C.c_int64
    L.hw_column_gaps.restype = C.c_int64
    L.hw_code_ray.argtypes = [C.c_int64, C.c_void_p, C.c_void_p, C.c_int, C.c_void_p]
    L.hw_column_major.argtypes = [C.c_int, C.c_int, C.c_int64]
    L.hw_column_major.restype = C.c_int64
    return L


# rings per group of the library's device layout (uspg_internal.hpp kRingGroup)
GROUP = 4


class Walk:
    def __init__(self, L, w, o, grp=GROUP):
        self.L, self.w, self.o = L, w, o
        q = round(w.n_views * 2 * math.pi / w.span)
        self.q, self.grp = q, grp
        ng = np.ascontiguousarray(o.ng, dtype=np.int32)
        rc = L.hw_setup(w.n_rings, w.n_slices, w.radius, w.height, ng.ctypes.data, q, GEOM[w.geometry],
                        int(w.is3d), w.det_u, w.det_v, w.det_half_u, w.det_half_v, w.src_axis, w.src_det,
                        grp)
        assert rc == 0
        self.kq = np.zeros(w.n_rings, dtype=np.int32)
        self.hq = np.zeros(w.n_rings, dtype=np.int32)
        self.Cq = int(L.hw_tables(self.kq.ctypes.data, self.hq.ctypes.data, None))
        self.ring_of = np.zeros(self.Cq, dtype=np.int32)
        L.hw_tables(self.kq.ctypes.data, self.hq.ctypes.data, self.ring_of.ctypes.data)
        # the layout: every grid cell has exactly one slot, the rest is padding
        assert (self.ring_of >= 0).sum() * q == o.head[-1]
        self.Wc = w.n_slices * self.Cq
        self.cap = 8 * (w.n_rings + w.n_slices) + 64

    def row(self, r):
        ids = np.zeros(self.cap, dtype=np.uint32)
        lens = np.zeros(self.cap)
        n = self.L.hw_trace(r, ids.ctypes.data, lens.ctypes.data, self.cap)
        assert n >= 0
        return ids[:n].astype(np.int64), lens[:n]

    def to_paper(self, x, view=0):
        x = (x + view * self.Wc) % (self.q * self.Wc)
        a, rem = x // self.Wc, x % self.Wc
        k, off = rem // self.Cq, rem % self.Cq
        i = self.ring_of[off]
        assert np.all(i >= 0)
        s = a * self.kq[i] + (off - self.hq[i]) // self.grp
        return k * self.o.head[-1] + self.o.head[i] + s


def compare(c1, l1, c2, l2):
    assert len(c1) == len(set(c1.tolist()))
    ia, ib = np.argsort(c1), np.argsort(c2)
    assert np.array_equal(c1[ia], c2[ib])
    assert np.allclose(l1[ia], l2[ib], rtol=LEN_RTOL, atol=LEN_ATOL)


def cases():
    return {
        "par2d": synth.get("par2d-32r-8v"),
        "par2d-paper-rule": synth.Workload(name="pp", geometry="parallel2d", n_rings=16,
                                           sector_rule="paper", n_views=2, span=math.pi, det_u=33),
        "fan2d-odd": synth.Workload(name="fan", geometry="fan2d", n_rings=20, sector_multiple=10,
                                    n_views=10, span=2 * math.pi, det_u=41, det_half_u=2.2,
                                    src_axis=4.0, src_det=8.0),
        "cone-small": synth.small_cone(n_rings=16, n_views=8, det=32, m=8),
        "cone-odd": synth.small_cone(n_rings=10, n_views=4, det=15, m=4, n_slices=7),
    }


@pytest.mark.parametrize("name", list(cases()))
def test_walk_equals_oracle_all_views(hw, name):
    w = cases()[name]
    o = Oracle(w)
    wk = Walk(hw, w, o)
    rows = [wk.row(r) for r in range(o.n_rays)]
    for v in range(w.n_views):
        direct = o.trace_view(v)
        for r in range(o.n_rays):
            ids, lens = rows[r]
            c2, l2 = direct.row(r)
            compare_rows(o, r, wk.to_paper(ids, v), lens, c2, l2, view=v)


@pytest.mark.parametrize("name,step", [("cone-128r-16v", 331), ("cone-256r-32v-hc", 2609)])
def test_walk_equals_oracle_sampled_full_size(hw, name, step):
    w = synth.get(name)
    o = Oracle(w)
    wk = Walk(hw, w, o)
    rng = np.random.default_rng(1)
    rays = list(range(0, o.n_rays, step)) + list(rng.integers(0, o.n_rays, 40))
    for r in rays:
        ids, lens = wk.row(int(r))
        for v in (0, w.n_views - 1):
            S, D = o.ray(v, int(r))
            c2, l2 = o.trace_line(S, D)
            compare(wk.to_paper(ids, v), lens, c2, l2)


def test_walk_random_and_near_tangent_lines(hw):
    # arbitrary lines, including ones that dip just below a circle in the middle
    # of a sector of the ring outside it (that sector is entered twice and the
    # two visits must be merged into one entry)
    from test_oracle_trace import _near_tangent_rays, cell_of_points
    hw.hw_trace_line.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int]
    for w in (synth.Workload(name="pp", geometry="parallel2d", n_rings=5, sector_rule="paper",
                             n_views=1, span=2 * math.pi, det_u=8),
              synth.small_cone(n_rings=6, n_views=8, det=8, m=8, n_slices=5)):
        o = Oracle(w)
        wk = Walk(hw, w, o)
        rng = np.random.default_rng(3)
        lines = _near_tangent_rays(o, rng, 300)
        for _ in range(300):
            lines.append((np.array([*rng.uniform(-3, 3, 2), rng.uniform(-0.9, 0.9) if w.is3d else 0]),
                          np.array([*rng.uniform(-3, 3, 2), rng.uniform(-0.9, 0.9) if w.is3d else 0])))
        reentries = 0
        for S, D in lines:
            S = np.ascontiguousarray(S, dtype=np.float64)
            D = np.ascontiguousarray(D, dtype=np.float64)
            ids = np.zeros(wk.cap, dtype=np.uint32)
            lens = np.zeros(wk.cap)
            n = hw.hw_trace_line(S.ctypes.data, D.ctypes.data, ids.ctypes.data, lens.ctypes.data, wk.cap)
            assert n >= 0
            c2, l2 = o.trace_line(S, D)
            compare(wk.to_paper(ids[:n].astype(np.int64)), lens[:n], c2, l2)
            # does the line enter some cell twice (two separate runs)?
            t = np.linspace(0, 1, 200001)
            cells = cell_of_points(o, S[None] + t[:, None] * (D - S)[None])
            inside = np.hypot(*(S[None, :2] + t[:, None] * (D - S)[None, :2]).T) < w.radius
            ci = cells[inside]
            if len(ci):
                runs = ci[np.r_[True, np.diff(ci) != 0]]
                reentries += len(runs) != len(set(runs.tolist()))
        assert reentries > 10     # the merge path was exercised


@pytest.mark.parametrize("grp", [1, 3, 8])
def test_layout_group_size_is_a_bijection(hw, grp):
    # any ring-group size gives the same rows once mapped back to the paper's
    # numbering, and every grid cell has exactly one slot in the layout
    for w in (synth.get("par2d-32r-8v"), synth.small_cone(n_rings=13, n_views=4, det=10, m=4, n_slices=5)):
        o = Oracle(w)
        wk = Walk(hw, w, o, grp=grp)
        ref = Walk(hw, w, o, grp=1)
        wk = Walk(hw, w, o, grp=grp)
        for r in range(0, o.n_rays, 3):
            ids, lens = wk.row(r)
            c2, l2 = o.trace_view(0).row(r) if r == 0 else o.trace_line(*o.ray(0, r))
            compare_rows(o, r, wk.to_paper(ids), lens, c2, l2)
        assert ref.Cq <= wk.Cq


@pytest.mark.parametrize("name,step", [("cone-small", 1), ("cone-odd", 1), ("cone-128r-16v", 7),
                                       ("cone-256r-32v-hc", 97)])
def test_coded_rows_rebuild_the_walk(hw, name, step):
    # coded rows (a column's in-plane path shared by its rays, plus per ray
    # piece / slice bits) rebuilt without the stored row equal the walk's row
    # bit for bit; every ray of the configured scans codes (none explicit)
    w = cases()[name] if name in cases() else synth.get(name)
    o = Oracle(w)
    wk = Walk(hw, w, o)
    m = hw.hw_columns()
    assert m > 0 and hw.hw_column_gaps() == 0
    ids = np.zeros(wk.cap, dtype=np.uint32)
    lens = np.zeros(wk.cap, dtype=np.float32)
    info = np.zeros(4, dtype=np.int64)
    coded = 0
    for r in range(0, o.n_rays, step):
        n = hw.hw_code_ray(r, ids.ctypes.data, lens.ctypes.data, wk.cap, info.ctypes.data)
        assert n >= 0, (r, n)          # -1: rebuilt row differs, -2: left explicit
        if n:
            coded += 1
            c2, l2 = wk.row(r)
            assert np.array_equal(ids[:n].astype(np.int64), c2)
            assert np.array_equal(lens[:n], l2.astype(np.float32))
    assert coded > 0


@pytest.mark.parametrize("U,V", [(512, 512), (7, 5), (20, 1), (1, 9)])
def test_column_major_threads_cover_every_ray_once(hw, U, V):
    # the per-ray launches give the rays of one detector column to
    # neighbouring threads: thread -> ray must be a bijection of [0, U V),
    # with ray = v U + u and thread = u V + v
    rays = np.array([hw.hw_column_major(U, V, t) for t in range(U * V)], dtype=np.int64)
    assert np.array_equal(np.sort(rays), np.arange(U * V))
    t = np.arange(U * V)
    if V > 1:
        assert np.array_equal(rays, (t % V) * U + t // V)
    else:
        assert np.array_equal(rays, t)
