"""The library's segment records and per-view re-binning (host build of
segments.hpp) against the oracle's literal variant, on the CPU: the same
records (slice, ring; azimuths equal up to rounding) and, for every view,
the same re-binned rows, on generic cone, fan and parallel scans whose view
steps are not whole sectors."""
import ctypes as C
import os
import subprocess

import numpy as np
import pytest

import synth
from oracle import Oracle
from oracle.oracle import SANITIZE

HERE = os.path.dirname(os.path.abspath(__file__))
BUILD = os.path.join(HERE, "_build")
GEOM = {"parallel2d": 0, "fan2d": 1, "cone3d": 2}


@pytest.fixture(scope="module")
def hs():
    os.makedirs(BUILD, exist_ok=True)
    # USPG_HOST_SANITIZE=1: the build with the sanitizers (test_sanitizers.py)
    san = os.environ.get("USPG_HOST_SANITIZE") == "1"
    so = os.path.join(BUILD, "host_segments" + ("_asan" if san else "") + ".so")
    opt = SANITIZE if san else ["-O2"]
    subprocess.run(["g++", *opt, "-std=c++17", "-fPIC", "-shared", "-ffp-contract=off",
                    "-Wno-unknown-pragmas", os.path.join(HERE, "host_segments.cpp"), "-o", so], check=True)
    L = C.CDLL(so)
    L.hs_setup.argtypes = [C.c_int, C.c_int, C.c_double, C.c_double, C.c_void_p, C.c_int, C.c_int, C.c_int,
                           C.c_int, C.c_double, C.c_double, C.c_double, C.c_double, C.c_double, C.c_int]
    L.hs_segments.argtypes = [C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int]
    L.hs_row.argtypes = [C.c_int, C.c_int64, C.c_void_p, C.c_int]
    L.hs_segments_mirrored.argtypes = L.hs_segments.argtypes
    return L


def P(a):
    return a.ctypes.data_as(C.c_void_p)


class Lib:
    def __init__(self, L, w, o):
        self.L, self.w = L, w
        ng = np.ascontiguousarray(o.ng, dtype=np.int32)
        self.ng = ng
        L.hs_setup(w.n_rings, w.n_slices, w.radius, w.height, P(ng), GEOM[w.geometry], int(w.is3d), w.det_u,
                   w.det_v, w.det_half_u, w.det_half_v, w.src_axis, w.src_det, w.span, w.n_views)

    def segments(self, r, cap=8192, mirrored=False):
        sl, rg, pr = (np.zeros(cap, dtype=np.int32) for _ in range(3))
        pa, pb = np.zeros(cap), np.zeros(cap)
        fn = self.L.hs_segments_mirrored if mirrored else self.L.hs_segments
        n = fn(r, P(sl), P(rg), P(pa), P(pb), P(pr), cap)
        assert n >= 0
        return sl[:n], rg[:n], pa[:n], pb[:n], pr[:n]

    def row(self, view, r, cap=1 << 16):
        cells = np.zeros(cap, dtype=np.int64)
        n = self.L.hs_row(view, r, P(cells), cap)
        assert n >= 0, n
        return cells[:n]


def cases():
    return [
        synth.small_cone("sc-cone7", n_rings=7, n_views=7, det=10, m=7).with_(sector_rule="paper", n_slices=5),
        synth.small_cone("sc-cone50", n_rings=12, n_views=50, det=18, m=1).with_(sector_rule="paper", n_slices=9),
        synth.small_cone("sc-fan", n_rings=9, n_views=5, det=14, m=5).with_(
            geometry="fan2d", n_slices=1, height=0.0, det_v=1, sector_rule="paper"),
        synth.parallel("sc-par70", 16, 70, 30, 1, phantom="none").with_(sector_rule="paper"),
        synth.parallel("sc-dip", 4, 5, 102, 5, phantom="none").with_(sector_rule="paper"),
        # detector much wider than the disk: most rays miss, the central ones
        # have up to 47 records
        synth.parallel("sc-wide", 24, 50, 121, 1, phantom="none").with_(sector_rule="paper", det_half_u=3.7),
        # few long rays (up to 155 records)
        synth.small_cone("sc-fanlong", n_rings=80, n_views=20, det=30, m=5).with_(
            geometry="fan2d", n_slices=1, height=0.0, det_v=1, sector_rule="paper"),
    ]


@pytest.mark.parametrize("w", cases(), ids=lambda w: w.name)
def test_records_and_rows_equal_oracle(hs, w):
    o = Oracle(w.with_(binary=True))
    lib = Lib(hs, w, o)
    seg = o.segments_view()
    partners = 0
    for r in range(o.n_rays):
        sl, rg, pa, pb, pr = lib.segments(r)
        osl, org, opa, opb = seg.ray(r)
        assert np.array_equal(sl, osl) and np.array_equal(rg, org), r
        assert np.allclose(pa, opa, rtol=0, atol=1e-14) and np.allclose(pb, opb, rtol=0, atol=1e-14), r
        # a partner is an earlier record of the same ring and slice
        for j in np.nonzero(pr >= 0)[0]:
            assert pr[j] < j and rg[pr[j]] == rg[j] and sl[pr[j]] == sl[j]
        partners += int((pr >= 0).sum())
    for v in range(w.n_views):
        rows = o.rebin_view(seg, v)
        for r in range(o.n_rays):
            assert np.array_equal(lib.row(v, r), rows.row(r)[0]), (v, r)
    if w.name == "sc-dip":
        assert partners > 0


@pytest.mark.parametrize("w", cases()[:3] + [synth.paper_fan(64, 50), synth.paper_cone(24, 70)],
                         ids=lambda w: w.name)
def test_quarter_tracing_mirrors_records(hs, w):
    """Sec. III.C: the records of the other three quadrants are the mirror
    images of the traced quadrant's (same rings, mirrored slices, azimuths
    2 pi - phi up to rounding), so the re-binned rows are the same."""
    o = Oracle(w.with_(binary=True))
    lib = Lib(hs, w, o)
    for r in range(o.n_rays):
        a = lib.segments(r)
        b = lib.segments(r, mirrored=True)
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]) and np.array_equal(a[4], b[4]), r
        d = np.abs(a[2] - b[2])
        d = np.minimum(d, 2 * np.pi - d)           # 0 and 2 pi are one azimuth
        assert d.max(initial=0) <= 1e-13, r
        d = np.abs(a[3] - b[3])
        d = np.minimum(d, 2 * np.pi - d)
        assert d.max(initial=0) <= 1e-13, r
