"""Workload descriptions: grid, scan geometry, phantom recipe and solver settings.

Every workload is a plain record.  Geometry conventions (the readings of the
paper's problem statement that the oracle and the library both follow):

* The reconstruction domain is a disk (2D) or a cylinder (3D) of radius R
  centred on the z axis; a cylinder spans z in [-H/2, H/2] with H = 2R.
* Rings have equal radial spacing r = R / n_rings (Sec. II.A).  With the
  ``multiple`` sector rule ring i (0-based) holds m * ceil(2*pi*(i+1/2)/m)
  sectors, so every cell has area close to r^2 and every ring's sector count is
  a multiple of m; with the ``paper`` rule ring i holds 4(2i+1) sectors (eq. 1).
* View v sits at angle v * span / n_views, anticlockwise about z.
* parallel2d: view-0 ray b is the line y = t_b, t_b = -W + (b+1/2) 2W/B.
* fan2d / cone3d: view-0 source at (-D_so, 0, 0), flat detector at
  x = D_sd - D_so; detector pixel (u, w) has centre
  (D_sd - D_so, -W_u + (u+1/2) 2W_u/U, -W_v + (w+1/2) 2W_v/V), ray index
  r = w * U + u.  The detector bounds the cylinder's shadow:
  W_u = D_sd R / sqrt(D_so^2 - R^2) and W_v = D_sd (H/2) / (D_so - R).
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field, replace
from typing import Optional


@dataclass(frozen=True)
class Workload:
    name: str
    geometry: str                 # "parallel2d" | "fan2d" | "cone3d"
    n_rings: int
    n_slices: int = 1
    radius: float = 1.0
    height: float = 0.0           # cylinder height (3D); 0 for 2D
    sector_rule: str = "multiple"  # "paper" | "multiple" | "explicit"
    sector_multiple: int = 8
    n_views: int = 8
    span: float = math.pi
    det_u: int = 64
    det_v: int = 1
    det_half_u: float = 1.0
    det_half_v: float = 0.0
    src_axis: float = 0.0
    src_det: float = 0.0
    binary: bool = False
    rebin: bool = False           # the paper's literal scheme: segment records re-binned per view
    quarter: bool = False         # literal scheme: trace one detector quadrant, mirror the rest
    phantom_scale: float = 1.0    # phantom size relative to the grid (field of view smaller than the grid)
    phantom: str = "ellipses"     # "ellipses" | "ellipsoids" | "body_inclusions" | "none"
    n_objects: int = 6
    seed: int = 1
    noise: float = 0.01
    sweeps: int = 10
    beta: float = 0.1
    dtype: str = "f32"
    remap_nc: int = 0
    extra: dict = field(default_factory=dict)

    @property
    def n_rays(self) -> int:
        return self.det_u * self.det_v

    @property
    def is3d(self) -> bool:
        return self.geometry == "cone3d"

    def with_(self, **kw) -> "Workload":
        return replace(self, **kw)


def cone(name: str, n_rings: int, n_views: int, det: int, m: int, **kw) -> Workload:
    """Cone-beam USCG workload with the fixed geometry ratios
    (source-to-axis 4R, source-to-detector 8R, cylinder height 2R)."""
    R, H, dso, dsd = 1.0, 2.0, 4.0, 8.0
    return Workload(
        name=name, geometry="cone3d", n_rings=n_rings, n_slices=kw.pop("n_slices", n_rings),
        radius=R, height=H, sector_rule="multiple", sector_multiple=m,
        n_views=n_views, span=2 * math.pi, det_u=det, det_v=det,
        det_half_u=dsd * R / math.sqrt(dso * dso - R * R),
        det_half_v=dsd * (H / 2) / (dso - R),
        src_axis=dso, src_det=dsd, **kw)


def parallel(name: str, n_rings: int, n_views: int, bins: int, m: int, **kw) -> Workload:
    """2D parallel-beam USPG workload over a half turn; bins span the diameter."""
    return Workload(
        name=name, geometry="parallel2d", n_rings=n_rings, n_slices=1, radius=1.0,
        sector_rule="multiple", sector_multiple=m, n_views=n_views, span=math.pi,
        det_u=bins, det_v=1, det_half_u=1.0, **kw)


def paper_fan(n_cart: int, n_views: int = 50, **kw) -> Workload:
    """The paper's 2D phantom scans (Table 1): fan beam from (-8, 0) to a flat
    detector centred at (8, 0), 101 detectors 0.05 apart, p views over a full
    turn, relaxation 0.4, on the paper's grid with Nr = N / 2 rings for an
    N x N Cartesian image, reconstructed with the literal segment scheme
    (binary coefficients re-binned per view).  R = 1.2 keeps the disk inside
    the fan (its edge rays reach +-2.43 of the +-2.525 detector)."""
    nr = n_cart // 2
    return Workload(
        name=kw.pop("name", f"paper-fan-{n_cart}-{n_views}v"), geometry="fan2d", n_rings=nr, n_slices=1,
        radius=kw.pop("radius", 1.2), height=0.0, sector_rule="paper", sector_multiple=1, n_views=n_views,
        span=2 * math.pi, det_u=101, det_v=1, det_half_u=101 * 0.05 / 2, src_axis=8.0, src_det=16.0,
        binary=True, rebin=True, quarter=kw.pop("quarter", True), phantom=kw.pop("phantom", "ellipses"),
        n_objects=kw.pop("n_objects", 8),
        seed=kw.pop("seed", 41), sweeps=kw.pop("sweeps", 20), beta=kw.pop("beta", 0.4),
        remap_nc=n_cart, **kw)


def paper_cone(n_cart: int, n_views: int = 70, **kw) -> Workload:
    """The paper's 3D phantom scan (Table 1): cone beam from (-3, 0, 0) to a
    flat detector centred at (10, 0, 0), 101 x 101 detectors 0.05 apart, p
    views over a full turn, relaxation 0.4, on the paper's grid with N / 2
    rings and N slices for an N^3 Cartesian volume, literal segment scheme.
    R = 0.5, H = 1 keeps the cylinder inside the cone but for its rims next
    to the source."""
    nr = n_cart // 2
    return Workload(
        name=kw.pop("name", f"paper-cone-{n_cart}-{n_views}v"), geometry="cone3d", n_rings=nr, n_slices=n_cart,
        radius=kw.pop("radius", 0.5), height=kw.pop("height", 1.0), sector_rule="paper", sector_multiple=1,
        n_views=n_views, span=2 * math.pi, det_u=101, det_v=101, det_half_u=101 * 0.05 / 2,
        det_half_v=101 * 0.05 / 2, src_axis=3.0, src_det=13.0, binary=True, rebin=True,
        quarter=kw.pop("quarter", True),
        phantom=kw.pop("phantom", "ellipsoids"), n_objects=kw.pop("n_objects", 10), seed=kw.pop("seed", 43),
        sweeps=kw.pop("sweeps", 20), beta=kw.pop("beta", 0.4), remap_nc=n_cart, **kw)


def paper_specimen(which: str, **kw) -> Workload:
    """The geometry of the paper's two experimental scans (Table 3) with a
    synthetic phantom in place of the specimen: Cu lump (source (-8.2, 0, 0),
    detector centre (38.4, 0, 0), 128^3 grid of spacing 0.03125, 101 x 101
    detectors 0.121 apart, 50 views) and frog (source (-22.5, 0, 0),
    detector centre (24.1, 0, 0), 256^3 grid of spacing 0.0078, 201 x 201
    detectors 0.06 apart, 70 views); relaxation 0.4, literal scheme, paper
    grid with N / 2 rings and N slices, the cylinder inscribed in the cube.
    The Cu-lump scan sees only the central 1.07 of the 2.0 radius, so its
    phantom is drawn at 0.4 of the grid's size."""
    if which == "culump":
        n, h, det, pitch, p, dso, dsd = 128, 0.03125, 101, 0.121, 50, 8.2, 46.6
    elif which == "frog":
        n, h, det, pitch, p, dso, dsd = 256, 0.0078, 201, 0.06, 70, 22.5, 46.6
    else:
        raise ValueError(which)
    R = n * h / 2
    return Workload(
        name=kw.pop("name", f"paper-{which}-geometry"), geometry="cone3d", n_rings=n // 2, n_slices=n, radius=R,
        height=2 * R, sector_rule="paper", sector_multiple=1, n_views=p, span=2 * math.pi, det_u=det, det_v=det,
        det_half_u=det * pitch / 2, det_half_v=det * pitch / 2, src_axis=dso, src_det=dsd, binary=True,
        rebin=True, quarter=kw.pop("quarter", True), phantom=kw.pop("phantom", "ellipsoids"),
        phantom_scale=kw.pop("phantom_scale", 1.0 if which == "frog" else 0.4),
        n_objects=kw.pop("n_objects", 10), seed=kw.pop("seed", 47 if which == "frog" else 45),
        sweeps=kw.pop("sweeps", 20), beta=kw.pop("beta", 0.4), remap_nc=n, **kw)


WORKLOADS = {
    # 2D parallel beam, FP64 plain MART: 32 rings, 8 views over 180 degrees, 64 bins.
    # Sector counts are multiples of 16 so that the 22.5-degree view step is a
    # whole number of sectors in every ring.
    "par2d-32r-8v": parallel("par2d-32r-8v", 32, 8, 64, 16, phantom="ellipses",
                             n_objects=6, seed=1, sweeps=10, beta=0.1, dtype="f64"),
    # 3D cone beam USCG, FP32: 128 rings x 128 slices, 16 views, 256x256 detector.
    "cone-128r-16v": cone("cone-128r-16v", 128, 16, 256, 16, phantom="ellipsoids",
                          n_objects=10, seed=2, sweeps=20, beta=0.1, dtype="f32"),
    # 3D cone beam USCG, FP32, high contrast: 256 rings x 256 slices, 32 views,
    # 512x512 detector, body ellipsoid with 3 dense inclusions, then a remap to
    # a 512 x 512 x 256 Cartesian grid.
    "cone-256r-32v-hc": cone("cone-256r-32v-hc", 256, 32, 512, 32, phantom="body_inclusions",
                             n_objects=4, seed=3, sweeps=20, beta=0.05, dtype="f32",
                             remap_nc=512),
    # The paper's own scans (Table 1) with its literal coefficient scheme.
    "paper-fan-256-50v": paper_fan(256),
    "paper-fan-512-50v": paper_fan(512),
    "paper-fan-1024-50v": paper_fan(1024),
    "paper-cone-128-70v": paper_cone(128),
    "paper-culump-geometry": paper_specimen("culump"),
    "paper-frog-geometry": paper_specimen("frog"),
}


def batch2d_members(n: int = 64, seed: int = 4) -> list:
    """The many-slice 2D workload: ring counts from {32,64,128,256}, views
    from {8,16,32}, 2*Nr bins, sector multiple 2p (half-turn scan), 15 sweeps."""
    import numpy as np
    rng = np.random.default_rng(seed)
    out = []
    for k in range(n):
        nr = int(rng.choice([32, 64, 128, 256]))
        p = int(rng.choice([8, 16, 32]))
        out.append(parallel(f"batch2d-{k}", nr, p, 2 * nr, 2 * p, phantom="ellipses",
                            n_objects=6, seed=4000 + k, sweeps=15, beta=0.1, dtype="f32"))
    return out


def serve_request(k: int, nr: int, p: int, sweeps: int) -> Workload:
    """One request of the serving workload: cone-beam USCG, Nr = Nz, detector
    2Nr x 2Nr, sector multiple p, random ellipsoid phantom."""
    return cone(f"serve-{k}", nr, p, 2 * nr, p, phantom="ellipsoids", n_objects=10,
                seed=5000 + k, sweeps=sweeps, beta=0.1, dtype="f32")


def get(name: str) -> Workload:
    return WORKLOADS[name]


def small_cone(name: str = "cone-16r-8v", n_rings: int = 16, n_views: int = 8, det: int = 32,
               m: Optional[int] = None, **kw) -> Workload:
    """Scaled-down cone-beam workload with the same ratios, for fast tests."""
    return cone(name, n_rings, n_views, det, m if m is not None else n_views,
                phantom=kw.pop("phantom", "ellipsoids"), n_objects=kw.pop("n_objects", 10),
                seed=kw.pop("seed", 7), sweeps=kw.pop("sweeps", 5), beta=kw.pop("beta", 0.1),
                dtype=kw.pop("dtype", "f32"), **kw)
