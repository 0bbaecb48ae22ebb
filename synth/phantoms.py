"""Seeded phantoms (sums of constant ellipses / ellipsoids) and their exact line
integrals along the scan's rays, plus the additive noise model.

The draws use numpy's PCG64 generator in a fixed order so that every consumer
sees the same arrays:

* ellipses: centre radius 0.7*sqrt(U), centre angle 2*pi*U, two semi-axes
  U[0.05, 0.4], orientation U[0, pi), value U[0.1, 1.0];
* ellipsoids: centre radius 0.7*sqrt(U), centre angle 2*pi*U, centre z
  U[-0.7, 0.7], three semi-axes U[0.05, 0.4], orientation about z U[0, pi),
  value U[0.05, 1.0];
* body_inclusions: a centred body ellipsoid with semi-axes U[0.75, 0.9],
  U[0.6, 0.8], U[0.75, 0.9], orientation about z U[0, pi) and value
  U[0.1, 0.3], then three spheres of radius U[0.02, 0.06] whose centres are
  uniform in the body shrunk by 0.6; each sphere adds 5.0 - body value, so the
  inclusions read 5.0.

The draws describe a unit disk (a cylinder of half-height 1); they are
scaled by the workload's radius in x, y and by its half-height in z, times
its phantom_scale.

Noise: P <- max(P + sigma * max(P) * N(0, 1), 0), drawn in array order.
"""

from __future__ import annotations

import math

import numpy as np

from .workloads import Workload


def draw_phantom(w: Workload) -> list:
    """Return a list of objects (centre[3], semi-axes[3], angle, value)."""
    rng = np.random.default_rng(w.seed)
    objs = []
    if w.phantom == "none":
        return objs
    if w.phantom == "ellipses":
        for _ in range(w.n_objects):
            rc = 0.7 * math.sqrt(rng.uniform())
            pc = 2 * math.pi * rng.uniform()
            ax = rng.uniform(0.05, 0.4, size=2)
            ang = rng.uniform(0.0, math.pi)
            mu = rng.uniform(0.1, 1.0)
            objs.append((np.array([rc * math.cos(pc), rc * math.sin(pc), 0.0]),
                         np.array([ax[0], ax[1], np.inf]), ang, mu))
    elif w.phantom == "ellipsoids":
        for _ in range(w.n_objects):
            rc = 0.7 * math.sqrt(rng.uniform())
            pc = 2 * math.pi * rng.uniform()
            zc = rng.uniform(-0.7, 0.7)
            ax = rng.uniform(0.05, 0.4, size=3)
            ang = rng.uniform(0.0, math.pi)
            mu = rng.uniform(0.05, 1.0)
            objs.append((np.array([rc * math.cos(pc), rc * math.sin(pc), zc]), ax, ang, mu))
    elif w.phantom == "body_inclusions":
        ax = np.array([rng.uniform(0.75, 0.9), rng.uniform(0.6, 0.8), rng.uniform(0.75, 0.9)])
        ang = rng.uniform(0.0, math.pi)
        mub = rng.uniform(0.1, 0.3)
        objs.append((np.zeros(3), ax, ang, mub))
        c, s = math.cos(ang), math.sin(ang)
        for _ in range(3):
            rad = rng.uniform(0.02, 0.06)
            while True:
                q = rng.uniform(-1.0, 1.0, size=3)
                if q @ q <= 1.0:
                    break
            q = 0.6 * q * ax
            cen = np.array([c * q[0] - s * q[1], s * q[0] + c * q[1], q[2]])
            objs.append((cen, np.array([rad, rad, rad]), 0.0, 5.0 - mub))
    else:
        raise ValueError(f"unknown phantom {w.phantom!r}")
    # the draws describe a unit disk / a cylinder of half-height 1: scale to
    # the workload's radius and half-height (identity for R = 1, H = 2)
    sr = w.radius * w.phantom_scale
    sz = (w.height / 2 if w.height > 0 else 1.0) * w.phantom_scale
    if sr != 1.0 or sz != 1.0:
        scale = np.array([sr, sr, sz])
        objs = [(cen * scale, ax * scale, ang, mu) for cen, ax, ang, mu in objs]
    return objs


def scan_rays(w: Workload, view: int):
    """Source points S and far points D (arrays [n_rays, 3]) of one view."""
    th = view * w.span / w.n_views
    c, s = math.cos(th), math.sin(th)
    U, V = w.det_u, w.det_v
    u = np.arange(U, dtype=np.float64)
    if w.geometry == "parallel2d":
        t = -w.det_half_u + (u + 0.5) * (2 * w.det_half_u / U)
        S0 = np.stack([np.full(U, -2 * w.radius), t, np.zeros(U)], axis=1)
        D0 = np.stack([np.full(U, 2 * w.radius), t, np.zeros(U)], axis=1)
    else:
        yv = -w.det_half_u + (u + 0.5) * (2 * w.det_half_u / U)
        if w.geometry == "cone3d":
            wv = np.arange(V, dtype=np.float64)
            zv = -w.det_half_v + (wv + 0.5) * (2 * w.det_half_v / V)
        else:
            zv = np.zeros(1)
        Y, Z = np.meshgrid(yv, zv)            # [V, U]
        n = Y.size
        S0 = np.tile(np.array([-w.src_axis, 0.0, 0.0]), (n, 1))
        D0 = np.stack([np.full(n, w.src_det - w.src_axis), Y.ravel(), Z.ravel()], axis=1)
    rot = np.array([[c, -s, 0.0], [s, c, 0.0], [0.0, 0.0, 1.0]])
    return S0 @ rot.T, D0 @ rot.T


def project(objs: list, S: np.ndarray, D: np.ndarray, two_d: bool) -> np.ndarray:
    """Exact line integrals of a sum of constant quadrics along the full lines
    S + t (D - S): value times the chord length through each object."""
    e = D - S
    out = np.zeros(len(S))
    dims = 2 if two_d else 3
    elen = np.linalg.norm(e[:, :dims], axis=1)
    for cen, ax, ang, mu in objs:
        c, s = math.cos(ang), math.sin(ang)
        x = S - cen
        # rotate into the object frame (inverse rotation about z)
        xr = np.stack([c * x[:, 0] + s * x[:, 1], -s * x[:, 0] + c * x[:, 1], x[:, 2]], axis=1)
        er = np.stack([c * e[:, 0] + s * e[:, 1], -s * e[:, 0] + c * e[:, 1], e[:, 2]], axis=1)
        xs = xr[:, :dims] / ax[:dims]
        es = er[:, :dims] / ax[:dims]
        A = np.einsum("ij,ij->i", es, es)
        B = np.einsum("ij,ij->i", xs, es)
        C = np.einsum("ij,ij->i", xs, xs) - 1.0
        disc = B * B - A * C
        hit = disc > 0
        dt = np.zeros(len(S))
        dt[hit] = 2.0 * np.sqrt(disc[hit]) / A[hit]
        out += mu * dt * elen
    return out


def add_noise(P: np.ndarray, sigma: float, seed: int) -> np.ndarray:
    if sigma <= 0:
        return P.copy()
    rng = np.random.default_rng(seed + 7919)
    noisy = P + sigma * P.max() * rng.standard_normal(P.shape)
    return np.maximum(noisy, 0.0)


def make_projections(w: Workload, noise: bool = True) -> np.ndarray:
    """Projection data P[view][det_v][det_u] (float64) for the workload's phantom."""
    objs = draw_phantom(w)
    P = np.zeros((w.n_views, w.det_v, w.det_u))
    for v in range(w.n_views):
        S, D = scan_rays(w, v)
        P[v] = project(objs, S, D, two_d=not w.is3d).reshape(w.det_v, w.det_u)
    if noise:
        P = add_noise(P, w.noise, w.seed)
    return P


def phantom_value(w: Workload, pts: np.ndarray) -> np.ndarray:
    """Phantom value at points [n, 3] (for image-quality reporting)."""
    objs = draw_phantom(w)
    out = np.zeros(len(pts))
    two_d = not w.is3d
    for cen, ax, ang, mu in objs:
        c, s = math.cos(ang), math.sin(ang)
        x = pts - cen
        xr = np.stack([c * x[:, 0] + s * x[:, 1], -s * x[:, 0] + c * x[:, 1], x[:, 2]], axis=1)
        dims = 2 if two_d else 3
        q = np.sum((xr[:, :dims] / ax[:dims]) ** 2, axis=1)
        out += np.where(q <= 1.0, mu, 0.0)
    return out


def scan_rays_torch(w: Workload, device):
    """Ray geometry of every view with torch on `device`, in float64: the
    source points S and directions e = D - S ([views, rays, 3]) and the
    in-plane (2D) or full (3D) length of e ([views, rays]).  Same geometry
    as scan_rays."""
    import torch

    f64 = torch.float64
    U, V = w.det_u, w.det_v
    th = torch.arange(w.n_views, dtype=f64, device=device) * (w.span / w.n_views)
    c, s = torch.cos(th)[:, None], torch.sin(th)[:, None]       # [views, 1]
    u = torch.arange(U, dtype=f64, device=device)
    if w.geometry == "parallel2d":
        t = -w.det_half_u + (u + 0.5) * (2 * w.det_half_u / U)
        s0 = torch.stack([torch.full_like(t, -2 * w.radius), t, torch.zeros_like(t)], 1)
        d0 = torch.stack([torch.full_like(t, 2 * w.radius), t, torch.zeros_like(t)], 1)
    else:
        yv = -w.det_half_u + (u + 0.5) * (2 * w.det_half_u / U)
        if w.geometry == "cone3d":
            zv = -w.det_half_v + (torch.arange(V, dtype=f64, device=device) + 0.5) * (2 * w.det_half_v / V)
        else:
            zv = torch.zeros(1, dtype=f64, device=device)
        Z, Y = torch.meshgrid(zv, yv, indexing="ij")              # [V, U]
        n = Y.numel()
        s0 = torch.tensor([-w.src_axis, 0.0, 0.0], dtype=f64, device=device).expand(n, 3)
        d0 = torch.stack([torch.full((n,), w.src_det - w.src_axis, dtype=f64, device=device),
                          Y.reshape(-1), Z.reshape(-1)], 1)

    def rot(p):   # [n, 3] -> [views, n, 3], rotation by each view angle about z
        x, y, z = p[:, 0][None], p[:, 1][None], p[:, 2][None]
        return torch.stack([c * x - s * y, s * x + c * y, z.expand(c.shape[0], -1)], 2)

    S = rot(s0)
    e = rot(d0) - S
    dims = 2 if not w.is3d else 3
    return S, e, torch.linalg.vector_norm(e[..., :dims], dim=2)


def make_projections_torch(w: Workload, device, dtype=None, noise: bool = True, rays=None):
    """Projection data [view][det_v][det_u] computed with torch on `device`
    (same phantom draw, geometry and chord formula as make_projections, in
    float64, then cast to `dtype`).  For generating many large inputs
    directly in device memory; `rays` may pass scan_rays_torch(w, device) of
    an equal geometry to skip rebuilding it.  Noise uses torch's generator on
    `device` seeded with seed + 7919, so it differs from the numpy draw in
    value but not in distribution."""
    import torch

    f64 = torch.float64
    S, e, elen = rays if rays is not None else scan_rays_torch(w, device)
    dims = 2 if not w.is3d else 3
    out = torch.zeros(elen.shape, dtype=f64, device=device)
    for cen, ax, ang, mu in draw_phantom(w):
        ca, sa = math.cos(ang), math.sin(ang)
        x = S - torch.as_tensor(cen, dtype=f64, device=device)
        xr = torch.stack([ca * x[..., 0] + sa * x[..., 1], -sa * x[..., 0] + ca * x[..., 1], x[..., 2]], 2)
        er = torch.stack([ca * e[..., 0] + sa * e[..., 1], -sa * e[..., 0] + ca * e[..., 1], e[..., 2]], 2)
        axd = torch.as_tensor(ax[:dims], dtype=f64, device=device)
        xs, es = xr[..., :dims] / axd, er[..., :dims] / axd
        A = (es * es).sum(2)
        B = (xs * es).sum(2)
        Cq = (xs * xs).sum(2) - 1.0
        disc = B * B - A * Cq
        dt = torch.where(disc > 0, 2.0 * torch.sqrt(disc.clamp_min(0)) / A, torch.zeros_like(A))
        out += mu * dt * elen
    out = out.reshape(w.n_views, w.det_v, w.det_u)
    if noise and w.noise > 0:
        g = torch.Generator(device=device)
        g.manual_seed(w.seed + 7919)
        out = (out + w.noise * out.max() * torch.randn(out.shape, generator=g, dtype=f64, device=device)
               ).clamp_min(0.0)
    return out.to(dtype or f64).contiguous()
