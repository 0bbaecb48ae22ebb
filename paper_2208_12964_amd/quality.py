"""Image-quality figures of a reconstruction against its ground truth
(the measures the paper reports in Tables 2, 4 and 5).

Reporting only (torch on whatever device the images live on); nothing here
is part of the reconstruction.  Readings, since the paper names the measures
but not their parameters (and `report` first rescales binary-coefficient
images, whose values are per-cell shares of the line integrals):
  * MAE = mean |x - y|, RMSE = sqrt(mean (x - y)^2), over all pixels;
  * SSIM is Wang et al.'s structural similarity with an 11 x 11 Gaussian
    window (sigma 1.5), K1 = 0.01, K2 = 0.03 and dynamic range L = max - min
    of the ground truth, averaged over the window positions that fit inside
    the image ("valid" filtering) and, for a volume, over its axial slices.
"""
from __future__ import annotations

import math

import torch


def mae(x: torch.Tensor, y: torch.Tensor) -> float:
    return (x.double() - y.double()).abs().mean().item()


def rmse(x: torch.Tensor, y: torch.Tensor) -> float:
    return math.sqrt(((x.double() - y.double()) ** 2).mean().item())


def _gauss(win: int, sigma: float, device) -> torch.Tensor:
    t = torch.arange(win, dtype=torch.float64, device=device) - (win - 1) / 2
    g = torch.exp(-(t * t) / (2 * sigma * sigma))
    return g / g.sum()


def ssim(x: torch.Tensor, ref: torch.Tensor, win: int = 11, sigma: float = 1.5, k1: float = 0.01,
         k2: float = 0.03, data_range: float | None = None) -> float:
    """Mean SSIM of x against ref; 2D images [H, W] or stacks [S, H, W]."""
    x = x.double()
    ref = ref.double()
    if x.dim() == 2:
        x, ref = x[None], ref[None]
    L = float(ref.max() - ref.min()) if data_range is None else float(data_range)
    if L <= 0:
        L = 1.0
    c1, c2 = (k1 * L) ** 2, (k2 * L) ** 2
    g = _gauss(win, sigma, x.device)
    kern_h = g.view(1, 1, 1, win)
    kern_v = g.view(1, 1, win, 1)

    def filt(a):   # separable Gaussian, valid region
        a = a[:, None]
        return torch.nn.functional.conv2d(torch.nn.functional.conv2d(a, kern_h), kern_v)[:, 0]

    mx, my = filt(x), filt(ref)
    sxx = filt(x * x) - mx * mx
    syy = filt(ref * ref) - my * my
    sxy = filt(x * ref) - mx * my
    s = ((2 * mx * my + c1) * (2 * sxy + c2)) / ((mx * mx + my * my + c1) * (sxx + syy + c2))
    return s.mean().item()


def cartesian_truth(w, nc: int, device, dtype=torch.float64) -> torch.Tensor:
    """The phantom sampled at the pixel centres of the nc x nc (x n_slices)
    Cartesian grid that uspg_to_cartesian fills: pixel (ix, iy) of slice k
    at ((2 ix + 1 - nc) R / nc, (2 iy + 1 - nc) R / nc, slice centre);
    0 outside the disk."""
    import numpy as np

    from synth import phantom_value

    X = (2 * np.arange(nc) + 1 - nc) * w.radius / nc
    nz = w.n_slices
    zc = (-w.height / 2 + (np.arange(nz) + 0.5) * (w.height / nz)) if w.geometry == "cone3d" else np.zeros(1)
    Z, Y, Xg = np.meshgrid(zc, X, X, indexing="ij")
    pts = np.stack([Xg.ravel(), Y.ravel(), Z.ravel()], axis=1)
    v = phantom_value(w, pts).reshape(len(zc), nc, nc)
    v[:, np.hypot(Xg[0], Y[0]) >= w.radius] = 0.0
    return torch.as_tensor(v, dtype=dtype, device=device)


def report(w, cart: torch.Tensor) -> dict:
    """MAE, RMSE and SSIM of a Cartesian reconstruction [slices, nc, nc]
    against the phantom.  With binary coefficients a cell's value is its
    share of the line integral (about attenuation times the cell's chord),
    not an attenuation, so the image is first multiplied by the least-squares
    factor s = <x, t> / <x, x> that best matches the truth t (reported as
    "scale"; about 1 for length coefficients)."""
    truth = cartesian_truth(w, cart.shape[-1], cart.device)
    c = cart.double().reshape(truth.shape)
    den = float((c * c).sum())
    sc = float((c * truth).sum()) / den if den > 0 else 1.0
    c = c * sc
    return {"mae": mae(c, truth), "rmse": rmse(c, truth), "ssim": ssim(c, truth), "scale": sc,
            "truth_max": float(truth.max())}
