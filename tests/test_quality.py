"""Image-quality figures (MAE, RMSE, SSIM) used to report reconstructions of
the paper's scans: closed forms and a brute-force SSIM over every window."""
import math

import numpy as np
import torch

import synth
from paper_2208_12964_amd.quality import cartesian_truth, mae, rmse, ssim


def test_mae_rmse_closed_forms():
    x = torch.rand(7, 9, dtype=torch.float64)
    assert abs(mae(x + 0.25, x) - 0.25) < 1e-15
    assert abs(rmse(x - 0.5, x) - 0.5) < 1e-15
    d = torch.tensor([3.0, -4.0])
    assert abs(rmse(d, torch.zeros(2)) - math.sqrt(12.5)) < 1e-15 and mae(d, torch.zeros(2)) == 3.5


def brute_ssim(x, y, win=11, sigma=1.5, k1=0.01, k2=0.03):
    t = np.arange(win) - (win - 1) / 2
    g1 = np.exp(-t * t / (2 * sigma * sigma))
    w2 = np.outer(g1, g1)
    w2 /= w2.sum()
    L = y.max() - y.min()
    c1, c2 = (k1 * L) ** 2, (k2 * L) ** 2
    vals = []
    for i in range(x.shape[0] - win + 1):
        for j in range(x.shape[1] - win + 1):
            a, b = x[i:i + win, j:j + win], y[i:i + win, j:j + win]
            ma, mb = (w2 * a).sum(), (w2 * b).sum()
            va, vb = (w2 * (a - ma) ** 2).sum(), (w2 * (b - mb) ** 2).sum()
            cov = (w2 * (a - ma) * (b - mb)).sum()
            vals.append((2 * ma * mb + c1) * (2 * cov + c2) / ((ma * ma + mb * mb + c1) * (va + vb + c2)))
    return float(np.mean(vals))


def test_ssim_brute_force_and_identities():
    rng = np.random.default_rng(0)
    y = rng.random((20, 17))
    x = y + 0.1 * rng.standard_normal((20, 17))
    got = ssim(torch.as_tensor(x), torch.as_tensor(y))
    assert abs(got - brute_ssim(x, y)) < 1e-12
    assert abs(ssim(torch.as_tensor(y), torch.as_tensor(y)) - 1.0) < 1e-12
    assert got < 0.99
    # a stack averages its slices
    xs = torch.as_tensor(np.stack([x, y]))
    ys = torch.as_tensor(np.stack([y, y]))
    assert abs(ssim(xs, ys) - 0.5 * (got + 1.0)) < 1e-12


def test_cartesian_truth_matches_phantom():
    w = synth.paper_cone(16, 5)
    t = cartesian_truth(w, 16, "cpu").numpy()
    assert t.shape == (16, 16, 16)
    X = (2 * np.arange(16) + 1 - 16) * w.radius / 16
    zc = -w.height / 2 + (np.arange(16) + 0.5) * (w.height / 16)
    for k, iy, ix in [(3, 4, 5), (8, 8, 8), (12, 2, 9), (0, 0, 0)]:
        p = np.array([[X[ix], X[iy], zc[k]]])
        want = synth.phantom_value(w, p)[0] if math.hypot(X[ix], X[iy]) < w.radius else 0.0
        assert t[k, iy, ix] == want
    assert t.max() > 0


def test_report_rescales_by_least_squares():
    from paper_2208_12964_amd.quality import report
    w = synth.paper_fan(32, 5)
    t = cartesian_truth(w, 32, "cpu")
    q = report(w, 0.02 * t)
    assert abs(q["scale"] - 50.0) < 1e-9 and q["mae"] < 1e-12 and abs(q["ssim"] - 1.0) < 1e-12
