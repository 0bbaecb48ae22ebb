"""Writes cone256_sweeps20.npz: the FP64 oracle's image of the 256-ring,
32-view high-contrast cone-beam workload after its 20 MART sweeps
(Sec. III.D, eqs. 17-18; order: views, lattice classes, rays).

The stored values come from the oracle alone (``oracle/``, on inputs from
``synth/``).  Too many cells to store them all (53.76 M), so the file keeps:

* every cell of the three slices through each dense inclusion's centre whose
  in-plane centre lies within the inclusion's radius + 0.04 of the
  inclusion's axis (the high-contrast region where FP32 drift is largest);
* every 997th cell of the whole image;
* max |f| and min f over all cells (the parity metric's denominator and the
  positivity check).

Run once on a CPU (about 10 minutes on 8 threads, 6 GB of memory):
    python tests/golden/make_cone256_golden.py
"""
from __future__ import annotations

import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

OUT = os.path.join(HERE, "cone256_sweeps20.npz")
WORKLOAD = "cone-256r-32v-hc"
STRIDE = 997
MARGIN = 0.04


def cell_centres(o, w, cells):
    """Centres (x, y, z) of cells in the paper's numbering (slice-major,
    ring heads of eq. 2, sectors anticlockwise from +x)."""
    c2d = int(o.head[-1])
    k = cells // c2d
    rem = cells % c2d
    i = np.searchsorted(o.head, rem, side="right") - 1
    s = rem - o.head[i]
    r = w.radius / w.n_rings
    rho = (i + 0.5) * r
    phi = (s + 0.5) * 2 * math.pi / o.ng[i]
    h = w.height / w.n_slices
    z = -w.height / 2 + (k + 0.5) * h
    return rho * np.cos(phi), rho * np.sin(phi), z


def sample_cells(o, w):
    import synth
    objs = synth.draw_phantom(w)
    c2d = int(o.head[-1])
    h = w.height / w.n_slices
    slice_cells = np.arange(c2d, dtype=np.int64)
    x, y, _ = cell_centres(o, w, slice_cells)
    picks = [np.arange(0, o.n_cells, STRIDE, dtype=np.int64)]
    for cen, ax, _, _ in objs[1:]:            # the three inclusions (spheres)
        near = slice_cells[np.hypot(x - cen[0], y - cen[1]) <= ax[0] + MARGIN]
        k0 = int(math.floor((cen[2] + w.height / 2) / h))
        for k in (k0 - 1, k0, k0 + 1):
            if 0 <= k < w.n_slices:
                picks.append(k * c2d + near)
    return np.unique(np.concatenate(picks))


def main():
    import synth
    from oracle import Oracle
    from oracle.oracle import build_oracle

    build_oracle(force=False)
    w = synth.get(WORKLOAD)
    threads = os.cpu_count() or 1
    t0 = time.perf_counter()
    P = synth.make_projections(w)
    o = Oracle(w, nthreads=threads)
    csr = o.trace_view(0)
    lat = o.colour(csr)
    t1 = time.perf_counter()
    print(f"inputs + trace + colouring {t1 - t0:.0f} s: nnz {csr.nnz}, lattice {lat}", flush=True)
    f = o.mart(csr, lat, P, np.ones(o.n_cells), w.sweeps, w.beta)
    t2 = time.perf_counter()
    print(f"{w.sweeps} sweeps {t2 - t1:.0f} s on {threads} threads", flush=True)
    idx = sample_cells(o, w)
    np.savez_compressed(
        OUT, workload=np.array(WORKLOAD), sweeps=np.int64(w.sweeps), beta=np.float64(w.beta),
        lattice=np.array(lat, dtype=np.int64), nnz=np.int64(csr.nnz), n_cells=np.int64(o.n_cells),
        cells=idx, values=f[idx], max_abs=np.float64(np.max(np.abs(f))), min=np.float64(np.min(f)),
        cite=np.array("Sec. III.D eqs. 17-18, 20 sweeps, FP64 oracle, order views > classes > rays"))
    print(f"wrote {OUT}: {len(idx)} cells, max|f| {np.max(np.abs(f)):.6g}, min f {np.min(f):.6g}", flush=True)


if __name__ == "__main__":
    main()
