#!/usr/bin/env python3
"""Throughput of MART on the 256-ring cone-beam USCG (high-contrast phantom).

One step = the whole path on one synthetic input already resident in HBM:
grid build, reference-view trace + colouring, 20 MART sweeps over 32 views,
and the remap to a 512 x 512 x 256 Cartesian grid.  Prints one JSON line.

value = MART ray-cell updates per second of the whole step
        (views * reference nonzeros * sweeps / step time).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
PROFILE = os.path.join(ROOT, "profiles", "mart_batch-cone-256r-32v-hc.md")
KERNEL_SRC = os.path.join(ROOT, "paper_2208_12964_amd", "csrc", "mart.hip")


def counter_traffic():
    """HBM bytes per mart_batch launch from the committed rocprofv3 counter
    summary (FETCH_SIZE and WRITE_SIZE scaled by a plain copy), or None when
    the kernel source changed since the counters were taken."""
    import hashlib
    if not os.path.exists(PROFILE):
        return None
    fields = {}
    for line in open(PROFILE):
        if ":" in line and line.startswith("- `"):
            key, val = line[3:].split("`", 1)
            fields[key] = val.split(":", 1)[1].strip().strip("`")
    sha = hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()
    if fields.get("source_sha256") != sha or "traffic_bytes_per_launch" not in fields:
        return None
    return float(fields["traffic_bytes_per_launch"])


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="cone-256r-32v-hc")
    ap.add_argument("--mode", default="single", choices=["single", "batch2d", "serve"],
                    help="single: the 256-ring cone path (default); batch2d: 64 mixed 2D slices "
                         "one at a time vs one persistent launch; serve: the request loop")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-rows", type=int, default=20, help="detector rows in the oracle sample")
    ap.add_argument("--sweeps", type=int, default=0, help="override the sweep count (profiling runs)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB device copy (scale for HBM byte counters)")
    return ap.parse_args()


def cpu_baseline(w, lattice, P, rows):
    """The FP64 oracle on a bounded sample of the same workload: the rays of
    `rows` central detector rows, traced, then MART over all views and sweeps
    with every other row empty."""
    from oracle import Oracle
    from oracle.oracle import CSR
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    o = Oracle(w, nthreads=threads)
    V, U = w.det_v, w.det_u
    w0 = V // 2 - rows // 2
    rays = [wv * U + u for wv in range(w0, w0 + rows) for u in range(U)]
    t0 = time.perf_counter()
    counts = np.zeros(o.n_rays, dtype=np.int64)
    cells, lens = [], []
    for r in rays:
        S, D = o.ray(0, r)
        c, l = o.trace_line(S, D)
        counts[r] = len(c)
        cells.append(c)
        lens.append(l)
    rowptr = np.concatenate([[0], np.cumsum(counts)])
    order = np.argsort(rays)
    csr = CSR(rowptr, np.concatenate([cells[i] for i in order]), np.concatenate([lens[i] for i in order]))
    t1 = time.perf_counter()
    o.mart(csr, lattice, P, np.ones(o.n_cells), w.sweeps, w.beta)
    t2 = time.perf_counter()
    updates = w.n_views * csr.nnz * w.sweeps
    return {"value": updates / (t2 - t0), "unit": "updates/s", "cores": threads, "kind": "oracle",
            "sample": f"{rows} central detector rows ({len(rays)} rays, {csr.nnz} reference nonzeros) of "
                      f"{w.name}: trace {t1 - t0:.2f} s + {w.sweeps} MART sweeps over {w.n_views} views "
                      f"{t2 - t1:.2f} s, FP64"}


def bench_batch2d(args):
    """64 independent 2D slices (ring counts 32..256, 8..32 views, 2 Nr bins,
    15 sweeps): one mart_run per slice in sequence vs one autotuned
    persistent launch.  value = slices reconstructed per second (batched)."""
    import torch

    import paper_2208_12964_amd as U
    import synth

    dev = torch.device("cuda:0")
    ws = synth.batch2d_members(64)
    t0 = time.perf_counter()
    grids = [U.Grid.from_workload(w) for w in ws]
    cos = [U.Coeffs.from_workload(g, w) for g, w in zip(grids, ws)]
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t0
    projs = [torch.as_tensor(synth.make_projections(w), dtype=torch.float32, device=dev).contiguous()
             for w in ws]
    sweeps = [w.sweeps for w in ws]
    betas = [w.beta for w in ws]
    works = [torch.empty(c.workspace_bytes(), dtype=torch.uint8, device=dev) for c in cos]

    def one_at_a_time():
        out = []
        for co, proj, g, w, wk in zip(cos, projs, grids, ws, works):
            img = torch.ones(g.n_cells, device=dev)
            U.mart(co, proj, img, w.sweeps, w.beta, work=wk)
            out.append(img)
        return out

    b = U.Batch(cos)
    ones = [torch.ones(g.n_cells, device=dev) for g in grids]
    tune_ms = b.autotune(projs, ones, betas, probe_sweeps=1, works=works)

    def batched():
        imgs = [torch.ones(g.n_cells, device=dev) for g in grids]
        b.run(projs, imgs, sweeps, betas, works=works)
        return imgs

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(reps):
            res = fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t) / reps, res

    t_seq, alone = timed(one_at_a_time, max(1, args.steps))
    t_bat, multi = timed(batched, max(1, args.steps))
    same = all(torch.equal(a, m) for a, m in zip(alone, multi))
    updates = sum(w.n_views * c.nnz * w.sweeps for w, c in zip(ws, cos))
    info = b.info()
    out = {"metric": "USPG 2D slices reconstructed/s (64 mixed slices, 15 sweeps)",
           "value": len(ws) / t_bat, "unit": "slices/s", "n_gpus": 1, "steps": args.steps, "warmup": 1,
           "ms_per_step": t_bat * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32", "data": "synthetic",
           "config": {"workload": "batch2d-64", "rings": sorted(set(w.n_rings for w in ws)),
                      "views": sorted(set(w.n_views for w in ws)), "sweeps": 15},
           "one_at_a_time": {"slices_per_s": len(ws) / t_seq, "ms": t_seq * 1e3},
           "speedup_vs_one_at_a_time": t_seq / t_bat, "bitwise_equal_to_one_at_a_time": same,
           "updates_per_s": updates / t_bat, "autotuned": info, "autotune_probe_ms": tune_ms,
           "build_s": build_s}
    print(json.dumps(out), flush=True)


def main():
    args = parse()
    if args.mode == "batch2d" and args.gpus == 1:
        return bench_batch2d(args)
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(independent reconstructions shard with no communication; see the design notes).",
              file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_2208_12964_amd as U
    import synth

    w = synth.get(args.workload)
    if args.sweeps:
        w = w.with_(sweeps=args.sweeps)
    dev = torch.device("cuda:0")
    if args.copy_calibration:
        src = torch.ones(1 << 28, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(2):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    P = synth.make_projections(w)
    proj = torch.as_tensor(P, dtype=torch.float32).to(dev).contiguous()
    nc = w.remap_nc or 2 * w.n_rings
    stream = torch.cuda.current_stream()

    def step(record=None):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
        ev[0].record(stream)
        grid = U.Grid.from_workload(w)
        co = U.Coeffs.from_workload(grid, w, torch.float32)
        ev[1].record(stream)
        img = torch.ones(grid.n_cells, dtype=torch.float32, device=dev)
        U.mart(co, proj, img, w.sweeps, w.beta)
        ev[2].record(stream)
        cart = U.to_cartesian(grid, img, nc)
        ev[3].record(stream)
        if record is not None:
            record.append((ev, co.nnz, co.lattice, co.max_row))
        return img, cart, co, grid

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    rec = []
    U.mart_timing(True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        img, cart, co, grid = step(rec)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    batch_ms, batch_launches = U.mart_timing(False)
    ms_step = (t1 - t0) * 1e3 / args.steps
    nnz, lattice = rec[0][1], rec[0][2]
    updates = w.n_views * nnz * w.sweeps
    build_ms = np.mean([r[0][0].elapsed_time(r[0][1]) for r in rec])
    mart_ms = np.mean([r[0][1].elapsed_time(r[0][2]) for r in rec])
    remap_ms = np.mean([r[0][2].elapsed_time(r[0][3]) for r in rec])
    n_launch = w.sweeps * w.n_views * lattice[0] * lattice[1]
    assert batch_launches == n_launch * args.steps
    per_launch_s = batch_ms * 1e-3 / batch_launches
    bytes_per_launch = 16.0 * updates / n_launch
    achieved = bytes_per_launch / per_launch_s / 1e9
    traffic = counter_traffic()
    f = img.float().cpu().numpy()
    out = {
        "metric": "MART ray-cell updates/s", "value": updates / (ms_step * 1e-3), "unit": "updates/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "rings": w.n_rings, "slices": w.n_slices, "views": w.n_views,
                   "detector": f"{w.det_u}x{w.det_v}", "sweeps": w.sweeps, "beta": w.beta,
                   "nnz_ref": nnz, "lattice": list(lattice), "remap": f"{nc}x{nc}x{w.n_slices}"},
        "sweeps_per_s": w.sweeps / (mart_ms * 1e-3),
        "phases_ms": {"build": build_ms, "mart": mart_ms, "remap": remap_ms},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic,
                     "kernel": "mart_batch", "bytes_per_update": 16,
                     "launches_per_step": n_launch, "avg_launch_us": per_launch_s * 1e6},
        "image": {"min": float(f.min()), "max": float(f.max())},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, lattice, P, args.cpu_rows)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
