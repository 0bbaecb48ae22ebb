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
CSRC = os.path.join(ROOT, "paper_2208_12964_amd", "csrc")
# the batch kernel of each row form, its counter summary and its sources
# (the kernel, then the headers it includes from this library)
KERNELS = {
    "coded": ("mart_coded", ("mart_coded.hpp", "coded_rows.hpp", "trace_walk.hpp", "mart_batch.hpp", "mart_row.hpp")),
    "stored": ("mart_batch", ("mart_batch.hpp", "mart_row.hpp")),
}


def profile_path(kernel: str, workload: str) -> str:
    return os.path.join(ROOT, "profiles", f"{kernel}-{workload}.md")


def kernel_sha256(rows: str = "coded") -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNELS[rows][1]:
        h.update(open(os.path.join(CSRC, f), "rb").read())
    return h.hexdigest()


def counter_traffic(rows: str, workload: str):
    """HBM bytes per batch-kernel launch from the committed rocprofv3 counter
    summary (FETCH_SIZE and WRITE_SIZE scaled by a plain copy), or None when
    the kernel source changed since the counters were taken."""
    path = profile_path(KERNELS[rows][0], workload)
    if not os.path.exists(path):
        return None
    fields = {}
    for line in open(path):
        if ":" in line and line.startswith("- `"):
            key, val = line[3:].split("`", 1)
            fields[key] = val.split(":", 1)[1].strip().strip("`")
    if fields.get("source_sha256") != kernel_sha256(rows) or "traffic_bytes_per_launch" not in fields:
        return None
    return float(fields["traffic_bytes_per_launch"])


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="cone-256r-32v-hc")
    ap.add_argument("--mode", default="single",
                    choices=["single", "batch2d", "conebatch", "serve", "paper", "slabs"],
                    help="single: the 256-ring cone path (default); batch2d: 64 mixed 2D slices "
                         "one at a time vs one persistent launch; conebatch: n copies of a cone-beam "
                         "serving request, one at a time vs one lockstep batch; serve: the request "
                         "loop; paper: the paper's Table 1 scans with its literal segment scheme and "
                         "image quality; slabs: the same solve split into z-slabs (the multi-device "
                         "layout) on one GPU")
    ap.add_argument("--slabs", type=int, default=8, help="slabs: number of z-slabs")
    ap.add_argument("--rows", default="coded", choices=["coded", "stored"],
                    help="cone-beam rows: coded (rebuilt per column, the default) or stored (id, coefficient) pairs")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-rows", type=int, default=20, help="detector rows in the oracle sample")
    ap.add_argument("--sweeps", type=int, default=0, help="override the sweep count (profiling runs)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB device copy (scale for HBM byte counters)")
    ap.add_argument("--rate", type=float, default=20.0, help="serve: arrivals per second")
    ap.add_argument("--duration", type=float, default=120.0, help="serve: arrival window (s)")
    ap.add_argument("--budget-gib", type=float, default=16.0, help="serve: admission budget (GiB)")
    ap.add_argument("--steps-per-call", type=int, default=512, help="serve: engine steps per call")
    ap.add_argument("--lanes", default="split", choices=["rings", "split", "one"],
                    help="serve: one engine per ring count; the 256-ring requests (whose steps fill the "
                         "chip alone) in one engine and the rest in engine 0; or a single engine")
    ap.add_argument("--slots", default="256:1,0:40",
                    help="serve: slots per lane as lane:count pairs (lane = ring count with --lanes rings; "
                         "256 and 0 with --lanes split; 0 with --lanes one)")
    ap.add_argument("--fifo", action="store_true", help="serve: also run the one-at-a-time baseline")
    ap.add_argument("--streams", default="shared", choices=["lane", "shared"],
                    help="serve: one stream per lane (calls of different lanes overlap) or one shared stream")
    return ap.parse_args()


def copy_bandwidth(dev, mib: int = 1024, reps: int = 5) -> float:
    """Context for the roofline: GB/s (read + write bytes) of a plain device
    copy of `mib` MiB, median of `reps` timed copies after a warm-up."""
    import torch
    src = torch.ones(mib << 18, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    times = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        dst.copy_(src)
        b.record()
        b.synchronize()
        times.append(a.elapsed_time(b) * 1e-3)
    del src, dst
    return 2.0 * (mib << 20) / sorted(times)[len(times) // 2] / 1e9


def host_info() -> dict:
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "model": model}


def cpu_baseline(w, lattice, P, rows, sweeps_1: int = 2):
    """The FP64 oracle on a bounded sample of the same workload: the rays of
    `rows` central detector rows (every other row empty), traced once, then
    the MART sweep loop over all views timed on its own, with every host
    thread the oracle may use (all of the workload's sweeps) and with one
    thread (`sweeps_1` sweeps; the rate is per update either way).  The two
    runs give the same image bit for bit (the rays of a colour class share no
    cell)."""
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
    o.mart(csr, lattice, P, np.ones(o.n_cells), w.sweeps, w.beta, nthreads=threads)
    t2 = time.perf_counter()
    o.mart(csr, lattice, P, np.ones(o.n_cells), sweeps_1, w.beta, nthreads=1)
    t3 = time.perf_counter()
    per_sweep = w.n_views * csr.nnz
    rate_n = per_sweep * w.sweeps / (t2 - t1)
    rate_1 = per_sweep * sweeps_1 / (t3 - t2)
    return {"value": rate_n, "unit": "updates/s", "cores": threads, "kind": "oracle",
            "threads_n": {"threads": threads, "updates_per_s": rate_n, "sweeps": w.sweeps, "s": t2 - t1},
            "threads_1": {"threads": 1, "updates_per_s": rate_1, "sweeps": sweeps_1, "s": t3 - t2},
            "trace_s": t1 - t0, "host": host_info(),
            "sample": f"{rows} central detector rows ({len(rays)} rays, {csr.nnz} reference nonzeros) of "
                      f"{w.name}, FP64; MART sweep loop over {w.n_views} views timed alone: {w.sweeps} sweeps on "
                      f"{threads} threads {t2 - t1:.2f} s, {sweeps_1} sweeps on 1 thread {t3 - t2:.2f} s; "
                      f"trace (serial, not in the rate) {t1 - t0:.2f} s"}


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


def bench_serve(args):
    """The serving loop on the seeded Poisson stream of cone-beam requests:
    grids and coefficients of the nine geometries built and resident first,
    every request's projections generated in device memory before the clock
    starts, then requests served as they arrive.  value = completed requests
    per second (first arrival to last completion); p50 / p99 latency =
    completion minus arrival."""
    import torch

    import paper_2208_12964_amd as U
    import synth
    from paper_2208_12964_amd.serve import Request, Server, serve_fifo

    dev = torch.device("cuda:0")
    items = synth.serve_trace(rate=args.rate, duration=args.duration)
    say = lambda m: print(m, file=sys.stderr, flush=True)   # noqa: E731
    say(f"serve: {len(items)} requests over {args.duration:.0f} s at {args.rate}/s")
    t0 = time.perf_counter()
    geo, rays = {}, {}
    for key in sorted({it.key for it in items}):
        w = synth.serve_request(0, key[0], key[1], 1)
        g = U.Grid.from_workload(w)
        geo[key] = (g, U.Coeffs.from_workload(g, w))
        rays[key] = synth.scan_rays_torch(w, dev)
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t0
    coeff_bytes = sum(c.device_bytes for _, c in geo.values())
    say(f"serve: {len(geo)} geometries built in {build_s:.1f} s ({coeff_bytes / 2**30:.2f} GiB resident)")
    t0 = time.perf_counter()
    projs = []
    for i, it in enumerate(items):
        projs.append(synth.make_projections_torch(it.workload(), dev, torch.float32, rays=rays[it.key])
                     .reshape(-1))
        if i % 400 == 399:
            torch.cuda.synchronize()
            say(f"serve: generated {i + 1} projection sets")
    rays.clear()
    torch.cuda.synchronize()
    gen_s = time.perf_counter() - t0
    lane_of = {"rings": lambda key: key[0], "split": lambda key: key[0] if key[0] >= 256 else 0,
               "one": lambda key: 0}[args.lanes]

    def make(_items):
        return [Request(it.k, it.arrival, it.key, pr, it.sweeps, 0.1) for it, pr in zip(items, projs)]

    # warm-up: one short request per geometry through the engine
    warm = Server(geo.get, budget=1 << 62, lane_of=lane_of)
    warm.run([Request(-1 - j, 0.0, key, projs[next(i for i, it in enumerate(items) if it.key == key)], 1, 0.1)
              for j, key in enumerate(sorted(geo))])
    warm.close()
    budget = int(args.budget_gib * 2**30)
    slots = {int(a): int(b) for a, b in (x.split(":") for x in args.slots.split(",") if x)}
    srv = Server(geo.get, budget=budget, lane_of=lane_of, max_slots=slots, steps_per_call=args.steps_per_call,
                 keep_results=False, shared_stream=args.streams == "shared")
    reqs = make(items)
    report = lambda st: say("serve: t=%.0f s completed %d queued %d active %d" % (   # noqa: E731
        st["wall_s"], st["completed"], st.get("queued", 0), st.get("active", 0)))
    st = srv.run(reqs, progress=report)
    srv.close()
    updates = sum(it.sweeps * it.n_views * geo[it.key][1].nnz for it in items)
    out = {"metric": f"served cone-beam reconstructions/s (Poisson {args.rate:g}/s, {args.duration:g} s, "
                     "Nr in {64,128,256}, p in {8,16,32}, 10-20 sweeps)",
           "value": st["req_per_s"], "unit": "req/s", "n_gpus": 1, "steps": st["completed"], "warmup": len(geo),
           "ms_per_step": st["wall_s"] * 1e3 / max(1, st["completed"]), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "serve-poisson", "rate_per_s": args.rate, "duration_s": args.duration,
                      "requests": len(items), "budget_gib": args.budget_gib, "lanes": args.lanes, "streams": args.streams,
                      "slots": args.slots,
                      "steps_per_call": args.steps_per_call},
           "latency": {k: v for k, v in st.items() if k.endswith("_s") or k.endswith("_by_key_s")},
           "completed": st["completed"], "rejected": st["rejected"],
           "updates_per_s_while_serving": updates / st["wall_s"],
           "build_s": build_s, "input_generation_s": gen_s, "coeff_gib_resident": coeff_bytes / 2**30}
    if args.fifo:
        say("serve: one-at-a-time baseline")
        torch.cuda.synchronize()
        time.sleep(1.0)    # an idle second parts the two phases in a kernel trace
        fst = serve_fifo(geo.get, make(items), keep_results=False,
                         progress=lambda s: say("fifo: t=%.0f s completed %d" % (s["wall_s"], s["completed"])))
        out["one_at_a_time"] = fst
    print(json.dumps(out), flush=True)


def bench_paper(args):
    """The paper's own scans (Table 1: fan beam 256^2 / 512^2 / 1024^2 with
    50 views, cone beam 128^3 with 70 views; Table 3's Cu-lump and frog
    geometries with synthetic phantoms) with its literal scheme:
    segment records re-binned per view (rows kept, and timed again re-binned
    on the fly), binary MART, bijection remap, and MAE / RMSE / SSIM against
    the phantom on the Cartesian grid.
    value = ray-cell updates/s of the 128^3 cone-beam solve."""
    import torch

    import paper_2208_12964_amd as U
    import synth
    from paper_2208_12964_amd.quality import report

    dev = torch.device("cuda:0")
    say = lambda m: print(m, file=sys.stderr, flush=True)   # noqa: E731
    out_cfg = []
    head = None
    for name in ("paper-fan-256-50v", "paper-fan-512-50v", "paper-fan-1024-50v", "paper-culump-geometry",
                 "paper-frog-geometry", "paper-cone-128-70v"):
        w = synth.get(name)
        if args.sweeps:
            w = w.with_(sweeps=args.sweeps)
        P = synth.make_projections_torch(w, dev, torch.float32).reshape(-1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g = U.Grid.from_workload(w)
        co = U.Coeffs.from_workload(g, w)
        torch.cuda.synchronize()
        build_s = time.perf_counter() - t0
        work = torch.empty(co.workspace_bytes(), dtype=torch.uint8, device=dev)
        warm = torch.ones(g.n_cells, device=dev)
        U.mart(co, P, warm, 1, w.beta, work=work)
        torch.cuda.synchronize()
        best = None
        for _ in range(max(1, args.steps)):
            img = torch.ones(g.n_cells, device=dev)
            U.mart_timing(True)
            t0 = time.perf_counter()
            U.mart(co, P, img, w.sweeps, w.beta, work=work)
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
            ms, launches = U.mart_timing(False)
            best = el if best is None or el < best else best
        # the same solve re-binning every view's rows from the records on the
        # fly instead of reading the kept rows
        co_r = U.Coeffs.from_workload(g, w, view_rows="rebin")
        U.mart(co_r, P, torch.ones(g.n_cells, device=dev), 1, w.beta, work=work)
        img_r = torch.ones(g.n_cells, device=dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        U.mart(co_r, P, img_r, w.sweeps, w.beta, work=work)
        torch.cuda.synchronize()
        rebin_s = time.perf_counter() - t0
        rebin_diff = ((img - img_r).abs().max() / img.abs().max()).item()
        kept_mib = (co.device_bytes - co_r.device_bytes) / 2 ** 20
        del co_r
        cart_b = U.to_cartesian(g, img, 2 * w.n_rings, mode="bijection")   # the paper's display map
        cart = U.to_cartesian(g, img, 2 * w.n_rings)                       # geometric: for the figures
        torch.cuda.synchronize()
        q = report(w, cart)
        q_b = report(w, cart_b)
        upd = int(co.view_nnz().sum()) * w.sweeps
        rec = {"workload": name, "rings": w.n_rings, "slices": w.n_slices, "views": w.n_views,
               "detector": f"{w.det_u}x{w.det_v}", "sweeps": w.sweeps, "beta": w.beta,
               "segments": co.nnz, "lattice": list(co.lattice), "updates_per_sweep": upd // w.sweeps,
               "build_ms": build_s * 1e3, "mart_ms": best * 1e3, "avg_launch_us": ms * 1e3 / max(1, launches),
               "launches": launches, "updates_per_s": upd / best, "kept_rows_mib": kept_mib,
               "rebin_on_the_fly": {"mart_ms": rebin_s * 1e3, "updates_per_s": upd / rebin_s,
                                    "max_rel_diff": rebin_diff},
               "quality_vs_phantom": q, "quality_bijection_map": q_b}
        say(f"paper: {json.dumps(rec)}")
        out_cfg.append(rec)
        head = rec
    out = {"metric": "MART ray-cell updates/s, paper's 128^3 cone-beam scan (70 views, literal scheme)",
           "value": head["updates_per_s"], "unit": "updates/s", "n_gpus": 1, "steps": max(1, args.steps),
           "warmup": 1, "ms_per_step": head["mart_ms"], "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": head["workload"], "views": head["views"], "sweeps": head["sweeps"]},
           "configs": out_cfg}
    if not args.no_cpu_baseline:
        from oracle import Oracle
        w = synth.get("paper-cone-128-70v")
        threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        o = Oracle(w, nthreads=threads)
        Pn = synth.make_projections_torch(w, "cpu").numpy()
        seg = o.segments_view()
        lat = o.colour_rebin(seg)
        t0 = time.perf_counter()
        o.mart_rebin(seg, lat, Pn, np.ones(o.n_cells), 2, w.beta)
        el = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": 2 * head["updates_per_sweep"] / el, "unit": "updates/s", "cores": threads,
                               "kind": "oracle", "sample": f"2 MART sweeps of {w.name} (FP64, rows re-binned per view)"}
    print(json.dumps(out), flush=True)


def bench_slabs(args):
    """The single-GPU workload split into z-slabs as several devices would
    share it (every batch: each slab's part of the ray sums, their sum, each
    slab's correction), all run here.  Reports the emulated time against the
    fused path, the agreement of the two images and each slab's share of
    the nonzeros; value = ray-cell updates/s of the emulated split."""
    import torch

    import paper_2208_12964_amd as U
    import synth

    dev = torch.device("cuda:0")
    w = synth.get(args.workload)
    if args.sweeps:
        w = w.with_(sweeps=args.sweeps)
    g = U.Grid.from_workload(w)
    co = U.Coeffs.from_workload(g, w)
    proj = synth.make_projections_torch(w, dev, torch.float32).reshape(-1).contiguous()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sl = U.Slabs(co, args.slabs)
    build_ms = (time.perf_counter() - t0) * 1e3
    info = [sl.info(k) for k in range(args.slabs)]
    work = torch.empty(sl.workspace_bytes(), dtype=torch.uint8, device=dev)
    fwork = torch.empty(co.workspace_bytes(), dtype=torch.uint8, device=dev)

    def timed(fn):
        img = torch.ones(g.n_cells, device=dev)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        fn(img)
        b.record()
        b.synchronize()
        return a.elapsed_time(b), img

    timed(lambda im: U.mart(co, proj, im, 1, w.beta, work=fwork))
    timed(lambda im: sl.run(proj, im, 1, w.beta, work=work))
    t_fused, f_fused = timed(lambda im: U.mart(co, proj, im, w.sweeps, w.beta, work=fwork))
    t_slab, f_slab = timed(lambda im: sl.run(proj, im, w.sweeps, w.beta, work=work))
    diff = ((f_fused - f_slab).abs().max() / f_fused.abs().max()).item()
    updates = w.n_views * co.nnz * w.sweeps
    share = max(i["nnz"] for i in info) / co.nnz
    rays_per_class = -(-w.det_u // co.lattice[0]) * -(-w.det_v // co.lattice[1])
    out = {"metric": f"MART ray-cell updates/s, {args.slabs} z-slabs emulated on one GPU",
           "value": updates / (t_slab * 1e-3), "unit": "updates/s", "n_gpus": 1, "steps": 1, "warmup": 1,
           "ms_per_step": t_slab, "higher_is_better": True, "scaling": "strong", "vs_baseline": None,
           "dtype": "f32", "data": "synthetic",
           "config": {"workload": w.name, "slabs": args.slabs, "sweeps": w.sweeps, "views": w.n_views,
                      "lattice": list(co.lattice)},
           "fused_ms": t_fused, "emulated_over_fused": t_slab / t_fused,
           "max_rel_diff_vs_fused": diff, "build_ms": build_ms,
           "slab_nnz_share": [i["nnz"] / co.nnz for i in info],
           "largest_share_ms_per_sweep_est": t_slab / w.sweeps * share,
           "allreduce_bytes_per_batch": rays_per_class * 4,
           "allreduces_per_sweep": w.n_views * co.lattice[0] * co.lattice[1]}
    print(json.dumps(out), flush=True)


def bench_conebatch(args):
    """n copies (1, 2, 4, 8, 16) of cone-beam serving requests (128 rings,
    32 and 8 views; 64 rings, 32 and 8 views; 3 sweeps, one phantom each):
    one mart() after another vs one lockstep batch, ray-cell updates/s of
    each; the batch results are checked bit for bit against the requests
    alone.  value = updates/s of sixteen 128-ring, 32-view requests batched."""
    import torch

    import paper_2208_12964_amd as U
    import synth

    dev = torch.device("cuda:0")
    rows, head = [], None
    for nr, p in ((128, 32), (128, 8), (64, 32), (64, 8)):
        ws = [synth.serve_request(100 + k, nr, p, 3) for k in range(16)]
        g = U.Grid.from_workload(ws[0])
        co = U.Coeffs.from_workload(g, ws[0])
        projs = [synth.make_projections_torch(w, dev, torch.float32).reshape(-1).contiguous() for w in ws]
        per = ws[0].sweeps * ws[0].n_views * co.nnz

        def alone(n):
            imgs = [torch.ones(g.n_cells, device=dev) for _ in range(n)]
            torch.cuda.synchronize()
            t = time.perf_counter()
            for im, pr, w in zip(imgs, projs, ws):
                U.mart(co, pr, im, w.sweeps, w.beta)
            torch.cuda.synchronize()
            return time.perf_counter() - t, imgs

        alone(1)
        for n in (1, 2, 4, 8, 16):
            t_a, ref = min((alone(n) for _ in range(2)), key=lambda x: x[0])
            b = U.Batch([co] * n)
            b.set("lockstep", 256)
            works = b.work_buffers(dev)
            best, imgs = None, None
            for _ in range(3):
                imgs = [torch.ones(g.n_cells, device=dev) for _ in range(n)]
                torch.cuda.synchronize()
                t = time.perf_counter()
                b.run(projs[:n], imgs, [w.sweeps for w in ws[:n]], [w.beta for w in ws[:n]], works=works)
                torch.cuda.synchronize()
                dt = time.perf_counter() - t
                best = dt if best is None else min(best, dt)
            same = all(torch.equal(a, m) for a, m in zip(ref, imgs))
            b.close()
            row = {"rings": nr, "views": p, "n": n, "alone_updates_per_s": n * per / t_a,
                   "batched_updates_per_s": n * per / best, "batched_ms": best * 1e3, "bitwise_equal": same}
            rows.append(row)
            if nr == 128 and p == 32 and n == 16:
                head = row
            print(f"conebatch: {nr} rings, {p} views, n={n}: alone {row['alone_updates_per_s'] / 1e9:.1f} G/s, "
                  f"batched {row['batched_updates_per_s'] / 1e9:.1f} G/s, equal {same}", file=sys.stderr, flush=True)
    out = {"metric": "ray-cell updates/s of 16 batched 128-ring, 32-view cone-beam requests",
           "value": head["batched_updates_per_s"], "unit": "updates/s", "n_gpus": 1, "steps": 3, "warmup": 1,
           "ms_per_step": head["batched_ms"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32", "data": "synthetic", "config": {"workload": "conebatch", "sweeps": 3},
           "rows": rows}
    print(json.dumps(out), flush=True)


def main():
    args = parse()
    if args.mode == "conebatch" and args.gpus == 1:
        return bench_conebatch(args)
    if args.mode == "slabs" and args.gpus == 1:
        return bench_slabs(args)
    if args.mode == "paper" and args.gpus == 1:
        return bench_paper(args)
    if args.mode == "batch2d" and args.gpus == 1:
        return bench_batch2d(args)
    if args.mode == "serve" and args.gpus == 1:
        return bench_serve(args)
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path. Independent "
              "reconstructions would shard over GPUs with no communication; one cone-beam solve "
              "would split into z-slabs (mart_run_slabs shows that split on one GPU).",
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
        co = U.Coeffs.from_workload(grid, w, torch.float32, rows=args.rows)
        ev[1].record(stream)
        img = torch.ones(grid.n_cells, dtype=torch.float32, device=dev)
        U.mart(co, proj, img, w.sweeps, w.beta)
        ev[2].record(stream)
        cart = U.to_cartesian(grid, img, nc)
        ev[3].record(stream)
        if record is not None:
            record.append((ev, co.nnz, co.lattice, co.max_row, co.coded, co.explicit_rays))
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
    mart_each = [r[0][1].elapsed_time(r[0][2]) for r in rec]
    mart_ms = np.mean(mart_each)
    remap_ms = np.mean([r[0][2].elapsed_time(r[0][3]) for r in rec])
    solve_each = sorted(r[0][0].elapsed_time(r[0][3]) for r in rec)

    def solve_pct(q):
        return float(solve_each[max(0, min(len(solve_each) - 1, -(-q * len(solve_each) // 100) - 1))])
    n_launch = w.sweeps * w.n_views * lattice[0] * lattice[1]
    assert batch_launches == n_launch * args.steps
    per_launch_s = batch_ms * 1e-3 / batch_launches
    bytes_per_launch = 16.0 * updates / n_launch
    achieved = bytes_per_launch / per_launch_s / 1e9
    kernel = KERNELS["coded" if rec[0][4] else "stored"][0]
    traffic = counter_traffic("coded" if rec[0][4] else "stored", w.name)
    copy_gbs = copy_bandwidth(dev)
    f = img.float().cpu().numpy()
    out = {
        "metric": "MART ray-cell updates/s", "value": updates / (ms_step * 1e-3), "unit": "updates/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "rings": w.n_rings, "slices": w.n_slices, "views": w.n_views,
                   "detector": f"{w.det_u}x{w.det_v}", "sweeps": w.sweeps, "beta": w.beta,
                   "nnz_ref": nnz, "lattice": list(lattice), "remap": f"{nc}x{nc}x{w.n_slices}",
                   "rows": "coded" if rec[0][4] else "stored", "explicit_rays": rec[0][5]},
        "sweeps_per_s": w.sweeps / (mart_ms * 1e-3),
        "phases_ms": {"build": build_ms, "mart": mart_ms, "remap": remap_ms},
        "mart_ms_over_steps": {"median": float(np.median(mart_each)), "min": float(np.min(mart_each)),
                               "max": float(np.max(mart_each))},
        # one solve (build, sweeps, remap) per step, device time; nearest-rank
        # percentiles over the timed steps
        "solve_latency_ms": {"p50": solve_pct(50), "p99": solve_pct(99), "n": len(solve_each)},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic,
                     "kernel": kernel, "bytes_per_update": 16,
                     "launches_per_step": n_launch, "avg_launch_us": per_launch_s * 1e6,
                     "copy_GBs": copy_gbs, "frac_of_copy": achieved / copy_gbs if copy_gbs else None},
        "image": {"min": float(f.min()), "max": float(f.max())},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, lattice, P, args.cpu_rows)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
