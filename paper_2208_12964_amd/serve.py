"""Continuous-batching reconstruction server over the library's engine.

Requests (a geometry key, projections already in device memory, a sweep
count and a relaxation) arrive over time.  The server keeps one grid and one
coefficient set per geometry resident on the device, admits queued requests
in arrival order while their device footprint fits a byte budget, and runs
every admitted request through ``uspg_engine_step`` calls: each call advances
all admitted requests of a lane by a number of (view, colour class) steps,
so requests of different sizes and sweep counts overlap on the device and
leave as soon as their own sweeps are done.  A request's result is bit for
bit the one ``mart`` gives for it alone.

Lanes: requests are split by a lane function (default: by ring count) into
engines, so that small requests do not advance at the launch rate of the
largest one.  The lanes issue their calls on one shared stream (default),
where the calls of different lanes run one after another instead of
competing for the chip, or on a stream each (`shared_stream=False`).  All
streams keep the default priority.

Only host logic lives here (queues, budget, timing); every step of the
reconstruction runs in the library.
"""

from __future__ import annotations

import time
from collections import deque
from dataclasses import dataclass, field

import torch

from . import Coeffs, Engine, Grid, mart


@dataclass(eq=False)
class Request:
    k: int
    arrival: float          # seconds from the start of the run
    key: tuple              # geometry key
    proj: torch.Tensor      # device projections [views * rays]
    sweeps: int
    beta: float
    image: torch.Tensor | None = None     # result (paper numbering) once done
    footprint: int = 0
    t_admit: float | None = None
    t_done: float | None = None
    cancelled: bool = False
    lane: int = -1
    slot: int = -1
    steps: int = 0          # engine steps the request needs
    offset: int = 0         # lane step count at admission
    work: torch.Tensor | None = field(default=None, repr=False)


class GeometryCache:
    """Grid and coefficients per geometry key, built on first use and kept
    resident.  `factory(key) -> (Grid, Coeffs)`."""

    def __init__(self, factory):
        self.factory = factory
        self.entries = {}

    def get(self, key):
        if key not in self.entries:
            self.entries[key] = self.factory(key)
        return self.entries[key]

    def device_bytes(self) -> int:
        return sum(c.device_bytes for _, c in self.entries.values())


def footprint_bytes(coeffs: Coeffs, proj: torch.Tensor, dtype) -> int:
    """Device bytes a request holds while admitted: its projections, its
    result image and the engine's work buffer."""
    esz = torch.empty((), dtype=dtype).element_size()
    return (proj.numel() * proj.element_size() + coeffs.grid.n_cells * esz
            + coeffs.workspace_bytes(dtype))


class Admission:
    """Admission by device-memory footprint, first come first served within
    each lane.  The budget covers the resident coefficient sets (`reserve`,
    held until the server ends) and the admitted requests.  A queued request
    is admitted when it fits what the budget has left and its lane has a
    free slot.  A request waiting for a slot holds back only later requests
    of its own lane.  A request waiting for memory may be passed by later
    ones that fit (`skip_ahead`) until it has waited `max_wait` seconds; from
    then on nothing behind it is admitted, so the memory it needs drains
    free.  A request larger than the budget left after the resident sets is
    rejected."""

    def __init__(self, budget: int, skip_ahead: bool = True, max_wait: float = 1.0):
        self.budget = budget
        self.skip_ahead = skip_ahead
        self.max_wait = max_wait
        self.in_use = 0
        self.resident = 0

    def reserve(self, nbytes: int):
        """Charges a resident coefficient set to the budget for good."""
        self.resident += nbytes
        self.in_use += nbytes

    def pick(self, queue, now: float, free_slots) -> tuple:
        """Returns (admitted, rejected) lists; removes both from `queue`.
        `free_slots` maps lane -> free slot count, updated in place."""
        admitted, rejected, keep = [], [], []
        held_lanes = set()     # lanes whose earlier request is still queued
        blocked = False        # a starved request holds back everything after it
        for r in queue:
            if r.footprint > self.budget - self.resident:
                rejected.append(r)
                continue
            if blocked or r.lane in held_lanes:
                keep.append(r)
                continue
            slot = free_slots.get(r.lane, 0) > 0
            mem = self.in_use + r.footprint <= self.budget
            if slot and mem:
                admitted.append(r)
                self.in_use += r.footprint
                free_slots[r.lane] -= 1
                continue
            keep.append(r)
            held_lanes.add(r.lane)
            if not mem and (not self.skip_ahead or now - r.arrival > self.max_wait):
                blocked = True
        queue.clear()
        queue.extend(keep)
        return admitted, rejected

    def release(self, r: Request):
        self.in_use -= r.footprint


def percentile(xs, q: float) -> float:
    """Nearest-rank percentile (q in [0, 100]) of a non-empty list."""
    s = sorted(xs)
    i = max(0, min(len(s) - 1, int(-(-q * len(s) // 100)) - 1))
    return s[i]


class _Lane:
    def __init__(self, max_slots, dtype, device, stream=None):
        self.engine = Engine(max_slots, dtype)
        self.stream = stream if stream is not None else torch.cuda.Stream(device=device)
        self.max_slots = max_slots
        self.slots = {}        # slot -> Request
        self.gstep = 0
        self.inflight = deque()   # (event, [requests finished by that call])

    def next_steps(self, cap: int) -> int:
        rem = min(r.steps - (self.gstep - r.offset) for r in self.slots.values())
        return max(1, min(rem, cap))


class Server:
    """Continuous-batching server.  `geometry(key) -> (Grid, Coeffs)`;
    `lane_of(key) -> int`; `budget` bytes for the resident coefficient sets
    and the admitted requests together; at most
    `max_slots` requests per lane (an int, or a dict lane -> count with 64
    for lanes it does not name); each step call advances a lane by at most
    `steps_per_call` steps; at most `depth` calls per lane are in flight.
    `shared_stream` (default): every lane issues its step calls on one
    stream, so calls of different lanes run one after another instead of
    side by side (measured faster on the serving workload: overlapping
    launches slow the largest requests more than they gain)."""

    def __init__(self, geometry, budget: int, lane_of=lambda key: key[0], max_slots=64,
                 steps_per_call: int = 512, depth: int = 2, dtype=torch.float32, device="cuda:0",
                 skip_ahead: bool = True, max_wait: float = 1.0, keep_results: bool = True,
                 shared_stream: bool = True):
        self.cache = GeometryCache(geometry)
        self.lane_of = lane_of
        self.admission = Admission(budget, skip_ahead, max_wait)
        self.max_slots = max_slots
        self.steps_per_call = steps_per_call
        self.depth = depth
        self.dtype = dtype
        self.device = torch.device(device)
        self.keep_results = keep_results
        self.shared = torch.cuda.Stream(device=self.device) if shared_stream else None
        self.lanes = {}
        self.queue = deque()
        self.rejected = []
        self.done = []

    def _lane(self, lid):
        if lid not in self.lanes:
            ms = self.max_slots.get(lid, 64) if isinstance(self.max_slots, dict) else self.max_slots
            self.lanes[lid] = _Lane(ms, self.dtype, self.device, self.shared)
        return self.lanes[lid]

    def prepare(self, r: Request):
        fresh = r.key not in self.cache.entries
        _, co = self.cache.get(r.key)
        if fresh:    # a new resident coefficient set (its work space) counts in the budget
            self.admission.reserve(co.device_bytes)
        r.lane = self.lane_of(r.key)
        self._lane(r.lane)
        r.footprint = footprint_bytes(co, r.proj, self.dtype)
        ku, kv = co.lattice
        r.steps = r.sweeps * co.n_views * ku * kv

    def cancel(self, r: Request) -> bool:
        """Drops a request that has not been admitted (not yet arrived, or
        queued); admitted ones run to the end.  Returns whether it was
        dropped."""
        if r.t_admit is not None or r.t_done is not None:
            return False
        if r in self.queue:
            self.queue.remove(r)
        r.cancelled = True
        return True

    def _admit(self, r: Request, now: float):
        lane = self.lanes[r.lane]
        grid, co = self.cache.get(r.key)
        with torch.cuda.stream(lane.stream):
            r.image = torch.ones(grid.n_cells, dtype=self.dtype, device=self.device)
            r.work = torch.empty(co.workspace_bytes(self.dtype), dtype=torch.uint8, device=self.device)
        r.slot = lane.engine.admit(co, r.proj, r.image, r.sweeps, r.beta, work=r.work, stream=lane.stream)
        r.offset = lane.gstep
        r.t_admit = now
        lane.slots[r.slot] = r

    def _retire(self, lane, now_fn, block: bool) -> bool:
        progressed = False
        while lane.inflight and (block or lane.inflight[0][0].query()):
            ev, reqs = lane.inflight.popleft()
            ev.synchronize()
            t = now_fn()
            for r in reqs:
                r.t_done = t
                r.work = None
                self.admission.release(r)
                if not self.keep_results:
                    r.image = None
                self.done.append(r)
            progressed = True
            block = False
        return progressed

    def run(self, requests, progress=None, progress_every: float = 10.0, on_tick=None):
        """Serves `requests` (arrival times relative to the start of this
        call) until all are done, rejected or cancelled.  `progress(stats)`
        is called every `progress_every` seconds, `on_tick(server)` once per
        loop iteration.  Returns stats."""
        for r in requests:
            self.prepare(r)
        torch.cuda.synchronize(self.device)
        pending = deque(sorted(requests, key=lambda r: r.arrival))
        t0 = time.perf_counter()
        now = lambda: time.perf_counter() - t0   # noqa: E731
        next_report = progress_every
        while pending or self.queue or any(l.slots or l.inflight for l in self.lanes.values()):
            if on_tick:
                on_tick(self)
            t = now()
            while pending and pending[0].arrival <= t:
                r = pending.popleft()
                if not r.cancelled:
                    self.queue.append(r)
            if self.queue:
                free = {lid: l.max_slots - len(l.slots) for lid, l in self.lanes.items()}
                adm, rej = self.admission.pick(self.queue, t, free)
                self.rejected.extend(rej)
                for r in adm:
                    self._admit(r, t)
            issued = False
            for lane in self.lanes.values():
                if lane.slots and len(lane.inflight) < self.depth:
                    n = lane.next_steps(self.steps_per_call)
                    fin = lane.engine.step(n, stream=lane.stream)
                    lane.gstep += n
                    ev = torch.cuda.Event()
                    ev.record(lane.stream)
                    lane.inflight.append((ev, [lane.slots.pop(s) for s in fin]))
                    issued = True
            retired = False
            for lane in self.lanes.values():
                retired |= self._retire(lane, now, block=False)
            if not issued and not retired:
                busy = [l for l in self.lanes.values() if l.inflight]
                if len(busy) == 1 and not self.queue:
                    # one lane at its depth: wait for its oldest call
                    self._retire(busy[0], now, block=True)
                elif not busy and pending and not self.queue:
                    time.sleep(max(0.0, min(pending[0].arrival - now(), 0.01)))
                else:
                    time.sleep(2e-5)
            if progress and now() >= next_report:
                progress(self.stats(now()))
                next_report += progress_every
        return self.stats(now())

    def stats(self, wall: float) -> dict:
        done = [r for r in self.done]
        lat = [r.t_done - r.arrival for r in done]
        svc = [r.t_done - r.t_admit for r in done]
        out = {"completed": len(done), "rejected": len(self.rejected), "wall_s": wall,
               "queued": len(self.queue),
               "active": sum(len(l.slots) for l in self.lanes.values())}
        if done:
            first = min(r.arrival for r in done)
            last = max(r.t_done for r in done)
            out.update({"p50_s": percentile(lat, 50), "p99_s": percentile(lat, 99),
                        "mean_s": sum(lat) / len(lat),
                        "admit_to_done_p50_s": percentile(svc, 50),
                        "admit_to_done_p99_s": percentile(svc, 99),
                        "req_per_s": len(done) / max(last - first, 1e-9)})
            by = {}
            for r in done:
                by.setdefault(r.key, []).append(r.t_done - r.arrival)
            out["p50_by_key_s"] = {f"{k[0]}x{k[1]}": percentile(v, 50) for k, v in sorted(by.items())}
        return out

    def close(self):
        for lane in self.lanes.values():
            lane.stream.synchronize()
            lane.engine.close()
        self.lanes.clear()


def serve_fifo(geometry, requests, dtype=torch.float32, device="cuda:0", keep_results: bool = True,
               progress=None, progress_every: float = 10.0):
    """Baseline: one request at a time in arrival order through ``mart``,
    with the same geometry cache.  Returns stats of the same form."""
    cache = GeometryCache(geometry)
    dev = torch.device(device)
    for r in requests:
        cache.get(r.key)
    torch.cuda.synchronize(dev)
    order = sorted(requests, key=lambda r: r.arrival)
    t0 = time.perf_counter()
    now = lambda: time.perf_counter() - t0   # noqa: E731
    next_report = progress_every
    done = []
    for r in order:
        wait = r.arrival - now()
        if wait > 0:
            time.sleep(wait)
        grid, co = cache.get(r.key)
        r.t_admit = now()
        r.image = torch.ones(grid.n_cells, dtype=dtype, device=dev)
        mart(co, r.proj, r.image, r.sweeps, r.beta)
        torch.cuda.synchronize(dev)
        r.t_done = now()
        if not keep_results:
            r.image = None
        done.append(r)
        if progress and now() >= next_report:
            progress({"completed": len(done), "wall_s": now()})
            next_report += progress_every
    lat = [r.t_done - r.arrival for r in done]
    wall = now()
    out = {"completed": len(done), "rejected": 0, "wall_s": wall}
    if done:
        out.update({"p50_s": percentile(lat, 50), "p99_s": percentile(lat, 99), "mean_s": sum(lat) / len(lat),
                    "req_per_s": len(done) / max(max(r.t_done for r in done) - min(r.arrival for r in done),
                                                 1e-9)})
        # device time per geometry: one request at a time, so admission to
        # completion is that request's whole service time
        svc = {}
        for r in done:
            svc[r.key] = svc.get(r.key, 0.0) + (r.t_done - r.t_admit)
        out["service_s_by_key"] = {f"{k[0]}x{k[1]}": v for k, v in sorted(svc.items())}
    return out
