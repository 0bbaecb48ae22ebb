"""The serving workload: a seeded Poisson stream of cone-beam requests.

Each request is one cone-beam USCG reconstruction (Nr = Nz rings and slices,
detector 2Nr x 2Nr, p views over a full turn, sector multiple p, a random
ten-ellipsoid phantom seeded 5000 + k) with a sweep count drawn uniformly.
Draw order from numpy's PCG64 generator: for each request, the exponential
inter-arrival gap, then the ring-count index, the view-count index and the
sweep count.  Arrivals stop at the first one past the duration.
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .workloads import Workload, serve_request


@dataclass(frozen=True)
class ServeItem:
    k: int            # request id (phantom seed 5000 + k)
    arrival: float    # seconds from the start of the stream
    n_rings: int
    n_views: int
    sweeps: int

    @property
    def key(self) -> tuple:
        """Geometry key: requests with equal keys share grid and coefficients."""
        return (self.n_rings, self.n_views)

    def workload(self) -> Workload:
        return serve_request(self.k, self.n_rings, self.n_views, self.sweeps)


def serve_trace(rate: float = 20.0, duration: float = 120.0, seed: int = 5,
                rings=(64, 128, 256), views=(8, 16, 32), sweeps=(10, 20)) -> list:
    """Poisson arrivals at `rate` per second over `duration` seconds."""
    rng = np.random.default_rng(seed)
    out, t, k = [], 0.0, 0
    while True:
        t += float(rng.exponential(1.0 / rate))
        if t >= duration:
            return out
        nr = int(rings[int(rng.integers(len(rings)))])
        p = int(views[int(rng.integers(len(views)))])
        sw = int(rng.integers(sweeps[0], sweeps[1] + 1))
        out.append(ServeItem(k, t, nr, p, sw))
        k += 1
