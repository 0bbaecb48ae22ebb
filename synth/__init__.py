"""Seeded synthetic inputs shared by the oracle tests and the GPU path.

This package only describes workloads (grid and scan parameters) and draws
phantoms and their analytic projections.  It holds none of the reconstruction
method's arithmetic (no grid tracing, no MART): both the CPU oracle and the
HIP library consume the arrays it writes, so it must not depend on either.
"""

from .workloads import (  # noqa: F401
    Workload, WORKLOADS, get, small_cone, cone, parallel, batch2d_members, serve_request, paper_fan, paper_cone, paper_specimen,
)
from .phantoms import (  # noqa: F401
    draw_phantom,
    scan_rays,
    project,
    add_noise,
    make_projections,
    phantom_value,
    make_projections_torch,
    scan_rays_torch,
)
from .serving import ServeItem, serve_trace  # noqa: F401
