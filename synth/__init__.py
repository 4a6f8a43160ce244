"""Seeded synthetic workloads shaped like the paper's inputs.

This package only *generates inputs*: template meshes, vertex colours, cameras,
random draws, a ground-truth deformation field and the target images rendered
from it.  It holds none of the solver's arithmetic (no embedded deformation,
no residuals, no Gauss-Newton) so that both the FP64 oracle and the HIP path
can take their inputs from it without sharing any code with each other.

The paper captures real video (540x960, template of about 5000 vertices,
Sec. 3.1 and Sec. 5); that data is not available, so these generators stand
in for it with the same shapes.
"""
from .meshes import icosphere, fibonacci_ellipsoid, ellipsoid_icosphere  # noqa: F401
from .render import render_targets  # noqa: F401
from .workloads import Camera, make_nonrigid_frame, CONFIGS, batch_specs, make_batch  # noqa: F401
