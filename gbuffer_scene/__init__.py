"""Seeded synthetic G-buffers for the visibility-bitmask gather.

This package only *produces inputs*: a procedural world (ground plane, axis-aligned
boxes, thin slabs, one directional light) ray-cast analytically into a single-layer
G-buffer (linear view depth, view-space normals, direct-light radiance with shadows),
plus a few analytic scenes (planes, a crease) used by the pins.  It holds none of the
method's arithmetic; the oracle and the HIP path both consume its arrays.

The paper's own workloads use the Amazon Lumberyard Bistro scene (Section 4.1), which is
not available; these seeded procedural scenes stand in for it.
"""
from .procedural import (
    CameraSpec,
    Scene,
    make_camera,
    make_scene,
    render_gbuffer,
    plane_gbuffer,
    crease_gbuffer,
    workload,
    WORKLOADS,
    mixed_batch,
    small_batch,
    request_stream,
    render_pool,
    as_format,
    BATCH_RESOLUTIONS,
    SERVE_RESOLUTIONS,
)

__all__ = [
    "CameraSpec",
    "Scene",
    "make_camera",
    "make_scene",
    "render_gbuffer",
    "plane_gbuffer",
    "crease_gbuffer",
    "workload",
    "WORKLOADS",
    "mixed_batch",
    "small_batch",
    "request_stream",
    "render_pool",
    "as_format",
    "BATCH_RESOLUTIONS",
    "SERVE_RESOLUTIONS",
]
