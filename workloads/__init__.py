"""Seeded synthetic workloads shared by the HIP path and the FP64 oracle.

This package only produces input data (geometry, materials, sensor and
source descriptions, wavelength grids).  It contains none of the rendering
arithmetic: no propagation law, no scattering kernel, no sampling.
"""

from .scenes import (  # noqa: F401
    Scene,
    Sensor,
    Source,
    Material,
    Workload,
    wavelength_bins,
    tiny_grating,
    parallel_mirror,
    grating_relay,
    split_mirror,
    rough_box,
    terrain_scene,
    mid_terrain,
    large_scene,
    coherent_case,
    surrogate_query_box,
)
