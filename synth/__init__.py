"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the bench.

This package holds only input recipes (phantoms, their analytic line integrals,
noise, angle sets and workload descriptions). It contains none of the
reconstruction method's arithmetic and imports neither ``oracle`` nor the HIP
package.
"""
from .phantoms import (  # noqa: F401
    Workload,
    WORKLOADS,
    detector_bins_for,
    uniform_angles,
    ellipse_params,
    ellipsoid_params,
    rasterize_ellipses,
    ellipse_sinogram,
    ellipsoid_volume,
    ellipsoid_sinogram,
    gaussian_blob,
    gaussian_blob_sinogram,
    textured_slice,
    textured_batch,
    uneven_problems,
    add_noise,
    make_problem,
)
