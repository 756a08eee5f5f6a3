"""Seeded synthetic inputs for the multi-peak Bragg ptychography (MPBP) workloads.

This package is shared by the GPU library's callers (bench, binding tests) and by the
CPU oracle's tests.  It holds only input generation: workload descriptions, Bragg
vectors, exit-beam shear directions, raster-scan parameters, the probe, the
displacement / amplitude fields and the random streams.  It holds none of the method's
arithmetic (no object build, projection, Fourier transform, loss or gradient); the
measured intensities are produced by whichever forward model the caller owns.
"""
from .configs import CONFIG_NAMES, get_config
from .inputs import (
    Problem,
    make_problem,
    make_fields,
    photon_rng,
    poisson_counts,
    speckle_counts,
    crop_problem,
    band_problem,
    unwrap_field,
    lattice_jump,
    incident_probe_3d,
)

__all__ = [
    "CONFIG_NAMES",
    "get_config",
    "Problem",
    "make_problem",
    "make_fields",
    "photon_rng",
    "poisson_counts",
    "speckle_counts",
    "crop_problem",
    "band_problem",
]
