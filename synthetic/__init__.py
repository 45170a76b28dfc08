"""Seeded synthetic inputs for RM synthesis: frequency bands, channel weights,
Faraday-depth grids and Stokes Q/U cubes.

This package is shared by the FP64 oracle side and the GPU side.  It holds
only the *forward* model of the sky (Faraday-thin screens and Burn slabs,
eqs. (1), (3), (4) of the paper) and the noise; it holds none of the
Faraday-depth transform itself.
"""
from .cubes import (  # noqa: F401
    C_LIGHT,
    Workload,
    WORKLOADS,
    band_lambda2,
    phi_grid,
    flag_channels,
    thin_spectrum,
    slab_spectrum,
    make_cube,
    make_small_cube,
    noise_sigma_F,
    stratified_subsample,
    LOS_MAJOR,
    FREQ_MAJOR,
)
