"""Seeded synthetic hyperspectral cubes.

This module only draws random numbers and arranges them into cubes. It holds
none of the PCA arithmetic (no means, covariances, rotations or projections),
so both the FP64 oracle's tests and the GPU path's tests/benchmarks can use it
without sharing any of the method with each other.
"""

from .cubes import (  # noqa: F401
    CONFIGS,
    batch_shapes,
    endmember_spectra,
    haar_orthogonal,
    make_batch,
    make_config,
    mixture_cube,
    planted_cube,
    planted_spectrum,
    radiance_cube_u16,
    SWEEP_SHAPES,
    snr_mixture_cube,
    random_symmetric,
)
