"""Seeded synthetic map-making problems shared by the oracle and the GPU path.

This package draws inputs only: scan geometries, polarisation angles, sky maps, noise
realisations and the inverse-noise band derived from the known noise spectrum.  It holds none of
the solver's arithmetic (no pointing products, no Toeplitz products, no preconditioner, no CG).
"""

from .problems import (  # noqa: F401
    MASTER_SEED,
    Problem,
    make_raster,
    make_ground,
    make_satellite,
    make_random_small,
    make_templates,
    make_config,
    serving_pool,
    serving_trace,
    serving_views,
    GeometryView,
    inverse_noise_band,
    noise_psd,
    CONFIGS,
)
