"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This package produces *inputs only*: antenna layouts, earth-rotation uvw tracks,
frequencies, sky images, noise realisations, weights and prior power spectra.  It
contains none of the response operator's arithmetic (no gridding, no DFT, no PSF,
no likelihood), so the FP64 oracle and the HIP path can both consume it without
sharing any of the method's code.

The paper's datasets (VLA Cygnus A, MeerKAT ESO 137-006) are not available; the
generators below reproduce their *shapes* (row counts, channel counts, image sizes,
pixel sizes, w-extent) as listed in the paper's observation tables, Sec. 4.
"""

from .layouts import (  # noqa: F401
    C_LIGHT,
    enu_to_xyz,
    earth_rotation_uvw,
    layout_uniform_disc,
    layout_vla_y,
    layout_meerkat_like,
    n_baselines,
)
from .skies import (  # noqa: F401
    power_spectrum,
    inv_power_half,
    correlated_field,
    point_sources,
    gaussian_blob,
    complex_noise,
)
from .configs import (  # noqa: F401
    BASE_SEED,
    Observation,
    make_config,
    config_rng,
)
