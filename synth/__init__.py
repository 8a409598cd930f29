"""Seeded synthetic inputs shared by the oracle-side tests and the HIP path.

Holds none of the sampler's arithmetic: it only draws a Gaussian random field
with a chosen P(k), a survey response (angular mask times radial selection)
and mock galaxy counts from the linear data model, all from numpy's seeded
generators.  Both sides of every parity test receive exactly these arrays.
"""
from .mock import (CONFIGS, MockConfig, fiducial_shape, make_mock, mask_and_selection,  # noqa: F401
                   shell_centres)
