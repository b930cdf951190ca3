"""Seeded synthetic inputs shared by the tests, the bench and the smoke check.

This module draws specimens and noise only; it holds none of the imaging
method's arithmetic (no pupils, transfer functions, FFT models or solves), so
both the oracle and the GPU path can be fed from it without sharing code.
Every generator takes an explicit seed and returns float32 arrays (the values
both sides receive).
"""

from .objects import (  # noqa: F401
    beads, ellipsoids, fibres, fibres_on_device, thin_cells, poisson_gaussian, gaussian_noise,
    plane_waves,
)
