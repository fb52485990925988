"""Seeded synthetic workloads: array / transmit / grid parameter sets and
random draws (scatterer phantoms, reflectivity maps, noise, parameter
samples, initial weights).

This package holds no arithmetic of the method: no delays, pulses,
beamforming or convolutions.  Both the CPU oracle (through the tests) and the
device path (through the tests and the benchmark) take their inputs from
here, so the two sides always see identical inputs.
"""
from .configs import Setup, CONFIGS, config, field_grid  # noqa: F401
from . import generators  # noqa: F401
