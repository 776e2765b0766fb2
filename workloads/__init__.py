"""Seeded synthetic initial states (density, velocity, temperature fields).

This package holds only input generation: cell-centre coordinates, spherical
harmonic synthesis and random draws.  It contains none of the vLBM update's
arithmetic, so both the HIP path and the CPU oracle can be fed from it.
"""
from .fields import *  # noqa: F401,F403
