"""Seeded synthetic wide-band inputs (PSF cube, sky cube, dirty cube).

This package only draws inputs.  It holds none of the reconstruction's
arithmetic, and it is shared by the GPU path's tests and benchmark and by the
CPU oracle, which never import each other.
"""
from .generator import Instance, make_instance, band_frequencies
from .configs import CONFIGS, SolverParams, get_config

__all__ = ["Instance", "make_instance", "band_frequencies", "CONFIGS",
           "SolverParams", "get_config"]
