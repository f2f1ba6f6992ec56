"""Seeded synthetic inputs (fields and particle positions).

These generators stand in for the paper's DNS velocity fields and particle sets
(Sec. 4: N = 2048/4096 grids, 1e6 .. 2.2e9 tracers), which are not available.
They hold none of the interpolation method's arithmetic; both the GPU library's
tests and the oracle consume their output.
"""
from .fields import fourier_mode_field, fourier_mode_eval, spectral_field, single_mode_field
from .particles import uniform_particles

__all__ = ["fourier_mode_field", "fourier_mode_eval", "spectral_field", "single_mode_field",
           "uniform_particles"]
