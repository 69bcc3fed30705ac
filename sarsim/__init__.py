"""Seeded synthetic SAR echo scenes: the single source of input for both the
HIP path and the FP64 oracle.

This package holds scene *models* (point targets, chirps, geometry, noise) and
nothing of the Range Doppler Algorithm itself: no FFT, no matched filter, no
RCMC.  Both sides receive the same complex64 array and the same parameter
dictionary.
"""
from .configs import (CONFIGS, config, batch_configs, lfm_scene, poisson_arrivals,
                      serve_pool_configs)
from .scene import Scene, simulate, simulate_many

__all__ = ["CONFIGS", "config", "batch_configs", "lfm_scene", "poisson_arrivals",
           "serve_pool_configs", "Scene", "simulate", "simulate_many"]
