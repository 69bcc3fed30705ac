"""Workload definitions for the synthetic scenes.

The paper measures a private 4096 x 4096 complex float32 point-target
simulation with 5 targets and 20 dB additive Gaussian noise (Sec. V.A).  The
simulator and its parameters are not published, so the dictionaries below are
our stand-ins; every value that the paper leaves open carries the reading we
took for it.

A scene dictionary carries two kinds of keys:

* processing parameters, shared by both the oracle and the HIP path:
  ``Nr, Na, range_len, range_tbp, az_model, az_len, az_tbp, lam, v, r_near,
  rcmc_taps, rcmc_beta``;
* simulation-only keys: ``n_targets, spacing, sigma2, seed, exposure``.

Units are normalised: one range cell = 1, one pulse (PRI) = 1, so chirp rates
are in cycles/sample^2, ``v`` in cells/pulse and ``lam`` in cells.
"""
from __future__ import annotations

import copy
import math

import numpy as np

# Per-sample noise variance for "20 dB" relative to a unit-amplitude target.
SIGMA2_20DB = 10.0 ** (-20.0 / 10.0)

_C1 = dict(
    name="c1_256_lfm",
    Nr=256, Na=256,
    range_len=64, range_tbp=32.0,          # fs/B = 2 (64 samples, TBP 32)
    az_model="lfm", az_len=64, az_tbp=32.0,
    lam=0.0, v=0.0, r_near=0.0,
    rcmc_taps=0, rcmc_beta=2.5,
    n_targets=5, spacing=16, sigma2=SIGMA2_20DB, seed=1, exposure=0,
)

# Normalised geometry giving a 1024-pulse aperture with at most 8 cells of
# hyperbolic range migration at near range: V = sqrt(2) cells/pulse,
# lambda = 5/32 cells, near range 32768 cells.
_C2 = dict(
    name="c2_4096_hyperbolic",
    Nr=4096, Na=4096,
    range_len=512, range_tbp=200.0,
    az_model="hyperbolic", az_len=1024, az_tbp=0.0,
    lam=5.0 / 32.0, v=math.sqrt(2.0), r_near=32768.0,
    rcmc_taps=8, rcmc_beta=2.5,
    n_targets=5, spacing=64, sigma2=SIGMA2_20DB, seed=2, exposure=1024,
)

CONFIGS = {
    "c1": _C1,
    "c2": _C2,
    # The split-precision run processes exactly the c2 scene.
    "c3": dict(_C2, name="c3_4096_hyperbolic_split"),
}


def config(name: str, **overrides) -> dict:
    """Return a copy of a named config with keys overridden."""
    d = copy.deepcopy(CONFIGS[name])
    d.update(overrides)
    return d


def lfm_scene(Nr: int, Na: int, n_targets: int, seed: int, name: str) -> dict:
    """An LFM-azimuth scene whose chirps span 1/8 of each dimension, TBP = L/2."""
    Lr, La = Nr // 8, Na // 8
    return dict(
        name=name, Nr=Nr, Na=Na,
        range_len=Lr, range_tbp=Lr / 2.0,
        az_model="lfm", az_len=La, az_tbp=La / 2.0,
        lam=0.0, v=0.0, r_near=0.0, rcmc_taps=0, rcmc_beta=2.5,
        n_targets=n_targets, spacing=64, sigma2=SIGMA2_20DB, seed=seed,
        exposure=0,
    )


def batch_configs(seed: int = 4, n: int = 64,
                  nr_choices=(1024, 2048, 4096, 8192, 16384),
                  na_choices=(512, 1024, 2048, 4096, 8192)) -> list[dict]:
    """The batched workload: ``n`` scenes of uneven size.

    Draw order from PCG64(seed): range sizes, azimuth sizes, target counts
    (3..9), then one 63-bit seed per scene.  Each scene is then simulated from
    its own seed, so scene i can be generated without generating 0..i-1.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    nr = rng.choice(np.asarray(nr_choices), size=n)
    na = rng.choice(np.asarray(na_choices), size=n)
    nt = rng.integers(3, 10, size=n)
    seeds = rng.integers(0, 2**63 - 1, size=n, dtype=np.int64)
    return [lfm_scene(int(nr[i]), int(na[i]), int(nt[i]), int(seeds[i]),
                       f"batch{i:02d}_{int(na[i])}x{int(nr[i])}")
            for i in range(n)]


def serve_pool_configs(seed: int = 5, n: int = 32,
                       nr_choices=(1024, 2048, 4096, 8192, 16384),
                       na_choices=(1024, 2048, 4096, 8192)) -> list[dict]:
    """The pool of pre-generated scenes that served requests draw from."""
    rng = np.random.Generator(np.random.PCG64(seed))
    nr = rng.choice(np.asarray(nr_choices), size=n)
    na = rng.choice(np.asarray(na_choices), size=n)
    seeds = rng.integers(0, 2**63 - 1, size=n, dtype=np.int64)
    return [lfm_scene(int(nr[i]), int(na[i]), 5, int(seeds[i]),
                       f"pool{i:02d}_{int(na[i])}x{int(nr[i])}")
            for i in range(n)]


def poisson_arrivals(seed: int, n: int, rate_hz: float,
                     pool_size: int) -> tuple[np.ndarray, np.ndarray]:
    """Arrival times (seconds from 0) and pool indices for ``n`` requests."""
    rng = np.random.Generator(np.random.PCG64(seed))
    gaps = rng.exponential(1.0 / rate_hz, size=n)
    which = rng.integers(0, pool_size, size=n)
    return np.cumsum(gaps), which
