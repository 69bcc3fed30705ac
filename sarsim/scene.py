"""Point-target echo simulator (numpy, FP64 signal model, complex64 output).

Scene models (normalised units: range cell = 1, pulse = 1):

* chirp ``c(u) = exp(j*pi*K*u^2)`` on ``u in [-L/2, L/2)``, ``K = TBP / L^2``,
  zero outside its support;
* LFM azimuth (zero migration):
  ``s[m][n] = sum_k exp(j*phi_k) * c_r(n - n_k) * conj(c_a(m - m_k)) + w``;
* hyperbolic azimuth: ``R_k(m) = sqrt(R0_k^2 + V^2 (m - m_k)^2)``,
  ``R0_k = r_near + n_k`` and
  ``s[m][n] = sum_k exp(j*phi_k) exp(-j*4*pi*R_k(m)/lam)
  * c_r(n - (R_k(m) - r_near)) * [-E/2 <= m - m_k < E/2] + w``,
  with the range chirp evaluated analytically at the fractional delay;
* noise ``w``: circular complex Gaussian, variance ``sigma2``.

Random draws come from ``numpy.random.Generator(PCG64(seed))`` in the order:
target cells, target phases, noise real parts, noise imaginary parts.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

_MAX_TRIES = 200000


@dataclasses.dataclass
class Scene:
    params: dict                 # the config dictionary the scene came from
    raw: np.ndarray              # complex64, shape (Na, Nr), C-contiguous
    targets: list                # [{"m": int, "n": int, "phase": float}]

    @property
    def shape(self):
        return self.raw.shape


def _place_targets(rng, count, m_lo, m_hi, n_lo, n_hi, spacing):
    """Integer cells uniform on [m_lo, m_hi] x [n_lo, n_hi] (inclusive); a
    candidate closer than ``spacing`` rows or ``spacing`` columns to an
    accepted target is rejected.  The spacing shrinks to fit when the span
    cannot hold ``count`` targets at the requested spacing."""
    span = min(m_hi - m_lo, n_hi - n_lo)
    g = min(spacing, max(1, span // (2 * max(count, 1))))
    cells = []
    tries = 0
    while len(cells) < count:
        tries += 1
        if tries > _MAX_TRIES:
            raise RuntimeError("cannot place targets with the requested spacing")
        m = int(rng.integers(m_lo, m_hi + 1))
        n = int(rng.integers(n_lo, n_hi + 1))
        if all(abs(m - cm) >= g and abs(n - cn) >= g for cm, cn in cells):
            cells.append((m, n))
    return cells


def _chirp(u, K):
    return np.exp(1j * math.pi * K * u * u)


def _frac_turns_exp(turns, sign):
    """exp(sign * j * 2*pi * turns) with the argument reduced in FP64 first."""
    f = turns - np.floor(turns)
    return np.exp(sign * 2j * math.pi * f)


def simulate(cfg: dict, noise: bool = True, targets=None) -> Scene:
    """Simulate one scene.  ``targets`` (a list of (m, n) cells) overrides the
    seeded placement; phases are still drawn from the seeded stream."""
    Nr, Na = int(cfg["Nr"]), int(cfg["Na"])
    Lr, La = int(cfg["range_len"]), int(cfg["az_len"])
    Kr = float(cfg["range_tbp"]) / (Lr * Lr)
    rng = np.random.Generator(np.random.PCG64(int(cfg["seed"])))
    count = int(cfg["n_targets"])
    hyper = cfg["az_model"] == "hyperbolic"

    if targets is None:
        if hyper:
            E = int(cfg["exposure"])
            cells = _place_targets(rng, count, E // 2, Na - E // 2,
                                   Lr // 2, Nr - Lr // 2 - 9, cfg["spacing"])
        else:
            cells = _place_targets(rng, count, La // 2, Na - La // 2,
                                   Lr // 2, Nr - Lr // 2, cfg["spacing"])
    else:
        cells = [(int(m), int(n)) for m, n in targets]
        count = len(cells)
    phases = rng.uniform(0.0, 2.0 * math.pi, size=count)

    if noise and cfg["sigma2"] > 0:
        s = math.sqrt(cfg["sigma2"] / 2.0)
        raw = np.empty((Na, Nr), dtype=np.complex64)
        raw.real = rng.standard_normal((Na, Nr), dtype=np.float32) * np.float32(s)
        raw.imag = rng.standard_normal((Na, Nr), dtype=np.float32) * np.float32(s)
    else:
        raw = np.zeros((Na, Nr), dtype=np.complex64)

    tlist = []
    for (m_k, n_k), phi in zip(cells, phases):
        tlist.append({"m": m_k, "n": n_k, "phase": float(phi)})
        amp = np.exp(1j * phi)
        if not hyper:
            Ka = float(cfg["az_tbp"]) / (La * La)
            ua = np.arange(-La // 2, La // 2, dtype=np.float64)
            ur = np.arange(-Lr // 2, Lr // 2, dtype=np.float64)
            blk = amp * np.outer(np.conj(_chirp(ua, Ka)), _chirp(ur, Kr))
            rs = slice(m_k - La // 2, m_k + La // 2)
            cs = slice(n_k - Lr // 2, n_k + Lr // 2)
        else:
            E = int(cfg["exposure"])
            lam, V, r_near = float(cfg["lam"]), float(cfg["v"]), float(cfg["r_near"])
            R0 = r_near + n_k
            dm = np.arange(-E // 2, E // 2, dtype=np.float64)
            R = np.sqrt(R0 * R0 + (V * dm) ** 2)             # (E,)
            delay = R - r_near                                # echo centre cell
            n0 = n_k - Lr // 2
            ncols = Lr + int(math.ceil(delay.max() - n_k)) + 1
            if n0 < 0 or n0 + ncols > Nr:
                raise ValueError("target echo does not fit inside the scene")
            n = n0 + np.arange(ncols, dtype=np.float64)       # (ncols,)
            u = n[None, :] - delay[:, None]                   # (E, ncols)
            inside = (u >= -Lr / 2) & (u < Lr / 2)
            az = amp * _frac_turns_exp(2.0 * R / lam, -1.0)   # exp(-j 4 pi R / lam)
            blk = np.where(inside, az[:, None] * _chirp(u, Kr), 0.0)
            rs = slice(m_k - E // 2, m_k + E // 2)
            cs = slice(n0, n0 + ncols)
        acc = raw[rs, cs].astype(np.complex128) + blk
        raw[rs, cs] = acc.astype(np.complex64)

    return Scene(params=dict(cfg), raw=np.ascontiguousarray(raw), targets=tlist)


def simulate_many(cfgs, workers: int = 8, consume=None):
    """simulate() for many scenes on a thread pool (numpy's generators and
    array arithmetic release the GIL).  Each scene draws from its own seeded
    stream, so the result does not depend on ``workers``.  With ``consume``,
    each scene is passed to consume(index, scene) in order and not kept (at
    most 2 x workers scenes are held at once); else the list is returned."""
    import concurrent.futures as cf
    cfgs = list(cfgs)
    out = []
    window = 2 * max(1, workers)
    with cf.ThreadPoolExecutor(max_workers=max(1, workers)) as ex:
        futs = {i: ex.submit(simulate, cfgs[i]) for i in range(min(window, len(cfgs)))}
        for i in range(len(cfgs)):
            sc = futs.pop(i).result()
            if i + window < len(cfgs):
                futs[i + window] = ex.submit(simulate, cfgs[i + window])
            if consume is None:
                out.append(sc)
            else:
                consume(i, sc)
    return out if consume is None else None
