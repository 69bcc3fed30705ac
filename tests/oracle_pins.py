"""Pins of the FP64 oracle against facts that do not come from the oracle
itself: brute-force definitions, closed forms, invariants, textbook values.

Each ``pin_*`` function raises AssertionError when the oracle disagrees.  The
pins are run as ordinary tests (``test_oracle_pins.py``) and again against
copies of the oracle with planted mistakes (``test_oracle_mutations.py``),
which must each be caught by at least one pin.
"""
from __future__ import annotations

import math
import os

import numpy as np

from oracle import oracle as O

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def _cplx(rng, n):
    return rng.standard_normal(n) + 1j * rng.standard_normal(n)


def _rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / max(np.linalg.norm(np.ravel(b)), 1e-300))


def _golden(name):
    out = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                k, v = line.split()
                out[k] = float(v)
    return out


# --------------------------------------------------------------------------
# FFT (forward exp(-j), unnormalised; inverse = (1/N) conj(FFT(conj x)))
# --------------------------------------------------------------------------

def pin_fft_bruteforce():
    """O(N^2) DFT straight from its definition, N = 1 .. 64, both directions."""
    rng = _rng(11)
    for n in (1, 2, 4, 8, 16, 32, 64):
        x = _cplx(rng, n)
        k = np.arange(n)
        E = np.exp(-2j * np.pi * np.outer(k, k) / n)
        X = E @ x
        assert _rel(O.fft(x), X) < 1e-12, n
        Einv = np.exp(+2j * np.pi * np.outer(k, k) / n) / n
        assert _rel(O.ifft(X), Einv @ X) < 1e-12, n


def pin_fft_single_bins_longdouble():
    """Single bins of a 16384-point FFT against long-double direct sums."""
    rng = _rng(12)
    n = 16384
    x = _cplx(rng, n)
    X = O.fft(x)
    xr = x.real.astype(np.longdouble)
    xi = x.imag.astype(np.longdouble)
    idx = np.arange(n, dtype=np.int64)
    scale = math.sqrt(n) * float(np.sqrt(np.mean(np.abs(x) ** 2)))
    for k in (0, 1, 7, 4095, 8192, 12345, 16383):
        ang = (np.longdouble(-2) * np.longdouble(np.pi)
               * ((k * idx) % n).astype(np.longdouble) / np.longdouble(n))
        c, s = np.cos(ang), np.sin(ang)
        re = np.sum(xr * c - xi * s)
        im = np.sum(xr * s + xi * c)
        err = abs(complex(float(re), float(im)) - X[k]) / scale
        assert err < 1e-12, (k, err)


def pin_fft_parseval():
    rng = _rng(13)
    for n in (256, 4096, 16384):
        x = _cplx(rng, n)
        X = O.fft(x)
        e1 = np.sum(np.abs(x) ** 2)
        e2 = np.sum(np.abs(X) ** 2) / n
        assert abs(e1 - e2) / e1 < 1e-12, n


def pin_fft_impulse_and_shift():
    """delta[n - n0] -> exp(-2 pi j k n0 / N); circular shift theorem."""
    n = 1024
    k = np.arange(n)
    for n0 in (0, 1, 37, 511, 1023):
        x = np.zeros(n, complex)
        x[n0] = 1.0
        ref = np.exp(-2j * np.pi * ((k * n0) % n) / n)
        assert np.max(np.abs(O.fft(x) - ref)) < 1e-12, n0
    rng = _rng(14)
    x = _cplx(rng, n)
    X = O.fft(x)
    for s in (1, 100, 1000):
        Xs = O.fft(np.roll(x, s))
        assert _rel(Xs, X * np.exp(-2j * np.pi * ((k * s) % n) / n)) < 1e-12, s


def pin_fft_round_trip():
    rng = _rng(15)
    for n in (2, 64, 4096, 16384):
        x = _cplx(rng, n)
        assert _rel(O.ifft(O.fft(x)), x) < 1e-13, n


def pin_fft_cazac():
    """exp(j pi n^2 / N), N even, has a flat spectrum |X[k]| = sqrt(N)."""
    for n in (64, 4096):
        m = np.arange(n)
        x = np.exp(1j * np.pi * (m * m % (2 * n)) / n)
        X = O.fft(x)
        assert np.max(np.abs(np.abs(X) - math.sqrt(n))) / math.sqrt(n) < 1e-10, n


# --------------------------------------------------------------------------
# Matched filter H = conj(FFT(replica)), line compression IFFT(FFT(x) H)
# --------------------------------------------------------------------------

def _replica(n, length, tbp, sign):
    K = tbp / (length * length)
    h = np.zeros(n, complex)
    for u in range(-(length // 2), length - length // 2):
        h[u % n] = np.exp(sign * 1j * np.pi * K * u * u)
    return h


def _circ_xcorr(x, h):
    """rho[d] = sum_j x[(j + d) mod N] conj(h[j]), by direct summation over
    the support of h (O(N * L))."""
    n = x.size
    supp = np.nonzero(h)[0]
    d = np.arange(n)
    return np.sum(x[(supp[None, :] + d[:, None]) % n] * np.conj(h[supp])[None, :], axis=1)


def pin_cazac_self_compression():
    """A full-length CAZAC replica compresses to exactly N * delta."""
    for n in (64, 1024):
        H = O.matched_filter(n, n, float(n), +1)
        m = np.arange(n)
        x = np.exp(1j * np.pi * (m * m % (2 * n)) / n)
        y = O.compress_rows(x[None, :], H)[0]
        ref = np.zeros(n, complex)
        ref[0] = n
        assert np.max(np.abs(y - ref)) < 1e-9 * n, n


def pin_compression_is_correlation():
    """For L < N the compressed echo equals the direct circular correlation
    with the centred replica; its peak L sits at the echo centre."""
    n = 512
    for length, tbp, sign, d0 in ((64, 32.0, +1, 100), (64, 32.0, -1, 300), (200, 60.0, +1, 7)):
        h = _replica(n, length, tbp, sign)
        x = np.roll(h, d0)
        y = O.compress_rows(x[None, :], O.matched_filter(n, length, tbp, sign))[0]
        ref = _circ_xcorr(x, h)
        assert _rel(y, ref) < 1e-12, (length, sign)
        assert abs(y[d0] - length) < 1e-9 * length
        assert int(np.argmax(np.abs(y))) == d0


def pin_corner_turn_exact():
    rng = _rng(16)
    a = _cplx(rng, 37 * 53).reshape(37, 53)
    b = O.corner_turn(a)
    assert b.shape == (53, 37)
    assert np.array_equal(b, a.T)


# --------------------------------------------------------------------------
# Whole-RDA closed form: noise-free LFM scene (config-1 geometry)
# --------------------------------------------------------------------------

def pin_lfm_closed_form():
    """I[m][n] = sum_k exp(j phi_k) rho_r(n - n_k) rho_a(m - m_k), the two
    autocorrelations by direct sums (no FFT).  Peaks L_r * L_a at the cells."""
    from sarsim import config, simulate
    cfg = config("c1")
    sc = simulate(cfg, noise=False)
    img = O.rda(sc.raw, cfg)
    Nr, Na = cfg["Nr"], cfg["Na"]
    hr = _replica(Nr, cfg["range_len"], cfg["range_tbp"], +1)
    ha = _replica(Na, cfg["az_len"], cfg["az_tbp"], -1)
    rho_r = _circ_xcorr(hr, hr)
    rho_a = _circ_xcorr(ha, ha)
    ref = np.zeros((Na, Nr), complex)
    m = np.arange(Na)
    n = np.arange(Nr)
    for t in sc.targets:
        ref += (np.exp(1j * t["phase"])
                * np.outer(rho_a[(m - t["m"]) % Na], rho_r[(n - t["n"]) % Nr]))
    # the raw scene is stored as complex64: compare at that precision
    assert _rel(img, ref) < 1e-6
    peak = cfg["range_len"] * cfg["az_len"]
    for t in sc.targets:
        sub = np.abs(img[t["m"] - 8:t["m"] + 9, t["n"] - 8:t["n"] + 9])
        i = int(np.argmax(sub))
        assert (i // 17, i % 17) == (8, 8)
        assert abs(abs(img[t["m"], t["n"]]) - peak) < 1e-3 * peak


def pin_noise_gain():
    """Noise-only LFM scene: mean |I|^2 = sigma^2 * L_r * L_a (compression by
    unit-modulus replicas); the estimate's spread is under 1% here."""
    from sarsim import config, simulate
    cfg = config("c1", n_targets=0)
    sc = simulate(cfg)
    img = O.rda(sc.raw, cfg)
    expect = cfg["sigma2"] * cfg["range_len"] * cfg["az_len"]
    got = float(np.mean(np.abs(img) ** 2))
    assert abs(got / expect - 1.0) < 0.04, got / expect


# --------------------------------------------------------------------------
# RCMC: Kaiser-windowed sinc interpolation, exact-geometry azimuth filter
# --------------------------------------------------------------------------

def pin_bessel_i0():
    import scipy.special as sp
    for x, v in _golden("bessel_i0.txt").items():
        assert abs(O.bessel_i0(float(x)) - v) < 1e-14 * v, x
    for x in np.linspace(0.0, 10.0, 41):
        assert abs(O.bessel_i0(x) - sp.i0(x)) < 1e-13 * sp.i0(x), x


def pin_rcmc_weights_structure():
    """x = 0 collapses to the identity; weights sum to 1; mirror symmetry
    w_t(x) = w_{1-t}(1-x) of an even kernel on taps t = -3..4."""
    w0 = O.rcmc_weights(0.0)
    ref = np.zeros(8)
    ref[3] = 1.0
    assert np.max(np.abs(w0 - ref)) < 1e-15
    for x in (0.1, 0.25, 0.5, 0.77, 0.999):
        w = O.rcmc_weights(x)
        assert abs(np.sum(w) - 1.0) < 1e-14
        wm = O.rcmc_weights(1.0 - x)
        assert np.max(np.abs(w - wm[::-1])) < 1e-14, x
    # at x = 1/2 the two centre taps carry equal, largest weight
    w = O.rcmc_weights(0.5)
    assert abs(w[3] - w[4]) < 1e-15 and w[3] == np.max(w)


def pin_rcmc_weights_kaiser_values():
    """The normalised weights themselves, against an independent construction:
    scipy's Kaiser window (its own I0) times numpy's sinc, normalised to unit
    sum.  A symmetric Kaiser window of M = 2*4*D + 1 points spans offsets
    -4 .. 4 in steps of 1/D, so tap t = -3 .. 4 at fractional position x = c/D
    sits on window node (t - x)*D + 4*D.  x = 1/10, 1/4, 1/2 and 3/4 hit the
    nodes exactly; beta = 2.5, half-width 4 (Sec. IV.A step 3, our reading of
    the 8-tap sinc interpolator).  Catches a wrong beta, a wrong window shape
    (e.g. sqrt(1 - |r|)), a missing window or a wrong tap alignment."""
    from scipy.signal.windows import kaiser
    beta, half = 2.5, 4
    taps = np.arange(-3, 5)
    for num, den in ((1, 10), (1, 4), (1, 2), (3, 4)):
        x = num / den
        win = kaiser(2 * half * den + 1, beta, sym=True)
        nodes = (taps * den - num) + half * den
        ref = np.sinc(taps - x) * win[nodes]
        ref = ref / np.sum(ref)
        got = O.rcmc_weights(x)
        assert np.max(np.abs(got - ref)) < 1e-12, (x, np.max(np.abs(got - ref)))


def pin_rcmc_weights_interpolate_tones():
    """A band-limited tone exp(2 pi j f i), |f| <= 0.3, interpolated at
    fractional positions matches the analytic tone within the passband ripple
    of an 8-tap, beta = 2.5 Kaiser-sinc with unit-sum weights (about +-4.5%;
    a sanity band, not an exact pin).  DC is reproduced exactly."""
    for f in (0.0, 0.05, 0.2, 0.3, -0.25):
        for p in (10.0, 10.3, 10.5, 10.93):
            i0 = math.floor(p)
            w = O.rcmc_weights(p - i0)
            taps = np.arange(-3, 5) + i0
            y = np.sum(w * np.exp(2j * np.pi * f * taps))
            tol = 1e-14 if f == 0.0 else 5e-2
            assert abs(y - np.exp(2j * np.pi * f * p)) < tol, (f, p)


def _geometry_D(na, lam, v):
    k = np.arange(na)
    f = np.where(k < na // 2, k, k - na) / na
    x = lam * f / (2 * v)
    return np.sqrt(1 - x * x)


def pin_rcmc_pulse_returns_to_r0():
    """A synthetic range-Doppler pulse sitting at range R0/D(f) in every
    Doppler bin, carrying the phase exp(-j 4 pi R0 D / lam), is moved back to
    its cell and phase-flattened, so it focuses to ~1 at (n_t, m = 0)."""
    nr, na = 64, 64
    lam, v, r_near = 5.0 / 32.0, math.sqrt(2.0), 32768.0
    n_t = 20
    R0 = r_near + n_t
    D = _geometry_D(na, lam, v)
    pos = n_t + R0 * (1.0 / D - 1.0)                      # cell index of R0/D
    i = np.arange(nr)[:, None]
    g = np.sinc(0.5 * (i - pos[None, :]))                 # band-limited pulse
    A = g * np.exp(-1j * 4 * np.pi * R0 * D / lam)[None, :]
    img = O.rcmc_azimuth(A, lam, v, r_near, 8, 2.5)
    assert abs(img[n_t, 0] - 1.0) < 2e-2, img[n_t, 0]
    col = np.abs(img[:, 0])
    assert int(np.argmax(col)) == n_t
    # neighbours follow the pulse shape sinc(0.5 d): ~0.64 at +-1, ~0 at +-2
    assert abs(col[n_t + 1] - 2 / np.pi) < 3e-2 and abs(col[n_t - 1] - 2 / np.pi) < 3e-2
    assert col[n_t + 2] < 3e-2 and col[n_t - 2] < 3e-2
    # the energy of row n_t concentrates in m = 0
    assert np.sum(np.abs(img[n_t, 1:]) ** 2) < 1e-3


def pin_rcmc_disabled_is_phase_only():
    """taps = 0 skips interpolation: the output is IFFT(A * exp(+j 4 pi R0 D/lam))."""
    rng = _rng(17)
    nr, na = 8, 32
    lam, v, r_near = 5.0 / 32.0, math.sqrt(2.0), 32768.0
    A = _cplx(rng, nr * na).reshape(nr, na)
    img = O.rcmc_azimuth(A, lam, v, r_near, 0, 2.5)
    D = _geometry_D(na, lam, v)
    R0 = r_near + np.arange(nr)[:, None]
    Y = A * np.exp(1j * 4 * np.pi * R0 * D[None, :] / lam)
    k = np.arange(na)
    Einv = np.exp(2j * np.pi * np.outer(k, k) / na) / na
    assert _rel(img, Y @ Einv.T) < 1e-9


def pin_hyperbolic_point_target():
    """Noise-free hyperbolic scene, one target: the RDA focuses it exactly at
    its seeded cell, with peak phase phi - pi/4 (the stationary-phase constant
    of a down-chirp) and |peak| = L_r * sqrt(B_a * E) within a few percent."""
    from sarsim import config, simulate
    cfg = config("c2", Na=2048, Nr=1024, n_targets=1)
    m_t, n_t = 1000, 400
    sc = simulate(cfg, noise=False, targets=[(m_t, n_t)])
    img = O.rda(sc.raw, cfg)
    sub = np.abs(img[m_t - 8:m_t + 9, n_t - 8:n_t + 9])
    i = int(np.argmax(sub))
    assert (i // 17, i % 17) == (8, 8)
    pk = img[m_t, n_t]
    dphi = (np.angle(pk) - sc.targets[0]["phase"] + np.pi / 4 + np.pi) % (2 * np.pi) - np.pi
    assert abs(dphi) < 0.05, dphi
    R0 = cfg["r_near"] + n_t
    Ba = (2.0 / cfg["lam"]) * cfg["v"] ** 2 * cfg["exposure"] / R0
    expect = cfg["range_len"] * math.sqrt(Ba * cfg["exposure"])
    assert abs(abs(pk) / expect - 1.0) < 0.05, abs(pk) / expect


ALL_PINS = [
    pin_fft_bruteforce,
    pin_fft_single_bins_longdouble,
    pin_fft_parseval,
    pin_fft_impulse_and_shift,
    pin_fft_round_trip,
    pin_fft_cazac,
    pin_cazac_self_compression,
    pin_compression_is_correlation,
    pin_corner_turn_exact,
    pin_lfm_closed_form,
    pin_noise_gain,
    pin_bessel_i0,
    pin_rcmc_weights_structure,
    pin_rcmc_weights_kaiser_values,
    pin_rcmc_weights_interpolate_tones,
    pin_rcmc_pulse_returns_to_r0,
    pin_rcmc_disabled_is_phase_only,
    pin_hyperbolic_point_target,
]
