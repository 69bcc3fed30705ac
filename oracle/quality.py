"""Point-target image-quality metrics (numpy, FP64).

TEST INFRASTRUCTURE ONLY.  The paper reports a relative L2 error, a maximum
absolute error and a per-target SNR (Sec. V.D, Table IV) and claims PSLR/ISLR
validation without stating how either is measured.  The estimators below are
our readings:

* peak: argmax of |I| in a +-8 box around the seeded cell, ties to the
  lowest linear index;
* SNR_k = 10 log10(|I[peak]|^2 / P_n), where P_n is the mean |I|^2 over
  pixels at least ``guard`` rows from every target row *and* ``guard``
  columns from every target column;
* PSLR / ISLR on 1-D range and azimuth cuts of half-width ``half`` through
  the peak, upsampled x16 by band-limited (DFT zero-padding) interpolation;
  the main lobe spans the first minima on each side of the peak;
  PSLR = 20 log10(max sidelobe / peak), ISLR = 10 log10(E_side / E_main).
"""
from __future__ import annotations

import numpy as np


def rel_l2(a: np.ndarray, ref: np.ndarray) -> float:
    a = np.asarray(a, dtype=np.complex128)
    ref = np.asarray(ref, dtype=np.complex128)
    return float(np.linalg.norm((a - ref).ravel()) / np.linalg.norm(ref.ravel()))


def max_abs(a: np.ndarray, ref: np.ndarray) -> float:
    return float(np.max(np.abs(np.asarray(a, np.complex128) - np.asarray(ref, np.complex128))))


def peak_cell(img: np.ndarray, m: int, n: int, box: int = 8) -> tuple[int, int]:
    """Row/column of max |I| within +-box of (m, n); first in row-major order
    on ties (= lowest linear index in the full image)."""
    na, nr = img.shape
    m0, m1 = max(0, m - box), min(na, m + box + 1)
    n0, n1 = max(0, n - box), min(nr, n + box + 1)
    sub = np.abs(img[m0:m1, n0:n1])
    i = int(np.argmax(sub))
    return m0 + i // sub.shape[1], n0 + i % sub.shape[1]


def noise_power(img: np.ndarray, targets, guard: int) -> float:
    na, nr = img.shape
    rows = np.ones(na, dtype=bool)
    cols = np.ones(nr, dtype=bool)
    r = np.arange(na)
    c = np.arange(nr)
    for t in targets:
        rows &= np.abs(r - t["m"]) >= guard
        cols &= np.abs(c - t["n"]) >= guard
    sel = np.abs(img[np.ix_(rows, cols)]) ** 2
    if sel.size == 0:
        raise ValueError("no pixels left for the noise estimate")
    return float(np.mean(sel))


def snr_db(img: np.ndarray, targets, guard: int) -> list[float]:
    pn = noise_power(img, targets, guard)
    out = []
    for t in targets:
        pm, pn_ = peak_cell(img, t["m"], t["n"])
        out.append(float(10.0 * np.log10(np.abs(img[pm, pn_]) ** 2 / pn)))
    return out


def upsample(cut: np.ndarray, factor: int = 16) -> np.ndarray:
    """Band-limited interpolation of an even-length cut by DFT zero-padding;
    the Nyquist bin is split evenly between the two halves."""
    n = cut.size
    if n % 2:
        raise ValueError("cut length must be even")
    X = np.fft.fft(cut)
    m = n * factor
    Y = np.zeros(m, dtype=np.complex128)
    h = n // 2
    Y[:h] = X[:h]
    Y[m - h + 1:] = X[h + 1:]
    Y[h] = 0.5 * X[h]
    Y[m - h] = 0.5 * X[h]
    return np.fft.ifft(Y) * factor


def lobe_metrics(cut: np.ndarray, factor: int = 16) -> tuple[float, float]:
    """(PSLR dB, ISLR dB) of a 1-D cut whose peak is near its centre."""
    u = np.abs(upsample(np.asarray(cut, dtype=np.complex128), factor))
    c = cut.size // 2 * factor
    w = factor                       # search the peak within +-1 sample of centre
    p = c - w + int(np.argmax(u[c - w:c + w + 1]))
    lo = p
    while lo > 0 and u[lo - 1] <= u[lo]:
        lo -= 1
    hi = p
    while hi < u.size - 1 and u[hi + 1] <= u[hi]:
        hi += 1
    main = u[lo:hi + 1]
    side = np.concatenate([u[:lo], u[hi + 1:]])
    pslr = 20.0 * np.log10(np.max(side) / u[p])
    islr = 10.0 * np.log10(np.sum(side ** 2) / np.sum(main ** 2))
    return float(pslr), float(islr)


def cut_through(img: np.ndarray, m: int, n: int, half: int, axis: str) -> np.ndarray:
    """Even-length (2*half) cut centred on (m, n), wrapping circularly."""
    na, nr = img.shape
    off = np.arange(-half, half)
    if axis == "range":
        return img[m, (n + off) % nr]
    return img[(m + off) % na, n]


def point_target_report(img: np.ndarray, targets, guard: int, half: int) -> list[dict]:
    """Per target: peak cell, SNR, PSLR/ISLR in range and in azimuth."""
    pn = noise_power(img, targets, guard)
    rep = []
    for t in targets:
        pm, pr = peak_cell(img, t["m"], t["n"])
        r_p, r_i = lobe_metrics(cut_through(img, pm, pr, half, "range"))
        a_p, a_i = lobe_metrics(cut_through(img, pm, pr, half, "azimuth"))
        rep.append(dict(peak=(pm, pr),
                        snr_db=float(10.0 * np.log10(np.abs(img[pm, pr]) ** 2 / pn)),
                        pslr_range=r_p, islr_range=r_i,
                        pslr_azimuth=a_p, islr_azimuth=a_i))
    return rep
