"""ctypes wrapper around the FP64 C oracle (``oracle_rda.c``).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg.  The HIP product path never imports this module.

Arrays cross as interleaved doubles; complex inputs are promoted to
complex128, and every function returns new complex128 arrays.
"""
from __future__ import annotations

import contextlib
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle_rda.c")
_LIB_PATH = os.path.join(_HERE, "liboracle_rda.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle shared library with gcc + OpenMP."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-fopenmp", "-std=c11", "-Wall", "-Wextra",
             "-shared", "-fPIC", _SRC, "-lm", "-o", tmp])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def build_mutant(k: int, out_dir: str) -> str:
    """Compile a copy of the oracle with planted mistake ``k`` (pin-strength
    tests only)."""
    path = os.path.join(out_dir, f"liboracle_mut{k}.so")
    subprocess.check_call(
        ["gcc", "-O2", "-fopenmp", "-std=c11", f"-DORC_MUTANT={int(k)}",
         "-shared", "-fPIC", _SRC, "-lm", "-o", path])
    return path


@contextlib.contextmanager
def use_library(path: str):
    """Route every wrapper call through another build of the oracle."""
    global _lib
    saved = _lib
    _lib = _load(path)
    try:
        yield
    finally:
        _lib = saved


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        _lib = _load(_LIB_PATH)
    return _lib


def _load(path: str):
    L = ctypes.CDLL(path)
    dp = ctypes.POINTER(ctypes.c_double)
    fp = ctypes.POINTER(ctypes.c_float)
    i, d = ctypes.c_int, ctypes.c_double
    L.orc_fft.argtypes = [dp, i, i]
    L.orc_matched_filter.argtypes = [i, i, d, i, dp]
    L.orc_compress_rows.argtypes = [dp, i, i, dp, dp]
    L.orc_fft_rows.argtypes = [dp, i, i, dp]
    L.orc_corner_turn.argtypes = [dp, i, i, dp]
    L.orc_bessel_i0.argtypes = [d]
    L.orc_bessel_i0.restype = d
    L.orc_rcmc_weights.argtypes = [d, d, i, dp]
    L.orc_rcmc_azimuth.argtypes = [dp, i, i, d, d, d, i, d, dp]
    L.orc_rda.argtypes = [fp, i, i, i, d, i, i, d, d, d, d, i, d, dp]
    L.orc_num_threads.restype = i
    L.orc_set_num_threads.argtypes = [i]
    return L


def _c128(x) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(x, dtype=np.complex128))


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _check(rc, what):
    if rc != 0:
        raise ValueError(f"oracle {what} rejected its arguments (rc={rc})")


def set_threads(n: int) -> None:
    lib().orc_set_num_threads(int(n))


def num_threads() -> int:
    return int(lib().orc_num_threads())


def fft(x, inverse: bool = False) -> np.ndarray:
    a = _c128(x).copy()
    _check(lib().orc_fft(_dp(a), a.size, int(inverse)), "fft")
    return a


def ifft(x) -> np.ndarray:
    return fft(x, inverse=True)


def matched_filter(n: int, length: int, tbp: float, sign: int = +1) -> np.ndarray:
    H = np.empty(n, dtype=np.complex128)
    _check(lib().orc_matched_filter(n, length, float(tbp), int(sign), _dp(H)),
           "matched_filter")
    return H


def compress_rows(x, H) -> np.ndarray:
    a = _c128(x)
    rows, n = a.shape
    out = np.empty_like(a)
    h = _c128(H)
    _check(lib().orc_compress_rows(_dp(a), rows, n, _dp(h), _dp(out)), "compress_rows")
    return out


def fft_rows(x) -> np.ndarray:
    a = _c128(x)
    rows, n = a.shape
    out = np.empty_like(a)
    _check(lib().orc_fft_rows(_dp(a), rows, n, _dp(out)), "fft_rows")
    return out


def corner_turn(x) -> np.ndarray:
    a = _c128(x)
    rows, cols = a.shape
    out = np.empty((cols, rows), dtype=np.complex128)
    _check(lib().orc_corner_turn(_dp(a), rows, cols, _dp(out)), "corner_turn")
    return out


def bessel_i0(y: float) -> float:
    return float(lib().orc_bessel_i0(float(y)))


def rcmc_weights(x: float, beta: float = 2.5, taps: int = 8) -> np.ndarray:
    w = np.empty(taps, dtype=np.float64)
    _check(lib().orc_rcmc_weights(float(x), float(beta), taps, _dp(w)), "rcmc_weights")
    return w


def rcmc_azimuth(A, lam: float, v: float, r_near: float, taps: int = 8,
                 beta: float = 2.5) -> np.ndarray:
    """RCMC + exact-geometry azimuth phase + azimuth IFFT on A[range][Doppler]."""
    a = _c128(A)
    nr, na = a.shape
    out = np.empty_like(a)
    _check(lib().orc_rcmc_azimuth(_dp(a), nr, na, float(lam), float(v), float(r_near),
                                  int(taps), float(beta), _dp(out)), "rcmc_azimuth")
    return out


_AZ = {"lfm": 0, "hyperbolic": 1}


def rda(raw: np.ndarray, p: dict) -> np.ndarray:
    """The full FP64 RDA: complex64 raw [Na][Nr] -> complex128 image [Na][Nr]."""
    r = np.ascontiguousarray(raw, dtype=np.complex64)
    na, nr = r.shape
    img = np.empty((na, nr), dtype=np.complex128)
    rp = r.view(np.float32).ctypes.data_as(ctypes.POINTER(ctypes.c_float))
    _check(lib().orc_rda(rp, na, nr, int(p["range_len"]), float(p["range_tbp"]),
                         _AZ[p["az_model"]], int(p["az_len"]), float(p["az_tbp"]),
                         float(p["lam"]), float(p["v"]), float(p["r_near"]),
                         int(p["rcmc_taps"]), float(p["rcmc_beta"]), _dp(img)),
           "rda")
    return img
