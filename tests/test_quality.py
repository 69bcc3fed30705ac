"""Image-quality estimators against textbook closed forms (CPU only)."""
import os

import numpy as np
import pytest

from oracle import quality as Q

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _golden(name):
    out = {}
    for line in open(os.path.join(GOLDEN, name)):
        line = line.strip()
        if line and not line.startswith("#"):
            k, v = line.split()
            out[k] = float(v)
    return out


@pytest.mark.parametrize("offset", [0.0, 0.3, -0.45])
def test_sinc_pslr_islr(offset):
    """A sampled sinc of bandwidth 0.5 (2 samples per resolution cell) gives
    the textbook PSLR and the ISLR integrated over +-16 / +-25 cells."""
    g = _golden("sinc_lobes.txt")
    n = np.arange(-32, 32)
    p, i = Q.lobe_metrics(np.sinc(0.5 * (n - offset)))
    assert abs(p - g["pslr_db"]) < 0.02
    assert abs(i - g["islr_db_M16"]) < 0.02
    n = np.arange(-50, 50)
    p, i = Q.lobe_metrics(np.sinc(0.5 * (n - offset)))
    assert abs(p - g["pslr_db"]) < 0.02
    assert abs(i - g["islr_db_M25"]) < 0.02


def test_peak_tie_break_lowest_index():
    img = np.zeros((32, 32), complex)
    img[10, 12] = 5.0
    img[10, 14] = 5.0
    img[12, 11] = 5.0
    assert Q.peak_cell(img, 11, 12) == (10, 12)


def test_rel_l2_and_max_abs():
    a = np.array([3.0 + 4.0j, 0.0])
    b = np.array([3.0 + 4.0j, 1.0])
    assert Q.rel_l2(b, a) == pytest.approx(0.2)
    assert Q.max_abs(a, b) == 1.0


def test_c1_snr_near_closed_form(oracle_lib):
    """c1: SNR = 20 dB + 10 log10(L_r L_a) = 56.12 dB, within the spread of a
    noise estimate over ~2.3e3 independent samples (~0.1 dB)."""
    from sarsim import config, simulate
    cfg = config("c1")
    sc = simulate(cfg)
    img = oracle_lib.rda(sc.raw, cfg)
    expect = 20.0 + 10.0 * np.log10(cfg["range_len"] * cfg["az_len"])
    for s in Q.snr_db(img, sc.targets, 16):
        assert abs(s - expect) < 0.35
