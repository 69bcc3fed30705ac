"""Pin strength: copies of the oracle built with one planted mistake each
must fail at least one pin.  Mistakes (oracle_rda.c, MUT(k)):
 1 FFT twiddle sign flipped        7 RCMC weights not normalised
 2 bit reversal skipped            8 RCMC taps off by one cell
 3 IFFT without the 1/N scale      9 RCMC shift sign flipped
 4 matched filter not conjugated  10 azimuth phase sign flipped
 5 replica off-centre by a sample 11 I0 series with k! instead of k!^2
 6 corner turn writes untransposed 12 Doppler bins not in fftfreq order
13 Kaiser window with 2*beta       14 window sqrt(1 - |r|) instead of sqrt(1 - r^2)
15 window dropped (beta = 0, a truncated sinc)
"""
import pytest

import oracle_pins as P
from oracle import oracle as O

MUTANTS = list(range(1, 16))


@pytest.fixture(scope="module")
def mutant_dir(tmp_path_factory):
    return str(tmp_path_factory.mktemp("oracle_mutants"))


@pytest.mark.parametrize("k", MUTANTS)
def test_planted_mistake_is_caught(k, mutant_dir):
    path = O.build_mutant(k, mutant_dir)
    failed = []
    with O.use_library(path):
        for pin in P.ALL_PINS:
            try:
                pin()
            except (AssertionError, ValueError, FloatingPointError):
                failed.append(pin.__name__)
    assert failed, f"planted mistake {k} passed every pin"
