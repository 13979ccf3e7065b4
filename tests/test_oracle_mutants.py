"""The pins must catch plausible mistakes in the oracle.

Each case compiles the oracle with one planted mistake (ORACLE_MUTATION=n in
pfb_oracle.c) into a temporary directory, runs the pins of
test_oracle_pins.py against that build, and requires at least one of them to
fail.  Runs on the CPU only."""
import numpy as np
import pytest

import oracle as oracle_pkg
from oracle import Oracle

import test_oracle_pins as pins

MUTANTS = {
    1: "oldest tap dropped",
    2: "taps not reversed (h[m*P+p])",
    3: "conjugated twiddle for real input",
    4: "wrong quadrant rotation in the twiddle",
    5: "window centred at L/2",
    6: "DFT phase index slips",
    7: "sign of the complex cross term",
    8: "block-scaled DFT leaves the coefficients unquantised",
    9: "block scale one binade too small (saturates)",
}


def _run_pins(o):
    checks = [
        lambda: pins.test_window_matches_numpy(o, "hann", np.hanning, 16, 4),
        lambda: pins.test_twiddle_quarter_turns_exact(o, 16),
        lambda: pins.test_twiddle_quarter_turns_exact(o, 4096),
        lambda: pins.test_dft_of_delta(o, 16, 3),
        lambda: pins.test_dft_matches_numpy_fft(o, 16),
        lambda: pins.test_fir_impulse_reproduces_taps(o, 16, 4, 0, 5),
        lambda: pins.test_fir_branch_is_causal_convolution(o, True),
        lambda: pins.test_pfb_complex_tone_closed_form(o, 16, 4, 3, "hann"),
        lambda: pins.test_pfb_equals_bank_of_bandpass_filters(o, 8, 3, 200, True),
        lambda: pins.test_pfb_equals_bank_of_bandpass_filters(o, 16, 4, 512, False),
        lambda: pins.test_mx_exponent_is_smallest_fitting_power(o, 1.0),
        lambda: pins.test_mx_dft_of_delta_is_the_quantised_coefficient(o, 64, False, 37),
        lambda: pins.test_mx_dft_within_rounding_bound(o, 64, True),
    ]
    failed = []
    for i, c in enumerate(checks):
        try:
            c()
        except AssertionError:
            failed.append(i)
    return failed


@pytest.mark.parametrize("mid", sorted(MUTANTS))
def test_planted_mistake_is_caught(tmp_path, mid):
    path = oracle_pkg.build(str(tmp_path / f"liboracle_m{mid}.so"), defines=(f"ORACLE_MUTATION={mid}",))
    failed = _run_pins(Oracle(path))
    assert failed, f"no pin catches mutation {mid}: {MUTANTS[mid]}"


def test_unmutated_build_passes_all(tmp_path):
    path = oracle_pkg.build(str(tmp_path / "liboracle_m0.so"))
    assert _run_pins(Oracle(path)) == []
