"""The oracle's pins must reject plausible mistakes.

Each case plants one mistake in a copy of the oracle's C source (on the CPU,
in a temporary directory), builds it, points the oracle wrapper at it and runs
the pin battery of ``test_oracle_pins``; at least one pin has to fail.  The
unmodified source must pass the same battery.
"""
import os
import subprocess

import pytest

from oracle import build as obuild
from oracle import ols
from tests import test_oracle_pins as pins

SRC = open(obuild.SRC).read()

MUTANTS = {
    "idft_sign": [("accr += yr * wr[r] + yi * wi[r];", "accr += yr * wr[r] - yi * wi[r];"),
                  ("acci += yi * wr[r] - yr * wi[r];", "acci += yi * wr[r] + yr * wi[r];")],
    "idft_no_1_over_n": [("z[2 * i] = accr / (double)n;", "z[2 * i] = accr;"),
                         ("z[2 * i + 1] = acci / (double)n;", "z[2 * i + 1] = acci;")],
    "twiddle_sign": [("(*wi)[r] = -sin(a);", "(*wi)[r] = sin(a);")],
    "mirror_not_reversed": [("return v[n - k - k1];", "return v[k - (n - k1 - lv + 1)];")],
    "pass_edge_includes_k1": [("(k >= 0 && k <= k1 - 1)", "(k >= 0 && k <= k1)")],
    "upper_pass_edge": [("(k >= n - k1 + 1 && k <= n - 1)", "(k >= n - k1 + 2 && k <= n - 1)")],
    "delay_off_by_one": [("int64_t d = (n - hop) / 2;", "int64_t d = (n - hop) / 2 + 1;")],
    "framing_off_by_one": [("int64_t start = m * (int64_t)hop - (int64_t)(n - hop);",
                            "int64_t start = m * (int64_t)hop - (int64_t)(n - hop) + 1;")],
    "discard_off_by_one": [("out[2 * j] = z[2 * (n - hop + j)];", "out[2 * j] = z[2 * (n - hop + j - 1)];"),
                           ("out[2 * j + 1] = z[2 * (n - hop + j) + 1];",
                            "out[2 * j + 1] = z[2 * (n - hop + j - 1) + 1];")],
    "switch_one_block_early": [("if (from[i] <= m && (best < 0", "if (from[i] <= m + 1 && (best < 0")],
    "conjugated_coefficient": [("X[2 * k + 1] = hr * xi + hi * xr;", "X[2 * k + 1] = hr * xi - hi * xr;")],
    "last_sample_dropped": [("if (t >= 0 && t < len) {", "if (t >= 0 && t < len - 1) {")],
    "stopband_leak": [("    return 0.0;                             /* stopband k_s */",
                       "    return 1e-3;                            /* stopband k_s */")],
    "transition_value_shift": [("return v[k - k1];", "return v[k - k1 > 0 ? k - k1 - 1 : 0];")],
}


def battery():
    """Run the pins; return the names of those that fail."""
    cases = [
        ("dft_fft", lambda: pins.test_dft_matches_numpy_fft(64)),
        ("idft_sign", lambda: pins.test_idft_sign_and_scale(16)),
        ("parseval", lambda: pins.test_dft_parseval_and_tone(16)),
        ("ti_conv", lambda: pins.test_ti_case_is_linear_convolution(64, 48, 64 * 5 + 1)),
        ("ti_conv_ragged", lambda: pins.test_ti_case_is_linear_convolution(16, 10, 97)),
        ("allpass", lambda: pins.test_allpass_is_pure_delay(64, 48)),
        ("cosine", lambda: pins.test_coefficients_match_cosine_closed_form(128, 96, 41, 15)),
        ("regions", pins.test_magnitude_regions_and_mirror),
        ("brute", pins.test_brute_force_tiny_sizes),
        ("tones", lambda: pins.test_bin_centred_tones(64, 48, 10, 4)),
        ("switch", pins.test_bandwidth_switch_splices_whole_blocks),
        ("subset", pins.test_block_subset_equals_full_run),
        ("ragged", lambda: pins.test_ragged_and_empty_lengths(97)),
    ]
    failed = []
    for name, fn in cases:
        try:
            fn()
        except (AssertionError, ols.OracleError):
            failed.append(name)
    return failed


def _build(src_text, tmp_path, tag):
    c = tmp_path / f"{tag}.c"
    so = tmp_path / f"lib{tag}.so"
    c.write_text(src_text)
    subprocess.run(["gcc", "-O1", "-std=c11", "-fopenmp", "-shared", "-fPIC", "-o", str(so),
                    str(c), "-lm"], check=True)
    return str(so)


def test_unmodified_source_passes(tmp_path):
    with ols.use_library(_build(SRC, tmp_path, "orig")):
        assert battery() == []


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path):
    text = SRC
    for old, new in MUTANTS[name]:
        assert text.count(old) == 1, (name, old)
        text = text.replace(old, new)
    with ols.use_library(_build(text, tmp_path, name)):
        failed = battery()
    assert failed, f"planted mistake '{name}' passed every pin"
