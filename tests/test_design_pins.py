"""Design-side relations pinned to the numbers the paper prints for its
example (Sec. IV, Tables II and III); fixture: tests/golden/paper_example.json."""
import json
import math
import os

import pytest

from oracle import design

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_example.json")))


def test_bin_domain_width_and_range():
    spec, printed = GOLD["spec"], GOLD["printed"]
    n = printed["N"]
    delta = spec["Delta_over_pi"] * math.pi
    lo = design.bin_edges(spec["b_over_pi"][0] * math.pi, delta, n)
    hi = design.bin_edges(spec["b_over_pi"][1] * math.pi, delta, n)
    assert lo.delta_n == pytest.approx(printed["Delta_N"], abs=1e-9)
    assert round(lo.b_n) == printed["b_N"][0] and round(hi.b_n) == printed["b_N"][1]
    # eq. (7) in bins: k1 = b_N - Delta_N/2 + 1, k2 = k1 + Delta_N - 2
    assert lo.k1 == pytest.approx(48 - 8 + 1) and lo.k2 == pytest.approx(48 + 8 - 1)
    # L_V = Delta_N - 1 equals the memory of Table III
    assert lo.lv == pytest.approx(GOLD["table3_fdfd"]["memory"])
    # the upper end of the range is the largest admissible b_N
    assert design.b_n_range(printed["Delta_N"], n)[1] == printed["b_N"][1]
    assert design.b_n_range(printed["Delta_N"], n)[0] <= printed["b_N"][0]


def test_order_and_dft_size_estimates():
    spec, printed = GOLD["spec"], GOLD["printed"]
    nd = design.order_estimate(spec["delta_p"], spec["delta_s"], spec["Delta_over_pi"] * math.pi)
    assert nd == pytest.approx(80.0 / 3.0)          # closed form: 4*5/0.75
    assert design.even_order(nd) == printed["N_D_hat"]
    L0 = printed["N_D_hat"] + 1
    n_hat, n, m = design.dft_size(L0)
    assert round(n_hat) == printed["N_hat"] and n == printed["N"]
    assert (L0, m) == (GOLD["table2_tdfd"]["L"], GOLD["table2_tdfd"]["M"])
    assert printed["N"] - printed["L"] + 1 == printed["M"]


def test_table2_fdfd_row_from_table1():
    row = GOLD["table2_fdfd"]
    r = design.complexity(row["N"], row["L"], GOLD["table3_fdfd"]["memory"], odd_k_rule=True)
    assert (row["L"] - 1) / row["N"] == GOLD["odd_k_rule"]["L_minus_1_over_N"]
    assert round(r.r_mf, 1) == row["R_mf"]
    assert round(r.r_mv, 1) == row["R_mv"]
    assert round(r.r_a, 1) == row["R_a"]
    assert r.memory == GOLD["table3_fdfd"]["memory"]
    # Table I alone (no exponent shortcut) does not give the printed row
    plain = design.complexity(row["N"], row["L"], 15)
    assert round(plain.r_mf, 1) != row["R_mf"]
    assert plain.r_mv == r.r_mv
