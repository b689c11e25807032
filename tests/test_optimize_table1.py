"""The App. D closed-form cost functions, minimised over the admissible
quadrant, must reproduce Table 1 groups A and B (no GPU)."""
import json
import os

from paper_1107_4543_amd import optimize

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_tables.json")))


def test_dispersion_cost_minimum_is_table1_group_a():
    a = GOLD["table1"]["A"]
    se, sq, val = optimize.minimize("odd")
    assert se == 0.0                                # the minimum lies on the boundary sigma_eps = 0
    assert abs(sq - a["sigma_q"]) < 1e-4 * a["sigma_q"]
    assert abs(val - a["Fo"]) < 1e-8 * a["Fo"]
    # and the printed minimiser evaluates to the printed minimum
    assert abs(optimize.F_odd(a["sigma_eps"], a["sigma_q"]) - a["Fo"]) < 1e-9 * a["Fo"]


def test_total_cost_minimum_is_table1_group_b():
    b = GOLD["table1"]["B"]
    se, sq, val = optimize.minimize("total")
    assert se == 0.0
    assert abs(sq - b["sigma_q"]) < 1e-4 * b["sigma_q"]
    assert abs(val - b["F"]) < 1e-8 * b["F"]
    # App. D prints the coefficients to 10 significant digits: agreement to a
    # few 1e-9 is all their rounding allows
    assert abs(optimize.F_total(b["sigma_eps"], b["sigma_q"]) - b["F"]) < 5e-9 * b["F"]
    # sigma_eps = 0 means s_eps = 2, at the edge of the admissible range (0, 2]
    assert optimize.rates_from_sigma(0.0) == 2.0
