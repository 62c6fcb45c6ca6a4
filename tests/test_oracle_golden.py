"""Pins against numbers printed in the paper (tests/golden/paper_values.json)."""

import json
import math
import os

import oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")


def load():
    with open(GOLDEN) as f:
        return json.load(f)


def test_split_coefficients_match_printed_values():
    g = load()
    for order, key in ((1, "split_first_order"), (2, "split_second_order")):
        A, B = O.split_coefficients(order)
        assert A == g[key]["a"] and B == g[key]["b"]
    A, B = O.split_coefficients(4)
    t = A[1]
    assert round(t, g["split_fourth_order_t"]["digits"]) == g["split_fourth_order_t"]["value"]
    # printed layout: a = (0, t, 1-2t, t), b = (t/2, (1-t)/2, (1-t)/2, t/2)
    assert A == [0.0, t, 1 - 2 * t, t]
    assert B == [t / 2, (1 - t) / 2, (1 - t) / 2, t / 2]
    # t is the fourth-order (Forest-Ruth / Yoshida) root: 2 t^3 + (1-2t)^3 = 0
    assert abs(2 * t ** 3 + (1 - 2 * t) ** 3) < 1e-14


def test_interbranch_ratio_printed_value():
    g = load()["interbranch_ratio"]
    assert abs(math.exp(-2 * math.pi / g["beta_over_betac"]) - g["I_over_I0"]) < 5e-5
