"""Pins against numbers printed in the paper (tests/golden/paper_values.json).

* The Jakob number Ja = rho_l cp_l dT/(rho_v h_lg) (Sec. 3.1) reproduces the
  printed Ja of the Stefan, sucking and Scriven setups; the same definition
  sets h_lg for the synthetic workloads (Ja = 1).
* The Stefan closed form (Sec. 3.1) with the printed properties gives the
  printed initial vapour thickness 322.5 um at t = 0.282 s.
"""
import json
import math
import os

import pytest

from oracle import closed

HERE = os.path.dirname(os.path.abspath(__file__))
VALS = json.load(open(os.path.join(HERE, "golden", "paper_values.json")))


@pytest.mark.parametrize("key", ["stefan", "sucking", "scriven"])
def test_jakob_numbers(key):
    v = VALS[key]
    dT = v.get("dT", v.get("T_w", 0) - v.get("T_sat", 0))
    Ja = v["rho_l"] * v["cp_l"] * dT / (v["rho_v"] * v["h_lg"])
    assert abs(Ja - v["Ja"]) < 0.006, (key, Ja)


def test_stefan_initial_thickness():
    v = VALS["stefan"]
    dT = v["T_w"] - v["T_sat"]
    beta = closed.stefan_beta(v["cp_v"], dT, v["h_lg"])
    alpha_v = v["lam_v"] / (v["rho_v"] * v["cp_v"])
    X = closed.stefan_position(v["t0"], beta, alpha_v)
    # the paper prints four significant digits
    assert abs(X - v["X0"]) < 0.05e-6 * 10, (X, v["X0"])
    assert abs(X - v["X0"]) / v["X0"] < 2e-3
    # and the transcendental equation holds at the root
    lhs = beta * math.exp(beta ** 2) * math.erf(beta)
    assert abs(lhs - v["cp_v"] * dT / (math.sqrt(math.pi) * v["h_lg"])) < 1e-16
