"""The oracle against its own stored results (tests/golden/, written by
tests/golden/make_golden.py from oracle/ alone): a regression pin, so that
any later change to the oracle's arithmetic shows up here and has to be
justified. The independent pins of the same runs (the laminate's exact
finite-strain solution, the LCE pieces) live in test_oracle_admm.py and
test_oracle_lce.py."""
import json
import os
import sys

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))

import make_golden as G  # noqa: E402


def load(name):
    with open(os.path.join(HERE, "golden", name + ".json")) as f:
        return json.load(f)


def close(a, b, tol=1e-12):
    a, b = np.asarray(a, float), np.asarray(b, float)
    return np.max(np.abs(a - b)) <= tol * max(1.0, np.max(np.abs(b)))


def test_laminate16_reproduces_golden():
    g, r = load("oracle_laminate16"), G.laminate16()
    assert r["iters"] == g["iters"] and r["rc"] == g["rc"]
    assert close(r["r_p"], g["r_p"]) and close(r["r_d"], g["r_d"])
    assert close(r["P_mean"], g["P_mean"])


def test_lce16_reproduces_golden():
    g, r = load("oracle_lce16"), G.lce16()
    for k, c in g["cases"].items():
        assert close(r["cases"][k]["P_mean"], c["P_mean"])
        assert close(r["cases"][k]["r_p"], c["r_p"]) and close(r["cases"][k]["r_d"], c["r_d"])


@pytest.mark.slow
def test_wavy32_reproduces_golden():
    g, r = load("oracle_wavy32"), G.wavy32()
    for a, b in zip(r["steps"], g["steps"]):
        assert a["iters"] == b["iters"] and a["rc"] == b["rc"]
        assert close(a["P_mean"], b["P_mean"]) and close([a["rho"]], [b["rho"]])
