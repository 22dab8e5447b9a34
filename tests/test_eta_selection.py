"""The minibatch configurations' eta0 is the one the paper's selection rule
picks (Sec. 5, hyper-parameters: smallest angular error summed over the run):
tests/golden/eta_selection.json, written by tests/golden/select_eta.py with
the float64 oracle on a 50,000-row sample of each configuration's generator,
run for the configuration's own number of steps."""
import json
import math
import os

import numpy as np
import pytest

import bench
from tests.golden import select_eta as S

GOLD = os.path.join(os.path.dirname(__file__), "golden", "eta_selection.json")


def _gold():
    with open(GOLD) as f:
        return json.load(f)


def test_stored_selection_is_consistent():
    g = _gold()
    assert g["grid"] == list(S.GRID) and g["sample_rows"] == S.SAMPLE_ROWS
    for name, rec in g["configs"].items():
        scores = {float(k): v for k, v in rec["summed_angle"].items()}
        assert set(scores) == set(S.GRID)
        assert rec["eta0"] == min(scores, key=scores.get)
        c = S.CONFIGS[name]
        assert rec["steps"] == math.ceil(c["epochs"] * c["n"] / c["batch"])


@pytest.mark.parametrize("name", ["oja-f32", "eigengame-fp8"])
def test_bench_configuration_uses_selected_eta(name):
    g = _gold()
    c, s = bench.MINIBATCH[name], S.CONFIGS[name]
    assert c["eta0"] == g["configs"][name]["eta0"]
    for key in ("n", "d", "spectrum", "k", "l", "batch", "epochs", "t0", "seed"):
        assert c[key] == s[key], key


def test_oja_selection_recomputes():
    """The stored Oja scores come from the script: the winning and the runner-up
    rate recomputed here give the same summed angles."""
    from synthdata import make_problem
    g = _gold()["configs"]["oja-f32"]
    c = S.CONFIGS["oja-f32"]
    p = make_problem(S.SAMPLE_ROWS, c["d"], c["spectrum"], seed=c["seed"], mode="gaussian",
                     dtype=np.float64)
    x = p.x - p.x.mean(axis=0, keepdims=True)
    for eta in (1.0, 0.1):
        s, _ = S.summed_angle(x, p.q, c, eta)
        assert s == pytest.approx(g["summed_angle"][str(eta)], rel=1e-9)
