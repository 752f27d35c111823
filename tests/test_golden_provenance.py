"""The stored full-size values (tests/golden/*.json) are what the committed
script tests/golden/make_golden.py computes with the oracle: re-running it
reproduces the rank, the largest rank after every merge step, the root
singular values and the sampled error."""
import importlib.util
import json
import os

import numpy as np
import pytest

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _script():
    spec = importlib.util.spec_from_file_location("make_golden", os.path.join(HERE,
                                                                              "make_golden.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


@pytest.mark.parametrize("name", ["gauss3d", "helmholtz", "coherent"])
def test_golden_values_reproduce(name):
    mg = _script()
    with open(os.path.join(HERE, mg.WORKLOADS[name])) as f:
        stored = json.load(f)
    now = mg.record(name)
    for key in ("m", "n", "tol", "d", "leaf", "seed", "rank", "step_rank_max"):
        assert now[key] == stored[key], key
    s0, s1 = np.asarray(stored["sigma"]), np.asarray(now["sigma"])
    assert np.max(np.abs(s1 - s0)) <= 1e-12 * s0[0]
    assert abs(now["rel_err_rows7"] - stored["rel_err_rows7"]) <= 1e-8 * stored["rel_err_rows7"]
