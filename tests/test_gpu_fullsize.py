"""Full-size parity on the benchmark workload (Helmholtz, 20000 x 20000,
complex FP64, tol 1e-4, d = 16, leaf 625) in the configuration bench.py
times: rank, the maximum rank after every merge step and the singular values
against the oracle's values stored in tests/golden (written by
tests/golden/make_golden.py, which calls only the oracle), plus the relative
error on every 7th row recomputed on the device."""
import json
import os

import numpy as np
import pytest

from workloads import make_config

from _hbtest import run_gpu, say

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.mark.parametrize("name,file", [("helmholtz", "helmholtz_20000.json"),
                                       ("gauss3d", "gauss3d_2000.json")])
def test_full_size_matches_golden(lib, name, file):
    gold = json.load(open(os.path.join(GOLD, file)))
    wl = make_config(name)
    say(f"[full size] {name} {wl['m']} x {wl['n']}")
    res = run_gpu(lib, wl)
    U, S, Vh = res.factors(0)
    S = S.cpu().numpy()
    st = res.stats()
    assert res.rank(0) == gold["rank"]
    assert st["step_rank_max"][: len(gold["step_rank_max"])] == gold["step_rank_max"]
    sg = np.array(gold["sigma"])
    assert np.allclose(S, sg, rtol=0, atol=1e-10 * sg[0])
    e2, a2 = res.error(0, 7)
    err = float(np.sqrt(e2 / a2))
    say(f"  rank {res.rank(0)}, sampled error {err:.4e} (oracle {gold['rel_err_rows7']:.4e}), "
        f"{st['ms_total']:.1f} ms")
    assert abs(err - gold["rel_err_rows7"]) <= 1e-6 * gold["rel_err_rows7"]


def test_coherent_variant_full_size(lib):
    """The coherent variant at its full size (20000 x 20000: a rank-30 product
    of Gaussian factors plus 200 spikes of 1e3, tol 1e-4, d = 16, leaf 625)
    against the oracle's stored values.  Once the rank-30 part is captured
    the residual is rounding plus isolated spikes, so which spikes each run
    finds is decided by rounding; what is compared is the rank (within 5)
    and the sampled error (within 25 %), which both runs take from the spikes
    they miss.  Both stay far above tol: the paper's coherence failure of
    cross approximation (Section "Blocked Adaptive Cross Approximation"),
    reported rather than hidden."""
    gold = json.load(open(os.path.join(GOLD, "coherent_20000.json")))
    wl = make_config("coherent")
    say(f"[full size] coherent {wl['m']} x {wl['n']}, {len(wl['spike_lin'])} spikes")
    res = run_gpu(lib, wl)
    e2, a2 = res.error(0, 7)
    err = float(np.sqrt(e2 / a2))
    say(f"  rank {res.rank(0)} (oracle {gold['rank']}), sampled error {err:.4e} "
        f"(oracle {gold['rel_err_rows7']:.4e})")
    assert abs(res.rank(0) - gold["rank"]) <= 5
    assert 0.8 * gold["rel_err_rows7"] <= err <= 1.25 * gold["rel_err_rows7"]
