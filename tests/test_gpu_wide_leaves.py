"""Leaves whose BACA rank exceeds the register TSQR tile (128 real columns)
take the two-merge re-compression (V^H orthonormalised without truncation,
then an eps-truncated merge with column-panel QR).  The 8-D Gaussian mixture
at tol 1e-6 has leaf ranks up to 224 and merge widths up to 470; the FP64
result is held to the usual bars against the oracle."""
import numpy as np
import pytest

from workloads import generators as G

from _hbtest import factors_np, lowrank_diff, recon_norm, run_gpu, run_oracle, say

pytestmark = pytest.mark.gpu


def test_wide_leaves_match_oracle(lib):
    wl = G.make_gauss_mixture(n=2000, leaf=250, tol=1e-6, d=16, cfg=44)
    say("[wide leaves] 8-D mixture 2000 x 2000, leaf 250, d 16, tol 1e-6")
    res = run_gpu(lib, wl)
    _, ores = run_oracle(wl)
    st = res.stats()
    say(f"  leaf BACA rank max {st['leaf_rank_baca_max']}; rank gpu {res.rank(0)} oracle {ores.rank}")
    assert st["leaf_rank_baca_max"] > 128  # the wide path did run
    U, S, Vh = factors_np(res)
    assert S.size == ores.rank
    assert np.allclose(S, ores.S, rtol=0, atol=1e-10 * ores.S[0])
    diff = lowrank_diff(U * S, Vh, ores.U * ores.S, ores.V.T)
    assert diff <= 1e-10 * recon_norm(ores.U * ores.S, ores.V.T)
