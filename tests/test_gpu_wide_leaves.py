"""Leaves whose BACA rank exceeds the register TSQR tile (128 real columns)
take the column-panel route of the SVD re-compression (QR(U) and QR(V^H) by
column panels, the truncated SVD of T_U T_V^H).  The 8-D Gaussian mixture at
tol 1e-6 has leaf ranks up to 224 and merge widths up to 470; every leaf's
pivot tape and the FP64 result are held to the usual bars against the
oracle."""
import numpy as np
import pytest

from workloads import generators as G

from _hbtest import (compare_tape, divergence_nu, factors_np, lowrank_diff, parity_bar,
                     recon_norm, run_gpu, run_oracle, say)

pytestmark = pytest.mark.gpu


def test_wide_leaves_match_oracle(lib):
    wl = G.make_gauss_mixture(n=2000, leaf=250, tol=1e-6, d=16, cfg=44)
    say("[wide leaves] 8-D mixture 2000 x 2000, leaf 250, d 16, tol 1e-6")
    res = run_gpu(lib, wl, record_tape=1)
    _, ores = run_oracle(wl)
    nb = 1 << ores.L
    parted = 0.0
    for li in range(res.nleaves):
        info = res.leaf_info(li)
        b = info["t"] * nb + info["v"]
        tape = res.leaf_tape(li)
        msg = compare_tape(tape, info, ores.leaf_info[b])
        assert msg is None, f"leaf {b}: {msg}"
        parted += divergence_nu(tape, ores.leaf_info[b])
    st = res.stats()
    say(f"  leaf BACA rank max {st['leaf_rank_baca_max']}; rank gpu {res.rank(0)} oracle {ores.rank}")
    assert st["leaf_rank_baca_max"] > 128  # the wide path did run
    U, S, Vh = factors_np(res)
    assert S.size == ores.rank
    ref = recon_norm(ores.U * ores.S, ores.V.T)
    bar = parity_bar(ref, parted)
    assert np.allclose(S, ores.S, rtol=0, atol=max(bar, 1e-10 * ores.S[0]))
    diff = lowrank_diff(U * S, Vh, ores.U * ores.S, ores.V.T)
    say(f"  reconstruction difference {diff / ref:.2e} (bar {bar / ref:.2e})")
    assert diff <= bar
