"""The TSQR autotuner (hb_autotune): it times both lane layouts of every
width on synthetic batches and fills the layout table; whatever it picks,
the merges keep the FP64 parity bars against the oracle (the layouts differ
only in the order of partial sums)."""
import numpy as np
import pytest

from workloads import generators as G

from _hbtest import factors_np, lowrank_diff, recon_norm, run_gpu, run_oracle, say

pytestmark = pytest.mark.gpu


def test_autotune_then_parity(lib):
    out = lib.autotune()
    table, us = out["table"], np.asarray(out["us"]).reshape(2, 4, 2, 2)
    say(f"[autotune] layout table {table}")
    assert set(table) <= {0, 1}
    # every timed (scalar, width, batch) combination has both layouts measured
    for sc in range(2):
        for ki in range(4):
            if sc == 1 and ki == 3:
                continue
            assert np.all(us[sc, ki] > 0.0)
    for wl in (G.make_helmholtz_plates(n=1200, leaf=300, cfg=2),
               G.make_gauss3d(n=800, leaf=100, tol=1e-9, d=8, cfg=23)):
        res = run_gpu(lib, wl)
        _, ores = run_oracle(wl)
        U, S, Vh = factors_np(res)
        assert S.size == ores.rank
        Vo = ores.V.conj().T
        diff = lowrank_diff(U * S, Vh, ores.U * ores.S, Vo)
        assert diff <= 1e-10 * recon_norm(ores.U * ores.S, Vo)
