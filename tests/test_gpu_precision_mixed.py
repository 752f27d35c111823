"""Mixed precision (FP32 entries, residual blocks and leaf factors with FP64
accumulation; FP64 norm estimates, re-compression and merges) against the
FP64 oracle on the same seeded inputs, on single problems.

Pivots chosen from FP32 residuals may differ from the FP64 oracle's, so the
bar is on what the method promises: the compressed operators agree to
5 tol relative (Frobenius norm of the difference, computed from the
factors), the error against A stays within 5 tol of the oracle's, and the
ranks stay close."""
import numpy as np
import pytest

from workloads import generators as G

from _hbtest import check_mixed, run_gpu

pytestmark = pytest.mark.gpu


def _laplace_single(cfg, tol=1e-4, d=8):
    b = G.make_laplace_blocks(nblocks=1, cfg=cfg)
    m, n = int(b["row_cnt"][0]), int(b["col_cnt"][0])
    return dict(name="laplace", entry=2, X=b["X"][:m], Y=b["Y"][:n], m=m, n=n, h=0.0,
                gauss_c=0.0, wavenumber=0.0, tol=tol, d=d, leaf=max(32, max(m, n) // 3),
                seed=9, complex=False)


MIXED_CASES = {
    "gauss3d_1000_tol1e-6": lambda: G.make_gauss3d(n=1000, leaf=125, tol=1e-6, d=8, cfg=41),
    "gauss3d_ragged_d16": lambda: G.make_gauss3d(n=900, m=770, leaf=200, tol=1e-6, d=16, cfg=45),
    "adjoint_geometry_3200": lambda: G.make_gauss3d(n=3200, h=0.7, leaf=400, tol=1e-6, d=8,
                                                    cfg=46),
    "laplace_tol1e-4": lambda: _laplace_single(47),
    "lowrank_r25": lambda: G.make_lowrank_spikes(n=600, m=560, rank=25, n_spikes=0, tol=1e-6,
                                                 d=8, leaf=150, cfg=48),
}


@pytest.mark.parametrize("case", sorted(MIXED_CASES))
def test_mixed_precision_within_5tol_of_oracle(lib, case):
    check_mixed(lib, case, MIXED_CASES[case]())


def test_mixed_precision_rejects_complex_kernels(lib):
    wl = G.make_helmholtz_plates(n=200, leaf=100, cfg=50)
    with pytest.raises(lib.HBACAError) as e:
        run_gpu(lib, wl, precision=lib.HB_PREC_MIXED)
    assert e.value.status == -6
