"""Mixed precision on the 8-D Gaussian mixture (leaves whose entries reach
1e-14 and residual panels far below that), against the FP64 oracle at the
5 tol bar.

This case once faulted the GPU: in the FP32 leaf kernel a Householder
scale beta ~ 1/sigma^2 beyond the FP32 range became inf, the reflector
update gave inf - inf = NaN, and a NaN norm never won the pivot comparison,
leaving the pivot index unset.  The kernel now forms beta v w in FP64 and
every pivot argmax treats a NaN norm as zero, so a valid pivot always
exists.  It runs last among the GPU tests."""
import pytest

from workloads import generators as G

from _hbtest import check_mixed

pytestmark = pytest.mark.gpu


def test_mixed_precision_8d_mixture(lib):
    wl = G.make_gauss_mixture(n=2000, leaf=250, tol=1e-6, d=16, cfg=44)
    check_mixed(lib, "mixture_8d_2000", wl)
