"""Documented limits and error returns on the GPU: a leaf whose BACA rank
would pass rank_cap returns HB_ERANKCAP and no result; a cap that is not
reached changes nothing; leaves wider than the leaf kernel's 2048 rows
return HB_EUNSUPPORTED."""
import numpy as np
import pytest

from workloads import generators as G

from _hbtest import factors_np, run_gpu, say

pytestmark = pytest.mark.gpu


def test_rank_cap_exhausted(lib):
    wl = G.make_gauss3d(n=500, leaf=125, tol=1e-6, d=8, cfg=61)
    say("[limits] rank_cap 8 on leaves of rank ~30")
    with pytest.raises(lib.HBACAError) as e:
        run_gpu(lib, wl, rank_cap=8)
    assert e.value.status == -4


def test_rank_cap_not_reached_changes_nothing(lib):
    wl = G.make_gauss3d(n=500, leaf=125, tol=1e-6, d=8, cfg=61)
    a = run_gpu(lib, wl)
    b = run_gpu(lib, wl, rank_cap=125)
    Ua, Sa, Va = factors_np(a)
    Ub, Sb, Vb = factors_np(b)
    assert np.array_equal(Sa, Sb)
    assert np.array_equal(Ua, Ub) and np.array_equal(Va, Vb)


def test_leaves_wider_than_the_kernel_are_rejected(lib):
    # one leaf of 2100 x 2100 (L = 0)
    wl = G.make_gauss3d(n=2100, leaf=4096, tol=1e-6, d=8, cfg=62)
    with pytest.raises(lib.HBACAError) as e:
        run_gpu(lib, wl)
    assert e.value.status == -6
