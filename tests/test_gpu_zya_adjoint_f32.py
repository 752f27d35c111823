"""hbaca_adjoint, the adjoint for FP32 vectors, against hbaca_vjp on the same
vectors widened to FP64.  Widening is exact and the replay is deterministic,
so the FP64 gradients (h and the points) are identical and the w-gradient is
hbaca_vjp's rounded to FP32."""
import pytest

from workloads import generators as G

from _hbtest import run_gpu, say

pytestmark = pytest.mark.gpu


def test_fp32_entry_matches_vjp(lib):
    import torch
    wl = G.make_gauss3d(n=400, m=360, h=0.7, leaf=100, tol=1e-6, d=8, cfg=51)
    say("[adjoint fp32] 360 x 400")
    res = run_gpu(lib, wl, record_tape=2)
    g = torch.Generator(device="cuda").manual_seed(9)
    w = torch.randn(wl["n"], dtype=torch.float32, device="cuda", generator=g)
    yb = torch.randn(wl["m"], dtype=torch.float32, device="cuda", generator=g)
    gw, gh, gX, gY = res.adjoint(w, yb)
    vw, vh, vX, vY = res.vjp(w.double(), yb.double())
    assert gw.dtype == torch.float32 and gh.dtype == torch.float64
    assert torch.equal(gw, vw.float())
    assert torch.equal(gh, vh) and torch.equal(gX, vX) and torch.equal(gY, vY)
    # outputs left out are not formed
    nw, nh, nX, nY = res.adjoint(w, yb, want=("h",))
    assert nw is None and nX is None and nY is None
    assert torch.equal(nh, vh)


def test_fp32_entry_rejects_results_without_frozen_structure(lib):
    import torch
    wl = G.make_gauss3d(n=400, m=360, h=0.7, leaf=100, tol=1e-6, d=8, cfg=51)
    res = run_gpu(lib, wl)  # record_tape = 0
    w = torch.zeros(wl["n"], dtype=torch.float32, device="cuda")
    yb = torch.zeros(wl["m"], dtype=torch.float32, device="cuda")
    with pytest.raises(lib.HBACAError) as e:
        res.adjoint(w, yb)
    assert e.value.status == -1
