"""hbaca_apply_noalloc (the apply for callers that cannot allocate) against
hbaca_apply through the C ABI: two calls in a row on the same GPU, the
second on a smaller problem with a smaller rank, each equal to the
allocating entry point's output; complex and adjoint applies too."""
import numpy as np
import pytest

from workloads import generators as G

from _hbtest import run_gpu, say

pytestmark = pytest.mark.gpu


def _check(res, rng, adjoint):
    import torch
    m, n = res.shape(0)
    dt = torch.complex128 if res.is_complex else torch.float64
    nin, nout = (m, n) if adjoint else (n, m)
    w = torch.tensor(rng.standard_normal(nin), device="cuda").to(dt)
    ref = res.apply(w, adjoint=adjoint)
    out = torch.full((nout,), float("nan"), dtype=dt, device="cuda")
    res.apply_noalloc(w, out, adjoint=adjoint)
    torch.cuda.synchronize()
    assert torch.equal(out, ref)
    return ref


def test_noalloc_apply_matches_apply(lib):
    rng = np.random.default_rng(7)
    big = G.make_gauss3d(n=1500, m=1400, leaf=200, tol=1e-8, d=8, cfg=61)
    small = G.make_gauss3d(n=300, m=260, leaf=100, tol=1e-4, d=8, cfg=62)
    r1 = run_gpu(lib, big)
    r2 = run_gpu(lib, small)
    say(f"[noalloc] ranks {r1.rank(0)} then {r2.rank(0)}")
    assert r2.rank(0) < r1.rank(0)
    for res in (r1, r2):
        for adjoint in (False, True):
            _check(res, rng, adjoint)
    cx = run_gpu(lib, G.make_helmholtz_plates(n=800, leaf=200, cfg=63))
    for adjoint in (False, True):
        _check(cx, rng, adjoint)
    _check(r1, rng, False)  # and back to the larger rank
