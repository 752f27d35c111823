"""The compressed operator applied to vectors on the GPU (hbaca_apply) and
its autograd wrapper: y = U diag(S) Vh^H w and the w-gradient
Vh diag(S) U^H ybar, against plain torch products of the copied factors."""
import numpy as np
import pytest

from workloads import generators as G

from _hbtest import run_gpu, say

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("name", ["gauss3d", "helmholtz"])
def test_apply_and_adjoint_match_factor_products(lib, name):
    import torch
    wl = G.make_config(name, 0.05)
    say(f"[apply] {name} {wl['m']} x {wl['n']}")
    res = run_gpu(lib, wl)
    U, S, Vh = res.factors(0)
    dt = U.dtype
    g = torch.Generator(device="cuda").manual_seed(77)
    w = torch.randn(wl["n"], dtype=torch.float64, device="cuda", generator=g).to(dt)
    z = torch.randn(wl["m"], dtype=torch.float64, device="cuda", generator=g).to(dt)
    y = res.apply(w)
    y_ref = U @ (S.to(dt) * (Vh.conj().T @ w))
    assert torch.allclose(y, y_ref, rtol=0, atol=1e-11 * y_ref.abs().max().item())
    wt = res.apply(z, adjoint=True)
    wt_ref = Vh @ (S.to(dt) * (U.conj().T @ z))
    assert torch.allclose(wt, wt_ref, rtol=0, atol=1e-11 * wt_ref.abs().max().item())
    # <A w, z> = <w, A^H z>, to rounding relative to the norms involved
    lhs = torch.vdot(z, y).item()
    rhs = torch.vdot(wt, w).item()
    scale = (torch.linalg.norm(z) * torch.linalg.norm(y)
             + torch.linalg.norm(wt) * torch.linalg.norm(w)).item()
    assert abs(lhs - rhs) <= 1e-12 * scale


def test_autograd_w_gradient(lib):
    import torch
    wl = G.make_config("gauss3d", 0.1)
    res = run_gpu(lib, wl)
    op = lib.operator(res)
    w = torch.randn(wl["n"], dtype=torch.float64, device="cuda", requires_grad=True)
    b = torch.randn(wl["m"], dtype=torch.float64, device="cuda")
    loss = ((op(w) - b) ** 2).sum()
    loss.backward()
    r = res.apply(w.detach()) - b
    g_ref = 2 * res.apply(r, adjoint=True)
    assert torch.allclose(w.grad, g_ref, rtol=0, atol=1e-12 * g_ref.abs().max().item())
    assert np.isfinite(loss.item())
