"""Frozen-pivot adjoint on the GPU (hbaca_vjp and gaussian_operator) against
the adjoint oracle (oracle/adjoint.py).  The GPU forward run's frozen
structure (every I_k, J_k, pivot order, d_k and merge rank) is first checked
equal to the oracle's; with the same structure the gradients of
<ybar, A~ w> with respect to w, h and the points agree to FP64 rounding of
the two replays.  The task code itself is checked on the CPU by
tests/test_adjoint_host.py."""
import numpy as np
import pytest

from oracle import adjoint as adj
from workloads import generators as G

from _adjhost import records_from_oracle
from _hbtest import run_gpu, say

pytestmark = pytest.mark.gpu


def _same_structure(res, fs):
    """The GPU run recorded the oracle's pivots, d_k and ranks."""
    li, recs, ranks, dm, stride = records_from_oracle(fs)
    for b in range(li.shape[0]):
        g = res.leaf_frozen(b)
        o = recs.reshape(-1, stride)[li[b, 6]:li[b, 6] + li[b, 4]]
        assert g.shape[0] == o.shape[0], (b, g.shape, o.shape)
        assert g.shape[1] == stride
        for k in range(o.shape[0]):
            nI, nJ, dk = (int(x) for x in o[k, :3])
            assert tuple(g[k, :3]) == (nI, nJ, dk), (b, k)
            assert np.array_equal(g[k, 3:3 + nI], o[k, 3:3 + nI]), (b, k)
            assert np.array_equal(g[k, 3 + dm:3 + dm + nJ], o[k, 3 + dm:3 + dm + nJ]), (b, k)
            assert np.array_equal(g[k, 3 + 2 * dm:3 + 2 * dm + dk],
                                  o[k, 3 + 2 * dm:3 + 2 * dm + dk]), (b, k)
        assert res.leaf_info(b)["rank_leaf"] == li[b, 5], b
    assert np.array_equal(res.merge_ranks(), ranks)


def _rel(a, r):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(r)) / np.linalg.norm(np.asarray(r)))


CASES = {
    "gauss3d_400x360": lambda: G.make_gauss3d(n=400, m=360, h=0.7, leaf=100, tol=1e-6, d=8,
                                              cfg=51),
    "gauss3d_ragged_d16": lambda: G.make_gauss3d(n=700, m=650, h=0.6, leaf=90, tol=1e-5, d=16,
                                                 cfg=53),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_vjp_matches_frozen_oracle(lib, name):
    import torch
    wl = CASES[name]()
    say(f"[vjp] {name}: m={wl['m']} n={wl['n']} leaf={wl['leaf']} d={wl['d']}")
    fs = adj.FrozenStructure(wl)
    rng = np.random.default_rng(5105)
    w = rng.standard_normal(wl["n"])
    b = rng.standard_normal(wl["m"])
    _, gw, gh, gX, gY = adj.frozen_gradients(fs, w, b)
    res = run_gpu(lib, wl, record_tape=2)
    assert res.rank() == fs.res.rank
    _same_structure(res, fs)
    wd = torch.tensor(w, device="cuda")
    yb = 2.0 * (res.apply(wd) - torch.tensor(b, device="cuda"))
    hw, hh, hX, hY = res.vjp(wd, yb)
    torch.cuda.synchronize()
    assert _rel(hw.cpu().numpy(), gw) <= 1e-8
    assert abs(hh.item() - gh) <= 1e-8 * abs(gh)
    assert _rel(hX.cpu().numpy(), gX) <= 1e-8
    assert _rel(hY.cpu().numpy(), gY) <= 1e-8
    # only the h-gradient: the other outputs are skipped
    _, h2, x2, y2 = res.vjp(wd, yb, want=("h",))
    assert x2 is None and y2 is None
    assert abs(h2.item() - hh.item()) <= 1e-12 * abs(hh.item())


def test_autograd_function_matches_frozen_oracle(lib):
    import torch
    wl = CASES["gauss3d_400x360"]()
    fs = adj.FrozenStructure(wl)
    rng = np.random.default_rng(77)
    w = rng.standard_normal(wl["n"])
    b = rng.standard_normal(wl["m"])
    L, gw, gh, gX, gY = adj.frozen_gradients(fs, w, b)
    X = torch.tensor(wl["X"], device="cuda", requires_grad=True)
    Y = torch.tensor(wl["Y"], device="cuda", requires_grad=True)
    h = torch.tensor(float(wl["h"]), dtype=torch.float64, device="cuda", requires_grad=True)
    wt = torch.tensor(w, device="cuda", requires_grad=True)
    y = lib.gaussian_operator(X, Y, h, wt, wl["tol"], wl["d"], wl["leaf"],
                              gauss_c=wl.get("gauss_c", 1.0), seed=wl["seed"])
    loss = ((y - torch.tensor(b, device="cuda")) ** 2).sum()
    loss.backward()
    assert abs(loss.item() - L) <= 1e-10 * L
    assert _rel(wt.grad.cpu().numpy(), gw) <= 1e-8
    assert abs(h.grad.item() - gh) <= 1e-8 * abs(gh)
    assert _rel(X.grad.cpu().numpy(), gX) <= 1e-8
    assert _rel(Y.grad.cpu().numpy(), gY) <= 1e-8


def test_recompute_frozen_and_central_differences(lib):
    """hbaca_recompute_frozen at the recorded parameters reproduces the
    forward result; its central differences in h and along a random point
    direction match hbaca_vjp."""
    import torch
    wl = CASES["gauss3d_400x360"]()
    res = run_gpu(lib, wl, record_tape=2)
    X = torch.tensor(wl["X"], device="cuda")
    Y = torch.tensor(wl["Y"], device="cuda")
    h = float(wl["h"])
    c = wl.get("gauss_c", 1.0)
    same = res.recompute_frozen(X, Y, h, c)
    assert same.rank() == res.rank()
    U0, S0, V0 = res.factors(0)
    U1, S1, V1 = same.factors(0)
    ref = torch.linalg.norm((U0 * S0) @ V0.T)
    assert torch.linalg.norm((U1 * S1) @ V1.T - (U0 * S0) @ V0.T) <= 1e-11 * ref
    g = torch.Generator(device="cuda").manual_seed(3)
    w = torch.randn(wl["n"], dtype=torch.float64, device="cuda", generator=g)
    yb = torch.randn(wl["m"], dtype=torch.float64, device="cuda", generator=g)
    _, gh, gX, gY = res.vjp(w, yb)

    def f(Xp, Yp, hp):
        r = res.recompute_frozen(Xp, Yp, hp, c)
        return torch.dot(yb, r.apply(w)).item()

    dh = 1e-4
    c1 = (f(X, Y, h + dh) - f(X, Y, h - dh)) / (2 * dh)
    c2 = (f(X, Y, h + 2 * dh) - f(X, Y, h - 2 * dh)) / (4 * dh)
    assert abs((4 * c1 - c2) / 3 - gh.item()) <= 1e-8 * abs(gh.item())
    PX = torch.randn(X.shape, dtype=torch.float64, device="cuda", generator=g)
    PY = torch.randn(Y.shape, dtype=torch.float64, device="cuda", generator=g)
    an = (torch.sum(gX * PX) + torch.sum(gY * PY)).item()

    def cp(dp):
        return (f(X + dp * PX, Y + dp * PY, h) - f(X - dp * PX, Y - dp * PY, h)) / (2 * dp)

    fd = (4 * cp(1e-4) - cp(2e-4)) / 3
    assert abs(fd - an) <= 1e-8 * abs(an)


def test_reference_size_checks(lib):
    """n = 2000, leaf 250 (the differentiation workload's reference size):
    against the frozen oracle (1e-8), central differences of
    hbaca_recompute_frozen with step 1e-4 in FP64 (1e-5) on h, one random
    direction over all points and 20 random coordinates, and the exact
    dense gradient (1e-3)."""
    import torch
    wl = G.make_gauss3d(n=2000, h=0.7, leaf=250, tol=1e-6, d=8, cfg=5)
    say("[vjp reference] 2000 x 2000, leaf 250")
    fs = adj.FrozenStructure(wl)
    rng = np.random.default_rng(5)
    w = rng.standard_normal(wl["n"])
    b = rng.standard_normal(wl["m"])
    _, gw, gh, gX, gY = adj.frozen_gradients(fs, w, b)
    res = run_gpu(lib, wl, record_tape=2)
    _same_structure(res, fs)
    wd = torch.tensor(w, device="cuda")
    yb = 2.0 * (res.apply(wd) - torch.tensor(b, device="cuda"))
    hw, hh, hX, hY = res.vjp(wd, yb)
    assert _rel(hw.cpu().numpy(), gw) <= 1e-8
    assert abs(hh.item() - gh) <= 1e-8 * abs(gh)
    assert _rel(hX.cpu().numpy(), gX) <= 1e-8
    assert _rel(hY.cpu().numpy(), gY) <= 1e-8
    X = torch.tensor(wl["X"], device="cuda")
    Y = torch.tensor(wl["Y"], device="cuda")
    c = wl.get("gauss_c", 1.0)

    def f(Xp, Yp, hp):
        r = res.recompute_frozen(Xp, Yp, hp, c)
        return torch.dot(yb, r.apply(wd)).item()

    step = 1e-4
    h = float(wl["h"])
    fd = (f(X, Y, h + step) - f(X, Y, h - step)) / (2 * step)
    assert abs(fd - hh.item()) <= 1e-5 * abs(hh.item())
    PX = torch.tensor(rng.standard_normal(wl["X"].shape), device="cuda")
    PY = torch.tensor(rng.standard_normal(wl["Y"].shape), device="cuda")
    fd = (f(X + step * PX, Y + step * PY, h) - f(X - step * PX, Y - step * PY, h)) / (2 * step)
    an = (torch.sum(hX * PX) + torch.sum(hY * PY)).item()
    assert abs(fd - an) <= 1e-5 * abs(an)
    scale = max(hX.abs().max().item(), hY.abs().max().item())
    for _ in range(10):
        for side, G_, P_ in ((0, hX, X), (1, hY, Y)):
            i = int(rng.integers(P_.shape[0]))
            q = int(rng.integers(P_.shape[1]))
            E = torch.zeros_like(P_)
            E[i, q] = step
            if side == 0:
                fd = (f(X + E, Y, h) - f(X - E, Y, h)) / (2 * step)
            else:
                fd = (f(X, Y + E, h) - f(X, Y - E, h)) / (2 * step)
            g = G_[i, q].item()
            assert abs(fd - g) <= 1e-5 * max(abs(g), 1e-3 * scale)
    _, dw, dh, dX, dY = adj.dense_gradients(wl, w, b)
    say(f"  gap to the dense gradient: h {abs(hh.item() - dh) / abs(dh):.1e}, "
        f"X {_rel(hX.cpu().numpy(), dX):.1e}, Y {_rel(hY.cpu().numpy(), dY):.1e}")
    assert abs(hh.item() - dh) <= 1e-3 * abs(dh)
    assert _rel(hX.cpu().numpy(), dX) <= 1e-3
    assert _rel(hY.cpu().numpy(), dY) <= 1e-3


def test_vjp_rejects_results_without_frozen_structure(lib):
    import torch
    wl = CASES["gauss3d_400x360"]()
    res = run_gpu(lib, wl)  # record_tape = 0
    wd = torch.zeros(wl["n"], dtype=torch.float64, device="cuda")
    yb = torch.zeros(wl["m"], dtype=torch.float64, device="cuda")
    with pytest.raises(lib.HBACAError) as e:
        res.vjp(wd, yb)
    assert e.value.status == -1


def test_vjp_full_size_adjoint_geometry(lib):
    """50000 x 50000 (the differentiation workload): the w-gradient equals
    A~^T ybar of the forward factors, every gradient is finite."""
    import torch
    wl = G.make_config("gauss3d_adjoint", 1.0)
    say(f"[vjp full] {wl['m']} x {wl['n']}")
    res = run_gpu(lib, wl, record_tape=2)
    g = torch.Generator(device="cuda").manual_seed(5)
    wd = torch.randn(wl["n"], dtype=torch.float64, device="cuda", generator=g)
    yb = torch.randn(wl["m"], dtype=torch.float64, device="cuda", generator=g)
    hw, hh, hX, hY = res.vjp(wd, yb)
    ref = res.apply(yb, adjoint=True)
    assert torch.allclose(hw, ref, rtol=0, atol=1e-9 * ref.abs().max().item())
    for t in (hh, hX, hY):
        assert torch.isfinite(t).all()
