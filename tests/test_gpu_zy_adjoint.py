"""Frozen-pivot adjoint on the GPU (hbaca_vjp, hbaca_recompute_frozen and
gaussian_operator).

* The recorded frozen structure agrees with the pivot tape the leaf kernel
  writes (a check of the recording itself).
* Central differences of the GPU's own frozen map (hbaca_recompute_frozen)
  match hbaca_vjp: this needs no reference.
* The GPU run records the oracle's frozen structure (every I_k, J_k,
  pivot order, d_k and merge rank), and the gradients
  match the adjoint oracle (oracle/adjoint.py) to 1e-8.  The two runs must
  freeze the same structure on these cases: a difference fails the test and
  names the first leaf and iteration where they part.

The task code itself is checked on the CPU by tests/test_adjoint_host.py."""
import numpy as np
import pytest

from oracle import adjoint as adj
from workloads import generators as G

from _adjhost import records_from_oracle
from _hbtest import run_gpu, say

pytestmark = pytest.mark.gpu


def _rel(a, r):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(r)) / np.linalg.norm(np.asarray(r)))


def _records_match_tape(res):
    """Each iteration record holds the rows I_k(1:d_k) and columns
    J_k(pivots) of the pivot tape, in the tape's order."""
    for b in range(res.nleaves):
        rec = res.leaf_frozen(b)
        tape = res.leaf_tape(b)
        info = res.leaf_info(b)
        dm = (rec.shape[1] - 3) // 3
        r = 0
        assert rec.shape[0] == info["iters"], b
        for k in range(rec.shape[0]):
            nI, nJ, dk = (int(x) for x in rec[k, :3])
            assert 0 <= dk <= min(nI, nJ) <= dm, (b, k)
            assert dk == tape["dk"][k], (b, k)
            I = rec[k, 3:3 + nI]
            J = rec[k, 3 + dm:3 + dm + nJ]
            piv = rec[k, 3 + 2 * dm:3 + 2 * dm + dk]
            assert np.array_equal(I[:dk], tape["rows"][r:r + dk]), (b, k)
            assert np.array_equal(J[piv], tape["cols"][r:r + dk]), (b, k)
            r += dk
        assert r == info["rank_baca"], b


def _same_structure(res, fs):
    """'' if the GPU run recorded the oracle's frozen structure, else where
    they first differ."""
    li, recs, ranks, dm, stride = records_from_oracle(fs)
    for b in range(li.shape[0]):
        g = res.leaf_frozen(b)
        o = recs.reshape(-1, stride)[li[b, 6]:li[b, 6] + li[b, 4]]
        if g.shape != o.shape:
            return f"leaf {b}: {g.shape[0]} iterations, oracle {o.shape[0]}"
        for k in range(o.shape[0]):
            nI, nJ, dk = (int(x) for x in o[k, :3])
            same = (tuple(g[k, :3]) == (nI, nJ, dk)
                    and np.array_equal(g[k, 3:3 + nI], o[k, 3:3 + nI])
                    and np.array_equal(g[k, 3 + dm:3 + dm + nJ], o[k, 3 + dm:3 + dm + nJ])
                    and np.array_equal(g[k, 3 + 2 * dm:3 + 2 * dm + dk],
                                       o[k, 3 + 2 * dm:3 + 2 * dm + dk]))
            if not same:
                return f"leaf {b}, iteration {k}"
        if res.leaf_info(b)["rank_leaf"] != li[b, 5]:
            return f"leaf {b}: re-compression rank"
    if not np.array_equal(res.merge_ranks(), ranks):
        return "merge ranks"
    return ""


def _fd_checks(res, wl, wd, yb, grads, rng, ncoord, rtol, richardson, value_noise=0.0):
    """Central differences of the GPU's frozen map against hbaca_vjp.
    value_noise > 0 allows, in each difference, the rounding of the map's
    value: value_noise * |f| over the step (|f| is large at full size)."""
    import torch
    _, hh, hX, hY = grads
    X = torch.tensor(wl["X"], device="cuda")
    Y = torch.tensor(wl["Y"], device="cuda")
    c = wl.get("gauss_c", 1.0)
    h = float(wl["h"])

    def f(Xp, Yp, hp):
        r = res.recompute_frozen(Xp, Yp, hp, c)
        return torch.dot(yb, r.apply(wd)).item()

    def central(fun, step):
        d1 = (fun(step) - fun(-step)) / (2 * step)
        if not richardson:
            return d1
        d2 = (fun(2 * step) - fun(-2 * step)) / (4 * step)
        return (4 * d1 - d2) / 3

    step = 1e-4
    allow = value_noise * abs(f(X, Y, h)) / step if value_noise > 0 else 0.0
    fd = central(lambda s: f(X, Y, h + s), step)
    assert abs(fd - hh.item()) <= rtol * abs(hh.item()) + allow
    PX = torch.tensor(rng.standard_normal(wl["X"].shape), device="cuda")
    PY = torch.tensor(rng.standard_normal(wl["Y"].shape), device="cuda")
    fd = central(lambda s: f(X + s * PX, Y + s * PY, h), step)
    an = (torch.sum(hX * PX) + torch.sum(hY * PY)).item()
    assert abs(fd - an) <= rtol * abs(an) + allow
    scale = max(hX.abs().max().item(), hY.abs().max().item())
    worst = 0.0
    for _ in range(ncoord):
        for side, G_, P_ in ((0, hX, X), (1, hY, Y)):
            i = int(rng.integers(P_.shape[0]))
            q = int(rng.integers(P_.shape[1]))
            E = torch.zeros_like(P_)
            E[i, q] = 1.0
            if side == 0:
                fd = central(lambda s: f(X + s * E, Y, h), step)
            else:
                fd = central(lambda s: f(X, Y + s * E, h), step)
            g = G_[i, q].item()
            worst = max(worst, abs(fd - g) / max(abs(g), 1e-3 * scale))
            assert abs(fd - g) <= rtol * max(abs(g), 1e-3 * scale) + allow
    if value_noise > 0:
        say(f"  finite differences: worst coordinate difference {worst:.1e} of the gradient "
            f"scale; the value's rounding allows {allow:.1e} absolute")


CASES = {
    "gauss3d_400x360": lambda: G.make_gauss3d(n=400, m=360, h=0.7, leaf=100, tol=1e-6, d=8,
                                              cfg=51),
    "gauss3d_ragged_d16": lambda: G.make_gauss3d(n=700, m=650, h=0.6, leaf=90, tol=1e-5, d=16,
                                                 cfg=53),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_vjp(lib, name):
    import torch
    wl = CASES[name]()
    say(f"[vjp] {name}: m={wl['m']} n={wl['n']} leaf={wl['leaf']} d={wl['d']}")
    res = run_gpu(lib, wl, record_tape=2)
    _records_match_tape(res)
    rng = np.random.default_rng(5105)
    w = rng.standard_normal(wl["n"])
    b = rng.standard_normal(wl["m"])
    wd = torch.tensor(w, device="cuda")
    yb = 2.0 * (res.apply(wd) - torch.tensor(b, device="cuda"))
    grads = res.vjp(wd, yb)
    hw, hh, hX, hY = grads
    torch.cuda.synchronize()
    # w enters linearly: its gradient is A~^T ybar of the forward factors
    ref = res.apply(yb, adjoint=True)
    sig1 = res.factors(0)[1][0].item()
    assert torch.linalg.norm(hw - ref).item() <= 1e-10 * sig1 * torch.linalg.norm(yb).item()
    # only the h-gradient: the other outputs are skipped
    _, h2, x2, y2 = res.vjp(wd, yb, want=("h",))
    assert x2 is None and y2 is None
    assert abs(h2.item() - hh.item()) <= 1e-12 * abs(hh.item())
    _fd_checks(res, wl, wd, yb, grads, rng, ncoord=2, rtol=1e-6, richardson=True)
    fs = adj.FrozenStructure(wl)
    diff = _same_structure(res, fs)
    assert not diff, f"the GPU run and the oracle froze different structures ({diff})"
    _, gw, gh, gX, gY = adj.frozen_gradients(fs, w, b)
    assert _rel(hw.cpu().numpy(), gw) <= 1e-8
    assert abs(hh.item() - gh) <= 1e-8 * abs(gh)
    assert _rel(hX.cpu().numpy(), gX) <= 1e-8
    assert _rel(hY.cpu().numpy(), gY) <= 1e-8


def test_autograd_function_matches_vjp(lib):
    """gaussian_operator's backward returns hbaca_vjp of the same forward run
    (the compression is deterministic, so a second run freezes the same
    structure)."""
    import torch
    wl = CASES["gauss3d_400x360"]()
    rng = np.random.default_rng(77)
    w = rng.standard_normal(wl["n"])
    b = rng.standard_normal(wl["m"])
    X = torch.tensor(wl["X"], device="cuda", requires_grad=True)
    Y = torch.tensor(wl["Y"], device="cuda", requires_grad=True)
    h = torch.tensor(float(wl["h"]), dtype=torch.float64, device="cuda", requires_grad=True)
    wt = torch.tensor(w, device="cuda", requires_grad=True)
    bt = torch.tensor(b, device="cuda")
    y = lib.gaussian_operator(X, Y, h, wt, wl["tol"], wl["d"], wl["leaf"],
                              gauss_c=wl.get("gauss_c", 1.0), seed=wl["seed"])
    loss = ((y - bt) ** 2).sum()
    loss.backward()
    res = run_gpu(lib, wl, record_tape=2)
    wd = wt.detach()
    yb = 2.0 * (res.apply(wd) - bt)
    assert torch.allclose(y.detach(), res.apply(wd), rtol=0, atol=0)
    gw, gh, gX, gY = res.vjp(wd, yb)
    for a, r in ((wt.grad, gw), (h.grad.reshape(1), gh), (X.grad, gX), (Y.grad, gY)):
        assert torch.allclose(a, r, rtol=0, atol=1e-12 * r.abs().max().item())


def test_recompute_frozen_reproduces_the_forward_run(lib):
    import torch
    wl = CASES["gauss3d_400x360"]()
    res = run_gpu(lib, wl, record_tape=2)
    X = torch.tensor(wl["X"], device="cuda")
    Y = torch.tensor(wl["Y"], device="cuda")
    same = res.recompute_frozen(X, Y, float(wl["h"]), wl.get("gauss_c", 1.0))
    assert same.rank() == res.rank()
    U0, S0, V0 = res.factors(0)
    U1, S1, V1 = same.factors(0)
    ref = torch.linalg.norm((U0 * S0) @ V0.T)
    assert torch.linalg.norm((U1 * S1) @ V1.T - (U0 * S0) @ V0.T) <= 1e-11 * ref
    # the recomputed result carries the frozen structure too
    wd = torch.ones(wl["n"], dtype=torch.float64, device="cuda")
    yb = torch.ones(wl["m"], dtype=torch.float64, device="cuda")
    g0 = res.vjp(wd, yb)
    g1 = same.vjp(wd, yb)
    for a, r in zip(g0, g1):
        assert torch.allclose(a, r, rtol=0, atol=1e-10 * r.abs().max().item())


def test_reference_size_checks(lib):
    """n = 2000, leaf 250 (the differentiation workload's reference size):
    central differences of hbaca_recompute_frozen with step 1e-4 in FP64
    (1e-5) on h, one random direction over all points and 20 random
    coordinates; with the oracle's frozen structure, the frozen oracle
    (1e-8) and the exact dense gradient (1e-3)."""
    import torch
    wl = G.make_gauss3d(n=2000, h=0.7, leaf=250, tol=1e-6, d=8, cfg=5)
    say("[vjp reference] 2000 x 2000, leaf 250")
    res = run_gpu(lib, wl, record_tape=2)
    _records_match_tape(res)
    rng = np.random.default_rng(5)
    w = rng.standard_normal(wl["n"])
    b = rng.standard_normal(wl["m"])
    wd = torch.tensor(w, device="cuda")
    yb = 2.0 * (res.apply(wd) - torch.tensor(b, device="cuda"))
    grads = res.vjp(wd, yb)
    hw, hh, hX, hY = grads
    _fd_checks(res, wl, wd, yb, grads, rng, ncoord=20, rtol=1e-5, richardson=False)
    fs = adj.FrozenStructure(wl)
    diff = _same_structure(res, fs)
    assert not diff, f"the GPU run and the oracle froze different structures ({diff})"
    _, gw, gh, gX, gY = adj.frozen_gradients(fs, w, b)
    assert _rel(hw.cpu().numpy(), gw) <= 1e-8
    assert abs(hh.item() - gh) <= 1e-8 * abs(gh)
    assert _rel(hX.cpu().numpy(), gX) <= 1e-8
    assert _rel(hY.cpu().numpy(), gY) <= 1e-8
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
    A~^T ybar of the forward factors, every gradient is finite, and central
    differences (step 1e-4) of the GPU's frozen map agree with the VJP on h,
    one random direction over all points and 20 coordinates (10 row, 10
    column), to 1e-5 relative plus the rounding of the map's value (taken
    as 1e-14 |f|) over the step, the part of each difference that no step
    size removes."""
    import torch
    wl = G.make_config("gauss3d_adjoint", 1.0)
    say(f"[vjp full] {wl['m']} x {wl['n']}")
    res = run_gpu(lib, wl, record_tape=2)
    g = torch.Generator(device="cuda").manual_seed(5)
    wd = torch.randn(wl["n"], dtype=torch.float64, device="cuda", generator=g)
    yb = torch.randn(wl["m"], dtype=torch.float64, device="cuda", generator=g)
    import time
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    hw, hh, hX, hY = res.vjp(wd, yb)
    torch.cuda.synchronize()
    say(f"  rank {res.rank()}, forward {res.stats()['ms_total']:.1f} ms, "
        f"hbaca_vjp {1e3 * (time.perf_counter() - t0):.1f} ms")
    ref = res.apply(yb, adjoint=True)
    sig1 = res.factors(0)[1][0].item()
    assert torch.linalg.norm(hw - ref).item() <= 1e-10 * sig1 * torch.linalg.norm(yb).item()
    for t in (hh, hX, hY):
        assert torch.isfinite(t).all()
    say("  finite differences: h, one direction, 20 coordinates")
    _fd_checks(res, wl, wd, yb, (hw, hh, hX, hY), np.random.default_rng(7), ncoord=10, rtol=1e-5,
               richardson=False, value_noise=1e-14)
