"""Pins for the frozen-pivot adjoint oracle (oracle/adjoint.py): the frozen
replay reproduces the forward oracle's operator at the recorded parameters,
its automatic derivatives agree with central finite differences of the same
frozen map, the w-gradient has its closed form, and the gradients stay close
to those of the exact dense loss ||A w - b||^2 (the truncation level)."""
import numpy as np
import pytest
import torch

from oracle import adjoint as adj
from workloads import generators as G


@pytest.fixture(scope="module")
def case():
    wl = G.make_gauss3d(n=400, m=360, h=0.7, leaf=100, tol=1e-6, d=8, cfg=51)
    fs = adj.FrozenStructure(wl)
    rng = np.random.default_rng(5105)
    w = rng.standard_normal(wl["n"])
    b = rng.standard_normal(wl["m"])
    return wl, fs, w, b


def _loss(fs, X, Y, h, w, b):
    t = lambda a: torch.tensor(a, dtype=torch.float64)  # noqa: E731
    return float(adj.frozen_loss(fs, t(X), t(Y), t(h), t(w), t(b)))


def test_frozen_replay_reproduces_forward(case):
    wl, fs, _, _ = case
    f64 = dict(dtype=torch.float64)
    U, S, V = adj.frozen_operator(fs, torch.tensor(wl["X"], **f64), torch.tensor(wl["Y"], **f64),
                                  torch.tensor(wl["h"], **f64))
    assert S.shape[0] == fs.res.rank
    At = (U * S[None, :]) @ V
    Ao = fs.res.dense()
    assert np.linalg.norm(At.numpy() - Ao) <= 1e-11 * np.linalg.norm(Ao)


def test_gradients_match_central_differences(case):
    wl, fs, w, b = case
    L, gw, gh, gX, gY = adj.frozen_gradients(fs, w, b)
    X, Y, h = wl["X"], wl["Y"], wl["h"]
    # central differences with step 1e-4 (error O(step^2)), and their
    # Richardson extrapolation from steps 1e-4 and 2e-4 (error O(step^4))
    def central(dh):
        return (_loss(fs, X, Y, h + dh, w, b) - _loss(fs, X, Y, h - dh, w, b)) / (2 * dh)

    f1, f2 = central(1e-4), central(2e-4)
    assert abs(f1 - gh) <= 1e-5 * abs(gh)
    assert abs((4 * f1 - f2) / 3 - gh) <= 1e-8 * abs(gh)
    rng = np.random.default_rng(51051)
    PX = rng.standard_normal(X.shape)
    PY = rng.standard_normal(Y.shape)
    dp = 1e-5
    fd_p = (_loss(fs, X + dp * PX, Y + dp * PY, h, w, b)
            - _loss(fs, X - dp * PX, Y - dp * PY, h, w, b)) / (2 * dp)
    an_p = float(np.sum(gX * PX) + np.sum(gY * PY))
    assert abs(fd_p - an_p) <= 1e-6 * abs(an_p)
    # one coordinate of one row point and one column point (Richardson from
    # steps 1e-3 and 2e-3, large enough that rounding of L stays negligible)
    for g, which in ((gX, 0), (gY, 1)):
        E = np.zeros(X.shape if which == 0 else Y.shape)
        E[17, 1] = 1.0

        def c(dd):
            if which == 0:
                return (_loss(fs, X + dd * E, Y, h, w, b) - _loss(fs, X - dd * E, Y, h, w, b)) / (2 * dd)
            return (_loss(fs, X, Y + dd * E, h, w, b) - _loss(fs, X, Y - dd * E, h, w, b)) / (2 * dd)

        fd = (4 * c(1e-3) - c(2e-3)) / 3
        assert abs(fd - g[17, 1]) <= 1e-6 * abs(g[17, 1]) + 1e-12 * L


def test_w_gradient_closed_form(case):
    _, fs, w, b = case
    L, gw, _, _, _ = adj.frozen_gradients(fs, w, b)
    A = fs.res.dense()
    r = A @ w - b
    assert abs(L - r @ r) <= 1e-10 * (r @ r)
    assert np.allclose(gw, 2 * A.T @ r, rtol=0, atol=1e-9 * np.abs(2 * A.T @ r).max())


def test_close_to_dense_gradients(case):
    wl, fs, w, b = case
    _, gw, gh, gX, gY = adj.frozen_gradients(fs, w, b)
    _, dw, dh, dX, dY = adj.dense_gradients(wl, w, b)
    assert abs(gh - dh) <= 1e-3 * abs(dh)
    assert np.linalg.norm(gX - dX) <= 1e-3 * np.linalg.norm(dX)
    assert np.linalg.norm(gY - dY) <= 1e-3 * np.linalg.norm(dY)
    assert np.linalg.norm(gw - dw) <= 1e-3 * np.linalg.norm(dw)
