"""Adjoint of the compressed operator with frozen pivots and ranks (oracle).

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle``.

H-BACA output depends on the kernel parameters only through the entries it
samples: every leaf evaluates A(:, J_k) and A(I_k, :) for its blocks I_k,
J_k.  With the pivots (I_k, J_k, the pivot order of QR(W_k, eps) and d_k)
and every truncation rank frozen from a forward run, the compressed
operator A~(theta) is a smooth function of those entries, hence of
theta = (h, row points, column points).  This module replays that frozen
pipeline in PyTorch FP64 on the CPU, step by step as the forward oracle
computes it:

* leaf BACA (Algorithm 2): C_k = A(:, J_k) - U V(:, J_k),
  R_k = A(I_k, :) - U(I_k, :) V, W_k = C_k(I_k, :), U_k = C_k(:, Jbar),
  V_k = T11^{-1} Q1^H R_k (eqs. (8)-(9)) with the recorded pivot order and
  d_k (the QR of the pivoted W_k is taken without further pivoting; U_k V_k
  does not depend on the sign convention of that QR);
* the SVD re-compression truncated at the recorded leaf rank;
* the merges (Algorithm 3, eqs. (14)-(15)) truncated at the recorded ranks,
  in the forward oracle's order;

and differentiates L = ||A~ w - b||^2 with PyTorch's automatic
differentiation.  Gaussian kernels only (the differentiation workload has a
learnable length scale).

Parity: pinned in tests/test_oracle_adjoint.py against the forward oracle
(same operator at the recorded parameters), central finite differences of
the frozen replay, and the gradient of the dense loss ||A w - b||^2.
"""
from __future__ import annotations

import numpy as np
import torch

from .hbaca import cluster_tree, hbaca, tree_levels


def gauss_block(X, Y, h, c, I, J):
    """exp(-|x_i - y_j|^2 / (c h^2)) for index arrays I, J (torch, FP64)."""
    d = X[I][:, None, :] - Y[J][None, :, :]
    return torch.exp(-(d * d).sum(-1) / (c * h * h))


def _leaf_replay(blk, m0, n0, iters):
    """Leaf BACA with frozen pivots; returns U (m0 x r), V (r x n0)."""
    U = torch.zeros((m0, 0), dtype=torch.float64)
    V = torch.zeros((0, n0), dtype=torch.float64)
    allr = np.arange(m0)
    allc = np.arange(n0)
    for it in iters:
        dk = int(it["dk"])
        if dk == 0:
            break
        J = np.asarray(it["Jblock"], dtype=np.int64)
        I = np.asarray(it["Iblock"], dtype=np.int64)
        piv = np.asarray(it["piv"], dtype=np.int64)[:dk]
        C = blk(allr, J) - U @ V[:, J]
        R = blk(I, allc) - U[I, :] @ V
        W = C[I, :]
        Q1, T11 = torch.linalg.qr(W[:, piv])
        Uk = C[:, piv]
        Vk = torch.linalg.solve_triangular(T11, Q1.T @ R, upper=True)
        U = torch.cat([U, Uk], dim=1)
        V = torch.cat([V, Vk], dim=0)
    return U, V


def _empty(m, n):
    z = torch.zeros(0, dtype=torch.float64)
    return (torch.zeros((m, 0), dtype=torch.float64), z, torch.zeros((0, n), dtype=torch.float64))


def _recompress(U, V, r):
    if r == 0 or U.shape[1] == 0:
        return _empty(U.shape[0], V.shape[1])
    QU, TU = torch.linalg.qr(U)
    QV, TV = torch.linalg.qr(V.T)
    Xs, S, Yh = torch.linalg.svd(TU @ TV.T, full_matrices=False)
    return QU @ Xs[:, :r], S[:r], Yh[:r, :] @ QV.T


def _merge_h(b1, b2, r):
    U1, S1, V1 = b1
    U2, S2, V2 = b2
    r1 = S1.shape[0]
    if r == 0 or r1 + S2.shape[0] == 0:
        return _empty(U1.shape[0], V1.shape[1] + V2.shape[1])
    Q, R = torch.linalg.qr(torch.cat([U1 * S1[None, :], U2 * S2[None, :]], dim=1))
    Xs, S, Yh = torch.linalg.svd(R, full_matrices=False)
    Y = Yh[:r, :]
    return Q @ Xs[:, :r], S[:r], torch.cat([Y[:, :r1] @ V1, Y[:, r1:] @ V2], dim=1)


def _merge_v(b1, b2, r):
    U1, S1, V1 = b1
    U2, S2, V2 = b2
    r1 = S1.shape[0]
    if r == 0 or r1 + S2.shape[0] == 0:
        return _empty(U1.shape[0] + U2.shape[0], V1.shape[1])
    Q, R = torch.linalg.qr(torch.cat([S1[:, None] * V1, S2[:, None] * V2], dim=0).T)
    Xs, S, Zh = torch.linalg.svd(R.T, full_matrices=False)
    Xk = Xs[:, :r]
    return torch.cat([U1 @ Xk[:r1], U2 @ Xk[r1:]], dim=0), S[:r], Zh[:r, :] @ Q.T


class FrozenStructure:
    """Pivots and ranks of one forward H-BACA run (Gaussian kernel)."""

    def __init__(self, wl: dict):
        from .entries import EntrySource
        src = EntrySource(wl)
        self.wl = wl
        self.res = hbaca(src, wl["m"], wl["n"], wl["tol"], wl["d"], wl["leaf"], wl["seed"])
        self.L = tree_levels(wl["m"], wl["n"], wl["leaf"])
        self.rows = cluster_tree(wl["m"], self.L)[self.L]
        self.cols = cluster_tree(wl["n"], self.L)[self.L]


def frozen_operator(fs: FrozenStructure, X, Y, h):
    """(U, S, V) of the frozen pipeline at points X, Y and width h (torch)."""
    c = float(fs.wl.get("gauss_c", 1.0))
    nb = 1 << fs.L
    cur = {}
    for t in range(nb):
        ra, rs = fs.rows[t]
        for v in range(nb):
            ca, cs = fs.cols[v]
            info = fs.res.leaf_info[t * nb + v]

            def blk(I, J, ra=ra, ca=ca):
                return gauss_block(X, Y, h, c, np.asarray(I) + ra, np.asarray(J) + ca)

            U, V = _leaf_replay(blk, rs, cs, info["iters"])
            cur[(t, v)] = _recompress(U, V, int(info["rank"]))
    ranks = {k: list(v) for k, v in fs.res.ranks.items()}
    for lev in range(1, fs.L + 1):
        nbl = 1 << (fs.L - lev)
        nxt = {}
        hr = iter(ranks[lev - 0.5])
        vr = iter(ranks[lev])
        for t in range(nbl):
            for v in range(nbl):
                hs = [_merge_h(cur[(2 * t + i, 2 * v)], cur[(2 * t + i, 2 * v + 1)], next(hr))
                      for i in range(2)]
                nxt[(t, v)] = _merge_v(hs[0], hs[1], next(vr))
        cur = nxt
    return cur[(0, 0)]


def frozen_loss(fs: FrozenStructure, X, Y, h, w, b):
    """L = ||U diag(S) V w - b||^2 of the frozen compressed operator."""
    U, S, V = frozen_operator(fs, X, Y, h)
    y = U @ (S * (V @ w))
    return ((y - b) ** 2).sum()


def frozen_gradients(fs: FrozenStructure, w: np.ndarray, b: np.ndarray):
    """(L, dL/dw, dL/dh, dL/dX, dL/dY) of the frozen compressed operator."""
    X = torch.tensor(fs.wl["X"], dtype=torch.float64, requires_grad=True)
    Y = torch.tensor(fs.wl["Y"], dtype=torch.float64, requires_grad=True)
    h = torch.tensor(float(fs.wl["h"]), dtype=torch.float64, requires_grad=True)
    wt = torch.tensor(w, dtype=torch.float64, requires_grad=True)
    bt = torch.tensor(b, dtype=torch.float64)
    L = frozen_loss(fs, X, Y, h, wt, bt)
    L.backward()
    return (float(L.detach()), wt.grad.numpy(), float(h.grad), X.grad.numpy(), Y.grad.numpy())


def dense_gradients(wl: dict, w: np.ndarray, b: np.ndarray):
    """The same quantities for the exact dense loss ||A w - b||^2."""
    c = float(wl.get("gauss_c", 1.0))
    X = torch.tensor(wl["X"], dtype=torch.float64, requires_grad=True)
    Y = torch.tensor(wl["Y"], dtype=torch.float64, requires_grad=True)
    h = torch.tensor(float(wl["h"]), dtype=torch.float64, requires_grad=True)
    wt = torch.tensor(w, dtype=torch.float64, requires_grad=True)
    A = gauss_block(X, Y, h, c, np.arange(wl["m"]), np.arange(wl["n"]))
    L = ((A @ wt - torch.tensor(b, dtype=torch.float64)) ** 2).sum()
    L.backward()
    return (float(L.detach()), wt.grad.numpy(), float(h.grad), X.grad.numpy(), Y.grad.numpy())
