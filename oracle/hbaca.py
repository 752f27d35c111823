"""Hierarchical merge of leaf factors, H-BACA (Algorithm 3), oracle side.

* Cluster trees (Algorithm 3, first line; Section "Parallel Hierarchical
  Low-Rank Merge"): L-level binary trees on [0, m) and [0, n); a node of size
  s has children of sizes ceil(s/2) and floor(s/2).  Reading: one L for both
  trees, the smallest L >= 0 with leaf * 2^L >= max(m, n), lowered until
  2^L <= min(m, n) so no node is empty.  Leaf (t, v) has id b = t * 2^L + v.
* Leaf compression: BACA (Algorithm 2) then the SVD re-compression of the
  Section "Blocked Adaptive Cross Approximation": QR(U), QR(V^H), truncated
  SVD of T_U T_V^H.  Reading: always applied (the paper takes it as BACA's
  output).
* Merges, level l = 1..L: for every parent (tau, nu) first the two horizontal
  merges of eqs. (14)-(15) (rows tau_i, columns nu_1 | nu_2), then the vertical
  merge of the results.  SVD(X, eps) is computed as a thin QR followed by the
  SVD of the small triangular factor; for the short-fat vertical factor the
  QR is taken of its conjugate transpose.
* eps-rank: r = min{k : sigma_{k+1} < eps sigma_1}, relative to the block's
  own sigma_1 (Section "Notation"); r = 0 when sigma_1 = 0.

Blocks are triples (U, S, V) with A_block ~ U diag(S) V, U m x r, V r x n.
QR and SVD of the small factors use NumPy's LAPACK routines as steps.
"""
from __future__ import annotations

import numpy as np

from .baca import baca_leaf
from .entries import EntrySource
from .splitmix import first_column_block


def tree_levels(m: int, n: int, leaf: int) -> int:
    L = 0
    big = max(m, n)
    while leaf * (1 << L) < big:
        L += 1
    while L > 0 and (1 << L) > min(m, n):
        L -= 1
    return L


def cluster_tree(size: int, L: int) -> list[list[tuple[int, int]]]:
    """Nodes (offset, size) per depth 0..L; depth L are the leaves."""
    levels = [[(0, size)]]
    for _ in range(L):
        nxt = []
        for a, s in levels[-1]:
            h = (s + 1) // 2
            nxt.append((a, h))
            nxt.append((a + h, s - h))
        levels.append(nxt)
    return levels


def eps_rank(S: np.ndarray, eps: float) -> int:
    if S.size == 0 or not S[0] > 0.0:
        return 0
    r = 0
    while r < S.size and S[r] >= eps * S[0]:
        r += 1
    return r


def _empty(m, n, dt):
    return (np.zeros((m, 0), dt), np.zeros(0), np.zeros((0, n), dt))


def recompress(U: np.ndarray, V: np.ndarray, eps: float):
    """SVD re-compression of a BACA result U V (m0 x r, r x n0)."""
    m, r = U.shape
    n = V.shape[1]
    if r == 0:
        return _empty(m, n, U.dtype)
    QU, TU = np.linalg.qr(U)
    QV, TV = np.linalg.qr(V.conj().T)
    M = TU @ TV.conj().T
    X, S, Yh = np.linalg.svd(M)
    k = eps_rank(S, eps)
    return (QU @ X[:, :k], S[:k].copy(), Yh[:k, :] @ QV.conj().T)


def merge_horizontal(b1, b2, eps: float):
    """Blocks sharing rows: [A1, A2] from A_i = U_i S_i V_i (eqs. (14)-(15))."""
    U1, S1, V1 = b1
    U2, S2, V2 = b2
    r1, r2 = S1.size, S2.size
    m, n1, n2 = U1.shape[0], V1.shape[1], V2.shape[1]
    if r1 + r2 == 0:
        return _empty(m, n1 + n2, U1.dtype)
    Ubar = np.concatenate([U1 * S1[None, :], U2 * S2[None, :]], axis=1)
    Q, R = np.linalg.qr(Ubar)
    X, S, Yh = np.linalg.svd(R, full_matrices=False)
    k = eps_rank(S, eps)
    Y = Yh[:k, :]
    V = np.concatenate([Y[:, :r1] @ V1, Y[:, r1:] @ V2], axis=1)
    return (Q @ X[:, :k], S[:k].copy(), V)


def merge_vertical(b1, b2, eps: float):
    """Blocks sharing columns: [A1; A2] (Algorithm 3, vertical step)."""
    U1, S1, V1 = b1
    U2, S2, V2 = b2
    r1, r2 = S1.size, S2.size
    m1, m2, n = U1.shape[0], U2.shape[0], V1.shape[1]
    if r1 + r2 == 0:
        return _empty(m1 + m2, n, U1.dtype)
    Vbar = np.concatenate([S1[:, None] * V1, S2[:, None] * V2], axis=0)
    Q, R = np.linalg.qr(Vbar.conj().T)           # Vbar = R^H Q^H
    X, S, Zh = np.linalg.svd(R.conj().T, full_matrices=False)
    k = eps_rank(S, eps)
    Xk = X[:, :k]
    U = np.concatenate([U1 @ Xk[:r1], U2 @ Xk[r1:]], axis=0)
    return (U, S[:k].copy(), Zh[:k, :] @ Q.conj().T)


def merge_tree(leaves: dict, L: int, eps: float, ranks: dict | None = None,
               flops: list | None = None):
    """Merge leaf blocks {(t, v): (U, S, V)} at depth L up to the root."""
    cur = leaves
    for lev in range(1, L + 1):
        depth = L - lev
        nxt = {}
        nb = 1 << depth
        for t in range(nb):
            for v in range(nb):
                hs = []
                for i in range(2):
                    ti = 2 * t + i
                    a, b = cur[(ti, 2 * v)], cur[(ti, 2 * v + 1)]
                    if flops is not None:
                        m = a[0].shape[0]
                        k = a[1].size + b[1].size
                        flops.append(2 * m * k * k + 2 * m * k * k)
                    hs.append(merge_horizontal(a, b, eps))
                if flops is not None:
                    n = hs[0][2].shape[1]
                    k = hs[0][1].size + hs[1][1].size
                    flops.append(2 * n * k * k + 2 * n * k * k)
                nxt[(t, v)] = merge_vertical(hs[0], hs[1], eps)
                if ranks is not None:
                    ranks.setdefault(lev, []).append(nxt[(t, v)][1].size)
                    ranks.setdefault(lev - 0.5, []).extend(h[1].size for h in hs)
        cur = nxt
    return cur[(0, 0)]


class HBACAResult:
    def __init__(self, U, S, V, L, leaf_info, ranks, ops):
        self.U, self.S, self.V = U, S, V
        self.L = L
        self.leaf_info = leaf_info
        self.ranks = ranks
        self.ops = ops

    @property
    def rank(self):
        return self.S.size

    def dense(self):
        return (self.U * self.S[None, :]) @ self.V


def hbaca(src: EntrySource, m: int, n: int, eps: float, d: int, leaf: int,
          seed: int, keep_leaf_factors: bool = False, selector: int = 0,
          select_f: float = 2.0) -> HBACAResult:
    """H-BACA (Algorithm 3) of the m x n matrix whose entries ``src`` gives.
    ``selector``/``select_f`` choose the leaves' pivot selection (see
    baca_leaf)."""
    L = tree_levels(m, n, leaf)
    rows = cluster_tree(m, L)[L]
    cols = cluster_tree(n, L)[L]
    nb = 1 << L
    leaves, leaf_info = {}, {}
    ops = dict(entries=0, resid_flops=0, qrcp_flops=0, lrid_flops=0,
               norm_flops=0, bytes=0, merge_flops=0, recompress_flops=0)
    for t in range(nb):
        ra, rs = rows[t]
        for v in range(nb):
            ca, cs = cols[v]
            b = t * nb + v

            def blk(I, J, ra=ra, ca=ca):
                return src.block(np.asarray(I) + ra, np.asarray(J) + ca)

            J1 = first_column_block(seed, b, cs, d)
            res = baca_leaf(blk, rs, cs, d, eps, J1, selector=selector, select_f=select_f)
            for key in res.ops:
                ops[key] += res.ops[key]
            rb = res.rank
            ops["recompress_flops"] += 4 * (rs + cs) * rb * rb + 22 * rb ** 3
            blkres = recompress(res.U, res.V, eps)
            leaves[(t, v)] = blkres
            info = dict(rank_baca=rb, rank=blkres[1].size, iters=res.iters,
                        m0=rs, n0=cs, row0=ra, col0=ca,
                        swaps=sum(it["swaps_I"] + it["swaps_J"] for it in res.iters))
            if keep_leaf_factors:
                info["U"], info["V"] = res.U, res.V
            leaf_info[b] = info
    ranks = {0: [leaves[(t, v)][1].size for t in range(nb) for v in range(nb)]}
    mflops = []
    U, S, V = merge_tree(leaves, L, eps, ranks, mflops)
    ops["merge_flops"] = int(sum(mflops))
    return HBACAResult(U, S, V, L, leaf_info, ranks, ops)


def hbaca_batched(wl: dict, eps: float | None = None, d: int | None = None,
                  leaf: int | None = None, seed: int | None = None):
    """Independent H-BACA of every block of a batched workload.

    Block b uses rows ``X[row_off[b]:row_off[b]+row_cnt[b]]`` and columns
    ``Y[col_off[b]:...]``; its leaves draw J_1 from seed ``seed + b``."""
    eps = wl["tol"] if eps is None else eps
    d = wl["d"] if d is None else d
    leaf = wl["leaf"] if leaf is None else leaf
    seed = wl["seed"] if seed is None else seed
    out = []
    for b in range(int(wl["nblocks"])):
        ro, rc = int(wl["row_off"][b]), int(wl["row_cnt"][b])
        co, cc = int(wl["col_off"][b]), int(wl["col_cnt"][b])
        src = EntrySource(wl, X=wl["X"][ro:ro + rc], Y=wl["Y"][co:co + cc])
        out.append(hbaca(src, rc, cc, eps, d, leaf, seed + b))
    return out
