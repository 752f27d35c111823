"""Hierarchical matrix of a kernel matrix built with H-BACA (oracle side).

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle``.

The paper presents H-BACA as a building block for constructing hierarchical
matrices (Introduction) and applies it to one off-diagonal block of a
KD-permuted kernel matrix, noting that the permutation yields a hierarchical
representation of the whole matrix (Section "Numerical Results").  This
module builds that representation in its simplest form, a HODLR matrix
(every off-diagonal block of the cluster tree is low rank):

* the points are taken in the given (KD) order; the cluster tree of [0, N)
  splits a node of size s into ceil(s/2) and floor(s/2) (the split the
  H-BACA trees use), down to depth Lh, the smallest depth whose nodes hold
  at most ``nmin`` points;
* every internal node with children c1, c2 contributes the two blocks
  A(c1, c2) and A(c2, c1), each compressed by H-BACA (Algorithm 3) on its
  own; block p (numbered level by level from the root, nodes left to right,
  A(c1, c2) before A(c2, c1)) uses seed + p, as the library's batched call
  does;
* the diagonal blocks of the leaves are kept dense.

``hodlr_matvec`` applies the result: the dense leaves, then the low-rank
blocks.  Pinned in tests/test_oracle_hodlr.py: the blocks tile the matrix
exactly once, an exactly low-rank kernel is reproduced to rounding, and the
Gaussian kernel to the tolerance against a dense matrix.
"""
from __future__ import annotations

import numpy as np

from .entries import EntrySource
from .hbaca import cluster_tree, hbaca


def hodlr_depth(N: int, nmin: int) -> int:
    """Smallest depth Lh whose cluster-tree nodes hold at most nmin points."""
    L = 0
    while -(-N // (1 << L)) > nmin:
        L += 1
    return L


def hodlr_blocks(N: int, nmin: int):
    """(level, row_off, row_cnt, col_off, col_cnt) of every off-diagonal
    block in block order, and the leaves (offset, size)."""
    Lh = hodlr_depth(N, nmin)
    tree = cluster_tree(N, Lh)
    blocks = []
    for lev in range(Lh):
        for i in range(len(tree[lev])):
            c1, c2 = tree[lev + 1][2 * i], tree[lev + 1][2 * i + 1]
            blocks.append((lev, c1[0], c1[1], c2[0], c2[1]))
            blocks.append((lev, c2[0], c2[1], c1[0], c1[1]))
    return blocks, tree[Lh]


class HODLR:
    def __init__(self, N, blocks, factors, leaves, dense):
        self.N = N
        self.blocks = blocks      # (level, row_off, row_cnt, col_off, col_cnt)
        self.factors = factors    # H-BACA results (U, S, V) per block
        self.leaves = leaves      # (offset, size)
        self.dense = dense        # dense diagonal blocks

    def assemble(self) -> np.ndarray:
        """The dense matrix the representation stands for (small N only)."""
        dt = self.dense[0].dtype if self.dense else np.float64
        A = np.zeros((self.N, self.N), dtype=dt)
        for (off, s), D in zip(self.leaves, self.dense):
            A[off:off + s, off:off + s] = D
        for (_, ro, rc, co, cc), f in zip(self.blocks, self.factors):
            A[ro:ro + rc, co:co + cc] = (f.U * f.S[None, :]) @ f.V
        return A


def hodlr_build(wl: dict, nmin: int, eps: float, d: int, leaf: int, seed: int) -> HODLR:
    """HODLR matrix of the kernel matrix of the points wl["X"] with itself."""
    X = wl["X"]
    N = X.shape[0]
    blocks, leaves = hodlr_blocks(N, nmin)
    factors = []
    for p, (_, ro, rc, co, cc) in enumerate(blocks):
        src = EntrySource(wl, X=X[ro:ro + rc], Y=X[co:co + cc])
        factors.append(hbaca(src, rc, cc, eps, d, leaf, seed + p))
    full = EntrySource(wl, X=X, Y=X)
    dense = [full.block(np.arange(off, off + s), np.arange(off, off + s)) for off, s in leaves]
    return HODLR(N, blocks, factors, leaves, dense)


def hodlr_matvec(H: HODLR, x: np.ndarray) -> np.ndarray:
    """y = A_H x: dense diagonal leaves plus every low-rank block."""
    y = np.zeros(H.N, dtype=np.result_type(x.dtype, H.dense[0].dtype if H.dense else x.dtype))
    for (off, s), D in zip(H.leaves, H.dense):
        y[off:off + s] += D @ x[off:off + s]
    for (_, ro, rc, co, cc), f in zip(H.blocks, H.factors):
        y[ro:ro + rc] += f.U @ (f.S * (f.V @ x[co:co + cc]))
    return y
