"""Pins of the oracle's hierarchical (HODLR) matrix built with H-BACA
(oracle/hodlr.py), each against something other than the module itself:
the blocks and leaves tile the matrix exactly once, an exactly low-rank
kernel is reproduced to rounding, the Gaussian kernel of a curve to its
tolerance against the dense matrix, and the matrix-vector product equals the
assembled matrix times the vector."""
import numpy as np
import pytest

from oracle import EntrySource
from oracle.hodlr import hodlr_blocks, hodlr_build, hodlr_depth, hodlr_matvec
from workloads import generators as G


@pytest.mark.parametrize("N,nmin", [(37, 5), (64, 8), (100, 100), (101, 50), (1, 4)])
def test_blocks_and_leaves_tile_the_matrix_once(N, nmin):
    blocks, leaves = hodlr_blocks(N, nmin)
    cover = np.zeros((N, N), dtype=int)
    for _, ro, rc, co, cc in blocks:
        cover[ro:ro + rc, co:co + cc] += 1
    for off, s in leaves:
        cover[off:off + s, off:off + s] += 1
        assert s <= nmin
    assert np.all(cover == 1)
    L = hodlr_depth(N, nmin)
    assert len(blocks) == 2 * (2 ** L - 1) and len(leaves) == 2 ** L
    # blocks of one level cover disjoint rows
    for lev in range(L):
        rows = np.zeros(N, dtype=int)
        for lv, ro, rc, _, _ in blocks:
            if lv == lev:
                rows[ro:ro + rc] += 1
        assert rows.max() == 1


def test_exactly_low_rank_kernel_is_reproduced():
    wl = G.make_hodlr_polynomial(N=300, dim=2, nmin=40)
    H = hodlr_build(wl, 40, 1e-13, 8, 64, wl["seed"])
    A = EntrySource(wl, X=wl["X"], Y=wl["X"]).dense()
    assert np.linalg.norm(H.assemble() - A) <= 1e-12 * np.linalg.norm(A)
    assert max(f.rank for f in H.factors) <= 6  # quadratics in 2 variables


def test_gaussian_curve_within_tolerance_and_matvec():
    wl = G.make_hodlr_curve(N=700, nmin=64, tol=1e-6, leaf=128)
    H = hodlr_build(wl, wl["nmin"], wl["tol"], wl["d"], wl["leaf"], wl["seed"])
    A = EntrySource(wl, X=wl["X"], Y=wl["X"]).dense()
    AH = H.assemble()
    assert np.linalg.norm(AH - A) <= 10 * wl["tol"] * np.linalg.norm(A)
    x = np.random.default_rng(1).standard_normal(700)
    assert np.allclose(hodlr_matvec(H, x), AH @ x, rtol=0, atol=1e-13 * np.linalg.norm(AH @ x))


def test_single_leaf_is_dense():
    wl = G.make_hodlr_curve(N=50, nmin=64)
    H = hodlr_build(wl, 64, 1e-6, 8, 64, wl["seed"])
    assert H.blocks == [] and len(H.dense) == 1
    A = EntrySource(wl, X=wl["X"], Y=wl["X"]).dense()
    assert np.array_equal(H.assemble(), A)
