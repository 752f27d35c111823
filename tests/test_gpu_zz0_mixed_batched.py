"""Mixed precision on the batched call (one leaf launch over every block's
leaves in FP32, FP64 merges per step) against the FP64 oracle per block.

The bars are those of the single problems: the compressed operators agree
to 5 tol relative (Frobenius norm of the difference, from the factors), and
the ranks stay within max(3, 10 %) of the oracle's (FP32 residuals may
choose other pivots)."""
import pytest

from workloads import generators as G

from _hbtest import factors_np, lowrank_diff, recon_norm, say

pytestmark = pytest.mark.gpu


def test_mixed_batched_laplace_blocks(lib):
    import oracle
    import torch
    wl = G.make_laplace_blocks(nblocks=12, cfg=49)
    say("[mixed batched] 12 Laplace blocks")
    X = torch.tensor(wl["X"], device="cuda")
    Y = torch.tensor(wl["Y"], device="cuda")
    p = lib.params(dim=3, seed=wl["seed"], precision=lib.HB_PREC_MIXED)
    res = lib.compress_batched(wl["entry"], p, X, wl["row_off"], wl["row_cnt"], Y, wl["col_off"],
                               wl["col_cnt"], wl["tol"], wl["d"], wl["leaf"])
    refs = oracle.hbaca_batched(wl)
    assert res.nblocks == len(refs)
    for b, ref in enumerate(refs):
        U, S, Vh = factors_np(res, b)
        diff = lowrank_diff(U * S, Vh, ref.U * ref.S, ref.V.T)
        assert diff <= 5 * wl["tol"] * recon_norm(ref.U * ref.S, ref.V.T), b
        assert abs(S.size - ref.rank) <= max(3, ref.rank // 10), (b, S.size, ref.rank)
