"""Batched call over many blocks whose trees end at different depths.

A block whose tree is shallower than the deepest one finishes its merges
early; its root must survive the later merge levels of the other blocks.
256 Laplace blocks of the batched recipe with leaf 128 give trees of depth
0, 1, 2 and 3 in one call; every block is held to the FP64 parity bars
against the oracle (Algorithm 3 applied to each block on its own)."""
import collections

import numpy as np
import pytest

from workloads import generators as G

from _hbtest import factors_np, lowrank_diff, recon_norm, say

pytestmark = pytest.mark.gpu


def test_batched_mixed_depths_match_oracle(lib):
    import oracle
    import torch
    wl = G.make_laplace_blocks(nblocks=256, cfg=34, leaf=128)
    say("[batched depths] 256 Laplace blocks, leaf 128")
    X = torch.tensor(wl["X"], device="cuda")
    Y = torch.tensor(wl["Y"], device="cuda")
    p = lib.params(dim=3, seed=wl["seed"])
    res = lib.compress_batched(wl["entry"], p, X, wl["row_off"], wl["row_cnt"], Y, wl["col_off"],
                               wl["col_cnt"], wl["tol"], wl["d"], wl["leaf"])
    refs = oracle.hbaca_batched(wl)
    depths = collections.Counter(r.L for r in refs)
    say(f"  tree depths {dict(sorted(depths.items()))}")
    assert {0, 1, 2, 3} <= set(depths)
    assert res.nblocks == len(refs)
    worst = 0.0
    for b, ref in enumerate(refs):
        U, S, Vh = factors_np(res, b)
        assert S.size == ref.rank, (b, S.size, ref.rank)
        assert np.allclose(S, ref.S, rtol=0, atol=1e-10 * ref.S[0]), b
        diff = lowrank_diff(U * S, Vh, ref.U * ref.S, ref.V.T)
        rel = diff / recon_norm(ref.U * ref.S, ref.V.T)
        worst = max(worst, rel)
        assert rel <= 1e-10, (b, ref.L, rel)
    say(f"  largest relative difference over the blocks {worst:.2e}")
