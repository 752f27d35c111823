"""Hierarchical (HODLR) matrix built with the batched H-BACA path on the GPU
(hb_hodlr_build, hb_hodlr_matvec) against the oracle's (oracle/hodlr.py):
every off-diagonal block at the FP64 parity bars, the matrix-vector product
against the oracle's and against the dense kernel matrix."""
import numpy as np
import pytest

from workloads import generators as G

from _hbtest import lowrank_diff, recon_norm, say

pytestmark = pytest.mark.gpu

CASES = {
    "gauss_curve_4000": lambda: G.make_hodlr_curve(N=4000, nmin=256, tol=1e-6, leaf=256),
    "gauss_curve_ragged": lambda: G.make_hodlr_curve(N=2999, nmin=100, tol=1e-8, leaf=128, d=16,
                                                     cfg=81),
    "polynomial_1500": lambda: G.make_hodlr_polynomial(N=1500, nmin=128, tol=1e-6, leaf=128),
}


def _build(lib, wl):
    import torch
    X = torch.tensor(wl["X"], device="cuda")
    p = lib.params(dim=wl["X"].shape[1], h=wl["h"], gauss_c=wl["gauss_c"], seed=wl["seed"])
    return lib.hodlr_build(wl["entry"], p, X, wl["nmin"], wl["tol"], wl["d"], wl["leaf"])


@pytest.mark.parametrize("case", sorted(CASES))
def test_hodlr_matches_oracle(lib, case):
    import torch
    from oracle import EntrySource
    from oracle.hodlr import hodlr_build, hodlr_matvec
    wl = CASES[case]()
    N = wl["X"].shape[0]
    say(f"[HODLR] {case}: N={N} nmin={wl['nmin']} tol={wl['tol']} d={wl['d']} leaf={wl['leaf']}")
    H = _build(lib, wl)
    ref = hodlr_build(wl, wl["nmin"], wl["tol"], wl["d"], wl["leaf"], wl["seed"])
    assert H.nblocks == len(ref.blocks) and H.nleaves == len(ref.leaves)
    worst = 0.0
    for b, (blk, f) in enumerate(zip(ref.blocks, ref.factors)):
        assert H.block_info(b) == blk
        U, S, Vh = (t.cpu().numpy() for t in H.blocks.factors(b))
        assert S.size == f.rank, (b, S.size, f.rank)
        if f.rank:
            assert np.allclose(S, f.S, rtol=0, atol=1e-10 * f.S[0])
            rel = lowrank_diff(U * S, Vh, f.U * f.S, f.V.T) / recon_norm(f.U * f.S, f.V.T)
            worst = max(worst, rel)
    say(f"  {H.nblocks} blocks, largest rank {max(f.rank for f in ref.factors)}, "
        f"worst block difference {worst:.2e}")
    assert worst <= 1e-10
    x = np.random.default_rng(3).standard_normal(N)
    y = H.matvec(torch.tensor(x, device="cuda")).cpu().numpy()
    yo = hodlr_matvec(ref, x)
    assert np.linalg.norm(y - yo) <= 1e-10 * np.linalg.norm(yo)
    A = EntrySource(wl, X=wl["X"], Y=wl["X"]).dense()
    yd = A @ x
    err = np.linalg.norm(y - yd) / np.linalg.norm(yd)
    say(f"  matvec: against the oracle's {np.linalg.norm(y - yo) / np.linalg.norm(yo):.2e}, "
        f"against the dense matrix {err:.2e}")
    assert err <= 10 * wl["tol"]


def test_hodlr_single_leaf_and_rejected_kernels(lib):
    import torch
    from oracle import EntrySource
    wl = G.make_hodlr_curve(N=200, nmin=256)
    H = _build(lib, wl)
    assert H.nblocks == 0 and H.nleaves == 1 and H.blocks is None
    x = np.random.default_rng(4).standard_normal(200)
    y = H.matvec(torch.tensor(x, device="cuda")).cpu().numpy()
    A = EntrySource(wl, X=wl["X"], Y=wl["X"]).dense()
    assert np.allclose(y, A @ x, rtol=0, atol=1e-13 * np.linalg.norm(A @ x))
    X = torch.tensor(wl["X"], device="cuda")
    with pytest.raises(lib.HBACAError) as e:
        lib.hodlr_build(lib.HB_K_LAPLACE, lib.params(dim=3, seed=1), X, 64, 1e-6, 8, 64)
    assert e.value.status == -6
