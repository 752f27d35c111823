"""GPU parity: the HIP path (through the C ABI) against the CPU oracle on the
same seeded inputs.

Bars (FP64 path): every leaf's pivot tape and d_k equal to the oracle's
(except a terminating iteration at rounding level), every final rank equal,
singular values equal to 1e-10 sigma_1, reconstructions equal to 1e-10
relative.  Sizes span several tiles and ragged tails."""
import numpy as np
import pytest

from workloads import generators as G

from _hbtest import (compare_tape, factors_np, lowrank_diff, recon_norm, run_gpu, run_oracle,
                     say)

pytestmark = pytest.mark.gpu


def _lowrank(m, n, rank, tol=1e-8, d=8, leaf=128, seed=7, spikes=0):
    wl = G.make_lowrank_spikes(n=n, m=m, rank=rank, n_spikes=spikes, tol=tol, d=d, leaf=leaf,
                               cfg=seed)
    return wl


BACA_CASES = {
    "gauss_ragged_d8": lambda: G.make_gauss3d(n=700, m=600, leaf=150, d=8, cfg=11),
    "gauss_d1_aca": lambda: G.make_gauss3d(n=300, m=260, leaf=130, d=1, cfg=12),
    "gauss_d2": lambda: G.make_gauss3d(n=400, leaf=200, d=2, cfg=13),
    "gauss_d32": lambda: G.make_gauss3d(n=640, leaf=320, d=32, cfg=14),
    "gauss_d16_big_leaf": lambda: G.make_gauss3d(n=1600, leaf=800, d=16, h=0.7, cfg=15),
    "helmholtz_d16": lambda: G.make_helmholtz_plates(n=900, leaf=300, cfg=17),
    "helmholtz_d8_ragged": lambda: G.make_helmholtz_plates(n=700, m=650, leaf=170, d=8, cfg=18),
    "lowrank_r20": lambda: _lowrank(400, 380, 20, leaf=200),
}


def _laplace_single(cfg):
    b = G.make_laplace_blocks(nblocks=1, cfg=cfg)
    m, n = int(b["row_cnt"][0]), int(b["col_cnt"][0])
    return dict(name="laplace", entry=2, X=b["X"][:m], Y=b["Y"][:n], m=m, n=n, h=0.0,
                gauss_c=0.0, wavenumber=0.0, tol=1e-6, d=4, leaf=max(32, max(m, n) // 3),
                seed=5, complex=False)


BACA_CASES["laplace_d4"] = lambda: _laplace_single(16)


@pytest.mark.parametrize("case", sorted(BACA_CASES))
def test_leaf_baca_matches_oracle(lib, case):
    wl = BACA_CASES[case]()
    say(f"[leaf BACA] {case}: m={wl['m']} n={wl['n']} d={wl['d']} leaf={wl['leaf']}")
    res = run_gpu(lib, wl, record_tape=1, stop_after=1)
    _, ores = run_oracle(wl, keep_leaf_factors=True)
    assert res.nleaves == len(ores.leaf_info)
    worst = 0.0
    for li in range(res.nleaves):
        info = res.leaf_info(li)
        b = info["t"] * (1 << ores.L) + info["v"]
        oinfo = ores.leaf_info[b]
        assert (info["m0"], info["n0"]) == (oinfo["m0"], oinfo["n0"])
        msg = compare_tape(res.leaf_tape(li), info, oinfo)
        assert msg is None, f"leaf {b}: {msg}"
        U, S, Vh = factors_np(res, li)
        Uo, Vo = oinfo["U"], oinfo["V"]
        den = max(recon_norm(Uo, Vo.conj().T), 1e-300)
        worst = max(worst, lowrank_diff(U * S, Vh, Uo, Vo.conj().T) / den)
    say(f"  worst leaf reconstruction difference {worst:.2e}")
    assert worst <= 1e-10


FULL_CASES = {
    "gauss3d_2000_cfg1": lambda: G.make_gauss3d(n=2000, cfg=1),
    "gauss3d_ragged": lambda: G.make_gauss3d(n=1100, m=900, leaf=140, d=8, cfg=21),
    "helmholtz_1200": lambda: G.make_helmholtz_plates(n=1200, leaf=300, cfg=2),
    "helmholtz_5000": lambda: G.make_helmholtz_plates(n=5000, cfg=2),
    "laplace_single": lambda: _laplace_single(22),
    "gauss_tol1e8_two_panels": lambda: G.make_gauss3d(n=800, leaf=100, tol=1e-8, d=8, cfg=23),
    "gauss_tol1e9_three_panels": lambda: G.make_gauss3d(n=800, leaf=100, tol=1e-9, d=8, cfg=23),
}


@pytest.mark.parametrize("case", sorted(FULL_CASES))
def test_hbaca_matches_oracle(lib, case):
    wl = FULL_CASES[case]()

    say(f"[H-BACA] {case}: m={wl['m']} n={wl['n']} d={wl['d']} leaf={wl['leaf']} tol={wl['tol']}")
    res = run_gpu(lib, wl, record_tape=1)
    src, ores = run_oracle(wl)
    U, S, Vh = factors_np(res)
    say(f"  rank gpu {S.size} oracle {ores.rank}; leaf ranks max "
        f"{res.stats()['leaf_rank_max']}")
    assert S.size == ores.rank
    if S.size:
        assert np.allclose(S, ores.S, rtol=0, atol=1e-10 * ores.S[0])
    diff = lowrank_diff(U * S, Vh, ores.U * ores.S, ores.V.conj().T)
    ref = recon_norm(ores.U * ores.S, ores.V.conj().T)
    say(f"  reconstruction difference {diff / ref:.2e}")
    assert diff <= 1e-10 * ref
    # leaf ranks after re-compression equal too
    for li in range(res.nleaves):
        info = res.leaf_info(li)
        b = info["t"] * (1 << ores.L) + info["v"]
        assert info["rank_leaf"] == ores.leaf_info[b]["rank"]
    # device error check agrees with the dense one
    e2, a2 = res.error(0, 1)
    A = src.dense()
    dense_err = np.linalg.norm(A - (U * S) @ Vh.conj().T) / np.linalg.norm(A)
    assert abs(np.sqrt(e2 / a2) - dense_err) <= 1e-6 * dense_err + 1e-14


@pytest.mark.parametrize("panel", [8, 16, 40])
@pytest.mark.parametrize("case", ["helmholtz_1200", "gauss3d_ragged"])
def test_column_panel_qr_matches_oracle(lib, case, panel):
    """Merges forced through the column-panel Householder QR with narrow
    panels (many panels, ragged last panel) give the oracle's result."""
    wl = FULL_CASES[case]()
    say(f"[panel QR] {case} with {panel}-column panels")
    res = run_gpu(lib, wl, diag_panel=panel)
    _, ores = run_oracle(wl)
    U, S, Vh = factors_np(res)
    assert S.size == ores.rank
    assert np.allclose(S, ores.S, rtol=0, atol=1e-10 * ores.S[0])
    diff = lowrank_diff(U * S, Vh, ores.U * ores.S, ores.V.conj().T)
    assert diff <= 1e-10 * recon_norm(ores.U * ores.S, ores.V.conj().T)


@pytest.mark.parametrize("storage", [1, 2, 3])
def test_svd_storage_modes_agree(lib, storage):
    """The small SVD gives the same result with its matrices in HBM or in LDS,
    and on several workgroups per matrix."""
    wl = FULL_CASES["gauss3d_ragged"]()
    say(f"[svd storage] mode {storage}")
    a = factors_np(run_gpu(lib, wl))
    b = factors_np(run_gpu(lib, wl, diag_svd_storage=storage))
    assert a[1].size == b[1].size
    assert np.allclose(a[1], b[1], rtol=0, atol=1e-12 * a[1][0])


WIDE_SVD_CASES = {
    "gauss3d_ragged": lambda: G.make_gauss3d(n=1100, m=900, leaf=140, d=8, cfg=21),
    "helmholtz_1200": lambda: G.make_helmholtz_plates(n=1200, leaf=300, cfg=2),
    "polynomial_2000": lambda: G.make_polynomial(n=2000, leaf=250, tol=1e-4, d=8),
    "lowrank_r90_tol1e10": lambda: _lowrank(900, 800, 90, tol=1e-10, leaf=200),
}


@pytest.mark.parametrize("case", sorted(WIDE_SVD_CASES))
def test_multi_workgroup_svd_matches_oracle(lib, case):
    """Every SVD whose shape allows it (p >= k, p <= 512, more than one block
    pair) on several workgroups (storage mode 3): the result against the
    oracle at the FP64 bars."""
    wl = WIDE_SVD_CASES[case]()
    say(f"[multi-workgroup SVD] {case}: m={wl['m']} n={wl['n']} d={wl['d']} leaf={wl['leaf']}")
    res = run_gpu(lib, wl, diag_svd_storage=3)
    _, ores = run_oracle(wl)
    U, S, Vh = factors_np(res)
    st = res.stats()
    say(f"  rank gpu {S.size} oracle {ores.rank}; step ranks {st['step_rank_max']}; "
        f"sweeps max {st['svd_sweeps_max']}")
    assert max(st["step_rank_max"]) > 16  # merges wide enough for several blocks
    assert S.size == ores.rank
    assert np.allclose(S, ores.S, rtol=0, atol=1e-10 * ores.S[0])
    ref = recon_norm(ores.U * ores.S, ores.V.conj().T)
    diff = lowrank_diff(U * S, Vh, ores.U * ores.S, ores.V.conj().T)
    say(f"  reconstruction difference {diff / ref:.2e}")
    assert diff <= 1e-10 * ref


def test_zero_matrix_rank_zero(lib):
    wl = _lowrank(300, 260, 1, leaf=100)
    wl["G1"] = np.zeros_like(wl["G1"])
    say("[zero] 300 x 260 zero matrix")
    res = run_gpu(lib, wl)
    assert res.rank(0) == 0


@pytest.mark.parametrize("r0", [1, 7, 30])
def test_exact_recovery(lib, r0):
    wl = _lowrank(500, 450, r0, tol=1e-10, leaf=120)
    say(f"[exact] rank {r0} product of random factors, 500 x 450")
    res = run_gpu(lib, wl)
    U, S, Vh = factors_np(res)
    A = wl["G1"] @ wl["G2"]
    assert S.size == r0
    assert np.linalg.norm(A - (U * S) @ Vh.T) <= 1e-12 * np.linalg.norm(A)


def test_d1_reduces_to_aca(lib):
    """BACA with d = 1 is ACA: the GPU's leaf pivots equal the oracle's
    independent ACA (Algorithm 1)."""
    import oracle
    wl = G.make_gauss3d(n=240, m=200, leaf=240, d=1, tol=1e-6, cfg=31)
    say("[aca] d = 1 on a 200 x 240 Gaussian leaf")
    res = run_gpu(lib, wl, record_tape=1, stop_after=1)
    src = oracle.EntrySource(wl)
    J1 = oracle.first_column_block(wl["seed"], 0, wl["n"], 1)
    _, _, piv = oracle.aca(lambda I, J: src.block(I, J), wl["m"], wl["n"], wl["tol"], int(J1[0]))
    tape = res.leaf_tape(0)
    assert [int(x) for x in tape["rows"]] == [i for i, _ in piv]
    assert [int(x) for x in tape["cols"]] == [j for _, j in piv]


def test_repeatable_bitwise(lib):
    wl = G.make_helmholtz_plates(n=1500, leaf=375, cfg=32)
    say("[repeat] Helmholtz 1500 twice")
    a = factors_np(run_gpu(lib, wl))
    b = factors_np(run_gpu(lib, wl))
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def test_batched_matches_oracle(lib):
    import oracle
    import torch
    wl = G.make_laplace_blocks(nblocks=10, cfg=33)
    say("[batched] 10 Laplace blocks")
    X = torch.tensor(wl["X"], device="cuda")
    Y = torch.tensor(wl["Y"], device="cuda")
    p = lib.params(dim=3, seed=wl["seed"])
    res = lib.compress_batched(wl["entry"], p, X, wl["row_off"], wl["row_cnt"], Y, wl["col_off"],
                               wl["col_cnt"], wl["tol"], wl["d"], wl["leaf"])
    refs = oracle.hbaca_batched(wl)
    assert res.nblocks == len(refs)
    for b, ref in enumerate(refs):
        U, S, Vh = factors_np(res, b)
        assert S.size == ref.rank, (b, S.size, ref.rank)
        assert np.allclose(S, ref.S, rtol=0, atol=1e-10 * ref.S[0])
        diff = lowrank_diff(U * S, Vh, ref.U * ref.S, ref.V.T)
        assert diff <= 1e-10 * recon_norm(ref.U * ref.S, ref.V.T)


def test_coherent_variant_properties(lib):
    """Rank-30 product plus sparse spikes.  Once the rank-30 part is found the
    residual is rounding noise, so later pivots are chosen from noise on both
    sides and need not agree; compare what is unique: the error against A
    and the rank, which must stay close to the oracle's."""
    wl = _lowrank(2000, 2000, 30, tol=1e-4, d=16, leaf=625, spikes=20, seed=2)
    say("[coherent] 2000 x 2000 rank 30 + 20 spikes")
    res = run_gpu(lib, wl)
    src, ores = run_oracle(wl)
    U, S, Vh = factors_np(res)
    A = src.dense()
    eg = np.linalg.norm(A - (U * S) @ Vh.T) / np.linalg.norm(A)
    eo = np.linalg.norm(A - ores.dense()) / np.linalg.norm(A)
    say(f"  rank gpu {S.size} oracle {ores.rank}; error gpu {eg:.3e} oracle {eo:.3e}")
    assert abs(S.size - ores.rank) <= 3
    assert 0.5 * eo <= eg <= 2.0 * eo + 1e-12
