"""The strong rank-revealing pivot selection (HB_SEL_STRONG: greedy QRCP
refined by Gu-Eisenstat swaps) on the GPU against the oracle's
(oracle/qrcp.py strong_select) on the same seeded inputs.

Bars as for greedy QRCP: every leaf's pivot tape (which records the rows and
columns after the swaps) equal to the oracle's over the iterations the data
decides (swap decisions within 1e-6 of the threshold or of the runner-up
count as undecided), the FP64 reconstruction within 1e-10 of the operator's
norm plus twice the nu of iterations where the runs parted (plus four times
the oracle's own movement under rounding-level input changes, for problems
that amplify rounding past that); the total swap count equal where every
leaf is decided to the end."""
import numpy as np
import pytest

from workloads import generators as G

from _hbtest import (check_mixed, compare_tape, determined_iterations, divergence_nu,
                     factors_np, lowrank_diff, parity_bar, recon_norm, rounding_sensitivity,
                     run_gpu, run_oracle, say)

pytestmark = pytest.mark.gpu


def _laplace_single(cfg):
    b = G.make_laplace_blocks(nblocks=1, cfg=cfg)
    m, n = int(b["row_cnt"][0]), int(b["col_cnt"][0])
    return dict(name="laplace", entry=2, X=b["X"][:m], Y=b["Y"][:n], m=m, n=n, h=0.0,
                gauss_c=0.0, wavenumber=0.0, tol=1e-6, d=4, leaf=max(32, max(m, n) // 3),
                seed=5, complex=False)


CASES = {
    "gauss_ragged_d8": lambda: G.make_gauss3d(n=700, m=600, leaf=150, d=8, cfg=11),
    "gauss_d16_tol1e8": lambda: G.make_gauss3d(n=800, leaf=200, tol=1e-8, d=16, cfg=23),
    "gauss_d32": lambda: G.make_gauss3d(n=640, leaf=320, d=32, cfg=14),
    "helmholtz_d16": lambda: G.make_helmholtz_plates(n=900, leaf=300, cfg=17),
    "lowrank_r20": lambda: G.make_lowrank_spikes(n=380, m=400, rank=20, n_spikes=0, tol=1e-8,
                                                 d=8, leaf=200, cfg=7),
    "laplace_d4": lambda: _laplace_single(16),
    "efie2d_d8": lambda: G.make_efie2d_strips(n=1200, leaf=300, cfg=61),
}


def _compare(lib, wl, f, stop_after=0):
    res = run_gpu(lib, wl, record_tape=1, stop_after=stop_after, selector=lib.HB_SEL_STRONG,
                  select_f=f)
    _, ores = run_oracle(wl, keep_leaf_factors=stop_after == 1, selector=1, select_f=f)
    nb = 1 << ores.L
    parted, decided_all = 0.0, True
    for li in range(res.nleaves):
        info = res.leaf_info(li)
        b = info["t"] * nb + info["v"]
        oinfo = ores.leaf_info[b]
        tape = res.leaf_tape(li)
        msg = compare_tape(tape, info, oinfo)
        assert msg is None, f"leaf {b}: {msg}"
        parted += divergence_nu(tape, oinfo)
        decided_all = decided_all and determined_iterations(oinfo) == len(oinfo["iters"])
    return res, ores, parted, decided_all


@pytest.mark.parametrize("f", [1.05, 2.0])
@pytest.mark.parametrize("case", sorted(CASES))
def test_strong_selector_matches_oracle(lib, case, f):
    wl = CASES[case]()
    say(f"[strong selector] {case}: m={wl['m']} n={wl['n']} d={wl['d']} leaf={wl['leaf']} f={f}")
    res, ores, parted, decided_all = _compare(lib, wl, f)
    oswaps = sum(i["swaps"] for i in ores.leaf_info.values())
    st = res.stats()
    say(f"  swaps gpu {st['select_swaps']} oracle {oswaps}; rank gpu {res.rank(0)} oracle "
        f"{ores.rank}; parted nu {parted:.2e}")
    if decided_all:
        assert st["select_swaps"] == oswaps
    U, S, Vh = factors_np(res)
    ref = recon_norm(ores.U * ores.S, ores.V.conj().T)
    bar = parity_bar(ref, parted)
    if parted == 0.0:
        assert S.size == ores.rank
        assert np.allclose(S, ores.S, rtol=0, atol=1e-10 * ores.S[0])
    diff = lowrank_diff(U * S, Vh, ores.U * ores.S, ores.V.conj().T)
    if diff > bar and wl.get("X") is not None:
        # allow for the problem's own amplification of rounding
        sens = rounding_sensitivity(wl, selector=1, select_f=f)
        say(f"  oracle moves {sens / ref:.2e} under rounding-level input changes")
        bar += 4.0 * sens
    say(f"  reconstruction difference {diff / ref:.2e} (bar {bar / ref:.2e})")
    assert diff <= bar


def test_strong_selector_leaf_factors(lib):
    """Leaf factors of the strong selection straight after the leaf BACA."""
    wl = CASES["gauss_ragged_d8"]()
    res, ores, parted, _ = _compare(lib, wl, 1.05, stop_after=1)
    assert parted == 0.0
    nb = 1 << ores.L
    worst = 0.0
    for li in range(res.nleaves):
        info = res.leaf_info(li)
        oinfo = ores.leaf_info[info["t"] * nb + info["v"]]
        U, S, Vh = factors_np(res, li)
        Uo, Vo = oinfo["U"], oinfo["V"]
        den = max(recon_norm(Uo, Vo.conj().T), 1e-300)
        worst = max(worst, lowrank_diff(U * S, Vh, Uo, Vo.conj().T) / den)
    say(f"  worst leaf reconstruction difference {worst:.2e}")
    assert worst <= 1e-10


def test_swaps_happen(lib):
    """The workloads above exercise the swaps (not only the greedy picks)."""
    wl = CASES["gauss_d16_tol1e8"]()
    res = run_gpu(lib, wl, selector=lib.HB_SEL_STRONG, select_f=1.05)
    assert res.stats()["select_swaps"] > 0


def test_huge_threshold_is_qrcp(lib):
    """With f beyond every coefficient no swap is made and the tapes equal
    greedy QRCP's."""
    wl = CASES["helmholtz_d16"]()
    a = run_gpu(lib, wl, record_tape=1)
    b = run_gpu(lib, wl, record_tape=1, selector=lib.HB_SEL_STRONG, select_f=1e300)
    assert b.stats()["select_swaps"] == 0
    for li in range(a.nleaves):
        ta, tb = a.leaf_tape(li), b.leaf_tape(li)
        for key in ("rows", "cols", "dk"):
            assert np.array_equal(ta[key], tb[key])
    Ua, Sa, Va = factors_np(a)
    Ub, Sb, Vb = factors_np(b)
    assert lowrank_diff(Ua * Sa, Va, Ub * Sb, Vb) <= 1e-12 * recon_norm(Ua * Sa, Va)


def test_mixed_precision_with_strong_selector(lib):
    check_mixed(lib, "gauss_d8_strong", G.make_gauss3d(n=700, m=600, leaf=150, d=8, tol=1e-6,
                                                      cfg=11), selector=1, select_f=1.05)


@pytest.mark.parametrize("sel,f", [(2, 2.0), (1, 1.0), (1, float("nan")), (-1, 2.0)])
def test_invalid_selector_rejected(lib, sel, f):
    wl = G.make_gauss3d(n=200, leaf=100, d=4, cfg=3)
    with pytest.raises(lib.HBACAError) as e:
        run_gpu(lib, wl, selector=sel, select_f=f)
    assert e.value.status == -1
