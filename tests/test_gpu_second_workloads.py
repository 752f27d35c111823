"""The paper's EFIE2D and polynomial kernels (Section "Numerical Results",
kernels 2 and 5) on the GPU against the oracle.

They are the two rank regimes of the cost analysis (Table 1): the EFIE2D
strips (a high-frequency 2-D scattering kernel, complex) double their rank
at every merge level, the polynomial kernel (x^T y + h)^2 keeps a rank
bounded by the dimension of the quadratic polynomials at every level.  Both
are held to the FP64 parity bars: every leaf's pivot tape while the data
decides it, the ranks after every merge step, the singular values and the
reconstruction (1e-10 of the operator plus twice the nu of the leaf
iterations after the point where the two runs' picks part, which can happen
only where rounding decides a pick: the strips' close random nodes give a
few such leaves)."""
import numpy as np
import pytest

from workloads import generators as G

from _hbtest import (check_mixed, compare_tape, divergence_nu, factors_np, lowrank_diff,
                     parity_bar, recon_norm, run_gpu, run_oracle, say)

pytestmark = pytest.mark.gpu

HB_EUNSUPPORTED = -6

CASES = {
    "efie2d_2000": lambda: G.make_efie2d_strips(n=2000, leaf=125, tol=1e-4, d=8),
    "efie2d_ragged_d16": lambda: G.make_efie2d_strips(n=1500, m=1300, leaf=100, tol=1e-6, d=16),
    "polynomial_2000": lambda: G.make_polynomial(n=2000, leaf=250, tol=1e-4, d=8),
    "polynomial_d16_tol1e6": lambda: G.make_polynomial(n=1200, dim=8, leaf=150, tol=1e-6, d=16),
}


def _steps(ores):
    """The oracle's largest rank after every merge step, in the library's
    step order (0 leaves, then horizontal and vertical per level)."""
    out = [max(ores.ranks[0])]
    for lev in range(1, ores.L + 1):
        out.append(max(ores.ranks[lev - 0.5]))
        out.append(max(ores.ranks[lev]))
    return out


@pytest.mark.parametrize("case", sorted(CASES))
def test_second_workloads_match_oracle(lib, case):
    wl = CASES[case]()
    say(f"[second workloads] {case}: m={wl['m']} n={wl['n']} d={wl['d']} leaf={wl['leaf']} "
        f"tol={wl['tol']}")
    res = run_gpu(lib, wl, record_tape=1)
    _, ores = run_oracle(wl)
    nb = 1 << ores.L
    parted = 0.0
    for li in range(res.nleaves):
        info = res.leaf_info(li)
        b = info["t"] * nb + info["v"]
        tape = res.leaf_tape(li)
        msg = compare_tape(tape, info, ores.leaf_info[b])
        assert msg is None, f"leaf {b}: {msg}"
        parted += divergence_nu(tape, ores.leaf_info[b])
    st = res.stats()
    assert st["step_rank_max"] == _steps(ores)
    U, S, Vh = factors_np(res)
    Vo = ores.V.conj().T
    ref = recon_norm(ores.U * ores.S, Vo)
    bar = parity_bar(ref, parted)
    diff = lowrank_diff(U * S, Vh, ores.U * ores.S, Vo)
    say(f"  ranks per step {st['step_rank_max']}; reconstruction difference {diff / ref:.2e} "
        f"(bar {bar / ref:.2e})")
    assert S.size == ores.rank
    assert np.allclose(S, ores.S, rtol=0, atol=bar)
    assert diff <= bar


def test_rank_regimes_of_the_cost_analysis(lib):
    """Table 1's two regimes as the GPU runs them: the EFIE2D ranks grow by
    about 2 per level (from leaf rank to root rank over four levels at least
    eight-fold), the polynomial ranks stay within 20 % of the leaf rank."""
    e = run_gpu(lib, G.make_efie2d_strips(n=2000, leaf=125, tol=1e-4, d=8)).stats()
    p = run_gpu(lib, G.make_polynomial(n=2000, leaf=250, tol=1e-4, d=8)).stats()
    se, sp = e["step_rank_max"], p["step_rank_max"]
    say(f"  EFIE2D {se}; polynomial {sp}")
    assert se[-1] >= 8 * se[0]
    assert sp[-1] <= 1.2 * sp[0]


def test_polynomial_mixed_precision(lib):
    check_mixed(lib, "polynomial_1200", G.make_polynomial(n=1200, leaf=150, tol=1e-4, d=8))


def test_efie2d_mixed_precision_is_rejected(lib):
    wl = G.make_efie2d_strips(n=400, leaf=100)
    with pytest.raises(lib.HBACAError) as e:
        run_gpu(lib, wl, precision=lib.HB_PREC_MIXED)
    assert e.value.status == HB_EUNSUPPORTED
