"""Pins of the oracle's strong rank-revealing selector (oracle/qrcp.py
strong_select) and of BACA run with it (oracle/baca.py, selector 1).

What fixes the selector independently of its own code:
* a worked 2 x 3 example computed by hand (greedy QRCP picks columns 0, 1;
  column 2 has coefficients (1.2, -1) in that basis, so with f = 1.1 column
  2 replaces column 0 and the selection stops at coefficients 5/6);
* Cramer's rule: swapping chosen column i for candidate j scales the volume
  of the chosen columns by |W(i, j)|, so at exit every single swap,
  measured by brute-force determinants, gains at most a factor f, and the
  volume never falls below greedy QRCP's;
* special cases: a one-row panel (the largest entry, as QRCP), no candidate
  left to swap, a rank-deficient panel (only the numerical-rank picks are
  refined, the rest are the lowest free positions).
"""
import itertools

import numpy as np
import pytest

from oracle.qrcp import SWAP_CAP, qrcp, strong_select


def _vol(M, S):
    """Volume of the columns S of M: sqrt(det(M_S^H M_S))."""
    B = M[:, list(S)]
    return float(np.sqrt(abs(np.linalg.det(B.conj().T @ B))))


def test_worked_example():
    M = np.array([[1.0, 0.6, 0.6], [0.0, 0.75, -0.75]])
    assert list(qrcp(M, 2).piv) == [0, 1]
    s = strong_select(M, 2, 1.1)
    assert list(s.piv) == [2, 1] and s.swaps == 1
    # margins: (1.2 - 1.1) / 1.1 at the swap (runner-up 1.0 is further),
    # (1.1 - 5/6) / 1.1 at the exit
    assert s.margin == pytest.approx(0.1 / 1.1, rel=1e-12)
    s = strong_select(M, 2, 1.25)
    assert list(s.piv) == [0, 1] and s.swaps == 0
    assert s.margin == pytest.approx(0.05 / 1.25, rel=1e-12)


@pytest.mark.parametrize("cplx", [False, True])
@pytest.mark.parametrize("seed", range(6))
def test_local_maximum_volume(cplx, seed):
    rng = np.random.default_rng(seed)
    p, q = 4, 11
    # graded columns so that greedy QRCP is often not locally maximal
    M = rng.standard_normal((p, q)) * np.exp(rng.uniform(-2, 2, q))
    if cplx:
        M = M + 1j * rng.standard_normal((p, q)) * np.exp(rng.uniform(-2, 2, q))
    f = 1.05
    s = strong_select(M, p, f)
    S = list(s.piv)
    assert len(set(S)) == p
    v = _vol(M, S)
    assert v >= _vol(M, qrcp(M, p).piv) * (1 - 1e-12)
    for i, j in itertools.product(range(p), [c for c in range(q) if c not in S]):
        T = S.copy()
        T[i] = j
        assert _vol(M, T) <= f * v * (1 + 1e-10), (i, j)
    assert s.swaps < SWAP_CAP * p


def test_swaps_happen_and_ratio_is_the_coefficient():
    """Across seeds some selections swap, and every swap multiplies the
    volume (brute-force determinants) by more than f."""
    total = 0
    for seed in range(20):
        rng = np.random.default_rng(100 + seed)
        M = rng.standard_normal((8, 60))
        g = list(qrcp(M, 8).piv)
        s = strong_select(M, 8, 1.01)
        total += s.swaps
        if s.swaps:
            assert _vol(M, s.piv) > 1.01 ** s.swaps * _vol(M, g) * (1 - 1e-12)
    assert total > 0


def test_one_row_panel_is_qrcp():
    M = np.array([[0.3, -2.0, 1.5, 2.0, -0.1]])
    s = strong_select(M, 4, 1.01)
    assert list(s.piv) == list(qrcp(M, 4).piv) == [1] and s.swaps == 0


def test_no_candidate_left():
    rng = np.random.default_rng(7)
    M = rng.standard_normal((5, 3))
    s = strong_select(M, 5, 1.01)
    assert list(s.piv) == list(qrcp(M, 5).piv) and s.swaps == 0


def test_rank_deficient_panel():
    rng = np.random.default_rng(8)
    M = rng.standard_normal((6, 3)) @ (rng.standard_normal((3, 15)) * np.exp(rng.uniform(-2, 2, 15)))
    g = qrcp(M, 6)
    assert g.nz == 3
    s = strong_select(M, 6, 1.02)
    S = list(s.piv[:3])
    free = [c for c in range(15) if c not in S]
    assert list(s.piv[3:]) == free[:3]
    v = _vol(M, S)
    for i, j in itertools.product(range(3), free):
        T = S.copy()
        T[i] = j
        assert _vol(M, T) <= 1.02 * v * (1 + 1e-9)


def test_threshold_must_exceed_one():
    with pytest.raises(ValueError):
        strong_select(np.eye(3), 3, 1.0)


def test_baca_with_strong_selector():
    """BACA with the strong selector on a Gaussian kernel block: every
    recorded selection swapped at most SWAP_CAP * d times, some swapped, and
    the factors meet the tolerance against the dense block."""
    from oracle.baca import baca_leaf
    rng = np.random.default_rng(9)
    X = rng.random((300, 3))
    Y = rng.random((280, 3)) + np.array([1.2, 0.0, 0.0])
    A = np.exp(-((X[:, None, :] - Y[None, :, :]) ** 2).sum(-1) / 0.5)

    def blk(I, J):
        return A[np.ix_(np.asarray(I, np.int64), np.asarray(J, np.int64))]

    for d in (4, 8):
        J1 = rng.choice(280, size=d, replace=False)
        res = baca_leaf(blk, 300, 280, d, 1e-8, J1, selector=1, select_f=1.05)
        err = np.linalg.norm(A - res.U @ res.V) / np.linalg.norm(A)
        assert err < 1e-6
        sw = [it["swaps_I"] + it["swaps_J"] for it in res.iters]
        assert sum(sw) > 0
        assert all(x <= 2 * SWAP_CAP * d for x in sw)
        ref = baca_leaf(blk, 300, 280, d, 1e-8, J1)
        assert abs(res.rank - ref.rank) <= d
