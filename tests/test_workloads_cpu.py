"""The seeded inputs (workloads/, shared by the oracle and the GPU path)
follow their recipes: seeds 1000 cfg + s, each point set is the stated draw
put in KD order, and the geometry the recipes state holds (separations,
planes, block sizes, the mixture's split)."""
import numpy as np

from workloads import generators as G


def _same_rows(A, B):
    """A and B hold the same rows, in any order."""
    A, B = np.asarray(A), np.asarray(B)
    return A.shape == B.shape and np.array_equal(A[np.lexsort(A.T[::-1])],
                                                 B[np.lexsort(B.T[::-1])])


def _is_kd_ordered(P, min_size=16):
    """Every node of more than min_size points splits at ceil(s/2) with the
    first half below the second along the node's widest coordinate."""
    stack = [(0, len(P))]
    while stack:
        a, b = stack.pop()
        s = b - a
        if s <= min_size:
            continue
        sub = P[a:b]
        ax = int(np.argmax(sub.max(axis=0) - sub.min(axis=0)))
        h = (s + 1) // 2
        if sub[:h, ax].max() > sub[h:, ax].min():
            return False
        stack += [(a, a + h), (a + h, b)]
    return True


def test_kd_order_is_a_permutation_and_a_split_order():
    P = np.random.default_rng(7).random((1000, 3))
    perm = G.kd_order(P)
    assert np.array_equal(np.sort(perm), np.arange(1000))
    assert _is_kd_ordered(P[perm])
    assert not _is_kd_ordered(P)


def test_gauss3d_recipe():
    wl = G.make_config("gauss3d")
    assert (wl["m"], wl["n"], wl["h"], wl["gauss_c"], wl["tol"], wl["d"], wl["leaf"]) == \
        (2000, 2000, 0.5, 1.0, 1e-6, 8, 250)
    assert wl["seed"] == 1002 and wl["entry"] == G.ENTRY_GAUSS
    X = np.random.default_rng(1000).random((2000, 3))
    Y = np.random.default_rng(1001).random((2000, 3))
    Y[:, 0] += 2.0
    assert _same_rows(wl["X"], X) and _same_rows(wl["Y"], Y)
    assert _is_kd_ordered(wl["X"]) and _is_kd_ordered(wl["Y"])
    # unit cubes whose centres are 2.0 apart: the gap is at least 1.0
    assert wl["X"][:, 0].max() <= 1.0 and wl["Y"][:, 0].min() >= 2.0


def test_differentiation_workload_recipe():
    wl = G.make_config("gauss3d_adjoint", 0.02)
    assert (wl["m"], wl["n"], wl["h"], wl["tol"], wl["d"], wl["leaf"], wl["seed"]) == \
        (1000, 1000, 0.7, 1e-6, 8, 1563, 5002)
    X = np.random.default_rng(5000).random((1000, 3))
    assert _same_rows(wl["X"], X)


def test_helmholtz_recipe():
    wl = G.make_config("helmholtz", 0.05)
    m, n = wl["m"], wl["n"]
    assert (m, n, wl["wavenumber"], wl["tol"], wl["d"], wl["leaf"], wl["seed"]) == \
        (1000, 1000, 20.0, 1e-4, 16, 625, 2002)
    assert wl["complex"] and wl["entry"] == G.ENTRY_HELMHOLTZ
    X, Y = wl["X"], wl["Y"]
    assert np.all(X[:, 2] == 0.0) and np.all(Y[:, 2] == 1.0)
    assert _same_rows(X[:, :2], np.random.default_rng(2000).random((m, 2)))
    assert _same_rows(Y[:, :2], np.random.default_rng(2001).random((n, 2)))
    assert _is_kd_ordered(X) and _is_kd_ordered(Y)


def test_coherent_recipe():
    wl = G.make_lowrank_spikes(n=300, m=250, rank=30, n_spikes=40, cfg=2)
    assert wl["G1"].shape == (250, 30) and wl["G2"].shape == (30, 300)
    lin = wl["spike_lin"]
    assert np.all(np.diff(lin) > 0) and lin.min() >= 0 and lin.max() < 250 * 300
    assert set(np.abs(wl["spike_val"]).tolist()) == {1e3}
    assert wl["seed"] == 2002


def test_laplace_blocks_recipe():
    wl = G.make_laplace_blocks(nblocks=24, cfg=3)
    ms, ns = wl["row_cnt"], wl["col_cnt"]
    assert np.all(ms != ns)
    assert ms.min() >= 64 and ns.min() >= 64 and ms.max() <= 1024 and ns.max() <= 1024
    assert np.array_equal(wl["row_off"], np.concatenate([[0], np.cumsum(ms)[:-1]]))
    assert np.array_equal(wl["col_off"], np.concatenate([[0], np.cumsum(ns)[:-1]]))
    assert wl["X"].shape == (ms.sum(), 3) and wl["Y"].shape == (ns.sum(), 3)
    for b in range(24):
        X = wl["X"][wl["row_off"][b]:wl["row_off"][b] + ms[b]]
        Y = wl["Y"][wl["col_off"][b]:wl["col_off"][b] + ns[b]]
        assert X.min() >= 0.0 and X.max() <= 1.0
        # targets: a unit cube moved by s in [3, 4]; gap >= 3 - sqrt(3) > 1.2
        gap = np.sqrt(((X[:, None, :] - Y[None, :, :]) ** 2).sum(-1)).min()
        assert gap > 1.2, (b, gap)
        assert _is_kd_ordered(X) and _is_kd_ordered(Y)


def test_gauss_mixture_recipe():
    wl = G.make_gauss_mixture(n=400, cfg=4)
    X, Y = wl["X"], wl["Y"]
    assert X.shape == (400, 8) and Y.shape == (400, 8)
    assert (wl["h"], wl["gauss_c"], wl["tol"], wl["d"], wl["seed"]) == (1.0, 2.0, 1e-6, 16, 4002)
    # rows and columns are the two halves of one cloud split at the median
    # of its widest coordinate
    P = np.vstack([X, Y])
    ax = int(np.argmax(P.max(axis=0) - P.min(axis=0)))
    assert X[:, ax].max() <= Y[:, ax].min()
    assert _is_kd_ordered(X) and _is_kd_ordered(Y)
