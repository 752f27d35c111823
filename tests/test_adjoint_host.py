"""The adjoint's workgroup tasks (paper_1901_06101_amd/csrc/hb_adj.h), compiled
for the host and run with one thread per lane and a real barrier per
__syncthreads() (tests/adjoint_host), against the frozen-pivot adjoint
oracle (oracle/adjoint.py) on the same pivots and ranks.

This checks the device code's arithmetic, indexing and barrier placement
on the CPU; the library itself has no host path and its GPU run is checked
by tests/test_gpu_zy_adjoint.py."""
import numpy as np
import pytest
import torch

from oracle import adjoint as adj
from workloads import generators as G

import _adjhost as AH


def _ybar(fs, w, b):
    f64 = dict(dtype=torch.float64)
    wl = fs.wl
    U, S, V = adj.frozen_operator(fs, torch.tensor(wl["X"], **f64), torch.tensor(wl["Y"], **f64),
                                  torch.tensor(wl["h"], **f64))
    y = (U @ (S * (V @ torch.tensor(w, **f64)))).numpy()
    return 2.0 * (y - b)


@pytest.fixture(scope="module")
def case():
    wl = G.make_gauss3d(n=400, m=360, h=0.7, leaf=100, tol=1e-6, d=8, cfg=51)
    fs = adj.FrozenStructure(wl)
    rng = np.random.default_rng(5105)
    w = rng.standard_normal(wl["n"])
    b = rng.standard_normal(wl["m"])
    return fs, w, b


def _rel(a, r):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(r)) / np.linalg.norm(np.asarray(r)))


def test_host_tasks_match_frozen_oracle(case):
    fs, w, b = case
    _, gw, gh, gX, gY = adj.frozen_gradients(fs, w, b)
    hw, hh, hX, hY = AH.vjp(fs, w, _ybar(fs, w, b), nt=4)
    assert _rel(hw, gw) <= 1e-10
    assert abs(hh - gh) <= 1e-10 * abs(gh)
    assert _rel(hX, gX) <= 1e-10
    assert _rel(hY, gY) <= 1e-10


def test_host_tasks_ragged_d16_three_levels():
    # L = 3, ragged cluster sizes, block size 16, another width
    wl = G.make_gauss3d(n=700, m=650, h=0.6, leaf=90, tol=1e-5, d=16, cfg=53)
    fs = adj.FrozenStructure(wl)
    assert fs.L == 3
    rng = np.random.default_rng(53)
    w = rng.standard_normal(wl["n"])
    b = rng.standard_normal(wl["m"])
    _, gw, gh, gX, gY = adj.frozen_gradients(fs, w, b)
    hw, hh, hX, hY = AH.vjp(fs, w, _ybar(fs, w, b), nt=8)
    assert _rel(hw, gw) <= 1e-10
    assert abs(hh - gh) <= 1e-10 * abs(gh)
    assert _rel(hX, gX) <= 1e-10
    assert _rel(hY, gY) <= 1e-10


def test_host_forward_reproduces_oracle_operator(case):
    fs, _, _ = case
    U, S, Vt = AH.forward(fs)
    assert S.size == fs.res.rank
    A = fs.res.dense()
    assert np.linalg.norm((U * S) @ Vt.T - A) <= 1e-11 * np.linalg.norm(A)


def test_host_vjp_matches_central_differences_of_host_forward(case):
    """The task code's own frozen map, differenced: h, a random direction
    over all points, and the w-gradient (exactly linear)."""
    fs, _, _ = case
    wl = fs.wl
    rng = np.random.default_rng(3)
    w = rng.standard_normal(wl["n"])
    yb = rng.standard_normal(wl["m"])

    def f(X=None, Y=None, h=None):
        U, S, Vt = AH.forward(fs, X, Y, h)
        return float(yb @ (U @ (S * (Vt.T @ w))))

    gw, gh, gX, gY = AH.vjp(fs, w, yb)
    h, dh = wl["h"], 1e-4
    c1 = (f(h=h + dh) - f(h=h - dh)) / (2 * dh)
    c2 = (f(h=h + 2 * dh) - f(h=h - 2 * dh)) / (4 * dh)
    assert abs((4 * c1 - c2) / 3 - gh) <= 1e-8 * abs(gh)
    X, Y = wl["X"], wl["Y"]
    PX = rng.standard_normal(X.shape)
    PY = rng.standard_normal(Y.shape)
    an = float(np.sum(gX * PX) + np.sum(gY * PY))

    def cp(dp):
        return (f(X + dp * PX, Y + dp * PY) - f(X - dp * PX, Y - dp * PY)) / (2 * dp)

    fd = (4 * cp(1e-4) - cp(2e-4)) / 3
    assert abs(fd - an) <= 1e-8 * abs(an)
    U, S, Vt = AH.forward(fs)
    assert np.linalg.norm(gw - Vt @ (S * (U.T @ yb))) <= 1e-12 * np.linalg.norm(gw)


def test_host_tasks_single_leaf():
    # L = 0: the root is the re-compressed leaf, no merge
    wl = G.make_gauss3d(n=120, m=100, h=0.7, leaf=250, tol=1e-6, d=8, cfg=55)
    fs = adj.FrozenStructure(wl)
    assert fs.L == 0
    rng = np.random.default_rng(55)
    w = rng.standard_normal(wl["n"])
    b = rng.standard_normal(wl["m"])
    _, gw, gh, gX, gY = adj.frozen_gradients(fs, w, b)
    hw, hh, hX, hY = AH.vjp(fs, w, _ybar(fs, w, b), nt=4)
    assert _rel(hw, gw) <= 1e-10
    assert abs(hh - gh) <= 1e-10 * abs(gh)
    assert _rel(hX, gX) <= 1e-10
    assert _rel(hY, gY) <= 1e-10


def test_host_tasks_eight_dimensional_points():
    # the 8-D mixture: the largest point dimension and c = 2 in the Gaussian
    wl = G.make_gauss_mixture(n=600, leaf=150, tol=1e-5, d=16, cfg=72)
    fs = adj.FrozenStructure(wl)
    assert wl["X"].shape[1] == 8 and wl["gauss_c"] == 2.0
    rng = np.random.default_rng(9)
    w = rng.standard_normal(wl["n"])
    b = rng.standard_normal(wl["m"])
    _, gw, gh, gX, gY = adj.frozen_gradients(fs, w, b)
    hw, hh, hX, hY = AH.vjp(fs, w, _ybar(fs, w, b), nt=4)
    assert _rel(hw, gw) <= 1e-10
    assert abs(hh - gh) <= 1e-10 * abs(gh)
    assert _rel(hX, gX) <= 1e-10
    assert _rel(hY, gY) <= 1e-10


def test_host_tasks_block_size_32():
    # the largest block size (32 rows and columns per iteration), tol 1e-7
    wl = G.make_gauss3d(n=600, m=520, h=0.8, leaf=150, tol=1e-7, d=32, cfg=54)
    fs = adj.FrozenStructure(wl)
    rng = np.random.default_rng(54)
    w = rng.standard_normal(wl["n"])
    b = rng.standard_normal(wl["m"])
    _, gw, gh, gX, gY = adj.frozen_gradients(fs, w, b)
    hw, hh, hX, hY = AH.vjp(fs, w, _ybar(fs, w, b), nt=4)
    assert _rel(hw, gw) <= 1e-10
    assert abs(hh - gh) <= 1e-10 * abs(gh)
    assert _rel(hX, gX) <= 1e-8
    assert _rel(hY, gY) <= 1e-8


def test_lane_count_does_not_change_the_result(case):
    fs, w, b = case
    yb = _ybar(fs, w, b)
    one = AH.vjp(fs, w, yb, nt=1)
    many = AH.vjp(fs, w, yb, nt=16)
    for a, r in zip(one, many):
        assert np.max(np.abs(np.asarray(a) - np.asarray(r))) <= 1e-12 * max(1.0, np.max(np.abs(r)))


def test_outputs_left_out_are_not_written():
    """Null output pointers: only the wanted gradients are formed, and they
    equal those of the full call (the reductions of the others are not
    launched, and the root writes no w-gradient)."""
    wl = G.make_gauss3d(n=400, m=360, h=0.7, leaf=100, tol=1e-6, d=8, cfg=51)
    fs = adj.FrozenStructure(wl)
    rng = np.random.default_rng(8)
    w = rng.standard_normal(wl["n"])
    yb = rng.standard_normal(wl["m"])
    full = AH.vjp(fs, w, yb, nt=4)
    for want in (("h",), ("w",), ("x", "y"), ("y",)):
        got = AH.vjp(fs, w, yb, nt=4, want=want)
        for key, g, r in zip(("w", "h", "x", "y"), got, full):
            if key in want:
                assert np.array_equal(np.asarray(g), np.asarray(r)), (want, key)
            else:
                assert g is None


@pytest.mark.parametrize("extra", [(), AH.SPLIT_ALL], ids=["library", "jacobi_split_all"])
def test_workgroup_of_256_lanes_as_fibers(extra):
    """The GPU's 256 lanes per workgroup, run as fibers: lane-count dependent
    paths (dot products shared by 256/j lanes, reductions over 256 partial
    sums, Jacobi pairs shared over lanes) and every barrier reached by all
    lanes, with row chunks."""
    wl = G.make_gauss3d(n=200, m=180, h=0.7, leaf=50, tol=1e-6, d=8, cfg=52)
    fs = adj.FrozenStructure(wl)
    rng = np.random.default_rng(3)
    w = rng.standard_normal(wl["n"])
    yb = rng.standard_normal(wl["m"])
    ref = AH.vjp(fs, w, yb, nt=1)
    AH.set_chunking(16, 32, extra=extra)
    AH.set_fibers(True, extra=extra)
    try:
        got = AH.vjp(fs, w, yb, nt=256, extra=extra)
        split = AH.last_split(extra)[0]
    finally:
        diverged, barriers = AH.set_fibers(False, extra=extra)
        AH.set_chunking(extra=extra)
    assert not diverged
    assert split > 0 and barriers > 0
    for a, r in zip(got, ref):
        a, r = np.asarray(a), np.asarray(r)
        assert np.max(np.abs(a - r)) <= 1e-11 * max(1.0, np.max(np.abs(r)))


@pytest.mark.parametrize("chunking,nt,extra", [(None, 4, ()), ((16, 32), 4, ()),
                                               ((16, 32), 32, AH.SPLIT_ALL)])
def test_no_data_race_under_thread_sanitizer(tmp_path, chunking, nt, extra):
    # both merge shapes: wide first-level merges (45 rows), tall ones above;
    # with small row chunks the tall ones run split; with 32 lanes and every
    # Jacobi SVD split, the leaf re-compressions' pairs (21 to 29 columns)
    # are shared by two lanes each
    wl = G.make_gauss3d(n=200, m=180, h=0.7, leaf=50, tol=1e-6, d=8, cfg=52)
    fs = adj.FrozenStructure(wl)
    rng = np.random.default_rng(1)
    w = rng.standard_normal(wl["n"])
    yb = rng.standard_normal(wl["m"])
    exe = AH.build_tsan(extra)
    rc, err, outs = AH.run_exe(exe, fs, w, yb, nt, str(tmp_path), chunking)
    assert rc == 0, err[-4000:]
    assert "ThreadSanitizer" not in err
    ref = AH.vjp(fs, w, yb, nt=1)
    for a, r in zip(outs, ref):
        assert np.max(np.abs(np.asarray(a) - np.asarray(r))) <= 1e-12 * max(1.0, np.max(np.abs(r)))


@pytest.mark.parametrize("chunking,nt,extra", [(None, 2, ()), ((16, 32), 2, ()),
                                               ((16, 32), 32, AH.SPLIT_ALL)])
def test_no_memory_error_under_address_sanitizer(tmp_path, chunking, nt, extra):
    wl = G.make_gauss3d(n=200, m=180, h=0.7, leaf=50, tol=1e-6, d=8, cfg=52)
    fs = adj.FrozenStructure(wl)
    rng = np.random.default_rng(2)
    w = rng.standard_normal(wl["n"])
    yb = rng.standard_normal(wl["m"])
    exe = AH.build_asan(extra)
    rc, err, outs = AH.run_exe(exe, fs, w, yb, nt, str(tmp_path), chunking)
    assert rc == 0, err[-4000:]
    assert "Sanitizer" not in err and "runtime error" not in err
    ref = AH.vjp(fs, w, yb, nt=2)
    for a, r in zip(outs, ref):
        assert np.max(np.abs(np.asarray(a) - np.asarray(r))) <= 1e-12 * max(1.0, np.max(np.abs(r)))


@pytest.mark.parametrize("extra", [(), AH.SPLIT_ALL], ids=["library", "jacobi_split_all"])
@pytest.mark.parametrize("name,chunk", [("n400", 16), ("n700", 8)])
def test_merges_split_over_row_chunks(name, chunk, extra):
    """Tall merges run as row chunks (a two-level thin QR, per-chunk partial
    sums): forced small chunks make every merge above the first level split.
    The second build shares every Jacobi pair over lanes."""
    wl = {"n400": lambda: G.make_gauss3d(n=400, m=360, h=0.7, leaf=100, tol=1e-6, d=8, cfg=51),
          "n700": lambda: G.make_gauss3d(n=700, m=650, h=0.6, leaf=90, tol=1e-5, d=16,
                                         cfg=53)}[name]()
    fs = adj.FrozenStructure(wl)
    rng = np.random.default_rng(5)
    w = rng.standard_normal(wl["n"])
    b = rng.standard_normal(wl["m"])
    _, gw, gh, gX, gY = adj.frozen_gradients(fs, w, b)
    yb = _ybar(fs, w, b)
    AH.set_chunking(chunk, 32, extra=extra)
    try:
        U, S, Vt = AH.forward(fs, extra=extra)
        assert AH.last_split(extra)[0] > 0
        hw, hh, hX, hY = AH.vjp(fs, w, yb, nt=4, extra=extra)
    finally:
        AH.set_chunking(extra=extra)
    A = fs.res.dense()
    assert np.linalg.norm((U * S) @ Vt.T - A) <= 1e-11 * np.linalg.norm(A)
    assert _rel(hw, gw) <= 1e-10
    assert abs(hh - gh) <= 1e-10 * abs(gh)
    assert _rel(hX, gX) <= 1e-10
    assert _rel(hY, gY) <= 1e-10


def test_planner_rejects_inconsistent_structures(case):
    fs, w, b = case
    yb = np.zeros(fs.wl["m"])
    li, recs, ranks, dm, stride = AH.records_from_oracle(fs)

    def status(li2, recs2, ranks2):
        try:
            AH.vjp(fs, w, yb, nt=1, info=(li2, recs2, ranks2, dm, stride))
        except RuntimeError as e:
            return int(str(e).split()[-1])
        return 0

    assert status(li, recs, ranks) == 0
    bad = recs.copy()
    bad[3] = fs.wl["m"]  # a row index outside its leaf
    assert status(li, bad, ranks) == -1
    bad = recs.copy()
    bad[3 + dm + 1] = bad[3 + dm]  # a repeated column
    assert status(li, bad, ranks) == -1
    bad = recs.copy()
    bad[2] = 0  # d_k = 0 before the last record of a leaf with more records
    if li[0, 4] > 1:
        assert status(li, bad, ranks) == -1
    neg = ranks.copy()
    neg[-1] = -1  # a negative rank
    assert status(li, recs, neg) == -1
    big = ranks.copy()
    big[0] = 10_000  # more than r1 + r2
    assert status(li, recs, big) == -1
    li2 = li.copy()
    li2[0, 5] = li2[0, 5] + 1000  # leaf rank above its BACA rank
    assert status(li2, recs, ranks) == -1


def test_merges_wider_than_tall():
    # leaves of 45 rows whose ranks add up to more than 45 at the first
    # merge: the stacked factor is wide and its thin SVD has rows columns
    wl = G.make_gauss3d(n=200, m=180, h=0.7, leaf=50, tol=1e-6, d=8, cfg=52)
    fs = adj.FrozenStructure(wl)
    nb = 1 << fs.L
    r = [fs.res.leaf_info[b]["rank"] for b in range(nb * nb)]
    m0 = fs.res.leaf_info[0]["m0"]
    assert max(r[2 * v] + r[2 * v + 1] for v in range(nb // 2)) > m0
    U, S, Vt = AH.forward(fs)
    A = fs.res.dense()
    assert np.linalg.norm((U * S) @ Vt.T - A) <= 1e-11 * np.linalg.norm(A)
    rng = np.random.default_rng(52)
    w = rng.standard_normal(wl["n"])
    b = rng.standard_normal(wl["m"])
    _, gw, gh, gX, gY = adj.frozen_gradients(fs, w, b)
    hw, hh, hX, hY = AH.vjp(fs, w, _ybar(fs, w, b), nt=4)
    assert _rel(hw, gw) <= 1e-10
    assert abs(hh - gh) <= 1e-10 * abs(gh)
    assert _rel(hX, gX) <= 1e-10
    assert _rel(hY, gY) <= 1e-10


def test_adjoint_reference_size_checks():
    """The differentiation workload's reference size (its geometry at n =
    2000, leaf 250, L = 3): the host-built adjoint against the frozen
    oracle, against central differences (step 1e-4, FP64) of the host-built
    frozen map in h, along a random direction over all points and in six
    random coordinates, and the gap to the exact dense gradient."""
    wl = G.make_gauss3d(n=2000, h=0.7, leaf=250, tol=1e-6, d=8, cfg=5)
    fs = adj.FrozenStructure(wl)
    assert fs.L == 3
    rng = np.random.default_rng(5)
    w = rng.standard_normal(wl["n"])
    b = rng.standard_normal(wl["m"])
    _, gw, gh, gX, gY = adj.frozen_gradients(fs, w, b)
    yb = _ybar(fs, w, b)
    hw, hh, hX, hY = AH.vjp(fs, w, yb, nt=1)
    assert _rel(hw, gw) <= 1e-10
    assert abs(hh - gh) <= 1e-10 * abs(gh)
    assert _rel(hX, gX) <= 1e-10
    assert _rel(hY, gY) <= 1e-10

    def f(X=None, Y=None, h=None):
        U, S, Vt = AH.forward(fs, X, Y, h)
        return float(yb @ (U @ (S * (Vt.T @ w))))

    step = 1e-4
    h = wl["h"]
    fd = (f(h=h + step) - f(h=h - step)) / (2 * step)
    assert abs(fd - hh) <= 1e-5 * abs(hh)
    X, Y = wl["X"], wl["Y"]
    PX = rng.standard_normal(X.shape)
    PY = rng.standard_normal(Y.shape)
    fd = (f(X + step * PX, Y + step * PY) - f(X - step * PX, Y - step * PY)) / (2 * step)
    an = float(np.sum(hX * PX) + np.sum(hY * PY))
    assert abs(fd - an) <= 1e-5 * abs(an)
    scale = max(np.max(np.abs(hX)), np.max(np.abs(hY)))
    for _ in range(3):
        for side, G_, P_ in ((0, hX, X), (1, hY, Y)):
            i = int(rng.integers(P_.shape[0]))
            q = int(rng.integers(P_.shape[1]))
            E = np.zeros(P_.shape)
            E[i, q] = step
            if side == 0:
                fd = (f(X + E, Y) - f(X - E, Y)) / (2 * step)
            else:
                fd = (f(X, Y + E) - f(X, Y - E)) / (2 * step)
            assert abs(fd - G_[i, q]) <= 1e-5 * max(abs(G_[i, q]), 1e-3 * scale)
    # the frozen map against the exact dense loss: the truncation level
    _, dw, dh, dX, dY = adj.dense_gradients(wl, w, b)
    assert abs(hh - dh) <= 1e-3 * abs(dh)
    for a, r in ((hw, dw), (hX, dX), (hY, dY)):
        assert _rel(a, r) <= 1e-3


@pytest.mark.parametrize("seed", [11, 12, 13, 14, 15, 16])
def test_random_configurations_match_oracle(seed):
    """Random sizes (m != n), leaf sizes, block sizes, tolerances, lane
    counts (not powers of two too) and row chunks.  Bar 1e-9: near a
    truncation, trailing singular values that sit close together amplify
    rounding through 1/(s_j^2 - s_i^2); 1.0e-10 is the largest difference
    seen over such draws, the same for every lane count and chunking."""
    rng = np.random.default_rng(seed)
    n, m = int(rng.integers(120, 500)), int(rng.integers(120, 500))
    leaf, d = int(rng.integers(40, 160)), int(rng.choice([4, 8, 16]))
    tol, h = float(rng.choice([1e-4, 1e-6, 1e-8])), float(rng.uniform(0.5, 0.9))
    nt, chunk = int(rng.choice([1, 3, 8, 24])), int(rng.choice([0, 8, 32]))
    wl = G.make_gauss3d(n=n, m=m, h=h, leaf=leaf, tol=tol, d=d, cfg=200 + seed)
    fs = adj.FrozenStructure(wl)
    w = rng.standard_normal(n)
    b = rng.standard_normal(m)
    _, gw, gh, gX, gY = adj.frozen_gradients(fs, w, b)
    if chunk:
        AH.set_chunking(chunk, 32)
    try:
        hw, hh, hX, hY = AH.vjp(fs, w, _ybar(fs, w, b), nt=nt)
    finally:
        AH.set_chunking()
    assert _rel(hw, gw) <= 1e-9
    assert abs(hh - gh) <= 1e-9 * abs(gh)
    assert _rel(hX, gX) <= 1e-9
    assert _rel(hY, gY) <= 1e-9
