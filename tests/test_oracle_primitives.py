"""Pins for the oracle's building blocks, each against something other than
the oracle itself: published generator output, brute-force least squares,
closed forms and dense products."""
import numpy as np
import pytest

import oracle
from oracle.entries import EntrySource
from oracle.qrcp import householder, qrcp
from oracle.splitmix import first_column_block, splitmix64_stream


def test_splitmix64_published_vector():
    # First outputs of SplitMix64 from state 0, as published with the
    # generator (Steele, Lea and Flood 2014; Vigna's reference code).
    out = splitmix64_stream(0, 3)
    assert out == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


@pytest.mark.parametrize("n0,d", [(250, 8), (7, 16), (1, 1), (625, 16)])
def test_first_column_block_is_partial_permutation(n0, d):
    for b in range(5):
        J = first_column_block(1002, b, n0, d)
        assert J.size == min(d, n0)
        assert len(set(J.tolist())) == J.size
        assert J.min() >= 0 and J.max() < n0
    assert not np.array_equal(first_column_block(1002, 0, 250, 8),
                              first_column_block(1002, 1, 250, 8))


@pytest.mark.parametrize("cplx", [False, True])
def test_householder_maps_to_e1(cplx):
    rng = np.random.default_rng(0)
    x = rng.standard_normal(9) + (1j * rng.standard_normal(9) if cplx else 0)
    v, beta, alpha = householder(x)
    H = np.eye(9) - beta * np.outer(v, v.conj())
    e = np.zeros(9, dtype=H.dtype)
    e[0] = alpha
    assert np.allclose(H @ x, e, atol=1e-14)
    assert np.allclose(H.conj().T @ H, np.eye(9), atol=1e-14)
    assert abs(abs(alpha) - np.linalg.norm(x)) < 1e-14


def _greedy_by_least_squares(M, k):
    """Pivots chosen by recomputing every residual norm with lstsq."""
    sel = []
    norms = []
    for _ in range(k):
        best, bestn = None, -1.0
        for c in range(M.shape[1]):
            if c in sel:
                continue
            if sel:
                B = M[:, sel]
                coef = np.linalg.lstsq(B, M[:, c], rcond=None)[0]
                res = M[:, c] - B @ coef
            else:
                res = M[:, c]
            nr = np.linalg.norm(res)
            if nr > bestn * (1 + 1e-12):
                best, bestn = c, nr
        sel.append(best)
        norms.append(bestn)
    return sel, np.array(norms)


@pytest.mark.parametrize("cplx", [False, True])
@pytest.mark.parametrize("shape", [(8, 40), (16, 16), (5, 30)])
def test_qrcp_matches_bruteforce_greedy(cplx, shape):
    rng = np.random.default_rng(42 + shape[0])
    p, q = shape
    M = rng.standard_normal((p, q)) + (1j * rng.standard_normal((p, q)) if cplx else 0)
    # make it rank-revealing-interesting: decaying column scales
    M = M * np.exp(-0.2 * np.arange(q))[None, :]
    k = min(p, q)
    res = qrcp(M, k)
    sel, norms = _greedy_by_least_squares(M, k)
    assert res.piv.tolist() == sel
    assert np.allclose(np.abs(res.tdiag), norms, rtol=1e-10)
    # Q T reproduces the pivoted columns:  Q^H M(:, piv) = T11 (upper)
    QhM = res.apply_qh(M)
    order = list(res.piv) + [c for c in range(q) if c not in set(res.piv)]
    assert np.allclose(QhM[:k, order], res.T, atol=1e-12)
    assert np.allclose(np.tril(res.T[:k, :k], -1), 0, atol=1e-12)
    if p > k:
        assert np.allclose(QhM[k:, :], 0, atol=1e-12)


def test_qrcp_ties_go_to_lowest_position():
    M = np.zeros((3, 5))
    M[0, 1] = 2.0
    M[0, 3] = 2.0
    res = qrcp(M, 3)
    assert res.piv[0] == 1
    # after the first step every trailing norm is zero: lowest remaining
    assert res.piv[1] == 0


@pytest.mark.parametrize("cplx", [False, True])
def test_qrcp_rounding_level_norms_tie_to_lowest_position(cplx):
    """An exactly rank-2 panel: after two steps every trailing norm is
    rounding only (the reading counts it as zero), so the later picks are the
    lowest remaining positions, whatever the rounding left behind.  A panel
    whose third column is small but well above rounding keeps its greedy
    pick."""
    rng = np.random.default_rng(3)

    def rnd(*s):
        return rng.standard_normal(s) + (1j * rng.standard_normal(s) if cplx else 0)

    M = rnd(6, 2) @ rnd(2, 12)
    res = qrcp(M, 6)
    assert set(res.piv[:2].tolist()) <= set(range(12))
    rest = [c for c in range(12) if c not in res.piv[:2]]
    assert res.piv[2:].tolist() == rest[:4]
    assert np.all(np.abs(res.tdiag[2:]) < 1e-13 * np.abs(res.tdiag[0]))
    # a third direction at 1e-9 of the panel is information, not rounding
    M2 = M + 1e-9 * np.linalg.norm(M) * np.outer(rnd(6), np.eye(12)[7])
    res2 = qrcp(M2, 3)
    assert res2.piv[2] == 7 or 7 in res2.piv[:2]


def test_jacobi_closed_forms():
    # diagonal
    s = oracle.jacobi_svd(np.diag([3.0, -1.0, 2.0]))[1]
    assert np.allclose(s, [3, 2, 1])
    # 2x2: singular values from the closed form of the 2x2 Gram eigenvalues
    A = np.array([[1.0, 2.0], [3.0, 4.0]])
    G = A.T @ A
    tr, det = np.trace(G), np.linalg.det(G)
    lam = np.array([(tr + np.sqrt(tr * tr - 4 * det)) / 2,
                    (tr - np.sqrt(tr * tr - 4 * det)) / 2])
    assert np.allclose(oracle.jacobi_svd(A)[1], np.sqrt(lam), rtol=1e-14)
    # constructed U diag(s) V^H with known s (real and complex, tall and wide)
    rng = np.random.default_rng(3)
    for (m, n, cplx) in [(30, 12, False), (12, 30, True), (20, 20, True)]:
        k = min(m, n)
        X = rng.standard_normal((m, k)) + (1j * rng.standard_normal((m, k)) if cplx else 0)
        Y = rng.standard_normal((n, k)) + (1j * rng.standard_normal((n, k)) if cplx else 0)
        Qx, _ = np.linalg.qr(X)
        Qy, _ = np.linalg.qr(Y)
        sv = np.sort(np.exp(-rng.uniform(0, 20, k)))[::-1]
        A = (Qx * sv) @ Qy.conj().T
        U, s, V = oracle.jacobi_svd(A)
        assert np.allclose(s, sv, rtol=1e-10, atol=1e-15 * sv[0])
        assert np.allclose((U * s) @ V.conj().T, A, atol=1e-13)


def test_eps_rank_definition():
    s = np.array([10.0, 5.0, 1e-5, 9.99e-6, 1e-7])
    assert oracle.eps_rank(s, 1e-6) == 3
    assert oracle.eps_rank(s, 1e-1) == 2
    assert oracle.eps_rank(np.zeros(3), 1e-6) == 0
    assert oracle.eps_rank(np.zeros(0), 1e-6) == 0
    # exactly on the threshold is kept
    assert oracle.eps_rank(np.array([1.0, 0.5]), 0.5) == 2


@pytest.mark.parametrize("cplx", [False, True])
def test_lrnorm_and_update_equal_dense_norms(cplx):
    rng = np.random.default_rng(7)

    def rnd(*s):
        return rng.standard_normal(s) + (1j * rng.standard_normal(s) if cplx else 0)

    U, V = rnd(40, 9), rnd(9, 33)
    Uk, Vk = rnd(40, 5), rnd(5, 33)
    nu = oracle.lrnorm(Uk, Vk)
    assert abs(nu - np.linalg.norm(Uk @ Vk)) <= 1e-13 * nu
    mu2 = np.linalg.norm(U @ V) ** 2
    mu2n = oracle.lrnorm_update(U, V, mu2, Uk, Vk, nu)
    full = np.linalg.norm(np.hstack([U, Uk]) @ np.vstack([V, Vk])) ** 2
    assert abs(mu2n - full) <= 1e-12 * full


@pytest.mark.parametrize("cplx", [False, True])
@pytest.mark.parametrize("where", ["U_zero_column", "V_zero_row", "U_repeated_column"])
def test_lrnorm_cholesky_breakdown_fallback(cplx, where):
    """Reading of a Cholesky breakdown in LRnorm (eqs. (11)-(12)): a Gram
    matrix that is only positive semidefinite (a zero column of U_k, a zero
    row of V_k, or a repeated column) stops the factorisation, and nu comes
    from nu^2 = Re sum(G_U o conj(G_V)), which is ||U_k V_k||_F^2 exactly.
    The breakdown is checked to happen, so the fallback branch is what runs;
    a dropped conjugate or a transposed Gram matrix fails the complex cases."""
    from oracle.baca import _chol_upper
    rng = np.random.default_rng(11)

    def rnd(*s):
        return rng.standard_normal(s) + (1j * rng.standard_normal(s) if cplx else 0)

    Uk, Vk = rnd(30, 4), rnd(4, 25)
    if where == "U_zero_column":
        Uk[:, 2] = 0.0
    elif where == "V_zero_row":
        Vk[1, :] = 0.0
    else:
        Uk[:, 3] = Uk[:, 0]
        Uk[:, 1] = 0.0  # a repeated column alone may factor by rounding
    GU = Uk.conj().T @ Uk
    GV = Vk @ Vk.conj().T
    assert _chol_upper(GU) is None or _chol_upper(GV) is None
    nu = oracle.lrnorm(Uk, Vk)
    ref = np.linalg.norm(Uk @ Vk)
    assert abs(nu - ref) <= 1e-13 * ref


def test_entries_closed_values():
    X = np.array([[0.0, 0.0, 0.0]])
    Y = np.array([[0.5, 0.0, 0.0], [0.0, 2.0, 0.0]])
    g = EntrySource(dict(entry=1, X=X, Y=Y, h=0.5, gauss_c=1.0)).block([0], [0, 1])
    assert np.allclose(g, [[np.exp(-1.0), np.exp(-16.0)]], rtol=1e-15)
    g2 = EntrySource(dict(entry=1, X=X, Y=Y, h=1.0, gauss_c=2.0)).block([0], [1])
    assert np.allclose(g2, [[np.exp(-2.0)]])
    lap = EntrySource(dict(entry=2, X=X, Y=Y)).block([0], [0, 1])
    assert np.allclose(lap, [[2.0, 0.5]])
    hh = EntrySource(dict(entry=3, X=X, Y=Y, wavenumber=20.0)).block([0], [1])[0, 0]
    assert np.isclose(abs(hh), 1.0 / (8 * np.pi))
    assert np.isclose(np.angle(hh), np.angle(np.exp(40j)))
    G1 = np.arange(6.0).reshape(3, 2)
    G2 = np.ones((2, 4))
    src = EntrySource(dict(entry=4, G1=G1, G2=G2, spike_lin=np.array([1 * 4 + 2]),
                           spike_val=np.array([100.0])))
    D = src.dense()
    ref = G1 @ G2
    ref[1, 2] += 100.0
    assert np.array_equal(D, ref)


def test_efie2d_entries_against_hankel_closed_forms():
    """EFIE2D entries H_0^(2)(k r) = J_0(k r) - i Y_0(k r) (Section "Numerical
    Results", kernel 2), pinned without re-calling the library routine: the
    first zeros of J_0 and Y_0 (2.404825557695773 and 0.8935769662791675,
    Abramowitz and Stegun, Table 9.5) make the real and imaginary parts
    vanish; for small arguments J_0 -> 1 and Y_0 ~ (2/pi)(ln(x/2) + gamma);
    for large arguments H_0^(2)(x) ~ sqrt(2/(pi x)) exp(-i(x - pi/4)) (the
    sign of the exponent tells the second kind from the first)."""
    def entry(x, k=1.0):
        X = np.array([[0.0, 0.0]])
        Y = np.array([[x, 0.0]])
        return EntrySource(dict(entry=5, X=X, Y=Y, wavenumber=k)).block([0], [0])[0, 0]

    assert abs(entry(2.404825557695773).real) < 1e-15
    assert abs(entry(0.8935769662791675).imag) < 1e-15
    # the zero of J_0 through k and r: k = 2, r = x / 2
    assert abs(entry(2.404825557695773 / 2, k=2.0).real) < 1e-15
    x = 1e-6
    h = entry(x)
    assert abs(h.real - 1.0) < 1e-12
    assert abs(-h.imag - (2 / np.pi) * (np.log(x / 2) + np.euler_gamma)) < 1e-10
    x = 4000.0
    asym = np.sqrt(2 / (np.pi * x)) * np.exp(-1j * (x - np.pi / 4))
    assert abs(entry(x) - asym) < 1e-4 * abs(asym)


def test_polynomial_entries_and_rank():
    """(x^T y + h)^2 (Section "Numerical Results", kernel 5): a closed value,
    and the rank of the matrix is at most D (D + 3) / 2 + 1, the dimension
    of the quadratic polynomials in D variables."""
    X = np.array([[1.0, 2.0]])
    Y = np.array([[3.0, -1.0]])
    v = EntrySource(dict(entry=6, X=X, Y=Y, h=0.5)).block([0], [0])[0, 0]
    assert v == (3.0 - 2.0 + 0.5) ** 2
    rng = np.random.default_rng(4)
    for D in (2, 5):
        wl = dict(entry=6, X=rng.random((60, D)), Y=rng.random((70, D)), h=0.2)
        s = np.linalg.svd(EntrySource(wl).dense(), compute_uv=False)
        assert np.sum(s > 1e-12 * s[0]) == D * (D + 3) // 2 + 1


def test_cluster_tree_and_levels():
    assert oracle.tree_levels(2000, 2000, 250) == 3
    assert oracle.tree_levels(20000, 20000, 625) == 5
    assert oracle.tree_levels(50000, 50000, 1563) == 5
    assert oracle.tree_levels(100000, 100000, 1563) == 6
    assert oracle.tree_levels(300, 300, 1000) == 0
    assert oracle.tree_levels(3, 1000, 100) == 1  # capped so no node is empty
    lv = oracle.cluster_tree(7, 2)
    assert lv[1] == [(0, 4), (4, 3)]
    assert lv[2] == [(0, 2), (2, 2), (4, 2), (6, 1)]
