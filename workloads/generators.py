"""Seeded workload generators.

Every workload mirrors one of the paper's experiment families (Section
"Numerical Results"): kernel matrices between two point clouds whose rows and
columns are KD-permuted, and a product of random factors.  The paper's own
datasets (SUSY, MNIST, EFIE/Frontal meshes) are not available; the synthetic
stand-ins here reproduce their shape (dimension, separation, spectrum class).

Seeds follow one rule: a workload with id ``cfg`` uses ``1000*cfg + s`` with
s = 0 (row points), 1 (column points), 2 (the method's own seed for its random
first column block), 3 (factors, spikes, cluster centres), 4 (w) and 5 (b).

The dictionaries returned here carry plain NumPy arrays only.
"""
from __future__ import annotations

import math

import numpy as np

# Entry-function identifiers shared by the C ABI and the oracle's dispatcher.
ENTRY_GAUSS = 1
ENTRY_LAPLACE = 2
ENTRY_HELMHOLTZ = 3
ENTRY_LOWRANK_SPIKES = 4
ENTRY_EFIE2D = 5
ENTRY_POLYNOMIAL = 6

CONFIG_NAMES = ("gauss3d", "helmholtz", "coherent", "laplace_batched",
                "gauss_mixture", "gauss3d_adjoint", "efie2d", "polynomial")


def kd_order(points: np.ndarray, min_size: int = 16) -> np.ndarray:
    """Permutation that orders ``points`` along a binary KD split tree.

    A node of size s is split at its ceil(s/2)-th point along its widest
    coordinate (ties broken by index, stable sort), first half first.  The
    recursion stops at ``min_size`` points.  Because every level uses the
    same ceil(s/2) split that the cluster trees use, the ordering is
    consistent with a cluster tree of any depth whose leaves hold at least
    ``min_size`` points.
    """
    n = points.shape[0]
    perm = np.arange(n)
    stack = [(0, n)]
    while stack:
        a, b = stack.pop()
        s = b - a
        if s <= min_size:
            continue
        idx = perm[a:b]
        sub = points[idx]
        widths = sub.max(axis=0) - sub.min(axis=0)
        ax = int(np.argmax(widths))
        order = np.argsort(sub[:, ax], kind="stable")
        perm[a:b] = idx[order]
        h = (s + 1) // 2
        stack.append((a, a + h))
        stack.append((a + h, b))
    return perm


def _kd(points: np.ndarray) -> np.ndarray:
    return np.ascontiguousarray(points[kd_order(points)])


def make_gauss3d(n: int = 2000, m: int | None = None, h: float = 0.5,
                 gauss_c: float = 1.0, tol: float = 1e-6, d: int = 8,
                 leaf: int = 250, cfg: int = 1) -> dict:
    """Gaussian kernel exp(-|x-y|^2/(c h^2)) between two unit cubes in R^3
    whose centres are 2.0 apart (minimum gap 1.0)."""
    m = n if m is None else m
    X = np.random.default_rng(1000 * cfg + 0).random((m, 3))
    Y = np.random.default_rng(1000 * cfg + 1).random((n, 3))
    Y[:, 0] += 2.0
    return dict(name="gauss3d", entry=ENTRY_GAUSS, X=_kd(X), Y=_kd(Y), m=m, n=n,
                h=h, gauss_c=gauss_c, wavenumber=0.0, tol=tol, d=d, leaf=leaf,
                seed=1000 * cfg + 2, complex=False)


def make_helmholtz_plates(n: int = 20000, m: int | None = None, k: float = 20.0,
                          tol: float = 1e-4, d: int = 16, leaf: int = 625,
                          cfg: int = 2) -> dict:
    """Helmholtz free-space kernel exp(i k r)/(4 pi r) between two parallel
    unit squares 1.0 apart (z=0 and z=1)."""
    m = n if m is None else m
    X = np.zeros((m, 3))
    Y = np.ones((n, 3))
    X[:, :2] = np.random.default_rng(1000 * cfg + 0).random((m, 2))
    Y[:, :2] = np.random.default_rng(1000 * cfg + 1).random((n, 2))
    return dict(name="helmholtz", entry=ENTRY_HELMHOLTZ, X=_kd(X), Y=_kd(Y),
                m=m, n=n, h=0.0, gauss_c=0.0, wavenumber=k, tol=tol, d=d,
                leaf=leaf, seed=1000 * cfg + 2, complex=True)


def make_lowrank_spikes(n: int = 20000, m: int | None = None, rank: int = 30,
                        n_spikes: int = 200, spike_mag: float = 1e3,
                        tol: float = 1e-4, d: int = 16, leaf: int = 625,
                        cfg: int = 2) -> dict:
    """Product of i.i.d. N(0,1) factors G1 (m x rank) G2 (rank x n) plus
    ``n_spikes`` distinct entries of magnitude ``spike_mag`` with random sign.

    Spikes are returned sorted by their linear index i*n + j."""
    m = n if m is None else m
    rng = np.random.default_rng(1000 * cfg + 3)
    G1 = rng.standard_normal((m, rank))
    G2 = rng.standard_normal((rank, n))
    n_spikes = min(n_spikes, m * n)
    lin = rng.choice(m * n, size=n_spikes, replace=False) if n_spikes else \
        np.zeros(0, dtype=np.int64)
    lin = np.sort(lin.astype(np.int64))
    sign = rng.choice(np.array([-1.0, 1.0]), size=n_spikes)
    vals = sign * spike_mag
    return dict(name="coherent", entry=ENTRY_LOWRANK_SPIKES, X=None, Y=None,
                m=m, n=n, G1=np.ascontiguousarray(G1),
                G2=np.ascontiguousarray(G2), spike_lin=lin,
                spike_val=np.ascontiguousarray(vals), tol=tol, d=d, leaf=leaf,
                seed=1000 * cfg + 2, complex=False, h=0.0, gauss_c=0.0,
                wavenumber=0.0)


def make_laplace_blocks(nblocks: int = 4096, lo: int = 64, hi: int = 1024,
                        tol: float = 1e-4, d: int = 8, leaf: int = 256,
                        cfg: int = 3) -> dict:
    """Independent Laplace blocks 1/r between separated clusters in R^3.

    Block b has m_b sources in U[0,1]^3 and n_b targets in U[0,1]^3 shifted
    by s_b * u_b (u_b uniform on the sphere, s_b ~ U[3,4]); m_b, n_b are
    log-uniform in [lo, hi] and redrawn until they differ.  Points of all
    blocks are concatenated; ``row_off``/``col_off`` index them."""
    rng = np.random.default_rng(1000 * cfg + 3)
    ms = np.empty(nblocks, dtype=np.int64)
    ns = np.empty(nblocks, dtype=np.int64)
    for b in range(nblocks):
        while True:
            mb = int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))
            nb = int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))
            if mb != nb:
                break
        ms[b], ns[b] = mb, nb
    rx = np.random.default_rng(1000 * cfg + 0)
    ry = np.random.default_rng(1000 * cfg + 1)
    Xs, Ys = [], []
    for b in range(nblocks):
        X = rx.random((ms[b], 3))
        u = rng.standard_normal(3)
        u /= np.linalg.norm(u)
        s = rng.uniform(3.0, 4.0)
        Y = ry.random((ns[b], 3)) + s * u
        Xs.append(_kd(X))
        Ys.append(_kd(Y))
    row_off = np.concatenate([[0], np.cumsum(ms)[:-1]]).astype(np.int64)
    col_off = np.concatenate([[0], np.cumsum(ns)[:-1]]).astype(np.int64)
    return dict(name="laplace_batched", entry=ENTRY_LAPLACE,
                X=np.ascontiguousarray(np.concatenate(Xs)),
                Y=np.ascontiguousarray(np.concatenate(Ys)),
                row_off=row_off, row_cnt=ms, col_off=col_off, col_cnt=ns,
                nblocks=nblocks, tol=tol, d=d, leaf=leaf,
                seed=1000 * cfg + 2, complex=False, h=0.0, gauss_c=0.0,
                wavenumber=0.0)


def make_gauss_mixture(n: int = 100000, dim: int = 8, ncent: int = 10,
                       sigma: float = 0.3, h: float = 1.0, tol: float = 1e-6,
                       d: int = 16, leaf: int = 1563, cfg: int = 4) -> dict:
    """Gaussian kernel exp(-r^2/(2 h^2)) on an 8-D mixture of Gaussians.

    2n points are drawn from ``ncent`` equally weighted isotropic clusters with
    centres in U[-3,3]^dim; the cloud is split at the median of its widest
    coordinate: the lower half gives the rows, the upper half the columns
    (the off-diagonal block of a KD-permuted 2n x 2n kernel matrix)."""
    rng = np.random.default_rng(1000 * cfg + 3)
    cent = rng.uniform(-3.0, 3.0, size=(ncent, dim))
    lab = rng.integers(0, ncent, size=2 * n)
    P = cent[lab] + sigma * rng.standard_normal((2 * n, dim))
    ax = int(np.argmax(P.max(axis=0) - P.min(axis=0)))
    order = np.argsort(P[:, ax], kind="stable")
    X = P[order[:n]]
    Y = P[order[n:]]
    return dict(name="gauss_mixture", entry=ENTRY_GAUSS, X=_kd(X), Y=_kd(Y),
                m=n, n=n, h=h, gauss_c=2.0, wavenumber=0.0, tol=tol, d=d,
                leaf=leaf, seed=1000 * cfg + 2, complex=False)


def make_efie2d_strips(n: int = 4000, m: int | None = None, ppw: float = 15.0,
                       tol: float = 1e-4, d: int = 8, leaf: int = 250, cfg: int = 6) -> dict:
    """EFIE2D kernel H_0^(2)(k r) between two parallel strips of length 1 at
    distance 1 in the plane (y = 0 and y = 1), each carrying nodes drawn
    uniformly along it and sorted (which is their KD order); k gives ``ppw``
    points per wavelength on average on the longer strip, 2 pi max(m, n) /
    ppw.  Random rather than evenly spaced nodes: the mirror symmetry of
    evenly spaced strips makes pairs of residual rows of exactly equal norm,
    ties that rounding would decide."""
    m = n if m is None else m
    k = 2.0 * math.pi * max(m, n) / ppw
    X = np.zeros((m, 2))
    Y = np.ones((n, 2))
    X[:, 0] = np.sort(np.random.default_rng(1000 * cfg + 0).random(m))
    Y[:, 0] = np.sort(np.random.default_rng(1000 * cfg + 1).random(n))
    return dict(name="efie2d", entry=ENTRY_EFIE2D, X=X, Y=Y, m=m, n=n, h=0.0, gauss_c=0.0,
                wavenumber=k, tol=tol, d=d, leaf=leaf, seed=1000 * cfg + 2, complex=True)


def make_polynomial(n: int = 4000, dim: int = 16, h: float = 0.2, tol: float = 1e-4,
                    d: int = 8, leaf: int = 500, cfg: int = 7) -> dict:
    """Polynomial kernel (x^T y + h)^2 on 2n points uniform in [0, 1]^dim,
    split at the median of the widest coordinate: the lower half gives the
    rows, the upper half the columns (the off-diagonal block of the
    KD-permuted 2n x 2n matrix); each half is KD-ordered.  The matrix has
    rank at most dim (dim + 3) / 2 + 1 at every size: the constant-rank
    regime of the paper's cost analysis."""
    P = np.random.default_rng(1000 * cfg + 3).random((2 * n, dim))
    ax = int(np.argmax(P.max(axis=0) - P.min(axis=0)))
    order = np.argsort(P[:, ax], kind="stable")
    X = P[order[:n]]
    Y = P[order[n:]]
    return dict(name="polynomial", entry=ENTRY_POLYNOMIAL, X=_kd(X), Y=_kd(Y), m=n, n=n, h=h,
                gauss_c=0.0, wavenumber=0.0, tol=tol, d=d, leaf=leaf, seed=1000 * cfg + 2,
                complex=False)


def make_hodlr_curve(N: int = 32768, h: float = 0.25, nmin: int = 256, tol: float = 1e-6,
                     d: int = 8, leaf: int = 256, cfg: int = 8) -> dict:
    """One point set for a hierarchical matrix of the Gaussian kernel
    exp(-|x - y|^2 / h^2) with itself: N points on the closed space curve
    (cos t, sin t, 0.1 sin 3t), t uniform on [0, 2 pi), in KD order."""
    t = np.random.default_rng(1000 * cfg + 0).random(N) * 2.0 * math.pi
    X = np.stack([np.cos(t), np.sin(t), 0.1 * np.sin(3.0 * t)], axis=1)
    return dict(name="hodlr_curve", entry=ENTRY_GAUSS, X=_kd(X), N=N, h=h, gauss_c=1.0,
                wavenumber=0.0, nmin=nmin, tol=tol, d=d, leaf=leaf, seed=1000 * cfg + 2,
                complex=False)


def make_hodlr_polynomial(N: int = 4000, dim: int = 8, h: float = 0.2, nmin: int = 256,
                          tol: float = 1e-6, d: int = 16, leaf: int = 256, cfg: int = 9) -> dict:
    """One point set for a hierarchical matrix of the polynomial kernel
    (x^T y + h)^2 with itself: N points uniform in [0, 1]^dim, KD order."""
    X = np.random.default_rng(1000 * cfg + 0).random((N, dim))
    return dict(name="hodlr_polynomial", entry=ENTRY_POLYNOMIAL, X=_kd(X), N=N, h=h,
                gauss_c=0.0, wavenumber=0.0, nmin=nmin, tol=tol, d=d, leaf=leaf,
                seed=1000 * cfg + 2, complex=False)


def make_config(name: str, scale: float = 1.0) -> dict:
    """Workload by name at full size (scale=1) or shrunk in n (scale<1, at
    least a few leaves) for parity runs.  Names: gauss3d, helmholtz,
    coherent, laplace_batched, gauss_mixture, gauss3d_adjoint, efie2d,
    polynomial."""
    def sz(full, minimum):
        return max(minimum, int(round(full * scale)))
    if name == "gauss3d":
        return make_gauss3d(n=sz(2000, 64), cfg=1)
    if name == "helmholtz":
        return make_helmholtz_plates(n=sz(20000, 64), cfg=2)
    if name == "coherent":
        n = sz(20000, 64)
        return make_lowrank_spikes(n=n, n_spikes=max(1, int(200 * n / 20000)),
                                   cfg=2)
    if name == "laplace_batched":
        return make_laplace_blocks(nblocks=sz(4096, 4), cfg=3)
    if name == "gauss_mixture":
        return make_gauss_mixture(n=sz(100000, 256), cfg=4)
    if name == "gauss3d_adjoint":
        return make_gauss3d(n=sz(50000, 64), h=0.7, leaf=1563, cfg=5)
    if name == "efie2d":
        return make_efie2d_strips(n=sz(4000, 64), cfg=6)
    if name == "polynomial":
        return make_polynomial(n=sz(8000, 64), cfg=7)
    raise KeyError(name)
