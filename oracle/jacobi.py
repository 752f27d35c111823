"""LAPACK-free one-sided Jacobi SVD (brute force for tiny matrices).

Hestenes' method (Hestenes 1958; convergence and accuracy in Demmel and
Veselic 1992): sweep over all column pairs (i, j) of A, and rotate the pair by
a 2x2 unitary that makes it orthogonal, accumulating the same rotations in V.
For columns x, y with a = |x|^2, b = |y|^2, g = x^H y = |g| e^{i phi}, the
rotation first turns y by e^{-i phi}, then applies the real rotation with
zeta = (b - a) / (2 |g|), t = sign(zeta) / (|zeta| + sqrt(1 + zeta^2)),
c = 1 / sqrt(1 + t^2), s = c t:  x' = c x - s y', y' <- s x + c y'.
Sweeps stop when every pair satisfies |g| <= tol sqrt(a b).  The singular
values are the final column norms.

Used as an independent brute force for the oracle's pins; it never runs on
anything larger than about 100 x 100.
"""
from __future__ import annotations

import numpy as np


def jacobi_svd(A: np.ndarray, tol: float = 1e-15, max_sweeps: int = 60):
    """Return (U, s, V) with A = U diag(s) V^H, s sorted descending."""
    W = np.array(A, dtype=np.result_type(A.dtype, np.float64), copy=True)
    m, n = W.shape
    transposed = m < n
    if transposed:
        W = W.conj().T
        m, n = n, m
    V = np.eye(n, dtype=W.dtype)
    for _ in range(max_sweeps):
        rotated = False
        for i in range(n - 1):
            for j in range(i + 1, n):
                x = W[:, i]
                y = W[:, j]
                a = float(np.sum(np.abs(x) ** 2))
                b = float(np.sum(np.abs(y) ** 2))
                g = np.vdot(x, y)
                ag = abs(g)
                if ag == 0.0 or ag <= tol * np.sqrt(a * b):
                    continue
                rotated = True
                ph = g / ag
                zeta = (b - a) / (2.0 * ag)
                t = (1.0 if zeta >= 0 else -1.0) / (abs(zeta) + np.sqrt(1.0 + zeta * zeta))
                c = 1.0 / np.sqrt(1.0 + t * t)
                s = c * t
                yr = y * np.conj(ph)
                W[:, i], W[:, j] = c * x - s * yr, s * x + c * yr
                vi = V[:, i].copy()
                vj = V[:, j] * np.conj(ph)
                V[:, i], V[:, j] = c * vi - s * vj, s * vi + c * vj
        if not rotated:
            break
    s = np.sqrt(np.sum(np.abs(W) ** 2, axis=0))
    order = np.argsort(-s, kind="stable")
    s = s[order]
    W = W[:, order]
    V = V[:, order]
    U = np.zeros_like(W)
    nz = s > 0
    U[:, nz] = W[:, nz] / s[nz][None, :]
    if transposed:
        return V, s, U
    return U, s, V
