"""Greedy Householder QR with column pivoting (QRCP), oracle side.

The paper selects skeleton rows and columns with "QR(., d)" and compresses
the cross block with "QR(W, eps)" (Algorithm 2 and the LRID function, eqs.
(6)-(9)), citing LAPACK's QRCP as a greedy picker of well-conditioned columns
by the column norms of the trailing factor.

Reading used here (the paper is silent on norm downdating and ties):
at step t the pivot is the remaining column whose trailing part (rows t..)
has the largest 2-norm, recomputed exactly at every step rather than
downdated; equal norms go to the lowest column position.  A Householder
reflector H = I - beta v v^H maps the pivot's trailing part to alpha e_1 with
alpha = -exp(i arg x_0) |x|, and is applied to every remaining column.  The
number of steps is min(kmax, rows, columns).

Reading for trailing norms at the rounding level: a trailing norm below
NOISE times the largest column norm of the panel (taken at the first step)
is no information about the column, only rounding left by the earlier
reflectors.  Such norms count as zero, so the pick among them is a tie and
goes to the lowest column position.  Without this, two correct runs of the
method (here and on the GPU) would pick different noise columns whenever a
block's numerical rank falls below d, and the picks that follow would part.
The reflector itself is formed from the column's actual values.

Pinned in the tests against a brute-force selection that recomputes every
residual norm by least squares, and (for the full factorisation) against
Q T = W(:, pivots); the rounding-level reading against exactly rank-deficient
panels.
"""
from __future__ import annotations

import numpy as np

NOISE = 1e-12


def householder(x: np.ndarray):
    """Reflector (v, beta, alpha) with (I - beta v v^H) x = alpha e_1."""
    sigma = float(np.sqrt(np.sum(np.abs(x) ** 2)))
    v = x.astype(np.result_type(x.dtype, np.float64), copy=True)
    if sigma == 0.0:
        return v * 0, 0.0, 0.0 * x[0]
    x0 = x[0]
    a0 = abs(x0)
    phase = x0 / a0 if a0 != 0.0 else 1.0
    alpha = -phase * sigma
    v[0] = x0 - alpha
    beta = 1.0 / (sigma * (sigma + a0))
    return v, beta, alpha


class QRCPResult:
    """Pivots (column positions), diagonal of T, reflectors and T itself.

    ``T`` has one row per step and one column per input column, arranged in
    pivot order for the pivoted columns followed by the untouched ones, so
    ``T[:k, :k]`` is the leading upper-triangular block T11.
    """

    def __init__(self, piv, tdiag, refl, T):
        self.piv = piv
        self.tdiag = tdiag
        self.refl = refl
        self.T = T

    def apply_qh(self, B: np.ndarray, nsteps: int | None = None) -> np.ndarray:
        """Q^H B using the first ``nsteps`` reflectors (all by default)."""
        B = B.astype(np.result_type(B.dtype, self.T.dtype), copy=True)
        steps = self.refl if nsteps is None else self.refl[:nsteps]
        for t, (v, beta) in enumerate(steps):
            if beta == 0.0:
                continue
            w = v.conj() @ B[t:, :]
            B[t:, :] -= beta * np.outer(v, w)
        return B


def qrcp(M: np.ndarray, kmax: int) -> QRCPResult:
    """Greedy QRCP of M (p x q) for at most ``kmax`` steps."""
    A = np.array(M, dtype=np.result_type(M.dtype, np.float64), copy=True)
    p, q = A.shape
    steps = min(kmax, p, q)
    remaining = np.ones(q, dtype=bool)
    piv, tdiag, refl = [], [], []
    ref2 = 0.0
    for t in range(steps):
        cols = np.nonzero(remaining)[0]
        sub = A[t:, cols]
        norm2 = np.sum(sub.real ** 2 + sub.imag ** 2, axis=0) if np.iscomplexobj(sub) \
            else np.sum(sub * sub, axis=0)
        if t == 0:
            ref2 = float(norm2.max())
        else:  # rounding-level trailing norms count as zero
            norm2 = np.where(norm2 < NOISE * NOISE * ref2, 0.0, norm2)
        j = int(cols[int(np.argmax(norm2))])  # first maximum = lowest position
        v, beta, alpha = householder(A[t:, j])
        if beta != 0.0:
            w = v.conj() @ A[t:, cols]
            A[t:, cols] -= beta * np.outer(v, w)
        A[t, j] = alpha
        A[t + 1:, j] = 0.0
        remaining[j] = False
        piv.append(j)
        tdiag.append(alpha)
        refl.append((v, beta))
    order = piv + [c for c in range(q) if remaining[c]]
    T = A[:steps, order] if steps else np.zeros((0, q), dtype=A.dtype)
    return QRCPResult(np.array(piv, dtype=np.int64), np.array(tdiag), refl, T)
