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

``strong_select`` is the alternative selector the paper names beside QRCP
(Section "Blocked Adaptive Cross Approximation": strong rank-revealing QR):
greedy QRCP followed by the column swaps of Gu and Eisenstat (SIAM J. Sci.
Comput. 17 (1996), "Efficient algorithms for computing a strong
rank-revealing QR factorization").  Readings, since the paper gives no
details:

* k is the number of leading QRCP picks whose trailing norm is above the
  rounding level (the reading above); the panel has numerical rank k, so the
  trailing block R22 of the pivoted QR counts as zero and Gu and Eisenstat's
  swap test reduces to |W(i, j)| > f for W = R11^-1 R12, the coefficients of
  every other candidate column in the basis of the k chosen ones (a least
  squares solve, exact when the chosen columns span the panel).  Swapping
  chosen column i for candidate j multiplies |det R11| (the volume of the
  chosen columns) by |W(i, j)|;
* each round takes the largest |W(i, j)| (ties to the lowest candidate
  position, then the lowest i), swaps in place (candidate j takes the slot
  of chosen column i, so the pick order is otherwise kept) while it exceeds
  f > 1, at most SWAP_CAP * k times;
* the remaining picks past k (rounding-level norms, a tie) are the lowest
  positions not chosen, as QRCP's reading gives them.
"""
from __future__ import annotations

import numpy as np

NOISE = 1e-12
SWAP_CAP = 4


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

    def __init__(self, piv, tdiag, refl, T, nz=0):
        self.piv = piv
        self.tdiag = tdiag
        self.refl = refl
        self.T = T
        self.nz = nz  # leading picks whose trailing norm is above the rounding level

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
    nz, noise_reached = 0, False
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
        if norm2.max() > 0.0 and not noise_reached:
            nz += 1
        else:
            noise_reached = True
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
    return QRCPResult(np.array(piv, dtype=np.int64), np.array(tdiag), refl, T, nz)


class StrongSelection:
    """Picks of ``strong_select``, the swaps made, and two measures of how
    firmly its decisions were taken (instrumentation only):

    * margin: the smallest relative margin, (|W|max - f) / f or
      (f - |W|max) / f at every round and (|W|max - runner-up) / |W|max at
      every swap;
    * flip: the smallest panel perturbation that could reverse a decision,
      estimated per round as delta * sigma_min(M_S) / (1 + sqrt(k) |W|max),
      delta the absolute margin of the round: a change dM of the panel
      changes W by about M_S^+ (dM_rest - dM_S W).

    A decision whose flip is near the rounding of the panel's entries may go
    the other way in another correct run."""

    def __init__(self, piv, qr, swaps, margin, flip):
        self.piv = piv
        self.qr = qr
        self.swaps = swaps
        self.margin = margin
        self.flip = flip


def strong_select(M: np.ndarray, kmax: int, f: float) -> StrongSelection:
    """Strong rank-revealing selection of at most ``kmax`` columns of M:
    greedy QRCP, then Gu-Eisenstat swaps with threshold f > 1."""
    if not f > 1.0:
        raise ValueError("the swap threshold f must exceed 1")
    res = qrcp(M, kmax)
    piv = [int(c) for c in res.piv]
    k = res.nz
    q = M.shape[1]
    S = piv[:k]
    swaps, margin, flip = 0, np.inf, np.inf
    while k > 0 and swaps < SWAP_CAP * k:
        chosen = set(S)
        rest = np.array([c for c in range(q) if c not in chosen], dtype=np.int64)
        if rest.size == 0:
            break
        W = np.linalg.lstsq(M[:, S], M[:, rest], rcond=None)[0]  # k x |rest|
        A = np.abs(W)
        # the largest entry; ties to the lowest candidate position, then the
        # lowest chosen slot (column-major scan of A)
        flat = A.T.ravel()
        pos = int(np.argmax(flat))
        best = float(flat[pos])
        j, i = divmod(pos, k)
        smin = float(np.linalg.svd(M[:, S], compute_uv=False)[-1])
        scale = smin / (1.0 + np.sqrt(k) * best)
        if best <= f:
            margin = min(margin, (f - best) / f)
            flip = min(flip, (f - best) * scale)
            break
        second = float(np.max(np.delete(flat, pos))) if flat.size > 1 else 0.0
        margin = min(margin, (best - f) / f, (best - second) / best)
        flip = min(flip, min(best - f, best - second) * scale)
        S[i] = int(rest[j])
        swaps += 1
    chosen = set(S)
    noise = [c for c in range(q) if c not in chosen][:len(piv) - k]
    return StrongSelection(np.array(S + noise, dtype=np.int64), res, swaps, margin, flip)
