"""Blocked adaptive cross approximation of one leaf (Algorithm 2), oracle side.

Follows Algorithm 2 step by step in the paper's notation: U is m0 x r,
V is r x n0, A ~ U V.  Each iteration k

1. forms the residual column block C_k = A(:, J_k) - U V(:, J_k);
2. picks d skeleton rows I_k by QRCP of C_k^H over the rows not yet used
   (eq. (6));
3. forms the residual row block R_k = A(I_k, :) - U(I_k, :) V;
4. takes the cross block W_k = C_k(I_k, :) (it equals E_{k-1}(I_k, J_k));
5. LRID: QRCP(W_k, eps) gives d_k and pivots Jbar, U_k = C_k(:, Jbar),
   V_k = T11^{-1} Q1^H R_k (eqs. (8)-(9));
6. nu = LRnorm(U_k, V_k) (eqs. (11)-(12)); mu updated by LRnormUp (eq. (13));
7. appends U_k, V_k and updates the used rows/columns (eq. (10));
8. stops when nu < eps * mu; otherwise picks J_{k+1} by QRCP of R_k over the
   columns not used (eq. (7)).

Readings where the paper is silent or garbled:

* QR(C^t, d) returns min(d, #panel rows, #candidates) pivots, candidates being
  the rows not in any earlier I_i(1:d_i).
* J_{k+1} excludes every earlier J_i(Jbar_i) and all of the current J_k
  (this reduces exactly to eq. (3) when d = 1); afterwards only J_k(Jbar)
  stays excluded.
* QR(W, eps): d_k is the number of leading pivots before the first one with
  |T_jj| < eps |T_11| (the paper's own eps-rank rule for SVDs); T^{-1} means
  the leading d_k x d_k block and Q its first d_k columns.
* d_k = 0 ends the leaf without appending (the paper requires d_k > 0).
* A Cholesky breakdown in LRnorm falls back to nu^2 = Re sum(G_U o conj(G_V)).
* mu^2 is clamped at 0 against rounding.
* The loop also ends when no candidate rows or columns remain or the rank
  reaches min(m0, n0) (the paper's loop bound).
* Complex matrices: every transpose is a conjugate transpose and the cross
  term of eq. (13) takes the real part.

Instrumentation (no effect on the arithmetic): every iteration records its
pivots, d_k, nu, mu, the trailing norms of the row picks (sel_I) and of the
column picks that chose the next block (sel_J), and the whole blocks I_k,
J_k with the pivot order of QR(W_k, eps) (Iblock, Jblock, piv), which is
what a replay with frozen pivots needs; with the strong selector also the
swaps and decision margins of both selections (swaps_I, margin_I, flip_I,
swaps_J, margin_J, flip_J).
"""
from __future__ import annotations

import numpy as np

from .qrcp import qrcp, strong_select


def _chol_upper(G: np.ndarray):
    """Upper Cholesky factor T with G = T^H T, or None on a pivot <= 0."""
    n = G.shape[0]
    T = np.zeros_like(G)
    for j in range(n):
        s = G[j, j].real - np.sum(np.abs(T[:j, j]) ** 2)
        if not s > 0.0:
            return None
        T[j, j] = np.sqrt(s)
        for c in range(j + 1, n):
            T[j, c] = (G[j, c] - np.sum(T[:j, j].conj() * T[:j, c])) / T[j, j]
    return T


def lrnorm(Uk: np.ndarray, Vk: np.ndarray) -> float:
    """||U_k V_k||_F via Cholesky factors of the two Gram matrices
    (eqs. (11)-(12))."""
    GU = Uk.conj().T @ Uk
    GV = Vk @ Vk.conj().T
    T1 = _chol_upper(GU)
    T2 = _chol_upper(GV)
    if T1 is None or T2 is None:
        return float(np.sqrt(max(0.0, float(np.sum(GU * GV.conj()).real))))
    return float(np.sqrt(np.sum(np.abs(T1 @ T2.conj().T) ** 2)))


def lrnorm_update(U, V, mu2, Uk, Vk, nu) -> float:
    """mu^2 after appending (U_k, V_k) to (U, V) (eq. (13)); returns mu^2."""
    if U.shape[1] == 0:
        cross = 0.0
    else:
        cross = float(np.sum((U.conj().T @ Uk) * (V @ Vk.conj().T).conj()).real)
    return max(0.0, mu2 + nu * nu + 2.0 * cross)


def _back_substitute(T: np.ndarray, B: np.ndarray) -> np.ndarray:
    """Solve T X = B for upper-triangular T by back substitution."""
    n = T.shape[0]
    X = np.zeros((n, B.shape[1]), dtype=np.result_type(T.dtype, B.dtype))
    for i in range(n - 1, -1, -1):
        X[i] = (B[i] - T[i, i + 1:] @ X[i + 1:]) / T[i, i]
    return X


class LeafResult:
    def __init__(self, U, V, iters, ops):
        self.U = U
        self.V = V
        self.iters = iters
        self.ops = ops

    @property
    def rank(self):
        return self.U.shape[1]


def _select(M: np.ndarray, d: int, selector: int, f: float):
    """Pivots of the d-pick selection of eqs. (6)-(7) on panel M, the QRCP
    trailing norms of the greedy picks, the swaps made and the decision
    measures (margin, flip) of strong_select: selector 0 is greedy QRCP (the
    paper's choice), 1 the strong rank-revealing selection (QRCP then
    Gu-Eisenstat swaps, threshold f)."""
    if selector == 0:
        res = qrcp(M, d)
        return res.piv, np.abs(res.tdiag), 0, (np.inf, np.inf)
    ss = strong_select(M, d, f)
    return ss.piv, np.abs(ss.qr.tdiag), ss.swaps, (ss.margin, ss.flip)


def baca_leaf(block, m0: int, n0: int, d: int, eps: float, J1: np.ndarray,
              record: bool = True, selector: int = 0, select_f: float = 2.0) -> LeafResult:
    """BACA of the m0 x n0 leaf whose entries ``block(I, J)`` returns for
    leaf-local index arrays.  ``J1`` is the first column block.  ``selector``
    picks the row and column selection (0 greedy QRCP, 1 strong
    rank-revealing with swap threshold ``select_f``)."""
    probe = block(np.zeros(0, dtype=np.int64), np.zeros(0, dtype=np.int64))
    dt = probe.dtype
    U = np.zeros((m0, 0), dtype=dt)
    V = np.zeros((0, n0), dtype=dt)
    mu2 = 0.0
    used_r = np.zeros(m0, dtype=bool)
    used_c = np.zeros(n0, dtype=bool)
    allr = np.arange(m0)
    allc = np.arange(n0)
    J = np.asarray(J1, dtype=np.int64)
    iters = []
    phi = 4 if np.iscomplexobj(probe) else 1
    ops = dict(entries=0, resid_flops=0, qrcp_flops=0, lrid_flops=0,
               norm_flops=0, bytes=0)
    rmax = min(m0, n0)
    while J.size:
        r = U.shape[1]
        # (1) residual column block C_k = A(:, J_k) - U V(:, J_k)
        C = block(allr, J) - U @ V[:, J]
        ops["entries"] += m0 * J.size
        ops["resid_flops"] += 2 * phi * m0 * r * J.size
        # (2) skeleton rows by QRCP of C^H over unused rows (eq. (6))
        Pr = allr[~used_r]
        if Pr.size == 0:
            break
        pivI, normsI, swI, marI = _select(C[Pr, :].conj().T, d, selector, select_f)
        I = Pr[pivI]
        ops["qrcp_flops"] += 4 * phi * J.size * Pr.size * I.size
        # (3) residual row block R_k = A(I_k, :) - U(I_k, :) V
        R = block(I, allc) - U[I, :] @ V
        ops["entries"] += n0 * I.size
        ops["resid_flops"] += 2 * phi * n0 * r * I.size
        ops["bytes"] += (m0 + n0) * r * 8 * (2 if phi == 4 else 1)
        # (4) cross block W_k = E_{k-1}(I_k, J_k) = C_k(I_k, :)
        W = C[I, :]
        # (5) LRID (eqs. (8)-(9))
        full = qrcp(W, min(W.shape))
        t = np.abs(full.tdiag)
        dk = 0
        if t.size and t[0] > 0.0:
            while dk < t.size and t[dk] >= eps * t[0]:
                dk += 1
        if dk == 0:
            if record:
                iters.append(dict(I=np.zeros(0, np.int64), J=np.zeros(0, np.int64),
                                  dk=0, nu=0.0, mu=float(np.sqrt(mu2)), r=r,
                                  sel_I=normsI, sel_J=np.zeros(0),
                                  Iblock=I.copy(), Jblock=J.copy(), piv=full.piv.copy(),
                                  swaps_I=swI, margin_I=marI[0], flip_I=marI[1],
                                  swaps_J=0, margin_J=np.inf, flip_J=np.inf))
            break
        jbar = full.piv[:dk]
        Uk = C[:, jbar]
        QhR = full.apply_qh(R, dk)[:dk]
        Vk = _back_substitute(full.T[:dk, :dk], QhR)
        ops["lrid_flops"] += phi * (4 * n0 * I.size * dk + dk * dk * n0)
        # (6) norms (eqs. (11)-(13))
        nu = lrnorm(Uk, Vk)
        mu2 = lrnorm_update(U, V, mu2, Uk, Vk, nu)
        ops["norm_flops"] += 2 * phi * (m0 + n0) * (r + dk) * dk
        # (7) append and update the exclusion sets (eq. (10))
        U = np.concatenate([U, Uk], axis=1)
        V = np.concatenate([V, Vk], axis=0)
        Pc = allc[~used_c & ~np.isin(allc, J)]
        used_r[I[:dk]] = True
        used_c[J[jbar]] = True
        mu = float(np.sqrt(mu2))
        if record:
            iters.append(dict(I=I[:dk].copy(), J=J[jbar].copy(), dk=dk, nu=nu,
                              mu=mu, r=U.shape[1], sel_I=normsI,
                              sel_J=np.zeros(0), Iblock=I.copy(), Jblock=J.copy(),
                              piv=full.piv.copy(), swaps_I=swI, margin_I=marI[0],
                              flip_I=marI[1], swaps_J=0, margin_J=np.inf, flip_J=np.inf))
        # (8) stopping test, then the next column block (eq. (7))
        if nu < eps * mu or Pc.size == 0 or U.shape[1] >= rmax:
            break
        pivJ, normsJ, swJ, marJ = _select(R[:, Pc], d, selector, select_f)
        if record:
            iters[-1]["sel_J"] = normsJ
            iters[-1]["swaps_J"] = swJ
            iters[-1]["margin_J"] = marJ[0]
            iters[-1]["flip_J"] = marJ[1]
        ops["qrcp_flops"] += 4 * phi * I.size * Pc.size * pivJ.size
        J = Pc[pivJ]
    return LeafResult(U, V, iters, ops)
