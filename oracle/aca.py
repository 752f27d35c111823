"""Partially pivoted adaptive cross approximation (Algorithm 1), oracle side.

Written independently of the BACA code: rank-1 updates, the row pivot
i_k = argmax |E_{k-1}(:, j_k)| over rows not chosen before (eq. (2)), u_k
normalised by its pivot entry, v_k = E_{k-1}(i_k, :), the next column
j_{k+1} = argmax |v_k| over columns not chosen before (eq. (3)), and the stop
nu < eps mu with nu = ||u_k|| ||v_k|| and mu from the rank-1 form of the norm
update (eq. (4) and the algorithm's mu line).  Equal magnitudes go to the
lowest index.  A zero pivot ends the loop.

Used only as a pin: the paper states BACA with d = 1 is exactly this
algorithm.
"""
from __future__ import annotations

import numpy as np


def aca(block, m: int, n: int, eps: float, j1: int):
    us, vs = [], []
    mu2 = 0.0
    chosen_rows = np.zeros(m, dtype=bool)
    chosen_cols = np.zeros(n, dtype=bool)
    j = int(j1)
    pivots = []
    for _ in range(min(m, n)):
        chosen_cols[j] = True
        u = block(np.arange(m), np.array([j]))[:, 0].copy()
        for uu, vv in zip(us, vs):
            u -= uu * vv[j]
        mag = np.abs(u)
        mag[chosen_rows] = -1.0
        i = int(np.argmax(mag))
        if u[i] == 0.0:
            break
        chosen_rows[i] = True
        u = u / u[i]
        v = block(np.array([i]), np.arange(n))[0, :].copy()
        for uu, vv in zip(us, vs):
            v -= uu[i] * vv
        nu2 = float(np.sum(np.abs(u) ** 2) * np.sum(np.abs(v) ** 2))
        cross = 0.0
        for uu, vv in zip(us, vs):
            cross += float((np.vdot(uu, u) * np.vdot(vv, v)).real)
        mu2 = max(0.0, mu2 + nu2 + 2.0 * cross)
        us.append(u)
        vs.append(v)
        pivots.append((i, j))
        if np.sqrt(nu2) < eps * np.sqrt(mu2):
            break
        magv = np.abs(v)
        magv[chosen_cols] = -1.0
        if np.all(chosen_cols):
            break
        j = int(np.argmax(magv))
    U = np.array(us).T if us else np.zeros((m, 0))
    V = np.array(vs) if vs else np.zeros((0, n))
    return U, V, pivots
