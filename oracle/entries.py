"""Matrix entries evaluated on demand (oracle side).

The paper assumes any entry A(i, j) costs O(1) (Abstract; Section
"Numerical Results" lists its kernels).  The kernels here:

* Gaussian  exp(-|x_i - y_j|^2 / (c h^2)).  The paper writes c = 2; the 3-D
  workloads use c = 1 (their stated formula), so c is a parameter.
* Laplace   1 / |x_i - y_j|.
* Helmholtz exp(i k r) / (4 pi r), r = |x_i - y_j|   (complex).
* Product of random factors G1 G2 (the paper's "Product-of-random" kernel)
  plus a sparse set of spikes (coherent entries).
* EFIE2D    H_0^(2)(k |x_i - y_j|), the Hankel function of the second kind
  and order 0 (complex), between points of two 2-D strips.
* Polynomial (x_i^T y_j + h)^2.

Every function evaluates a full sub-block A(I, J) for global index arrays.
Parity: these are the plain definitions; the HIP side evaluates the same
formulas independently.
"""
from __future__ import annotations

import numpy as np

GAUSS, LAPLACE, HELMHOLTZ, LOWRANK_SPIKES, EFIE2D, POLYNOMIAL = 1, 2, 3, 4, 5, 6


class EntrySource:
    """Evaluates sub-blocks of one kernel matrix.

    ``wl`` is a workload dictionary (see the ``workloads`` package): it names
    the entry kind and carries the points (rows ``X``, columns ``Y``) or the
    factors and spikes.  ``row0``/``col0`` shift local to global indices so
    that one source can describe a block of a larger point set.
    """

    def __init__(self, wl: dict, X=None, Y=None):
        self.kind = int(wl["entry"])
        self.X = wl.get("X") if X is None else X
        self.Y = wl.get("Y") if Y is None else Y
        self.h = float(wl.get("h", 0.0))
        self.c = float(wl.get("gauss_c", 1.0))
        self.k = float(wl.get("wavenumber", 0.0))
        self.is_complex = self.kind in (HELMHOLTZ, EFIE2D)
        self.dtype = np.complex128 if self.is_complex else np.float64
        if self.kind == LOWRANK_SPIKES:
            self.G1 = wl["G1"]
            self.G2 = wl["G2"]
            self.spike_lin = np.asarray(wl["spike_lin"], dtype=np.int64)
            self.spike_val = np.asarray(wl["spike_val"], dtype=np.float64)
            self.m, self.n = self.G1.shape[0], self.G2.shape[1]
        else:
            self.m, self.n = self.X.shape[0], self.Y.shape[0]
        self.n_evals = 0

    def _r2(self, I, J):
        dx = self.X[I][:, None, :] - self.Y[J][None, :, :]
        return np.sum(dx * dx, axis=2)

    def block(self, I, J) -> np.ndarray:
        I = np.asarray(I, dtype=np.int64)
        J = np.asarray(J, dtype=np.int64)
        self.n_evals += I.size * J.size
        if I.size == 0 or J.size == 0:
            return np.zeros((I.size, J.size), dtype=self.dtype)
        if self.kind == GAUSS:
            return np.exp(-self._r2(I, J) / (self.c * self.h * self.h))
        if self.kind == LAPLACE:
            return 1.0 / np.sqrt(self._r2(I, J))
        if self.kind == HELMHOLTZ:
            r = np.sqrt(self._r2(I, J))
            return np.exp(1j * self.k * r) / (4.0 * np.pi * r)
        if self.kind == EFIE2D:
            from scipy.special import hankel2
            return hankel2(0, self.k * np.sqrt(self._r2(I, J)))
        if self.kind == POLYNOMIAL:
            return (self.X[I] @ self.Y[J].T + self.h) ** 2
        if self.kind == LOWRANK_SPIKES:
            A = self.G1[I] @ self.G2[:, J]
            if self.spike_lin.size:
                lin = I[:, None] * self.n + J[None, :]
                pos = np.searchsorted(self.spike_lin, lin)
                pos = np.minimum(pos, self.spike_lin.size - 1)
                hit = self.spike_lin[pos] == lin
                A = A + np.where(hit, self.spike_val[pos], 0.0)
            return A
        raise ValueError(f"unknown entry kind {self.kind}")

    def dense(self) -> np.ndarray:
        return self.block(np.arange(self.m), np.arange(self.n))
