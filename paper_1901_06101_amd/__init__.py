"""H-BACA on MI355X: hierarchical blocked adaptive cross approximation.

Python front end of libhbaca.so.  ``compress`` and ``compress_batched`` take
torch tensors that already live on the GPU and return a ``Result`` whose
factors come back as torch tensors:  A ~ U diag(S) Vh^H.

There is no CPU path: if the HIP library or the GPU is missing the calls
raise.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _binding as B
from ._binding import (HB_K_EFIE2D, HB_K_GAUSS, HB_K_HELMHOLTZ3D,  # noqa: F401
                       HB_K_LAPLACE, HB_K_LOWRANK_SPIKES, HB_K_POLYNOMIAL, HB_PREC_FP64,
                       HB_PREC_MIXED, HB_SEL_QRCP, HB_SEL_STRONG, HBACAError, HbParams,
                       HbStats, load)

__all__ = ["compress", "compress_batched", "Result", "operator", "gaussian_operator",
           "hodlr_build", "Hodlr", "autotune",
           "partition", "require_gpu", "params", "load",
           "HBACAError", "HB_K_GAUSS", "HB_K_LAPLACE", "HB_K_HELMHOLTZ3D",
           "HB_K_LOWRANK_SPIKES", "HB_K_EFIE2D", "HB_K_POLYNOMIAL", "HB_PREC_FP64",
           "HB_PREC_MIXED", "HB_SEL_QRCP", "HB_SEL_STRONG"]


def partition(m: int, n: int, leaf: int, d: int, seed: int):
    """The partition hbaca_compress uses (host only): (L, leaves, j1) with
    leaves[b] = (first row, rows, first column, columns) and j1[b] the first
    column block of leaf b = t 2^L + v (-1 past min(d, n0))."""
    lib = load()
    L = C.c_int32(0)
    B._check(lib.hb_partition(int(m), int(n), int(leaf), int(d),
                              int(seed) & ((1 << 64) - 1), C.byref(L), None, None), "hb_partition")
    nl = 4 ** L.value
    leaves = np.zeros((nl, 4), dtype=np.int64)
    j1 = np.zeros((nl, int(d)), dtype=np.int32)
    B._check(lib.hb_partition(int(m), int(n), int(leaf), int(d), int(seed) & ((1 << 64) - 1),
                              C.byref(L), leaves.ctypes.data_as(C.c_void_p),
                              j1.ctypes.data_as(C.c_void_p)), "hb_partition")
    return L.value, leaves, j1


def require_gpu():
    """Raise unless a GPU and the built library are both present."""
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("H-BACA needs a ROCm GPU (torch.cuda.is_available() is False)")
    load()


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def params(dim=3, h=1.0, gauss_c=1.0, wavenumber=0.0, seed=0, rank_cap=0, record_tape=0,
           stop_after=0, G1=None, G2=None, spike_lin=None, spike_val=None, diag_panel=0,
           diag_svd_storage=0, precision=B.HB_PREC_FP64, selector=0, select_f=2.0) -> dict:
    return dict(dim=dim, h=h, gauss_c=gauss_c, wavenumber=wavenumber, seed=seed,
                rank_cap=rank_cap, record_tape=record_tape, stop_after=stop_after, G1=G1,
                G2=G2, spike_lin=spike_lin, spike_val=spike_val, diag_panel=diag_panel,
                diag_svd_storage=diag_svd_storage, precision=precision, selector=selector,
                select_f=select_f)


def _hb_params(p: dict, keep: list) -> HbParams:
    hp = HbParams()
    hp.dim = int(p.get("dim", 3))
    hp.h = float(p.get("h", 1.0))
    hp.gauss_c = float(p.get("gauss_c", 1.0))
    hp.wavenumber = float(p.get("wavenumber", 0.0))
    G1, G2 = p.get("G1"), p.get("G2")
    if G1 is not None:
        keep += [G1, G2]
        hp.lr_rank = int(G1.shape[1])
        hp.lr_G1 = G1.data_ptr()
        hp.lr_G2 = G2.data_ptr()
    sl, sv = p.get("spike_lin"), p.get("spike_val")
    if sl is not None and sl.numel() > 0:
        keep += [sl, sv]
        hp.n_spikes = int(sl.numel())
        hp.spike_lin = sl.data_ptr()
        hp.spike_val = sv.data_ptr()
    hp.seed = int(p.get("seed", 0)) & ((1 << 64) - 1)
    hp.precision = int(p.get("precision", 0))
    hp.rank_cap = int(p.get("rank_cap", 0))
    hp.record_tape = int(p.get("record_tape", 0))
    hp.stop_after = int(p.get("stop_after", 0))
    hp.diag_panel = int(p.get("diag_panel", 0))
    hp.diag_svd_storage = int(p.get("diag_svd_storage", 0))
    hp.selector = int(p.get("selector", 0))
    hp.select_f = float(p.get("select_f", 2.0))
    return hp


class Result:
    """Owns an hb_result handle; frees it on close() or garbage collection
    (a view of a result another object owns frees nothing)."""

    def __init__(self, handle, keep, owned=True):
        self._h = handle
        self._keep = keep
        self._owned = owned
        self._lib = load()

    def close(self):
        if self._h:
            if self._owned:
                self._lib.hb_result_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def nblocks(self):
        return int(self._lib.hb_result_nblocks(self._h))

    @property
    def is_complex(self):
        return bool(self._lib.hb_result_is_complex(self._h))

    def rank(self, block=0):
        return int(self._lib.hb_result_rank(self._h, block))

    def shape(self, block=0):
        return (int(self._lib.hb_result_rows(self._h, block)),
                int(self._lib.hb_result_cols(self._h, block)))

    def factors(self, block=0):
        """(U, S, Vh) as torch tensors on the GPU with A ~ U diag(S) Vh^H."""
        import torch
        m, n = self.shape(block)
        r = self.rank(block)
        dt = torch.complex128 if self.is_complex else torch.float64
        dev = torch.device("cuda")
        Ub = torch.empty((r, m), dtype=dt, device=dev)   # column-major m x r
        Vb = torch.empty((r, n), dtype=dt, device=dev)
        S = torch.empty((r,), dtype=torch.float64, device=dev)
        if r > 0:
            B._check(self._lib.hb_result_copy(self._h, block, _ptr(Ub), _ptr(S), _ptr(Vb),
                                              _stream()), "hb_result_copy")
        return Ub.T, S, Vb.T

    def stats(self):
        st = HbStats()
        B._check(self._lib.hb_result_stats(self._h, C.byref(st)), "hb_result_stats")
        return st.as_dict()

    @property
    def nleaves(self):
        return int(self._lib.hb_result_nleaves(self._h))

    def leaf_info(self, leaf):
        buf = (C.c_int64 * 12)()
        B._check(self._lib.hb_result_leaf_info(self._h, leaf, buf), "hb_result_leaf_info")
        keys = ("block", "t", "v", "row0", "col0", "m0", "n0", "rank_baca", "rank_leaf",
                "iters", "status", "tape_len")
        return dict(zip(keys, [int(x) for x in buf]))

    def leaf_tape(self, leaf):
        info = self.leaf_info(leaf)
        n = info["rank_baca"]
        it = info["iters"]
        rows = np.zeros(max(n, 1), np.int32)
        cols = np.zeros(max(n, 1), np.int32)
        dk = np.zeros(max(it, 1), np.int32)
        nu = np.zeros(max(it, 1), np.float64)
        mu = np.zeros(max(it, 1), np.float64)
        B._check(self._lib.hb_result_leaf_tape(
            self._h, leaf, rows.ctypes.data_as(C.c_void_p), cols.ctypes.data_as(C.c_void_p),
            dk.ctypes.data_as(C.c_void_p), nu.ctypes.data_as(C.c_void_p),
            mu.ctypes.data_as(C.c_void_p)), "hb_result_leaf_tape")
        return dict(rows=rows[:n], cols=cols[:n], dk=dk[:it], nu=nu[:it], mu=mu[:it])

    def leaf_frozen(self, leaf):
        """Iteration records of one leaf (record_tape=2): int32 array of
        shape (iterations, stride), see hb_result_leaf_frozen."""
        stride = C.c_int32(0)
        B._check(self._lib.hb_result_leaf_frozen(self._h, leaf, C.byref(stride), None),
                 "hb_result_leaf_frozen")
        it = self.leaf_info(leaf)["iters"]
        rec = np.zeros((max(it, 1), stride.value), dtype=np.int32)
        B._check(self._lib.hb_result_leaf_frozen(self._h, leaf, C.byref(stride),
                                                 rec.ctypes.data_as(C.c_void_p)),
                 "hb_result_leaf_frozen")
        return rec[:it]

    def merge_ranks(self):
        """Every merge rank (record_tape=2), in hb_result_merge_ranks order."""
        n = C.c_int64(0)
        B._check(self._lib.hb_result_merge_ranks(self._h, None, C.byref(n)),
                 "hb_result_merge_ranks")
        out = np.zeros(max(n.value, 1), dtype=np.int32)
        B._check(self._lib.hb_result_merge_ranks(self._h, out.ctypes.data_as(C.c_void_p),
                                                 C.byref(n)), "hb_result_merge_ranks")
        return out[:n.value]

    def apply(self, w, block=0, adjoint=False):
        """U diag(S) Vh^H w (adjoint=False) or Vh diag(S) U^H w (adjoint=True)
        for a device vector w; returns a new device vector."""
        import torch
        m, n = self.shape(block)
        dt = torch.complex128 if self.is_complex else torch.float64
        w = w.to(dtype=dt).contiguous()
        if w.numel() != (m if adjoint else n):
            raise ValueError(f"vector of length {w.numel()} for a {m} x {n} block")
        out = torch.empty((n if adjoint else m,), dtype=dt, device=w.device)
        B._check(self._lib.hbaca_apply(self._h, block, _ptr(w), _ptr(out), int(bool(adjoint)),
                                       _stream()), "hbaca_apply")
        return out

    def apply_noalloc(self, w, out, block=0, adjoint=False):
        """apply() into the caller's device vector `out` through
        hbaca_apply_noalloc, which allocates no device memory."""
        m, n = self.shape(block)
        if w.numel() != (m if adjoint else n) or out.numel() != (n if adjoint else m):
            raise ValueError("vector lengths do not match the block")
        B._check(self._lib.hbaca_apply_noalloc(self._h, block, _ptr(w), _ptr(out),
                                               int(bool(adjoint)), _stream()),
                 "hbaca_apply_noalloc")
        return out

    def vjp(self, w, ybar, want=("w", "h", "x", "y")):
        """Gradients of <ybar, A~ w> with pivots and ranks frozen (needs a
        Gaussian result compressed with record_tape=2): (grad_w, grad_h,
        grad_X, grad_Y) as device tensors, None where not in `want`."""
        import torch
        m, n = self.shape(0)
        X, Y = self._keep[0], self._keep[1]
        dim = int(X.shape[1])
        w = w.to(dtype=torch.float64).contiguous()
        ybar = ybar.to(dtype=torch.float64).contiguous()
        if w.numel() != n or ybar.numel() != m:
            raise ValueError(f"w of length {w.numel()} and ybar of length {ybar.numel()} "
                             f"for a {m} x {n} operator")
        f64 = dict(dtype=torch.float64, device=w.device)
        gw = torch.empty((n,), **f64) if "w" in want else None
        gh = torch.empty((1,), **f64) if "h" in want else None
        gX = torch.empty((m, dim), **f64) if "x" in want else None
        gY = torch.empty((n, dim), **f64) if "y" in want else None
        B._check(self._lib.hbaca_vjp(self._h, _ptr(w), _ptr(ybar), _ptr(gw), _ptr(gh), _ptr(gX),
                                     _ptr(gY), _stream()), "hbaca_vjp")
        return gw, gh, gX, gY

    def adjoint(self, w, ybar, want=("w", "h", "x", "y")):
        """vjp for FP32 vectors (hbaca_adjoint): w and ybar in FP32, the
        w-gradient in FP32, the h and point gradients in FP64; None where
        not in `want`."""
        import torch
        m, n = self.shape(0)
        X = self._keep[0]
        dim = int(X.shape[1])
        w = w.to(dtype=torch.float32).contiguous()
        ybar = ybar.to(dtype=torch.float32).contiguous()
        if w.numel() != n or ybar.numel() != m:
            raise ValueError(f"w of length {w.numel()} and ybar of length {ybar.numel()} "
                             f"for a {m} x {n} operator")
        f64 = dict(dtype=torch.float64, device=w.device)
        gw = torch.empty((n,), dtype=torch.float32, device=w.device) if "w" in want else None
        gh = torch.empty((1,), **f64) if "h" in want else None
        gX = torch.empty((m, dim), **f64) if "x" in want else None
        gY = torch.empty((n, dim), **f64) if "y" in want else None
        B._check(self._lib.hbaca_adjoint(self._h, _ptr(w), _ptr(ybar), _ptr(gw), _ptr(gh),
                                         _ptr(gX), _ptr(gY), _stream()), "hbaca_adjoint")
        return gw, gh, gX, gY

    def recompute_frozen(self, X, Y, h, gauss_c=1.0):
        """The frozen operator (same pivots and ranks as this result, which
        needs record_tape=2) at new points X, Y and width h, as a new
        Result."""
        import torch
        X = X.detach().to(torch.float64).contiguous()
        Y = Y.detach().to(torch.float64).contiguous()
        keep = [X, Y]
        hp = _hb_params(params(dim=int(X.shape[1]), h=float(h), gauss_c=float(gauss_c)), keep)
        out = C.c_void_p()
        B._check(self._lib.hbaca_recompute_frozen(self._h, C.byref(hp), _ptr(X), _ptr(Y),
                                                  _stream(), C.byref(out)),
                 "hbaca_recompute_frozen")
        return Result(out, keep)

    def error(self, block=0, row_stride=1):
        """(sum |A - A~|^2, sum |A|^2) over rows 0, stride, ... (device FP64)."""
        e = C.c_double()
        a = C.c_double()
        B._check(self._lib.hb_result_error(self._h, block, row_stride, C.byref(e), C.byref(a),
                                           _stream()), "hb_result_error")
        return e.value, a.value


def operator(result: Result, block: int = 0):
    """y = A~ w as a differentiable function of w: its backward applies the
    adjoint Vh diag(S) U^H on the GPU (the gradient with respect to w; the
    factors are constants)."""
    import torch

    class _Apply(torch.autograd.Function):
        @staticmethod
        def forward(ctx, w):
            return result.apply(w, block, adjoint=False)

        @staticmethod
        def backward(ctx, ybar):
            # torch's complex convention: the vector-Jacobian product of a
            # linear map A is A^H ybar
            return result.apply(ybar.contiguous(), block, adjoint=True)

    return _Apply.apply


def gaussian_operator(X, Y, h, w, tol: float, d: int, leaf: int, gauss_c: float = 1.0,
                      seed: int = 0):
    """y = A~ w for the H-BACA compression A~ of A(i, j) = exp(-|x_i - y_j|^2 /
    (c h^2)), differentiable with respect to the points X (m x dim), Y
    (n x dim), the width h (a 0-dim or 1-element tensor) and w: the forward
    pass compresses on the GPU (recording its pivots and ranks) and applies
    the factors; the backward pass is hbaca_vjp, the adjoint of the same
    compression with those pivots and ranks frozen."""
    import torch

    class _GaussApply(torch.autograd.Function):
        @staticmethod
        def forward(ctx, X, Y, h, w):
            p = params(dim=int(X.shape[1]), h=float(h), gauss_c=gauss_c, seed=seed, record_tape=2)
            Xd = X.detach().to(torch.float64).contiguous()
            Yd = Y.detach().to(torch.float64).contiguous()
            res = compress(HB_K_GAUSS, p, Xd, Yd, Xd.shape[0], Yd.shape[0], tol, d, leaf)
            wd = w.detach().to(torch.float64).contiguous()
            ctx.res = res
            ctx.h_shape = h.shape
            ctx.save_for_backward(wd)
            return res.apply(wd)

        @staticmethod
        def backward(ctx, ybar):
            (wd,) = ctx.saved_tensors
            need = ctx.needs_input_grad
            want = tuple(k for k, f in zip(("x", "y", "h", "w"), need) if f)
            gw, gh, gX, gY = ctx.res.vjp(wd, ybar, want=want)
            return gX, gY, (gh.reshape(ctx.h_shape) if gh is not None else None), gw

    if not isinstance(h, torch.Tensor):
        h = torch.as_tensor(float(h), dtype=torch.float64, device=X.device)
    return _GaussApply.apply(X, Y, h, w)


def compress(entry: int, p: dict, X, Y, m: int, n: int, tol: float, d: int, leaf: int) -> Result:
    """H-BACA of an m x n kernel matrix (points X: m x dim, Y: n x dim, float64
    CUDA tensors; None for the low-rank-plus-spikes kernel)."""
    lib = load()
    keep = [X, Y]
    hp = _hb_params(p, keep)
    out = C.c_void_p()
    st = lib.hbaca_compress(int(entry), C.byref(hp), _ptr(X), _ptr(Y), int(m), int(n),
                            float(tol), int(d), int(leaf), _stream(), C.byref(out))
    B._check(st, "hbaca_compress")
    return Result(out, keep)


class Hodlr:
    """Owns an hb_hodlr handle (a HODLR matrix built with H-BACA)."""

    def __init__(self, handle, keep):
        self._h = handle
        self._keep = keep
        self._lib = load()
        hb = self._lib.hb_hodlr_blocks(self._h)
        # the off-diagonal blocks' H-BACA result, owned by the HODLR object
        self.blocks = Result(C.c_void_p(hb), [self], owned=False) if hb else None

    def close(self):
        if self._h:
            self.blocks = None
            self._lib.hb_hodlr_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def nblocks(self):
        return int(self._lib.hb_hodlr_nblocks(self._h))

    @property
    def nleaves(self):
        return int(self._lib.hb_hodlr_nleaves(self._h))

    def block_info(self, b):
        """(level, row_off, row_cnt, col_off, col_cnt) of off-diagonal block b."""
        buf = (C.c_int64 * 5)()
        B._check(self._lib.hb_hodlr_block_info(self._h, b, buf), "hb_hodlr_block_info")
        return tuple(int(v) for v in buf)

    def matvec(self, x, out=None):
        """A_H x for a float64 device vector of N entries."""
        import torch
        x = x.to(dtype=torch.float64).contiguous()
        if out is None:
            out = torch.empty_like(x)
        B._check(self._lib.hb_hodlr_matvec(self._h, _ptr(x), _ptr(out), _stream()),
                 "hb_hodlr_matvec")
        return out


def autotune():
    """Runs the library's TSQR autotuner (hb_autotune) on the current stream;
    returns {"table": [...16], "us": [...32]} (see include/hbaca.h)."""
    lib = load()
    table = np.zeros(16, dtype=np.int32)
    us = np.zeros(32, dtype=np.float64)
    B._check(lib.hb_autotune(_stream(), table.ctypes.data_as(C.c_void_p),
                             us.ctypes.data_as(C.c_void_p)), "hb_autotune")
    return dict(table=table.tolist(), us=us.tolist())


def hodlr_build(entry: int, p: dict, X, nmin: int, tol: float, d: int, leaf: int) -> Hodlr:
    """HODLR matrix of the kernel matrix of the KD-ordered points X (N x dim,
    float64 device tensor) with themselves; every off-diagonal block by
    H-BACA in one batched pass, dense diagonal leaves of at most nmin."""
    lib = load()
    keep = [X]
    hp = _hb_params(p, keep)
    out = C.c_void_p()
    st = lib.hb_hodlr_build(int(entry), C.byref(hp), _ptr(X), int(X.shape[0]), int(nmin),
                            float(tol), int(d), int(leaf), _stream(), C.byref(out))
    B._check(st, "hb_hodlr_build")
    return Hodlr(out, keep)


def compress_batched(entry: int, p: dict, X, row_off, row_cnt, Y, col_off, col_cnt, tol: float,
                     d: int, leaf: int) -> Result:
    """Independent H-BACA of many blocks in one pass (offsets/counts: host
    integer sequences)."""
    lib = load()
    keep = [X, Y]
    hp = _hb_params(p, keep)
    nb = len(row_off)
    arr = [np.ascontiguousarray(np.asarray(a, dtype=np.int64)) for a in
           (row_off, row_cnt, col_off, col_cnt)]
    ptrs = [a.ctypes.data_as(C.POINTER(C.c_int64)) for a in arr]
    out = C.c_void_p()
    st = lib.hbaca_compress_batched(int(entry), C.byref(hp), nb, _ptr(X), ptrs[0], ptrs[1],
                                    _ptr(Y), ptrs[2], ptrs[3], float(tol), int(d), int(leaf),
                                    _stream(), C.byref(out))
    B._check(st, "hbaca_compress_batched")
    return Result(out, keep)
