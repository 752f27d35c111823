"""ctypes binding of libhbaca.so (the C ABI declared in include/hbaca.h).

Argument marshalling only: every step of H-BACA runs in the library's HIP
kernels.  PyTorch supplies device memory and the current stream.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhbaca.so")

HB_OK, HB_EINVAL, HB_ENOMEM, HB_EDEVICE, HB_ERANKCAP, HB_ENONFINITE, HB_EUNSUPPORTED = \
    0, -1, -2, -3, -4, -5, -6
HB_K_GAUSS, HB_K_LAPLACE, HB_K_HELMHOLTZ3D, HB_K_LOWRANK_SPIKES = 1, 2, 3, 4
HB_K_EFIE2D, HB_K_POLYNOMIAL = 5, 6
HB_PREC_FP64, HB_PREC_MIXED = 0, 1
HB_SEL_QRCP, HB_SEL_STRONG = 0, 1

EXPORTED = (
    "hbaca_compress", "hbaca_compress_batched", "hb_result_nblocks", "hb_result_rank",
    "hb_result_rows", "hb_result_cols", "hb_result_is_complex", "hb_result_copy",
    "hb_result_stats", "hb_result_nleaves", "hb_result_leaf_info", "hb_result_leaf_tape",
    "hb_result_error", "hb_result_free", "hb_status_string", "hbaca_apply",
    "hbaca_apply_noalloc", "hbaca_vjp", "hbaca_adjoint",
    "hbaca_recompute_frozen", "hb_partition", "hb_result_leaf_frozen", "hb_result_merge_ranks",
    "hb_hodlr_build", "hb_hodlr_blocks", "hb_hodlr_nblocks", "hb_hodlr_nleaves",
    "hb_hodlr_block_info", "hb_hodlr_matvec", "hb_hodlr_free", "hb_autotune",
)


class HbParams(C.Structure):
    _fields_ = [
        ("dim", C.c_int32),
        ("h", C.c_double),
        ("gauss_c", C.c_double),
        ("wavenumber", C.c_double),
        ("lr_rank", C.c_int32),
        ("lr_G1", C.c_void_p),
        ("lr_G2", C.c_void_p),
        ("n_spikes", C.c_int32),
        ("spike_lin", C.c_void_p),
        ("spike_val", C.c_void_p),
        ("seed", C.c_uint64),
        ("precision", C.c_int32),
        ("rank_cap", C.c_int32),
        ("record_tape", C.c_int32),
        ("stop_after", C.c_int32),
        ("diag_panel", C.c_int32),
        ("diag_svd_storage", C.c_int32),
        ("selector", C.c_int32),
        ("select_f", C.c_double),
    ]


class HbStats(C.Structure):
    _fields_ = [
        ("n_blocks", C.c_int32),
        ("n_leaves", C.c_int32),
        ("levels_max", C.c_int32),
        ("leaf_rank_baca_max", C.c_int32),
        ("leaf_rank_max", C.c_int32),
        ("iters_max", C.c_int32),
        ("iters_total", C.c_int64),
        ("step_rank_max", C.c_int32 * 64),
        ("n_steps", C.c_int32),
        ("ms_setup", C.c_double),
        ("ms_baca", C.c_double),
        ("ms_recompress", C.c_double),
        ("ms_merge", C.c_double),
        ("ms_total", C.c_double),
        ("entries_evaluated", C.c_double),
        ("resid_bytes", C.c_double),
        ("resid_flops", C.c_double),
        ("svd_sweeps_max", C.c_int32),
        ("pad", C.c_int32),
        ("recompress_flops", C.c_double),
        ("merge_flops", C.c_double),
        ("resid_cr_bytes", C.c_double),
        ("ms_svd", C.c_double),
        ("ms_qr", C.c_double),
        ("ms_gemm", C.c_double),
        ("svd_flops", C.c_double),
        ("svd_launches", C.c_int32),
        ("qr_launches", C.c_int32),
        ("select_swaps", C.c_int64),
    ]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_ if k != "step_rank_max"}
        d["step_rank_max"] = list(self.step_rank_max[: max(self.n_steps, 1)])
        return d


class HBACAError(RuntimeError):
    def __init__(self, status, what=""):
        self.status = status
        super().__init__(f"{what}: {status_string(status)} ({status})")


_lib = None


def load(path: str = LIB_PATH):
    """Load the library (raises if it is missing: there is no CPU fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise OSError(f"{path} is missing; build it with paper_1901_06101_amd.build_lib.build()")
    lib = C.CDLL(path)
    vp, i64, i32, dbl = C.c_void_p, C.c_int64, C.c_int32, C.c_double
    lib.hbaca_compress.argtypes = [C.c_int, C.POINTER(HbParams), vp, vp, i64, i64, dbl, i32, i32,
                                   vp, C.POINTER(vp)]
    lib.hbaca_compress.restype = C.c_int
    lib.hbaca_compress_batched.argtypes = [C.c_int, C.POINTER(HbParams), i64, vp,
                                           C.POINTER(i64), C.POINTER(i64), vp, C.POINTER(i64),
                                           C.POINTER(i64), dbl, i32, i32, vp, C.POINTER(vp)]
    lib.hbaca_compress_batched.restype = C.c_int
    for name in ("hb_result_rank", "hb_result_rows", "hb_result_cols"):
        getattr(lib, name).argtypes = [vp, i64]
        getattr(lib, name).restype = i64
    lib.hb_result_nblocks.argtypes = [vp]
    lib.hb_result_nblocks.restype = i64
    lib.hb_result_nleaves.argtypes = [vp]
    lib.hb_result_nleaves.restype = i64
    lib.hb_result_is_complex.argtypes = [vp]
    lib.hb_result_is_complex.restype = i32
    lib.hb_result_copy.argtypes = [vp, i64, vp, vp, vp, vp]
    lib.hb_result_copy.restype = C.c_int
    lib.hb_result_stats.argtypes = [vp, C.POINTER(HbStats)]
    lib.hb_result_stats.restype = C.c_int
    lib.hb_result_leaf_info.argtypes = [vp, i64, C.POINTER(i64)]
    lib.hb_result_leaf_info.restype = C.c_int
    lib.hb_result_leaf_tape.argtypes = [vp, i64, vp, vp, vp, vp, vp]
    lib.hb_result_leaf_tape.restype = C.c_int
    lib.hb_result_error.argtypes = [vp, i64, i64, C.POINTER(dbl), C.POINTER(dbl), vp]
    lib.hb_result_error.restype = C.c_int
    lib.hbaca_apply.argtypes = [vp, i64, vp, vp, i32, vp]
    lib.hbaca_apply.restype = C.c_int
    lib.hbaca_apply_noalloc.argtypes = [vp, i64, vp, vp, i32, vp]
    lib.hbaca_apply_noalloc.restype = C.c_int
    lib.hb_hodlr_build.argtypes = [C.c_int, C.POINTER(HbParams), vp, i64, i32, dbl, i32, i32, vp,
                                   C.POINTER(vp)]
    lib.hb_hodlr_build.restype = C.c_int
    lib.hb_hodlr_blocks.argtypes = [vp]
    lib.hb_hodlr_blocks.restype = vp
    lib.hb_hodlr_nblocks.argtypes = [vp]
    lib.hb_hodlr_nblocks.restype = i64
    lib.hb_hodlr_nleaves.argtypes = [vp]
    lib.hb_hodlr_nleaves.restype = i64
    lib.hb_hodlr_block_info.argtypes = [vp, i64, vp]
    lib.hb_hodlr_block_info.restype = C.c_int
    lib.hb_hodlr_matvec.argtypes = [vp, vp, vp, vp]
    lib.hb_hodlr_matvec.restype = C.c_int
    lib.hb_hodlr_free.argtypes = [vp]
    lib.hb_hodlr_free.restype = None
    lib.hb_autotune.argtypes = [vp, vp, vp]
    lib.hb_autotune.restype = C.c_int
    lib.hbaca_vjp.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp]
    lib.hbaca_vjp.restype = C.c_int
    lib.hbaca_adjoint.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp]
    lib.hbaca_adjoint.restype = C.c_int
    lib.hbaca_recompute_frozen.argtypes = [vp, C.POINTER(HbParams), vp, vp, vp, C.POINTER(vp)]
    lib.hbaca_recompute_frozen.restype = C.c_int
    lib.hb_partition.argtypes = [i64, i64, i32, i32, C.c_uint64, C.POINTER(i32), vp, vp]
    lib.hb_partition.restype = C.c_int
    lib.hb_result_leaf_frozen.argtypes = [vp, i64, C.POINTER(i32), vp]
    lib.hb_result_leaf_frozen.restype = C.c_int
    lib.hb_result_merge_ranks.argtypes = [vp, vp, C.POINTER(i64)]
    lib.hb_result_merge_ranks.restype = C.c_int
    lib.hb_result_free.argtypes = [vp]
    lib.hb_result_free.restype = None
    lib.hb_status_string.argtypes = [C.c_int]
    lib.hb_status_string.restype = C.c_char_p
    _lib = lib
    return lib


def status_string(st: int) -> str:
    try:
        return load().hb_status_string(int(st)).decode()
    except OSError:
        return "library not loaded"


def _check(st, what):
    if st != HB_OK:
        raise HBACAError(st, what)
