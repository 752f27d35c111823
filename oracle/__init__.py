"""CPU oracle for the H-BACA hot path.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, step-by-step FP64 /
complex128 implementation of the paper's Algorithms 1-3 (ACA, BACA, H-BACA)
written from the paper's text.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import it.  It shares no code with the HIP
path and never imports it; the product path must not call into it.

Parity status of each function is stated in its module docstring.  Readings
of passages where the paper is silent or garbled are listed in the modules
that apply them.
"""
from .entries import EntrySource  # noqa: F401
from .splitmix import splitmix64_stream, first_column_block  # noqa: F401
from .qrcp import householder, qrcp  # noqa: F401
from .baca import baca_leaf, lrnorm, lrnorm_update  # noqa: F401
from .hbaca import (  # noqa: F401
    tree_levels, cluster_tree, eps_rank, recompress, merge_horizontal,
    merge_vertical, merge_tree, hbaca, hbaca_batched,
)
from .aca import aca  # noqa: F401
from .jacobi import jacobi_svd  # noqa: F401
