"""Seeded synthetic inputs for the H-BACA hot path.

This package is the only code shared by the CPU oracle and the HIP path.  It
draws point sets, factor matrices, sparse spikes and block lists, and orders
point sets along a KD split tree.  It holds none of the method's arithmetic:
no entry evaluation, no pivoting, no factorisation.
"""
from .generators import (  # noqa: F401
    kd_order,
    make_config,
    make_gauss3d,
    make_helmholtz_plates,
    make_lowrank_spikes,
    make_laplace_blocks,
    make_gauss_mixture,
    make_efie2d_strips,
    make_polynomial,
    make_hodlr_curve,
    make_hodlr_polynomial,
    CONFIG_NAMES,
)
