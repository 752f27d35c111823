"""Row a1 on the CPU: the library's partition (hb_partition: levels,
cluster trees, every leaf's first column block J_1) is the oracle's, index
for index, over sizes with m != n, ragged splits, leaves larger than the
matrix, d larger than the leaf and seeds with the high bit set."""
import os

import numpy as np
import pytest

from oracle.hbaca import cluster_tree, tree_levels
from oracle.splitmix import first_column_block

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1901_06101_amd", "libhbaca.so")

pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libhbaca.so not built")

CASES = [
    (2000, 2000, 250, 8, 1002),      # the Gaussian R^3 workload: L = 3
    (20000, 20000, 625, 16, 2002),   # the Helmholtz workload: L = 5
    (650, 700, 90, 16, 53),          # ragged, m != n
    (37, 1000, 8, 4, 7),             # L limited by min(m, n)
    (100, 100, 500, 8, 1),           # one leaf larger than the matrix
    (9, 9, 1, 3, 11),                # single-row leaves
    (300, 270, 75, 32, 2**63 + 5),   # d = 32, a seed with the high bit set
    (20, 20, 5, 8, 2**64 - 1),       # d above a 5-column leaf
]


@pytest.mark.parametrize("m,n,leaf,d,seed", CASES)
def test_partition_matches_oracle(m, n, leaf, d, seed):
    import paper_1901_06101_amd as hb
    L, leaves, j1 = hb.partition(m, n, leaf, d, seed)
    assert L == tree_levels(m, n, leaf)
    rows = cluster_tree(m, L)[L]
    cols = cluster_tree(n, L)[L]
    nb = 1 << L
    assert leaves.shape == (nb * nb, 4)
    for t in range(nb):
        for v in range(nb):
            b = t * nb + v
            assert tuple(leaves[b]) == (rows[t][0], rows[t][1], cols[v][0], cols[v][1])
            ref = np.asarray(first_column_block(seed, b, cols[v][1], d))
            q = min(d, cols[v][1])
            assert ref.size == q
            assert np.array_equal(j1[b, :q], ref)
            assert np.all(j1[b, q:] == -1)


def test_partition_rejects_bad_sizes():
    import ctypes as C

    from paper_1901_06101_amd import _binding
    lib = _binding.load(LIB)
    L = C.c_int32(0)
    for args in ((0, 5, 2, 2), (5, 0, 2, 2), (5, 5, 0, 2), (5, 5, 2, 0)):
        assert lib.hb_partition(*args, 1, C.byref(L), None, None) == -1
    assert lib.hb_partition(5, 5, 2, 2, 1, None, None, None) == -1
