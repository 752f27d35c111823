"""The random first column block J_1 of every leaf (Algorithm 2, first line).

The paper only says J_1 is a random index set of cardinality d.  Reading:
each leaf b draws it from SplitMix64 (Steele, Lea and Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014), a counter-based generator:
the state advances by the odd constant 0x9E3779B97F4A7C15 and each output is
the published 64-bit finaliser of the new state.  Leaf b starts from state
``seed + b * 0x632BE59BD9B4E019 (mod 2^64)`` and takes the first min(d, n0)
entries of a partial Fisher-Yates shuffle of 0..n0-1, position t swapping
with t + (next() mod (n0 - t)).

Pinned against the generator's published output for seed 0.
"""
from __future__ import annotations

import numpy as np

_MASK = (1 << 64) - 1
_GAMMA = 0x9E3779B97F4A7C15
_LEAF_STRIDE = 0x632BE59BD9B4E019


def splitmix64_stream(state: int, count: int) -> list[int]:
    """``count`` successive SplitMix64 outputs starting from ``state``."""
    out = []
    s = state & _MASK
    for _ in range(count):
        s = (s + _GAMMA) & _MASK
        z = s
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK
        out.append(z ^ (z >> 31))
    return out


def first_column_block(seed: int, leaf_id: int, n0: int, d: int) -> np.ndarray:
    """Leaf-local column indices of J_1 for leaf ``leaf_id`` of width n0."""
    q = min(d, n0)
    state = (seed + leaf_id * _LEAF_STRIDE) & _MASK
    draws = splitmix64_stream(state, q)
    perm = list(range(n0))
    for t in range(q):
        j = t + draws[t] % (n0 - t)
        perm[t], perm[j] = perm[j], perm[t]
    return np.array(perm[:q], dtype=np.int64)
