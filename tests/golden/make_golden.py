"""Writes the full-size golden values used by the GPU tests.

Calls only the CPU oracle (oracle/) on the seeded workloads (workloads/) and
stores, per workload, the final rank, the maximum rank after every merge
step, the root singular values and the relative Frobenius error on every
7th row.  Run:  python tests/golden/make_golden.py [name ...]
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from workloads import make_config  # noqa: E402

WORKLOADS = {"helmholtz": "helmholtz_20000.json", "gauss3d": "gauss3d_2000.json",
             "coherent": "coherent_20000.json"}


def sampled_error(src, res, stride=7):
    e2 = a2 = 0.0
    rows = np.arange(0, res.U.shape[0], stride)
    US = res.U * res.S
    for c0 in range(0, rows.size, 256):
        I = rows[c0:c0 + 256]
        A = src.block(I, np.arange(src.n))
        E = A - US[I] @ res.V
        e2 += float(np.sum(np.abs(E) ** 2))
        a2 += float(np.sum(np.abs(A) ** 2))
    return float(np.sqrt(e2 / a2))


def record(name):
    """The stored values of one workload, computed by the oracle."""
    wl = make_config(name)
    src = oracle.EntrySource(wl)
    t = time.perf_counter()
    res = oracle.hbaca(src, wl["m"], wl["n"], wl["tol"], wl["d"], wl["leaf"], wl["seed"])
    el = time.perf_counter() - t
    steps = [max(res.ranks[k]) for k in sorted(res.ranks)]
    return dict(workload=name, m=wl["m"], n=wl["n"], tol=wl["tol"], d=wl["d"],
                leaf=wl["leaf"], seed=wl["seed"], rank=int(res.rank),
                step_rank_max=[int(x) for x in steps],
                sigma=[float(x) for x in res.S],
                rel_err_rows7=sampled_error(src, res),
                oracle_seconds=el,
                source="oracle.hbaca on workloads.make_config(%r)" % name)


def main(names):
    for name in names:
        out = record(name)
        el = out["oracle_seconds"]
        with open(os.path.join(HERE, WORKLOADS[name]), "w") as f:
            json.dump(out, f, indent=1)
        print(name, "rank", out["rank"], "err", out["rel_err_rows7"], "time %.1fs" % el)


if __name__ == "__main__":
    main(sys.argv[1:] or list(WORKLOADS))
