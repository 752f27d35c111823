"""A second process on the device after this one has made cooperative
launches (the multi-workgroup SVD).  The runtime has refused cooperative
launches to such a process (error 401); the library then reruns the batch on
one workgroup per matrix and keeps to that for the process.  Either way the
child's result must meet the oracle bars of the parity tests."""
import os
import subprocess
import sys

import numpy as np
import pytest

from workloads import generators as G

from _hbtest import lowrank_diff, recon_norm, run_gpu, run_oracle, say

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
TESTS = os.path.join(ROOT, "tests")


def _workload():
    # merges wide enough for several workgroups per SVD (as in the parity
    # test of the multi-workgroup SVD)
    return G.make_gauss3d(n=1100, m=900, leaf=140, d=8, cfg=21)


CHILD = r"""
import sys
import numpy as np
import paper_1901_06101_amd as hb
from test_gpu_zw_coop_child import _workload
from _hbtest import factors_np, run_gpu
hb.require_gpu()
res = run_gpu(hb, _workload(), diag_svd_storage=3)
U, S, Vh = factors_np(res)
np.savez(sys.argv[1], U=U, S=S, Vh=Vh)
print("child: rank", S.size, flush=True)
"""


def test_child_after_cooperative_launches(lib, tmp_path):
    wl = _workload()
    say(f"[cooperative child] gauss3d {wl['m']} x {wl['n']}, this process first")
    res = run_gpu(lib, wl, diag_svd_storage=3)  # cooperative launches in this process
    assert res.rank(0) > 0
    out = str(tmp_path / "child.npz")
    env = dict(os.environ, HB_VERBOSE="1",
               PYTHONPATH=os.pathsep.join([ROOT, TESTS, os.environ.get("PYTHONPATH", "")]))
    say("  child process started")
    proc = subprocess.run([sys.executable, "-c", CHILD, out], env=env, cwd=ROOT,
                          capture_output=True, text=True, timeout=240)
    say(f"  child exit {proc.returncode}: {proc.stdout.strip()[-200:]}")
    refused = "falling back" in proc.stderr
    say(f"  cooperative launch refused in the child: {refused}")
    assert proc.returncode == 0, proc.stderr[-2000:]
    data = np.load(out)
    U, S, Vh = data["U"], data["S"], data["Vh"]
    _, ores = run_oracle(wl)
    assert S.size == ores.rank
    assert np.allclose(S, ores.S, rtol=0, atol=1e-10 * ores.S[0])
    ref = recon_norm(ores.U * ores.S, ores.V.conj().T)
    diff = lowrank_diff(U * S, Vh, ores.U * ores.S, ores.V.conj().T)
    say(f"  reconstruction difference {diff / ref:.2e}")
    assert diff <= 1e-10 * ref
