"""bench.py's host-side contract on a machine without a GPU: more than one
GPU is refused with a message and exit status 2 before anything touches a
GPU, and the CPU-baseline leg reports the oracle's time in the fields the
JSON line carries."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert p.returncode == 2
    assert "one GPU only" in p.stderr
    assert p.stdout.strip() == ""


def test_cpu_baseline_fields():
    sys.path.insert(0, ROOT)
    import bench
    from workloads import generators as G
    wl = G.make_gauss3d(n=300, leaf=75, tol=1e-6, d=8, cfg=63)
    out = bench.cpu_baseline(wl)
    assert out["kind"] == "oracle" and out["unit"] == "ms"
    assert out["value"] > 0 and out["cores"] >= 1
    assert out["rank"] > 0 and out["sample"]


def test_non_finite_values_become_null():
    sys.path.insert(0, ROOT)
    import json

    import bench
    out = bench._finite({"a": float("nan"), "b": [1.0, float("inf")], "c": {"d": -float("inf")},
                         "e": 2, "f": "x", "g": 0.5})
    assert out == {"a": None, "b": [1.0, None], "c": {"d": None}, "e": 2, "f": "x", "g": 0.5}
    json.loads(json.dumps(out), parse_constant=lambda c: (_ for _ in ()).throw(ValueError(c)))
