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


def test_adjoint_leg_runs_against_a_stand_in_library(monkeypatch, capsys):
    """The adjoint leg's own code (calls, timing, checks, JSON fields) run on
    the CPU against a stand-in for the library whose result applies the
    factors of a dense SVD; the library itself is tested on the GPU."""
    import json
    import types

    import numpy as np
    import torch

    sys.path.insert(0, ROOT)
    import bench
    import workloads
    from workloads import generators as G

    wl = G.make_gauss3d(n=120, m=100, h=0.7, leaf=30, tol=1e-6, d=8, cfg=71)

    class StandIn:
        def __init__(self, A):
            U, S, Vt = np.linalg.svd(A, full_matrices=False)
            r = int(np.sum(S > 1e-6 * S[0]))
            self.U, self.S, self.V = (torch.tensor(U[:, :r]), torch.tensor(S[:r]),
                                      torch.tensor(Vt[:r].T))

        def rank(self, block=0):
            return int(self.S.numel())

        def apply(self, w, block=0, adjoint=False):
            if adjoint:
                return self.V @ (self.S * (self.U.T @ w))
            return self.U @ (self.S * (self.V.T @ w))

        def vjp(self, w, ybar, want=("w", "h", "x", "y")):
            gw = self.apply(ybar, adjoint=True)
            return gw, torch.zeros(1, dtype=torch.float64), torch.zeros(wl["m"], 3), \
                torch.zeros(wl["n"], 3)

        def close(self):
            pass

    A = np.exp(-((wl["X"][:, None, :] - wl["Y"][None, :, :]) ** 2).sum(-1) / wl["h"] ** 2)
    fake = types.SimpleNamespace(
        require_gpu=lambda: None,
        params=lambda **kw: kw,
        compress=lambda entry, p, X, Y, m, n, tol, d, leaf: StandIn(A))
    monkeypatch.setitem(sys.modules, "paper_1901_06101_amd", fake)
    monkeypatch.setattr(workloads, "make_config", lambda name, scale=1.0: wl)
    orig_device = torch.device
    monkeypatch.setattr(torch, "device", lambda *a, **k: orig_device("cpu"))
    monkeypatch.setattr(torch.cuda, "synchronize", lambda *a, **k: None)
    bench.adjoint(steps=2, warmup=1)
    line = [s for s in capsys.readouterr().out.splitlines() if s.startswith("{")][-1]
    out = json.loads(line)
    for key in ("workload", "rank", "compress_recording_ms", "apply_ms", "vjp_ms",
                "loss_and_gradient_ms", "vjp_over_compression", "w_grad_vs_adjoint_apply_rel",
                "gradients_finite"):
        assert key in out, key
    assert out["w_grad_vs_adjoint_apply_rel"] == 0.0
    assert out["gradients_finite"] is True


def test_comparisons_leg_runs_against_a_stand_in_library(monkeypatch, capsys):
    """The comparisons leg's own code (mixed against FP64, batched against one
    call per block) run on the CPU against a stand-in for the library that
    returns fixed small factors; the library itself is tested on the GPU."""
    import json
    import types

    import numpy as np
    import torch

    sys.path.insert(0, ROOT)
    import bench
    import workloads
    from workloads import generators as G

    rng = np.random.default_rng(3)
    U0 = torch.tensor(np.linalg.qr(rng.standard_normal((40, 5)))[0])
    V0 = torch.tensor(np.linalg.qr(rng.standard_normal((30, 5)))[0])
    S0 = torch.tensor([5.0, 3.0, 1.0, 0.5, 0.1], dtype=torch.float64)

    class StandIn:
        def __init__(self, nblocks=1, shift=0.0):
            self.nblocks = nblocks
            self.shift = shift

        def rank(self, block=0):
            return 5

        def factors(self, block=0):
            return U0, S0 + self.shift, V0

        def error(self, block=0, row_stride=1):
            return 1e-14, 1.0

        def close(self):
            pass

    fake = types.SimpleNamespace(
        HB_PREC_FP64=0, HB_PREC_MIXED=1,
        require_gpu=lambda: None,
        params=lambda **kw: kw,
        compress=lambda *a: StandIn(1, 1e-9 * a[1].get("precision", 0)),
        compress_batched=lambda *a: StandIn(len(a[3])))
    nb = 1024
    cnt = np.full(nb, 2, dtype=np.int64)
    off = np.arange(nb, dtype=np.int64) * 2
    blocks = dict(X=rng.random((2 * nb, 3)), Y=rng.random((2 * nb, 3)) + 3.0, row_off=off,
                  row_cnt=cnt, col_off=off, col_cnt=cnt, seed=3000, entry=2, tol=1e-4, d=8,
                  leaf=64)
    wl = G.make_gauss3d(n=60, leaf=30, cfg=72)
    monkeypatch.setitem(sys.modules, "paper_1901_06101_amd", fake)
    monkeypatch.setattr(workloads, "make_config", lambda name, scale=1.0: wl)
    monkeypatch.setattr(G, "make_laplace_blocks", lambda nblocks, cfg: blocks)
    monkeypatch.setattr(G, "make_gauss_mixture", lambda **kw: wl)
    orig_device = torch.device
    monkeypatch.setattr(torch, "device", lambda *a, **k: orig_device("cpu"))
    monkeypatch.setattr(torch.cuda, "synchronize", lambda *a, **k: None)
    bench.comparisons(steps=1, warmup=1)
    line = [s for s in capsys.readouterr().out.splitlines() if s.startswith("{")][-1]
    out = json.loads(line)
    for key in ("mixed_vs_fp64_gauss_mixture", "mixed_vs_fp64_gauss3d"):
        mv = out[key]
        assert mv["fp64_rank"] == 5 and mv["mixed_within_5tol"] is True
        assert mv["speedup_counts"] is True and mv["eps"] == wl["tol"]
        assert 0.0 < mv["mixed_vs_fp64_operator_rel_diff"] < 1e-8
    bs = out["batched_vs_sequential"]
    for key in ("sequential_fp64_ms", "batched_fp64_ms", "batched_mixed_ms",
                "speedup_batched_fp64", "speedup_batched_mixed", "max_rel_err_rows7_fp64",
                "max_rel_err_rows7_mixed", "mixed_within_5tol", "speedup_fp64_counts",
                "speedup_mixed_counts", "fp64_vs_oracle_max_rel_diff", "eps"):
        assert key in bs, key


def test_json_line_contract_with_a_stand_in_library(monkeypatch, capsys):
    """main()'s line on the CPU with a stand-in library (the legs in child
    processes switched off): the fields the line must carry, the roofline
    object, and the CPU baseline from the oracle on a small workload."""
    import json
    import types

    import torch

    sys.path.insert(0, ROOT)
    import bench
    import workloads
    from workloads import generators as G

    wl = G.make_gauss3d(n=200, leaf=50, tol=1e-6, d=8, cfg=73)

    import time as _time

    class StandIn:
        def __init__(self):
            _time.sleep(0.005)  # a call takes longer than any of its phases

        def stats(self):
            return dict(ms_baca=1.0, resid_bytes=1.5e9, resid_cr_bytes=0.5e9, resid_flops=1e9,
                        recompress_flops=1e9, merge_flops=2e9, ms_setup=0.1,
                        ms_recompress=0.5, ms_merge=2.0, ms_total=3.6, ms_svd=0.4,
                        svd_flops=4e8, ms_qr=0.3, ms_gemm=0.05, svd_launches=3, qr_launches=9)

        def error(self, block=0, row_stride=1):
            return 1e-14, 1.0

        def rank(self, block=0):
            return 17

        def close(self):
            pass

    fake = types.SimpleNamespace(HB_K_LOWRANK_SPIKES=4, require_gpu=lambda: None,
                                 params=lambda **kw: kw, compress=lambda *a: StandIn())
    monkeypatch.setitem(sys.modules, "paper_1901_06101_amd", fake)
    monkeypatch.setattr(workloads, "make_config", lambda name, scale=1.0: wl)
    orig_device = torch.device
    monkeypatch.setattr(torch, "device", lambda *a, **k: orig_device("cpu"))
    monkeypatch.setattr(torch.cuda, "synchronize", lambda *a, **k: None)
    monkeypatch.setattr(bench, "copy_bandwidth", lambda torch: 5000.0)
    monkeypatch.setattr(sys, "argv", ["bench.py", "--steps", "2", "--warmup", "1",
                                      "--no-comparisons", "--no-adjoint", "--no-hodlr",
                                      "--no-sweep"])
    bench.main()
    lines = [s for s in capsys.readouterr().out.splitlines() if s.strip()]
    assert len(lines) == 1
    out = json.loads(lines[0])
    for key in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step",
                "higher_is_better", "scaling", "vs_baseline", "dtype", "data", "config"):
        assert key in out, key
    assert out["n_gpus"] == 1 and out["steps"] == 2 and out["warmup"] == 1
    assert out["value"] == out["ms_per_step"] and out["higher_is_better"] is False
    # the wall time of whole calls, not a phase of one
    assert out["value"] >= 5.0 and out["value"] != out["phases_ms"]["ms_merge"]
    assert out["eps"] == wl["tol"] and out["within_tol"] is True
    assert "workload" in out["config"]
    rf = out["roofline"]
    # the leaf kernel has the most device time here (1.0 ms against 0.4 and
    # 0.35): its bytes are the U/V streams plus the C_k, R_k writes
    assert rf["kernel"] == "baca_leaf_kernel"
    assert rf["bound"] == "hbm" and rf["unit"] == "GB/s" and rf["peak"] == 8000.0
    assert abs(rf["achieved"] - 2000.0) < 1e-9 and abs(rf["frac"] - 0.25) < 1e-12
    assert "traffic" in rf
    kc = {k["kernel"]: k for k in out["kernel_classes"]}
    assert abs(kc["svd_kernel"]["achieved"] - 1.0) < 1e-12 and kc["svd_kernel"]["bound"] == "alu"
    assert [k["launch_ms"] for k in out["kernel_classes"]] == sorted(
        [k["launch_ms"] for k in out["kernel_classes"]], reverse=True)
    cb = out["cpu_baseline"]
    assert cb["kind"] == "oracle" and cb["value"] > 0 and cb["cores"] >= 1
    assert "comparisons" not in out and "adjoint" not in out and "hodlr" not in out


def test_a_failing_leg_becomes_an_error_object(monkeypatch):
    sys.path.insert(0, ROOT)
    import subprocess
    import types

    import bench

    def failing(*a, **k):
        return types.SimpleNamespace(returncode=1, stdout="no json here\n")

    def slow(*a, **k):
        raise subprocess.TimeoutExpired(cmd="bench.py", timeout=k.get("timeout", 1))

    monkeypatch.setattr(subprocess, "run", failing)
    assert "error" in bench.run_child("--adjoint")
    monkeypatch.setattr(subprocess, "run", slow)
    assert "timed out" in bench.run_child("--comparisons", timeout=5)["error"]


def test_a_failing_headline_still_prints_the_line(monkeypatch, capsys):
    import json
    import types

    sys.path.insert(0, ROOT)
    import bench
    import workloads
    from workloads import generators as G

    wl = G.make_gauss3d(n=100, leaf=50, tol=1e-6, d=8, cfg=74)

    def broken(*a, **k):
        raise RuntimeError("device lost")

    fake = types.SimpleNamespace(HB_K_LOWRANK_SPIKES=4, require_gpu=broken,
                                 params=lambda **kw: kw, compress=broken)
    monkeypatch.setitem(sys.modules, "paper_1901_06101_amd", fake)
    monkeypatch.setattr(workloads, "make_config", lambda name, scale=1.0: wl)
    monkeypatch.setattr(sys, "argv", ["bench.py", "--no-comparisons", "--no-adjoint", "--no-hodlr", "--no-sweep",
                                      "--no-cpu-baseline"])
    bench.main()
    lines = [s for s in capsys.readouterr().out.splitlines() if s.strip()]
    assert len(lines) == 1
    out = json.loads(lines[0])
    assert out["value"] is None and "device lost" in out["error"]
    assert out["metric"] == bench.METRIC and out["n_gpus"] == 1


def test_hodlr_leg_runs_against_a_stand_in_library(monkeypatch, capsys):
    """The HODLR leg's own code (build and matvec timing, the sampled check
    against the dense kernel) on the CPU against a stand-in library whose
    matvec is the dense product."""
    import json
    import types

    import torch

    sys.path.insert(0, ROOT)
    import bench
    from workloads import generators as G

    small = G.make_hodlr_curve(N=300)

    class StandIn:
        def __init__(self, X, wl):
            d2 = ((X[:, None, :] - X[None, :, :]) ** 2).sum(-1)
            self.A = torch.exp(-d2 / (wl["gauss_c"] * wl["h"] ** 2))
            self.nblocks, self.nleaves = 2, 2
            self.blocks = types.SimpleNamespace(rank=lambda b: 7)

        def matvec(self, x):
            return self.A @ x

        def close(self):
            pass

    fake = types.SimpleNamespace(
        require_gpu=lambda: None, params=lambda **kw: kw,
        hodlr_build=lambda entry, p, X, nmin, tol, d, leaf: StandIn(X, small))
    monkeypatch.setitem(sys.modules, "paper_1901_06101_amd", fake)
    monkeypatch.setattr(G, "make_hodlr_curve", lambda N: small)
    orig_tensor = torch.tensor
    monkeypatch.setattr(torch, "tensor", lambda *a, **k: orig_tensor(
        *a, **{key: v for key, v in k.items() if key != "device"}))
    orig_arange = torch.arange
    monkeypatch.setattr(torch, "arange", lambda *a, **k: orig_arange(
        *a, **{key: v for key, v in k.items() if key != "device"}))
    monkeypatch.setattr(torch.cuda, "synchronize", lambda *a, **k: None)
    bench.hodlr(steps=1, warmup=1)
    line = [s for s in capsys.readouterr().out.splitlines() if s.startswith("{")][-1]
    out = json.loads(line)
    assert out["max_block_rank"] == 7 and out["blocks"] == 2
    assert out["matvec_rel_err_rows64"] < 1e-14 and out["within_10tol"] is True
