"""Benchmark: H-BACA compress time on one MI355X.

A step is one full H-BACA pass (leaf BACA, leaf SVD re-compression, every
merge level) over the benchmark workload with its inputs already resident in
HBM.  Prints one JSON line.  The roofline object rates the leaf BACA kernel:
its algorithmic bytes (U and V streamed once per iteration, counted by the
library from the per-iteration block ranks) over its duration from HIP events
on the call's stream, against the 8 TB/s HBM peak.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload helmholtz]
                  [--no-cpu-baseline] [--no-comparisons] [--no-adjoint]

Besides the headline workload, the line carries "comparisons": mixed
precision against plain FP64 (Gaussian 2000^2) and one batched call against
one call per block (1024 Laplace blocks); and "adjoint": the frozen-pivot
adjoint on the differentiation workload (Gaussian 50000^2 in R^3, h = 0.7),
that is the compression that records its pivots and ranks, the apply
y = A~w and the gradients of <ybar, A~w> with respect to w, h and every
point.  Each of the two runs in a child process of its own with a time
limit, after the headline measurement, so that neither can change it.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "H-BACA compress time at rel err\u2264tol, mixed/batched vs plain FP64; % roofline"
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6


def cpu_baseline(wl):
    """The CPU oracle, timed on this host on the same workload."""
    import numpy as np  # noqa: F401
    import oracle
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        threads = 1
    src = oracle.EntrySource(wl)
    t = time.perf_counter()
    res = oracle.hbaca(src, wl["m"], wl["n"], wl["tol"], wl["d"], wl["leaf"], wl["seed"])
    el = time.perf_counter() - t
    return dict(value=el * 1e3, unit="ms", cores=int(threads), kind="oracle",
                sample=f"the whole workload ({len(res.leaf_info)} leaves, all merge levels); "
                       "single Python thread, NumPy BLAS threads as counted",
                rank=int(res.rank))


def comparisons(steps=5, warmup=1):
    """Mixed precision and batching against the plain FP64 GPU path, each at
    the accuracy it reaches; prints one JSON object.  Runs in a child process
    of the benchmark so that its outcome cannot affect the headline line."""
    import numpy as np
    import torch

    import paper_1901_06101_amd as hb
    from workloads import generators as G
    from workloads import make_config

    hb.require_gpu()
    dev = torch.device("cuda:0")

    def timed(fn, steps, warmup):
        for _ in range(warmup):
            fn().close()
        torch.cuda.synchronize()
        t = time.perf_counter()
        res = None
        for _ in range(steps):
            if res is not None:
                res.close()
            res = fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t) * 1e3 / steps, res

    def rel_err(res, block=0):
        e2, a2 = res.error(block, 7)
        return float(np.sqrt(e2 / a2))

    out = {}
    # plain FP64 against mixed precision on the Gaussian R^3 workload
    wl = make_config("gauss3d")
    X = torch.tensor(wl["X"], device=dev)
    Y = torch.tensor(wl["Y"], device=dev)

    def single(prec):
        p = hb.params(dim=3, h=wl["h"], gauss_c=wl["gauss_c"], seed=wl["seed"], precision=prec)
        return hb.compress(wl["entry"], p, X, Y, wl["m"], wl["n"], wl["tol"], wl["d"], wl["leaf"])

    f_ms, f_res = timed(lambda: single(hb.HB_PREC_FP64), steps, warmup)
    _note(f"comparisons: gauss3d FP64 {f_ms:.1f} ms")
    m_ms, m_res = timed(lambda: single(hb.HB_PREC_MIXED), steps, warmup)
    _note(f"comparisons: gauss3d mixed {m_ms:.1f} ms")
    ef, em = rel_err(f_res), rel_err(m_res)

    def operator_rel_diff(a, b):
        # ||Ua Sa Va^T - Ub Sb Vb^T||_F / ||Ua Sa Va^T||_F from the factors
        Ua, Sa, Va = a.factors(0)
        Ub, Sb, Vb = b.factors(0)
        Qu, Ru = torch.linalg.qr(torch.cat([Ua, Ub], dim=1))
        Qv, Rv = torch.linalg.qr(torch.cat([Va, Vb], dim=1))
        M = Ru @ torch.diag(torch.cat([Sa, -Sb])) @ Rv.T
        return float(torch.linalg.norm(M) / torch.linalg.norm(Sa))

    out["mixed_vs_fp64"] = dict(
        workload=f"gauss3d {wl['m']}x{wl['n']} tol={wl['tol']} d={wl['d']} leaf={wl['leaf']}",
        fp64_ms=f_ms, mixed_ms=m_ms, speedup=f_ms / m_ms, fp64_rank=f_res.rank(0),
        mixed_rank=m_res.rank(0), fp64_rel_err_rows7=ef, mixed_rel_err_rows7=em,
        mixed_vs_fp64_operator_rel_diff=operator_rel_diff(f_res, m_res),
        mixed_within_5tol=bool(em <= 5 * wl["tol"]),
        # the speedup counts only where both reach rel. error <= tol
        speedup_counts=bool(ef <= wl["tol"] and em <= wl["tol"]))
    f_res.close()
    m_res.close()
    # one batched call against one call per block (Laplace blocks of the
    # batched workload's recipe), FP64 and mixed
    nb = 1024
    wb = G.make_laplace_blocks(nblocks=nb, cfg=3)
    Xb = torch.tensor(wb["X"], device=dev)
    Yb = torch.tensor(wb["Y"], device=dev)

    def batched(prec):
        p = hb.params(dim=3, seed=wb["seed"], precision=prec)
        return hb.compress_batched(wb["entry"], p, Xb, wb["row_off"], wb["row_cnt"], Yb,
                                   wb["col_off"], wb["col_cnt"], wb["tol"], wb["d"], wb["leaf"])

    bf_ms, bf_res = timed(lambda: batched(hb.HB_PREC_FP64), 3, 1)
    _note(f"comparisons: {nb} Laplace blocks batched FP64 {bf_ms:.1f} ms")
    bm_ms, bm_res = timed(lambda: batched(hb.HB_PREC_MIXED), 3, 1)
    _note(f"comparisons: {nb} Laplace blocks batched mixed {bm_ms:.1f} ms")

    def sequential():
        last = None
        for b in range(nb):
            r0, m = int(wb["row_off"][b]), int(wb["row_cnt"][b])
            c0, n = int(wb["col_off"][b]), int(wb["col_cnt"][b])
            p = hb.params(dim=3, seed=wb["seed"] + b)
            if last is not None:
                last.close()
            last = hb.compress(wb["entry"], p, Xb[r0:r0 + m], Yb[c0:c0 + n], m, n, wb["tol"],
                               wb["d"], wb["leaf"])
        return last

    s_ms, s_res = timed(sequential, 1, 1)
    s_res.close()
    _note(f"comparisons: {nb} Laplace blocks one call each {s_ms:.1f} ms")
    ebf = max(rel_err(bf_res, b) for b in range(nb))
    ebm = max(rel_err(bm_res, b) for b in range(nb))
    out["batched_vs_sequential"] = dict(
        workload=f"laplace_batched {nb} blocks, sizes 64-1024, tol={wb['tol']} d={wb['d']} "
                 f"leaf={wb['leaf']}",
        sequential_fp64_ms=s_ms, batched_fp64_ms=bf_ms, batched_mixed_ms=bm_ms,
        speedup_batched_fp64=s_ms / bf_ms, speedup_batched_mixed=s_ms / bm_ms,
        max_rel_err_rows7_fp64=ebf, max_rel_err_rows7_mixed=ebm,
        mixed_within_5tol=bool(ebm <= 5 * wb["tol"]),
        speedup_fp64_counts=bool(ebf <= wb["tol"]),
        speedup_mixed_counts=bool(ebf <= wb["tol"] and ebm <= wb["tol"]))
    print(json.dumps(out), flush=True)


def adjoint(steps=3, warmup=1):
    """The differentiation workload: compression with pivots and ranks
    recorded, y = A~w, and hbaca_vjp (gradients with respect to w, h and the
    points of both sides); prints one JSON object."""
    import numpy as np
    import torch

    import paper_1901_06101_amd as hb
    from workloads import make_config

    hb.require_gpu()
    dev = torch.device("cuda:0")
    wl = make_config("gauss3d_adjoint")
    X = torch.tensor(wl["X"], device=dev)
    Y = torch.tensor(wl["Y"], device=dev)
    p = hb.params(dim=3, h=wl["h"], gauss_c=wl["gauss_c"], seed=wl["seed"], record_tape=2)

    def compress():
        return hb.compress(wl["entry"], p, X, Y, wl["m"], wl["n"], wl["tol"], wl["d"],
                           wl["leaf"])

    def clock(fn, k):
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(k):
            out = fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t) * 1e3 / k, out

    _note(f"adjoint: {wl['m']}x{wl['n']} compression with pivots recorded")
    res = compress()
    for _ in range(warmup):
        compress().close()
    c_ms, r2 = clock(compress, steps)
    r2.close()
    rng = np.random.default_rng(wl["seed"])
    w = torch.tensor(rng.standard_normal(wl["n"]), device=dev)
    b = torch.tensor(rng.standard_normal(wl["m"]), device=dev)
    a_ms, y = clock(lambda: res.apply(w), steps)
    yb = 2.0 * (y - b)
    _note("adjoint: hbaca_vjp")
    for _ in range(warmup):
        res.vjp(w, yb)
    v_ms, (gw, gh, gX, gY) = clock(lambda: res.vjp(w, yb), steps)
    # w enters linearly: its gradient is the adjoint apply A~^T ybar
    ref = res.apply(yb, adjoint=True)
    check = float(torch.linalg.norm(gw - ref) / torch.linalg.norm(ref))
    finite = bool(torch.isfinite(gh).all() and torch.isfinite(gX).all()
                  and torch.isfinite(gY).all())
    out = dict(workload=f"gauss3d_adjoint {wl['m']}x{wl['n']} h={wl['h']} tol={wl['tol']} "
                        f"d={wl['d']} leaf={wl['leaf']}",
               steps=steps, warmup=warmup, rank=res.rank(0), compress_recording_ms=c_ms,
               apply_ms=a_ms, vjp_ms=v_ms, loss_and_gradient_ms=a_ms + v_ms,
               vjp_over_compression=v_ms / c_ms,
               w_grad_vs_adjoint_apply_rel=check, gradients_finite=finite)
    _note(f"adjoint: vjp {v_ms:.1f} ms")
    res.close()
    print(json.dumps(out), flush=True)


def copy_bandwidth(torch, nbytes=1 << 30, reps=5):
    """Device-to-device copy rate in GB/s (bytes read plus bytes written),
    the measured counterpart of the HBM peak."""
    try:
        src = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        dst.copy_(src)
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            dst.copy_(src)
        b.record()
        b.synchronize()
        ms = a.elapsed_time(b) / reps
        del src, dst
        return 2.0 * nbytes / (ms * 1e-3) / 1e9
    except Exception:
        return None


def _finite(x):
    """x with every non-finite float replaced by None (strict JSON)."""
    if isinstance(x, float):
        return x if x == x and abs(x) != float("inf") else None
    if isinstance(x, dict):
        return {k: _finite(v) for k, v in x.items()}
    if isinstance(x, (list, tuple)):
        return [_finite(v) for v in x]
    return x


def _note(msg):
    """Progress of the run on stderr (stdout carries only the JSON line)."""
    print(f"bench: {msg}", file=sys.stderr, flush=True)


def run_child(flag, timeout=300):
    """Runs this script with `flag` in a child process; its last JSON line,
    or an error object."""
    import subprocess
    _note(f"{flag[2:]} start in a child process")
    try:
        r = subprocess.run([sys.executable, os.path.abspath(__file__), flag],
                           stdout=subprocess.PIPE, text=True, timeout=timeout)
    except subprocess.TimeoutExpired:
        return {"error": f"timed out after {timeout} s"}
    for line in reversed(r.stdout.strip().splitlines()):
        if line.startswith("{"):
            return json.loads(line)
    return {"error": f"exit {r.returncode} (its messages are on stderr)"}


def headline(args, wl):
    """The timed compress calls on the headline workload: the measured
    fields of the line."""
    import numpy as np
    import torch

    import paper_1901_06101_amd as hb

    hb.require_gpu()
    dev = torch.device("cuda:0")
    X = torch.tensor(wl["X"], device=dev) if wl.get("X") is not None else None
    Y = torch.tensor(wl["Y"], device=dev) if wl.get("Y") is not None else None
    p = hb.params(dim=(wl["X"].shape[1] if wl.get("X") is not None else 0), h=wl.get("h", 0.0),
                  gauss_c=wl.get("gauss_c", 1.0), wavenumber=wl.get("wavenumber", 0.0),
                  seed=wl["seed"])
    if wl["entry"] == hb.HB_K_LOWRANK_SPIKES:
        p["G1"] = torch.tensor(wl["G1"], device=dev)
        p["G2"] = torch.tensor(wl["G2"], device=dev)
        p["spike_lin"] = torch.tensor(wl["spike_lin"], device=dev)
        p["spike_val"] = torch.tensor(wl["spike_val"], device=dev)

    def step():
        return hb.compress(wl["entry"], p, X, Y, wl["m"], wl["n"], wl["tol"], wl["d"],
                           wl["leaf"])

    _note(f"{wl['name']} {wl['m']}x{wl['n']}: warm-up")
    for _ in range(args.warmup):
        step().close()
    torch.cuda.synchronize()
    _note(f"{wl['name']}: {args.steps} timed steps")
    stats = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        r = step()
        stats.append(r.stats())
        last = r
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ms = el * 1e3 / args.steps
    e2, a2 = last.error(0, 7)
    rel_err = float(np.sqrt(e2 / a2))
    rank = last.rank(0)
    st = stats[-1]
    # dominant-kernel roofline: the leaf BACA kernel (residual passes), timed
    # with HIP events the library records on its stream around that launch
    ms_baca = float(np.mean([s["ms_baca"] for s in stats]))
    achieved = st["resid_bytes"] / (ms_baca * 1e-3) / 1e9
    roofline = dict(kernel="baca_leaf_kernel", bound="hbm", achieved=achieved,
                    peak=HBM_PEAK_GBS, unit="GB/s", frac=achieved / HBM_PEAK_GBS,
                    traffic=None,
                    algorithmic_bytes_per_launch=st["resid_bytes"],
                    launch_ms=ms_baca)
    copy = copy_bandwidth(torch)
    roofline["copy_GBps_measured"] = copy
    roofline["frac_of_copy"] = achieved / copy if copy else None
    phases = {k: float(np.mean([s[k] for s in stats])) for k in
              ("ms_setup", "ms_baca", "ms_recompress", "ms_merge", "ms_total")}
    # the other kernel classes against the FP64 peak: algorithmic flops of
    # the leaf residual passes, the re-compression and the merges (the
    # library's counters) over each phase's device time
    phase_rates = {}
    for name, flops, phase_ms in (("leaf_residuals", st["resid_flops"], phases["ms_baca"]),
                                  ("recompression", st["recompress_flops"], phases["ms_recompress"]),
                                  ("merges", st["merge_flops"], phases["ms_merge"])):
        tf = flops / (phase_ms * 1e-3) / 1e12 if phase_ms > 0 else None
        phase_rates[name] = dict(flops=flops, ms=phase_ms, achieved_TFLOPs=tf,
                                 peak_TFLOPs=FP64_PEAK_TFLOPS,
                                 frac=(tf / FP64_PEAK_TFLOPS) if tf is not None else None)
    out = {
        "value": ms,
        "ms_per_step": ms,
        "rank": rank,
        "rel_err_rows7": rel_err,
        "phases_ms": phases,
        "roofline": roofline,
        "phase_rates": phase_rates,
    }
    last.close()
    _note(f"{wl['name']}: {ms:.2f} ms per compress")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="helmholtz")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-comparisons", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--comparisons", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--adjoint", action="store_true", help=argparse.SUPPRESS)
    args = ap.parse_args()
    if args.comparisons:
        comparisons()
        return
    if args.adjoint:
        adjoint()
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for {args.gpus}); how H-BACA would "
              "shard over several GPUs is described in the design notes", file=sys.stderr)
        sys.exit(2)
    from workloads import make_config

    wl = make_config(args.workload)
    out = {
        "metric": METRIC,
        "value": None,
        "unit": "ms",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": None,
        "higher_is_better": False,
        "scaling": "strong",
        "vs_baseline": None,
        "dtype": "c128" if wl.get("complex") else "f64",
        "data": "synthetic",
        "config": {"workload": f"{wl['name']} {wl['m']}x{wl['n']} tol={wl['tol']} d={wl['d']} "
                               f"leaf={wl['leaf']}",
                   "precision": "plain FP64 (complex128 for Helmholtz)",
                   "parallelism": "single GPU"},
    }
    try:
        out.update(headline(args, wl))
    except Exception as e:  # the line is still printed, with the failure
        out["error"] = f"{type(e).__name__}: {e}"
        _note(f"headline failed: {out['error']}")
    if not args.no_cpu_baseline:
        _note("CPU baseline (the oracle on the same workload)")
        try:
            out["cpu_baseline"] = cpu_baseline(wl)
        except Exception as e:  # the GPU line is still reported
            out["cpu_baseline"] = {"value": None, "unit": "ms", "cores": None, "kind": "oracle",
                                   "sample": f"failed: {type(e).__name__}: {e}"}
    # the legs beside the headline, each in a child process with a time limit
    if not args.no_comparisons:
        out["comparisons"] = run_child("--comparisons")
    if not args.no_adjoint:
        out["adjoint"] = run_child("--adjoint")
    print(json.dumps(_finite(out)), flush=True)


if __name__ == "__main__":
    main()
