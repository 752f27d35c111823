"""Benchmark: H-BACA compress time on one MI355X.

A step is one full H-BACA call (leaf BACA, leaf SVD re-compression, every
merge level) over the benchmark workload with its inputs already resident in
HBM; `value` is the wall time per call.  The metric asks for the time at
rel. error <= tol: the truncation tolerance eps of the call is the largest of
tol, tol/2, tol/4, tol/8 whose result reaches a sampled relative Frobenius
error <= tol against A (the eps-rank is relative to sigma_1 of each block, so
eps = tol can leave a Frobenius error above tol); every path of the line is
run at that eps.  Prints one JSON line.

The roofline object rates the kernel class that takes the most device time
in the call (HIP events the library records on the call's stream around
each launch): the leaf BACA kernel against HBM (algorithmic bytes: U and V
streamed once per iteration plus the residual blocks C_k and R_k written),
or the small SVDs / the TSQR kernels against the FP64 vector peak.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload helmholtz]
                  [--no-cpu-baseline] [--no-comparisons] [--no-adjoint] [--no-hodlr]
                  [--no-sweep]

Besides the headline workload, the line carries "comparisons": mixed
precision against plain FP64 (the 8-D Gaussian mixture at 2000^2 and the
Gaussian R^3 2000^2 workload) and one batched call against one call per
block (the 4096 Laplace blocks of the batched workload), and "adjoint": the
frozen-pivot adjoint on the differentiation workload (Gaussian 50000^2 in
R^3, h = 0.7), and "hodlr": a hierarchical matrix of a Gaussian kernel
built with the batched path and its matrix-vector product, and "sweep": time,
rank and error over leaf counts and block sizes d on four kernels (the
paper's efficiency study, Fig. 5).  Each runs in a
child process of its own with a time limit,
after the headline measurement, so that neither can change it.
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
FP64_PEAK_TFLOPS = 78.6  # FP64 vector (and FP64 MFMA) peak of MI355X
EPS_DIVISORS = (1, 1.25, 1.6, 2, 4, 8)


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(wl, eps=None, single_thread=True):
    """The CPU oracle, timed on this host on the same workload at the same
    eps: once with the BLAS threads NumPy starts with (all cores) and once
    limited to one thread."""
    import oracle
    try:
        from threadpoolctl import threadpool_info, threadpool_limits
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        threadpool_limits = None
        threads = 1
    eps = wl["tol"] if eps is None else eps
    src = oracle.EntrySource(wl)

    def once():
        t = time.perf_counter()
        res = oracle.hbaca(src, wl["m"], wl["n"], eps, wl["d"], wl["leaf"], wl["seed"])
        return (time.perf_counter() - t) * 1e3, res

    ms, res = once()
    out = dict(value=ms, unit="ms", cores=int(threads), kind="oracle",
               sample=f"the whole workload ({len(res.leaf_info)} leaves, all merge levels, "
                      f"eps {eps:g}); one Python thread, NumPy BLAS on {threads} threads",
               rank=int(res.rank), cpu_model=_cpu_model(), logical_cpus=os.cpu_count())
    if single_thread and threadpool_limits is not None:
        with threadpool_limits(limits=1):
            ms1, _ = once()
        out["single_thread"] = dict(value=ms1, unit="ms", cores=1)
    return out


def _lowrank_rel_diff(X1, Y1, X2, Y2):
    """||X1 Y1^H - X2 Y2^H||_F / ||X2 Y2^H||_F from QR factors of the stacked
    factors (never the dense products)."""
    import numpy as np
    if X2.shape[1] == 0:
        return 0.0 if X1.shape[1] == 0 else float("inf")
    _, R1 = np.linalg.qr(np.hstack([X1, -X2]))
    _, R2 = np.linalg.qr(np.hstack([Y1, Y2]))
    _, Q1 = np.linalg.qr(X2)
    _, Q2 = np.linalg.qr(Y2)
    return float(np.linalg.norm(R1 @ R2.conj().T) / np.linalg.norm(Q1 @ Q2.conj().T))


def comparisons(steps=5, warmup=1):
    """Mixed precision and batching against the plain FP64 GPU path at equal
    accuracy: every pair runs at the largest eps (tol / 1, 2, 4, 8) where
    both sides reach a sampled relative error <= tol.  Prints one JSON object.
    Runs in a child process of the benchmark so that its outcome cannot
    affect the headline line."""
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
        return float(np.sqrt(e2 / a2)) if a2 > 0 else 0.0

    def max_err(res):
        return max(rel_err(res, b) for b in range(getattr(res, "nblocks", 1)))

    def equal_accuracy_eps(tol, makers):
        """Largest tol / f at which every maker's result is within tol."""
        eps = tol
        for f in EPS_DIVISORS:
            eps = tol / f
            ok = True
            for mk in makers:
                r = mk(eps)
                ok = ok and max_err(r) <= tol
                r.close()
            if ok:
                break
        return eps

    def operator_rel_diff(a, b):
        Ua, Sa, Va = (t.cpu().numpy() for t in a.factors(0))
        Ub, Sb, Vb = (t.cpu().numpy() for t in b.factors(0))
        return _lowrank_rel_diff(Ua * Sa, Va, Ub * Sb, Vb)

    out = {}
    # plain FP64 against mixed precision: the 8-D Gaussian mixture (the
    # mixed-precision workload's recipe at 2000^2) and the Gaussian R^3 case
    single_cases = (
        ("gauss_mixture", G.make_gauss_mixture(n=2000, leaf=250, tol=1e-6, d=16, cfg=4)),
        ("gauss3d", make_config("gauss3d")),
    )
    for key, wl in single_cases:
        X = torch.tensor(wl["X"], device=dev)
        Y = torch.tensor(wl["Y"], device=dev)
        tol = wl["tol"]

        def single(prec, eps, wl=wl, X=X, Y=Y):
            p = hb.params(dim=wl["X"].shape[1], h=wl["h"], gauss_c=wl["gauss_c"],
                          seed=wl["seed"], precision=prec)
            return hb.compress(wl["entry"], p, X, Y, wl["m"], wl["n"], eps, wl["d"], wl["leaf"])

        eps = equal_accuracy_eps(tol, [lambda e: single(hb.HB_PREC_FP64, e),
                                       lambda e: single(hb.HB_PREC_MIXED, e)])
        f_ms, f_res = timed(lambda: single(hb.HB_PREC_FP64, eps), steps, warmup)
        m_ms, m_res = timed(lambda: single(hb.HB_PREC_MIXED, eps), steps, warmup)
        _note(f"comparisons: {key} FP64 {f_ms:.1f} ms, mixed {m_ms:.1f} ms (eps {eps:g})")
        ef, em = rel_err(f_res), rel_err(m_res)
        out[f"mixed_vs_fp64_{key}"] = dict(
            workload=f"{key} {wl['m']}x{wl['n']} tol={tol} d={wl['d']} leaf={wl['leaf']}",
            eps=eps, fp64_ms=f_ms, mixed_ms=m_ms, speedup=f_ms / m_ms,
            fp64_rank=f_res.rank(0), mixed_rank=m_res.rank(0), fp64_rel_err_rows7=ef,
            mixed_rel_err_rows7=em,
            mixed_vs_fp64_operator_rel_diff=operator_rel_diff(m_res, f_res),
            mixed_within_5tol=bool(em <= 5 * tol),
            # the speedup counts only where both reach rel. error <= tol
            speedup_counts=bool(ef <= tol and em <= tol))
        f_res.close()
        m_res.close()
    # one batched call against one call per block: the batched workload's
    # 4096 Laplace blocks, FP64 and mixed
    wb = G.make_laplace_blocks(nblocks=4096, cfg=3)
    nb = len(wb["row_cnt"])
    Xb = torch.tensor(wb["X"], device=dev)
    Yb = torch.tensor(wb["Y"], device=dev)
    tol = wb["tol"]

    def batched(prec, eps):
        p = hb.params(dim=3, seed=wb["seed"], precision=prec)
        return hb.compress_batched(wb["entry"], p, Xb, wb["row_off"], wb["row_cnt"], Yb,
                                   wb["col_off"], wb["col_cnt"], eps, wb["d"], wb["leaf"])

    eps = equal_accuracy_eps(tol, [lambda e: batched(hb.HB_PREC_FP64, e),
                                   lambda e: batched(hb.HB_PREC_MIXED, e)])
    bf_ms, bf_res = timed(lambda: batched(hb.HB_PREC_FP64, eps), 3, 1)
    _note(f"comparisons: {nb} Laplace blocks batched FP64 {bf_ms:.1f} ms")
    bm_ms, bm_res = timed(lambda: batched(hb.HB_PREC_MIXED, eps), 3, 1)
    _note(f"comparisons: {nb} Laplace blocks batched mixed {bm_ms:.1f} ms")

    def sequential():
        last = None
        for b in range(nb):
            r0, m = int(wb["row_off"][b]), int(wb["row_cnt"][b])
            c0, n = int(wb["col_off"][b]), int(wb["col_cnt"][b])
            p = hb.params(dim=3, seed=wb["seed"] + b)
            if last is not None:
                last.close()
            last = hb.compress(wb["entry"], p, Xb[r0:r0 + m], Yb[c0:c0 + n], m, n, eps,
                               wb["d"], wb["leaf"])
        return last

    s_ms, s_res = timed(sequential, 1, 1)
    s_res.close()
    _note(f"comparisons: {nb} Laplace blocks one call each {s_ms:.1f} ms")
    ebf, ebm = max_err(bf_res), max_err(bm_res)
    # an evenly spaced sample of the blocks against the oracle (its H-BACA
    # of that block alone)
    sample = list(range(0, nb, max(1, nb // 128)))
    oracle_diff = None
    try:
        import oracle
        worst = 0.0
        for b in sample:
            ro, rc = int(wb["row_off"][b]), int(wb["row_cnt"][b])
            co, cc = int(wb["col_off"][b]), int(wb["col_cnt"][b])
            src = oracle.EntrySource(wb, X=wb["X"][ro:ro + rc], Y=wb["Y"][co:co + cc])
            ref = oracle.hbaca(src, rc, cc, eps, wb["d"], wb["leaf"], wb["seed"] + b)
            U, S, V = (t.cpu().numpy() for t in bf_res.factors(b))
            worst = max(worst, _lowrank_rel_diff(U * S, V, ref.U * ref.S, ref.V.T))
        oracle_diff = worst
    except Exception as e:  # reported, not fatal to the leg
        oracle_diff = f"{type(e).__name__}: {e}"
    out["batched_vs_sequential"] = dict(
        workload=f"laplace_batched {nb} blocks, sizes 64-1024, tol={tol} d={wb['d']} "
                 f"leaf={wb['leaf']}",
        eps=eps, sequential_fp64_ms=s_ms, batched_fp64_ms=bf_ms, batched_mixed_ms=bm_ms,
        speedup_batched_fp64=s_ms / bf_ms, speedup_batched_mixed=s_ms / bm_ms,
        max_rel_err_rows7_fp64=ebf, max_rel_err_rows7_mixed=ebm,
        fp64_vs_oracle_max_rel_diff=oracle_diff,
        fp64_vs_oracle_sample=f"{len(sample)} of the {nb} blocks, evenly spaced",
        mixed_within_5tol=bool(ebm <= 5 * tol),
        speedup_fp64_counts=bool(ebf <= tol),
        speedup_mixed_counts=bool(ebf <= tol and ebm <= tol))
    bf_res.close()
    bm_res.close()
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


def hodlr(steps=5, warmup=1):
    """A hierarchical (HODLR) matrix of the Gaussian kernel of 32768 points on
    a space curve built with the batched H-BACA path (every off-diagonal block
    of the cluster tree in one call), and its matrix-vector product; the
    product is checked against the dense kernel on every 64th row.  Prints
    one JSON object."""
    import numpy as np
    import torch

    import paper_1901_06101_amd as hb
    from workloads import generators as G

    hb.require_gpu()
    wl = G.make_hodlr_curve(N=32768)
    N = wl["X"].shape[0]
    X = torch.tensor(wl["X"], device="cuda")
    p = hb.params(dim=3, h=wl["h"], gauss_c=wl["gauss_c"], seed=wl["seed"])

    def build():
        return hb.hodlr_build(wl["entry"], p, X, wl["nmin"], wl["tol"], wl["d"], wl["leaf"])

    for _ in range(warmup):
        build().close()
    torch.cuda.synchronize()
    t = time.perf_counter()
    H = None
    for _ in range(steps):
        if H is not None:
            H.close()
        H = build()
    torch.cuda.synchronize()
    b_ms = (time.perf_counter() - t) * 1e3 / steps
    x = torch.tensor(np.random.default_rng(5).standard_normal(N), device="cuda")
    H.matvec(x)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(20):
        y = H.matvec(x)
    torch.cuda.synchronize()
    m_ms = (time.perf_counter() - t) * 1e3 / 20
    rows = torch.arange(0, N, 64, device="cuda")
    d2 = ((X[rows][:, None, :] - X[None, :, :]) ** 2).sum(-1)
    yd = torch.exp(-d2 / (wl["gauss_c"] * wl["h"] ** 2)) @ x
    err = float(torch.linalg.norm(y[rows] - yd) / torch.linalg.norm(yd))
    ranks = [H.blocks.rank(b) for b in range(H.nblocks)]
    out = dict(workload=f"hodlr_curve N={N} Gaussian h={wl['h']} nmin={wl['nmin']} "
                        f"tol={wl['tol']} d={wl['d']} leaf={wl['leaf']}",
               build_ms=b_ms, matvec_ms=m_ms, blocks=H.nblocks, leaves=H.nleaves,
               max_block_rank=max(ranks), matvec_rel_err_rows64=err,
               within_10tol=bool(err <= 10 * wl["tol"]))
    _note(f"hodlr: build {b_ms:.1f} ms, matvec {m_ms:.3f} ms")
    H.close()
    print(json.dumps(out), flush=True)


def _device_workload(hb, wl, **kw):
    """Device points and the parameter dict of a workload."""
    import numpy as np
    import torch
    dev = torch.device("cuda:0")
    X = torch.tensor(wl["X"], device=dev) if wl.get("X") is not None else None
    Y = torch.tensor(wl["Y"], device=dev) if wl.get("Y") is not None else None
    p = hb.params(dim=(wl["X"].shape[1] if wl.get("X") is not None else 0), h=wl.get("h", 0.0),
                  gauss_c=wl.get("gauss_c", 1.0), wavenumber=wl.get("wavenumber", 0.0),
                  seed=wl["seed"], **kw)
    if wl["entry"] == hb.HB_K_LOWRANK_SPIKES:
        p["G1"] = torch.tensor(wl["G1"], device=dev)
        p["G2"] = torch.tensor(wl["G2"], device=dev)
        p["spike_lin"] = torch.tensor(np.asarray(wl["spike_lin"], np.int64), device=dev)
        p["spike_val"] = torch.tensor(np.asarray(wl["spike_val"], np.float64), device=dev)
    return X, Y, p


def sweep(reps=2):
    """Time, rank and error of H-BACA for varying leaf counts n_b = 4^L and
    block sizes d, mirroring the paper's efficiency study (Section
    "Numerical Results", Fig. 5), on the 8-D Gaussian mixture (the Gaussian
    data-set runs), the polynomial kernel (constant-rank regime), a product
    of random factors, and the EFIE2D strips (increasing-rank regime); then,
    per workload, greedy QRCP against the strong rank-revealing selection
    at one (L, d).  Prints one JSON object."""
    import numpy as np
    import torch

    import paper_1901_06101_amd as hb
    from workloads import generators as G

    hb.require_gpu()
    cases = [
        ("gauss_mixture_20000_eps1e-2",
         G.make_gauss_mixture(n=20000, tol=1e-2, d=16, cfg=4), (4, 5, 6), 5),
        ("polynomial_8000_eps1e-4", G.make_polynomial(n=8000, tol=1e-4), (2, 3, 4, 5), 4),
        ("product_of_random_8000_r100",
         G.make_lowrank_spikes(n=8000, rank=100, n_spikes=0, tol=1e-4, cfg=10), (2, 3, 4, 5), 4),
        ("efie2d_4000_eps1e-4", G.make_efie2d_strips(n=4000, tol=1e-4), (1, 2, 3, 4), 3),
    ]

    def timed(wl, X, Y, p, d, leaf):
        def call():
            return hb.compress(wl["entry"], p, X, Y, wl["m"], wl["n"], wl["tol"], d, leaf)
        call().close()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(reps - 1):
            call().close()
        r = call()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t) * 1e3 / reps
        e2, a2 = r.error(0, 7)
        st = r.stats()
        row = dict(ms=ms, rank=r.rank(0), rel_err_rows7=float(np.sqrt(e2 / a2)),
                   swaps=st["select_swaps"], leaf_rank_max=st["leaf_rank_max"],
                   phases_ms={k: st[k] for k in ("ms_baca", "ms_recompress", "ms_merge",
                                                 "ms_svd", "ms_qr", "ms_gemm")})
        r.close()
        return row

    out = {}
    for name, wl, levels, Lsel in cases:
        X, Y, p = _device_workload(hb, wl)
        rows = []
        for L in levels:
            leaf = -(-max(wl["m"], wl["n"]) // (1 << L))
            for d in (1, 8, 16, 32):
                try:
                    rows.append(dict(L=L, n_b=4 ** L, leaf=leaf, d=d,
                                     **timed(wl, X, Y, p, d, leaf)))
                except Exception as e:  # a size the build does not take
                    rows.append(dict(L=L, n_b=4 ** L, leaf=leaf, d=d,
                                     error=f"{type(e).__name__}: {e}"))
        leaf = -(-max(wl["m"], wl["n"]) // (1 << Lsel))
        sel = []
        for f in (None, 2.0, 1.05):
            kw = {} if f is None else dict(selector=hb.HB_SEL_STRONG, select_f=f)
            X, Y, p = _device_workload(hb, wl, **kw)
            sel.append(dict(selector="qrcp" if f is None else "strong", f=f,
                            **timed(wl, X, Y, p, 16, leaf)))
        out[name] = dict(tol=wl["tol"], m=wl["m"], n=wl["n"], rows=rows,
                         selectors=dict(L=Lsel, leaf=leaf, d=16, rows=sel))
        _note(f"sweep: {name} done")
    print(json.dumps(_finite(out)), flush=True)


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


def _traffic(kernel, workload):
    """HBM bytes of one call's launches of a kernel class, measured with
    rocprofv3 --pmc (FETCH_SIZE plus WRITE_SIZE, scaled by the same
    counters' reading for a copy of known size), or None when no measurement
    of this class on this workload was taken with its current kernel source
    and launching code."""
    import hashlib
    rec = PMC_TRAFFIC.get((kernel, workload))
    if rec is None:
        return None
    h = hashlib.sha256()
    try:
        for src in rec["sources"]:
            with open(os.path.join(ROOT, src), "rb") as f:
                h.update(f.read())
    except OSError:
        return None
    sha = h.hexdigest()[:16]
    return rec["bytes_per_call"] if sha == rec["source_sha16"] else None


# rocprofv3 --pmc measurements (profiles/helmholtz_pmc.md): kernel class,
# workload -> HBM bytes of one call (FETCH_SIZE x 1024 x 2.0 + WRITE_SIZE x
# 1024 x 1.0, the factors of a 1 GiB copy) and the sha256 prefix of the
# class's kernel source and of the launching code when they were taken
PMC_TRAFFIC = {
    ("baca_leaf_kernel", "helmholtz"): dict(
        bytes_per_call=4543716896.0,
        sources=("paper_1901_06101_amd/csrc/hb_baca_impl.h", "paper_1901_06101_amd/csrc/hb_api.hip"),
        source_sha16="31bf566d39b4e826"),
    ("svd_kernel", "helmholtz"): dict(
        bytes_per_call=75910304.0,
        sources=("paper_1901_06101_amd/csrc/hb_merge.hip", "paper_1901_06101_amd/csrc/hb_api.hip"),
        source_sha16="c5e0c98aeef6d9b6"),
    ("tsqr_factor/apply + block_gemm", "helmholtz"): dict(
        bytes_per_call=4404459744.0,
        sources=("paper_1901_06101_amd/csrc/hb_merge.hip", "paper_1901_06101_amd/csrc/hb_api.hip"),
        source_sha16="c5e0c98aeef6d9b6"),
}


def rooflines(st, workload):
    """Rates of the three kernel classes of one call from the library's
    counters and HIP-event times; the dominant one by device time first."""
    ms_leaf = st["ms_baca"]
    leaf_bytes = st["resid_bytes"] + st.get("resid_cr_bytes", 0.0)
    out = []
    if ms_leaf > 0:
        a = leaf_bytes / (ms_leaf * 1e-3) / 1e9
        out.append(dict(kernel="baca_leaf_kernel", bound="hbm", achieved=a, peak=HBM_PEAK_GBS,
                        unit="GB/s", frac=a / HBM_PEAK_GBS,
                        traffic=_traffic("baca_leaf_kernel", workload),
                        algorithmic_bytes_per_launch=leaf_bytes, launch_ms=ms_leaf, launches=1))
    ms_svd = st.get("ms_svd", 0.0)
    if ms_svd > 0:
        a = st["svd_flops"] / (ms_svd * 1e-3) / 1e12
        out.append(dict(kernel="svd_kernel", bound="alu", achieved=a, peak=FP64_PEAK_TFLOPS,
                        unit="TFLOP/s", frac=a / FP64_PEAK_TFLOPS,
                        traffic=_traffic("svd_kernel", workload),
                        algorithmic_flops_per_call=st["svd_flops"], launch_ms=ms_svd,
                        launches=st.get("svd_launches")))
    ms_qr = st.get("ms_qr", 0.0) + st.get("ms_gemm", 0.0)
    if ms_qr > 0:
        fl = st["recompress_flops"] + st["merge_flops"]
        a = fl / (ms_qr * 1e-3) / 1e12
        out.append(dict(kernel="tsqr_factor/apply + block_gemm", bound="alu", achieved=a,
                        peak=FP64_PEAK_TFLOPS, unit="TFLOP/s", frac=a / FP64_PEAK_TFLOPS,
                        traffic=_traffic("tsqr_factor/apply + block_gemm", workload),
                        algorithmic_flops_per_call=fl, launch_ms=ms_qr,
                        launches=st.get("qr_launches")))
    out.sort(key=lambda r: -r["launch_ms"])
    return out


def headline(args, wl):
    """The timed compress calls on the headline workload: the measured
    fields of the line."""
    import numpy as np
    import torch

    import paper_1901_06101_amd as hb

    hb.require_gpu()
    # the library's TSQR autotuner (untimed): picks the lane layout of each
    # thin-QR width from measured times before the headline calls
    tune = hb.autotune() if hasattr(hb, "autotune") else None
    X, Y, p = _device_workload(hb, wl)
    tol = wl["tol"]

    def step(eps):
        return hb.compress(wl["entry"], p, X, Y, wl["m"], wl["n"], eps, wl["d"], wl["leaf"])

    def rel_err(res):
        e2, a2 = res.error(0, 7)
        return float(np.sqrt(e2 / a2))

    # the truncation tolerance that reaches rel. error <= tol (untimed)
    tried = []
    eps = tol
    for f in EPS_DIVISORS:
        eps = tol / f
        r = step(eps)
        e = rel_err(r)
        tried.append(dict(eps=eps, rel_err_rows7=e, rank=r.rank(0)))
        r.close()
        if e <= tol:
            break
    _note(f"{wl['name']} {wl['m']}x{wl['n']}: eps {eps:g} (tol {tol:g}); warm-up")
    for _ in range(args.warmup):
        step(eps).close()
    torch.cuda.synchronize()
    _note(f"{wl['name']}: {args.steps} timed steps")
    stats = []
    last = None
    t0 = time.perf_counter()
    for _ in range(args.steps):
        if last is not None:
            last.close()
        last = step(eps)
        stats.append(last.stats())
    torch.cuda.synchronize()
    wall_ms = (time.perf_counter() - t0) * 1e3 / args.steps
    rel = rel_err(last)
    rank = last.rank(0)
    keys = set(stats[-1])
    mean = {k: float(np.mean([s[k] for s in stats])) for k in keys
            if isinstance(stats[-1][k], (int, float))}
    rf = rooflines(mean, wl["name"])
    copy = copy_bandwidth(torch)
    for r in rf:
        if r["unit"] == "GB/s":
            r["copy_GBps_measured"] = copy
            r["frac_of_copy"] = r["achieved"] / copy if copy else None
    phases = {k: mean[k] for k in ("ms_setup", "ms_baca", "ms_recompress", "ms_merge", "ms_total",
                                   "ms_svd", "ms_qr", "ms_gemm") if k in mean}
    out = {
        "value": wall_ms,
        "ms_per_step": wall_ms,
        "eps": eps,
        "eps_search": tried,
        "rank": rank,
        "rel_err_rows7": rel,
        "within_tol": bool(rel <= tol),
        "phases_ms": phases,
        "roofline": rf[0] if rf else None,
        "kernel_classes": rf,
        "autotune_tsqr_layouts": tune["table"] if tune else None,
    }
    last.close()
    _note(f"{wl['name']}: {wall_ms:.2f} ms per compress (eps {eps:g}, rel. error {rel:.2e})")
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
    ap.add_argument("--no-hodlr", action="store_true")
    ap.add_argument("--no-sweep", action="store_true")
    ap.add_argument("--sweep", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--comparisons", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--adjoint", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--hodlr", action="store_true", help=argparse.SUPPRESS)
    args = ap.parse_args()
    if args.comparisons:
        comparisons()
        return
    if args.adjoint:
        adjoint()
        return
    if args.hodlr:
        hodlr()
        return
    if args.sweep:
        sweep()
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
                   "comparisons": "mixed precision vs plain FP64 and batched vs one call per "
                                  "block, in the 'comparisons' object",
                   "parallelism": "single GPU"},
    }
    # the legs beside the headline, each in a child process with a time limit,
    # before this process touches the GPU: the runtime has refused cooperative
    # launches to one process while another on the device had made some
    legs = {}
    if not args.no_comparisons:
        legs["comparisons"] = run_child("--comparisons")
    if not args.no_adjoint:
        legs["adjoint"] = run_child("--adjoint")
    if not args.no_hodlr:
        legs["hodlr"] = run_child("--hodlr")
    if not args.no_sweep:
        legs["sweep"] = run_child("--sweep")
    try:
        out.update(headline(args, wl))
    except Exception as e:  # the line is still printed, with the failure
        out["error"] = f"{type(e).__name__}: {e}"
        _note(f"headline failed: {out['error']}")
    if not args.no_cpu_baseline:
        _note("CPU baseline (the oracle on the same workload)")
        try:
            out["cpu_baseline"] = cpu_baseline(wl, eps=out.get("eps"))
        except Exception as e:  # the GPU line is still reported
            out["cpu_baseline"] = {"value": None, "unit": "ms", "cores": None, "kind": "oracle",
                                   "sample": f"failed: {type(e).__name__}: {e}"}
    out.update(legs)
    print(json.dumps(_finite(out)), flush=True)


if __name__ == "__main__":
    main()
