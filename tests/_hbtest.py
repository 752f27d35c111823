"""Shared helpers of the GPU parity tests: run the HIP path through the C ABI
and the CPU oracle on the same seeded inputs and compare them."""
from __future__ import annotations

import sys

import numpy as np

import oracle


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def device_inputs(wl):
    import torch
    dev = torch.device("cuda")
    X = torch.tensor(wl["X"], device=dev) if wl.get("X") is not None else None
    Y = torch.tensor(wl["Y"], device=dev) if wl.get("Y") is not None else None
    return X, Y


def gpu_params(hb, wl, **kw):
    import torch
    dim = wl["X"].shape[1] if wl.get("X") is not None else 0
    p = hb.params(dim=dim, h=wl.get("h", 0.0), gauss_c=wl.get("gauss_c", 1.0),
                  wavenumber=wl.get("wavenumber", 0.0), seed=wl["seed"], **kw)
    if wl["entry"] == 4:
        dev = torch.device("cuda")
        p["G1"] = torch.tensor(wl["G1"], device=dev)
        p["G2"] = torch.tensor(wl["G2"], device=dev)
        p["spike_lin"] = torch.tensor(np.asarray(wl["spike_lin"], np.int64), device=dev)
        p["spike_val"] = torch.tensor(np.asarray(wl["spike_val"], np.float64), device=dev)
    return p


def run_gpu(hb, wl, **kw):
    X, Y = device_inputs(wl)
    p = gpu_params(hb, wl, **kw)
    return hb.compress(wl["entry"], p, X, Y, wl["m"], wl["n"], wl["tol"], wl["d"], wl["leaf"])


def run_oracle(wl, keep_leaf_factors=False, selector=0, select_f=2.0):
    src = oracle.EntrySource(wl)
    return src, oracle.hbaca(src, wl["m"], wl["n"], wl["tol"], wl["d"], wl["leaf"], wl["seed"],
                             keep_leaf_factors=keep_leaf_factors, selector=selector,
                             select_f=select_f)


def factors_np(res, block=0):
    U, S, Vh = res.factors(block)
    return U.cpu().numpy(), S.cpu().numpy(), Vh.cpu().numpy()


def lowrank_diff(X1, Y1, X2, Y2):
    """||X1 Y1^H - X2 Y2^H||_F without forming the products (QR of the
    stacked factors, then the small core)."""
    Xs = np.hstack([X1, -X2])
    Ys = np.hstack([Y1, Y2])
    if Xs.shape[1] == 0:
        return 0.0
    _, R1 = np.linalg.qr(Xs)
    _, R2 = np.linalg.qr(Ys)
    return float(np.linalg.norm(R1 @ R2.conj().T))


def recon_norm(X, Y):
    if X.shape[1] == 0:
        return 0.0
    _, R1 = np.linalg.qr(X)
    _, R2 = np.linalg.qr(Y)
    return float(np.linalg.norm(R1 @ R2.conj().T))


PICK_NOISE = 1e-11
QRCP_ZERO = 1e-13
NU_DECIDED = 1e-7
PICK_FLOOR = 1e-11
MU_RTOL = 1e-9
NU_RTOL = 1e-6
SWAP_DECIDED = 1e-6
SWAP_FLIP = 1e-15


def _determined(norms):
    """A QRCP pick is unique while its trailing norm is well above the
    rounding level of its panel, or so far below it that both sides count
    every remaining norm as zero and pick the lowest index (the reading of
    rounding-level norms, QRCP_ZERO below the first pick).  Picks in the band
    between may differ."""
    norms = np.asarray(norms)
    if norms.size == 0 or not norms.max() > 0.0:
        return True
    rel = norms / norms.max()
    return not np.any((rel > QRCP_ZERO) & (rel <= PICK_NOISE))


def determined_iterations(oinfo):
    """How many leading iterations of the oracle's leaf are decided by the
    data rather than by rounding.  The comparison stops at the first
    iteration whose row picks, or the column picks that produced its block
    J_k, were made in the band of trailing norms that rounding can reorder
    (see _determined), or whose new block has nu < NU_DECIDED * mu: its
    residual panels are differences of entries some 1 / NU_DECIDED times
    larger, so their rounding (about 1e-16 mu) reaches 1e-9 of the panel and
    picks closer than that are a tie; likewise an iteration with a pick
    (among the rows I_k(1:d_k), or the columns that made J_k) whose trailing
    norm is below PICK_FLOOR * mu: rounding of order 1e-16 mu then moves
    that norm by 1e-5 of itself or more, enough to reorder close rows or
    columns (neighbouring nodes on the EFIE2D strips).  With the strong
    rank-revealing selector the comparison also stops at an iteration whose
    row selection, or the column selection that made J_k, took a swap
    decision within SWAP_DECIDED (relative) of the threshold f or of the
    runner-up coefficient, or one that a change of the panel's entries by
    less than SWAP_FLIP * mu could reverse (the oracle's flip estimate:
    the margin times the smallest singular value of the chosen columns):
    the residual panels carry rounding of about 1e-16 mu, and graded panels
    (the EFIE2D strips) have chosen columns with singular values far below
    mu.  An iteration with d_k = 0 ends the leaf and is counted like the
    others."""
    its = oinfo["iters"]
    nk = 0
    for k, it in enumerate(its):
        if not _determined(it["sel_I"]):
            break
        if k > 0 and not _determined(its[k - 1]["sel_J"]):
            break
        mu_k = max(it["mu"], its[k - 1]["mu"] if k else 0.0)
        if it.get("margin_I", np.inf) < SWAP_DECIDED or \
                it.get("flip_I", np.inf) < SWAP_FLIP * mu_k:
            break
        if k > 0 and (its[k - 1].get("margin_J", np.inf) < SWAP_DECIDED or
                      its[k - 1].get("flip_J", np.inf) < SWAP_FLIP * mu_k):
            break
        if it["dk"] > 0 and it["nu"] < NU_DECIDED * max(it["mu"], 1e-300):
            break
        # a trailing norm this close to the rounding of the matrix scale
        # (mu) decides nothing: two close rows or columns may trade places
        floor = PICK_FLOOR * max(it["mu"], its[k - 1]["mu"] if k else 0.0)
        sel = np.asarray(it["sel_I"])[:max(it["dk"], 1)]
        if sel.size and np.any((sel > QRCP_ZERO * sel.max()) & (sel < floor)):
            break
        if k > 0:
            sj = np.asarray(its[k - 1]["sel_J"])
            if sj.size and np.any((sj > QRCP_ZERO * sj.max()) & (sj < floor)):
                break
        nk += 1
    return nk


def divergence_nu(gtape, oinfo):
    """Sum of the oracle's nu over the iterations from the first one where
    the GPU's tape (d_k, I_k(1:d_k), J_k(Jbar)) differs from the oracle's; 0
    when the tapes agree.  compare_tape has checked that a difference comes
    only after the iterations the data decides.  Two valid runs that part at
    iteration k differ in that leaf by at most about twice this, before the
    re-compression and the merges (which do not enlarge a perturbation)."""
    its = oinfo["iters"]
    gdk = [int(x) for x in gtape["dk"]]
    r = 0
    for k, it in enumerate(its):
        dk = it["dk"]
        if k >= len(gdk) or gdk[k] != dk:
            break
        if not (np.array_equal(gtape["rows"][r:r + dk], it["I"])
                and np.array_equal(gtape["cols"][r:r + dk], it["J"])):
            break
        r += dk
    else:
        return 0.0 if len(gdk) == len(its) else float(its[-1]["nu"])
    return float(sum(x["nu"] for x in its[k:]))


def rounding_sensitivity(wl, **kw):
    """How far the oracle's own H-BACA result moves when its input points
    are perturbed at the rounding level (relative 2^-52, seeded): the
    reconstruction difference of the two oracle runs.  Two correct FP64 runs
    that round differently cannot be expected to agree more closely than a
    few times this; graded problems (the EFIE2D strips with large leaves)
    amplify rounding through the truncations well past 1e-10."""
    _, a = run_oracle(wl, **kw)
    w2 = dict(wl)
    rng = np.random.default_rng(12345)
    w2["X"] = wl["X"] * (1.0 + 2.0 ** -52 * rng.standard_normal(wl["X"].shape))
    _, b = run_oracle(w2, **kw)
    return lowrank_diff(a.U * a.S, a.V.conj().T, b.U * b.S, b.V.conj().T)


def parity_bar(ref_norm, diverged_nu=0.0):
    """The FP64 reconstruction bar: 1e-10 of the operator's norm, plus twice
    the nu of the leaf iterations where the two runs parted (sum of
    divergence_nu over the leaves)."""
    return 1e-10 * ref_norm + 2.0 * diverged_nu


def compare_tape(gtape, ginfo, oinfo):
    """Compare one leaf's GPU pivot tape with the oracle's iterations.

    Iterations are compared in order while the data decides their pivots
    (determined_iterations): d_k, I_k(1:d_k) and J_k(Jbar) must then be
    equal, and nu and mu agree to NU_RTOL and MU_RTOL.  Later iterations
    may legitimately differ; parity_bar accounts for them.
    Returns None or a text describing the first difference."""
    its = oinfo["iters"]
    gdk = list(int(x) for x in gtape["dk"])
    odk = [it["dk"] for it in its]
    nk = determined_iterations(oinfo)
    if gdk[:nk] != odk[:nk]:
        return f"d_k differ: gpu {gdk} oracle {odk}"
    r = int(sum(odk[:nk]))
    orows = np.concatenate([it["I"] for it in its[:nk]]) if nk else np.zeros(0, np.int64)
    ocols = np.concatenate([it["J"] for it in its[:nk]]) if nk else np.zeros(0, np.int64)
    if not np.array_equal(gtape["rows"][:r], orows):
        return "row pivots differ"
    if not np.array_equal(gtape["cols"][:r], ocols):
        return "column pivots differ"
    if nk == len(odk) and (len(gdk) != len(odk) or ginfo["rank_baca"] != oinfo["rank_baca"]):
        return f"iteration count differs: gpu {gdk} oracle {odk}"
    # the norm estimates of eqs. (11)-(13) on the compared iterations: both
    # sides form nu from Cholesky factors of Gram blocks of U_k and V_k, so
    # they agree to rounding amplified by the squared conditioning of those
    # blocks (V_k = T11^-1 Q1^H R_k inherits that of T11); mu is dominated by
    # the first, well-conditioned blocks
    gnu, gmu = np.asarray(gtape["nu"]), np.asarray(gtape["mu"])
    for k in range(nk):
        onu, omu = its[k]["nu"], its[k]["mu"]
        if abs(gmu[k] - omu) > MU_RTOL * omu:
            return f"iteration {k}: mu gpu {gmu[k]:.17e} oracle {omu:.17e}"
        if abs(gnu[k] - onu) > NU_RTOL * onu + 1e-13 * omu:
            return f"iteration {k}: nu gpu {gnu[k]:.17e} oracle {onu:.17e}"
    return None


def check_mixed(lib, case, wl, selector=0, select_f=2.0):
    """Mixed precision against the FP64 oracle on the same inputs: operator
    difference and error against A within 5 tol, ranks close."""
    tol = wl["tol"]
    say(f"[mixed] {case}: m={wl['m']} n={wl['n']} d={wl['d']} leaf={wl['leaf']} tol={tol}")
    res = run_gpu(lib, wl, precision=lib.HB_PREC_MIXED, selector=selector, select_f=select_f)
    src, ores = run_oracle(wl, selector=selector, select_f=select_f)
    U, S, Vh = factors_np(res)
    assert U.dtype == np.float64 and Vh.dtype == np.float64
    ref = recon_norm(ores.U * ores.S, ores.V.conj().T)
    diff = lowrank_diff(U * S, Vh, ores.U * ores.S, ores.V.conj().T)
    A = src.dense()
    nA = np.linalg.norm(A)
    eg = np.linalg.norm(A - (U * S) @ Vh.T) / nA
    eo = np.linalg.norm(A - ores.dense()) / nA
    say(f"  rank mixed {S.size} oracle {ores.rank}; operator difference {diff / ref:.2e}; "
        f"error mixed {eg:.2e} oracle {eo:.2e}")
    assert diff <= 5 * tol * ref
    assert eg <= eo + 5 * tol
    assert abs(S.size - ores.rank) <= max(3, ores.rank // 10)
    # the device error check sees the same error
    e2, a2 = res.error(0, 1)
    assert abs(np.sqrt(e2 / a2) - eg) <= 1e-6 * eg + 1e-12
