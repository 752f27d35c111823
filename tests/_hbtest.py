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


def run_oracle(wl, keep_leaf_factors=False):
    src = oracle.EntrySource(wl)
    return src, oracle.hbaca(src, wl["m"], wl["n"], wl["tol"], wl["d"], wl["leaf"], wl["seed"],
                             keep_leaf_factors=keep_leaf_factors)


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


NOISE = 1e-12
PICK_NOISE = 1e-11
QRCP_ZERO = 1e-13
NORM_RTOL = 1e-9


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


def compare_tape(gtape, ginfo, oinfo):
    """Compare one leaf's GPU pivot tape with the oracle's iterations.

    Iterations are compared in order while their pivots are unique: d_k,
    I_k(1:d_k) and J_k(Jbar) must then be equal.  Comparison stops at the
    first iteration whose row picks, or the column picks that produced its
    block J_k, were made among rounding-level trailing norms (an exactly
    low-rank residual), and a terminating iteration with nu < 1e-12 mu is
    never compared: in both cases several choices are equally valid.  On
    the compared iterations nu and mu must agree to NORM_RTOL as well.
    Returns None or a text describing the first difference."""
    its = oinfo["iters"]
    gdk = list(int(x) for x in gtape["dk"])
    odk = [it["dk"] for it in its]
    nk = 0
    for k, it in enumerate(its):
        if not _determined(it["sel_I"]):
            break
        if k > 0 and not _determined(its[k - 1]["sel_J"]):
            break
        if it["dk"] > 0 and it["nu"] < NOISE * max(it["mu"], 1e-300) and k == len(its) - 1:
            break
        nk += 1
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
    # sides form nu from Cholesky factors of Gram blocks, so they agree to
    # rounding amplified by the Gram blocks' conditioning
    gnu, gmu = np.asarray(gtape["nu"]), np.asarray(gtape["mu"])
    for k in range(nk):
        onu, omu = its[k]["nu"], its[k]["mu"]
        if abs(gmu[k] - omu) > NORM_RTOL * omu:
            return f"iteration {k}: mu gpu {gmu[k]:.17e} oracle {omu:.17e}"
        if abs(gnu[k] - onu) > NORM_RTOL * onu + 1e-13 * omu:
            return f"iteration {k}: nu gpu {gnu[k]:.17e} oracle {onu:.17e}"
    return None


def check_mixed(lib, case, wl):
    """Mixed precision against the FP64 oracle on the same inputs: operator
    difference and error against A within 5 tol, ranks close."""
    tol = wl["tol"]
    say(f"[mixed] {case}: m={wl['m']} n={wl['n']} d={wl['d']} leaf={wl['leaf']} tol={tol}")
    res = run_gpu(lib, wl, precision=lib.HB_PREC_MIXED)
    src, ores = run_oracle(wl)
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
