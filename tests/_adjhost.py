"""Host emulation of the adjoint's workgroup tasks (tests/adjoint_host).

Builds adj_host.cpp with g++ and feeds it a frozen structure in the record
format the leaf kernel writes (nI, nJ, d_k, I_k, J_k, pivot order), taken
here from the oracle's forward run."""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "adjoint_host", "adj_host.cpp")
OUT = os.path.join(HERE, "adjoint_host", "_build")

_libs = {}

# the build in which every Jacobi SVD shares its pairs over several lanes
# (the library does so from 64 columns on)
SPLIT_ALL = ("-DADJ_JACOBI_SPLIT_K=2",)


def build(extra=(), name="adj_host"):
    os.makedirs(OUT, exist_ok=True)
    so = os.path.join(OUT, name + ".so")
    cmd = ["g++", "-std=c++20", "-O2", "-pthread", "-shared", "-fPIC", *extra, SRC, "-o", so]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    return so


def load(extra=()):
    """The host build; `extra` are compile flags (SPLIT_ALL)."""
    key = tuple(extra)
    if key not in _libs:
        name = "adj_host" + ("_split_all" if key else "")
        lib = C.CDLL(build(key, name))
        p = C.c_void_p
        lib.adj_host_vjp.argtypes = [C.c_int64, C.c_int64, C.c_int, C.c_int, C.c_int, C.c_int,
                                     p, p, p, p, p, C.c_double, C.c_double, p, p, p, p, p, p,
                                     C.c_int, C.POINTER(C.c_int64)]
        lib.adj_host_vjp.restype = C.c_int
        lib.adj_host_forward.argtypes = [C.c_int64, C.c_int64, C.c_int, C.c_int, C.c_int, C.c_int,
                                         p, p, p, p, p, C.c_double, C.c_double, C.c_int, C.c_int,
                                         p, p, p, C.POINTER(C.c_int32)]
        lib.adj_host_forward.restype = C.c_int
        lib.adj_host_set_chunking.argtypes = [C.c_int64, C.c_int]
        lib.adj_host_set_chunking.restype = None
        lib.adj_host_last_split.argtypes = [C.POINTER(C.c_int), C.POINTER(C.c_int)]
        lib.adj_host_last_split.restype = None
        lib.adj_host_set_fibers.argtypes = [C.c_int, C.POINTER(C.c_int64)]
        lib.adj_host_set_fibers.restype = C.c_int
        lib.adj_host_fiber_profile.argtypes = [p, p, p]
        lib.adj_host_fiber_profile.restype = None
        _libs[key] = lib
    return _libs[key]


def fiber_profile(extra=()):
    """{task kind: (critical path ns, barriers on it, launches)} of the fiber
    runs since the last call."""
    ns = np.zeros(32)
    bar = np.zeros(32, dtype=np.int64)
    nl = np.zeros(32, dtype=np.int64)
    load(extra).adj_host_fiber_profile(ns.ctypes.data_as(C.c_void_p), bar.ctypes.data_as(C.c_void_p),
                                  nl.ctypes.data_as(C.c_void_p))
    return {k: (float(ns[k]), int(bar[k]), int(nl[k])) for k in range(32) if nl[k]}


def set_fibers(on, extra=()):
    """Lanes as fibers on one thread (on) or as threads; returns (diverged,
    barriers) for the calls since the last switch."""
    b = C.c_int64(0)
    e = load(extra).adj_host_set_fibers(1 if on else 0, C.byref(b))
    return bool(e), b.value


def set_chunking(chunk_rows=512, max_chunks=32, extra=()):
    """Row chunking of tall merges for later calls (512 and 32 are the
    library's defaults)."""
    load(extra).adj_host_set_chunking(int(chunk_rows), int(max_chunks))


def last_split(extra=()):
    """(merges split over row chunks, chunks) in the last plan."""
    a, b = C.c_int(0), C.c_int(0)
    load(extra).adj_host_last_split(C.byref(a), C.byref(b))
    return a.value, b.value


def dmax_for(d):
    return 8 if d <= 8 else (16 if d <= 16 else 32)


def records_from_oracle(fs):
    """(leaf_info int64 [nleaves, 7], records int32, ranks int32, dmax, stride)."""
    wl, res = fs.wl, fs.res
    dm = dmax_for(wl["d"])
    stride = 3 + 3 * dm
    nb = 1 << fs.L
    info, recs = [], []
    for b in range(nb * nb):
        li = res.leaf_info[b]
        first = len(recs)
        for it in li["iters"]:
            I = np.asarray(it["Iblock"], dtype=np.int64)
            J = np.asarray(it["Jblock"], dtype=np.int64)
            dk = int(it["dk"])
            piv = np.asarray(it["piv"], dtype=np.int64)[:dk]
            r = np.zeros(stride, dtype=np.int32)
            r[0], r[1], r[2] = I.size, J.size, dk
            r[3:3 + I.size] = I
            r[3 + dm:3 + dm + J.size] = J
            r[3 + 2 * dm:3 + 2 * dm + dk] = piv
            recs.append(r)
            if dk == 0:
                break
        info.append([li["row0"], li["col0"], li["m0"], li["n0"], len(recs) - first, li["rank"],
                     first])
    ranks = []
    for lev in range(1, fs.L + 1):
        nbl = 1 << (fs.L - lev)
        h = fs.res.ranks[lev - 0.5]  # order (t, v, i): block (2t + i, v)
        hp = np.zeros(2 * nbl * nbl, dtype=np.int32)
        for t in range(nbl):
            for v in range(nbl):
                for i in range(2):
                    hp[(2 * t + i) * nbl + v] = h[(t * nbl + v) * 2 + i]
        ranks.extend(hp.tolist())
        ranks.extend(fs.res.ranks[lev])
    recs = np.concatenate(recs) if recs else np.zeros(stride, dtype=np.int32)
    return (np.asarray(info, dtype=np.int64), recs.astype(np.int32),
            np.asarray(ranks, dtype=np.int32), dm, stride)


def vjp(fs, w, ybar, nt=8, info=None, want=("w", "h", "x", "y"), extra=()):
    """(gw, gh, gX, gY) of <ybar, A~ w> through the host emulation; None
    (a null output pointer) for what is not in `want`."""
    lib = load(extra)
    wl = fs.wl
    li, recs, ranks, dm, stride = info or records_from_oracle(fs)
    X = np.ascontiguousarray(np.asarray(wl["X"], dtype=np.float64).T)
    Y = np.ascontiguousarray(np.asarray(wl["Y"], dtype=np.float64).T)
    m, n, dim = wl["m"], wl["n"], X.shape[0]
    w = np.ascontiguousarray(w, dtype=np.float64)
    ybar = np.ascontiguousarray(ybar, dtype=np.float64)
    gw = np.zeros(n)
    gh = np.zeros(1)
    gX = np.zeros((m, dim))
    gY = np.zeros((n, dim))
    arena = C.c_int64(0)
    ptr = lambda a: None if a is None else a.ctypes.data_as(C.c_void_p)  # noqa: E731
    gw = gw if "w" in want else None
    gh = gh if "h" in want else None
    gX = gX if "x" in want else None
    gY = gY if "y" in want else None
    st = lib.adj_host_vjp(m, n, fs.L, dim, dm, stride, ptr(li), ptr(recs), ptr(ranks), ptr(X),
                          ptr(Y), float(wl["h"]), float(wl.get("gauss_c", 1.0)), ptr(w),
                          ptr(ybar), ptr(gw), ptr(gh), ptr(gX), ptr(gY), nt, C.byref(arena))
    if st != 0:
        raise RuntimeError(f"adj_host_vjp status {st}")
    return gw, (None if gh is None else float(gh[0])), gX, gY


def forward(fs, X=None, Y=None, h=None, nt=1, extra=()):
    """(U, S, Vt) of the frozen operator at points X, Y (point-major) and
    width h; the recorded ones by default."""
    lib = load(extra)
    wl = fs.wl
    li, recs, ranks, dm, stride = records_from_oracle(fs)
    X = np.ascontiguousarray(np.asarray(wl["X"] if X is None else X, dtype=np.float64).T)
    Y = np.ascontiguousarray(np.asarray(wl["Y"] if Y is None else Y, dtype=np.float64).T)
    h = float(wl["h"] if h is None else h)
    m, n = wl["m"], wl["n"]
    cap = int(max(1, min(m, n)))
    U = np.zeros((cap, m))
    Vt = np.zeros((cap, n))
    S = np.zeros(cap)
    rk = C.c_int32(0)
    ptr = lambda a: a.ctypes.data_as(C.c_void_p)  # noqa: E731
    st = lib.adj_host_forward(m, n, fs.L, X.shape[0], dm, stride, ptr(li), ptr(recs), ptr(ranks),
                              ptr(X), ptr(Y), h, float(wl.get("gauss_c", 1.0)), nt, cap, ptr(U),
                              ptr(S), ptr(Vt), C.byref(rk))
    if st != 0:
        raise RuntimeError(f"adj_host_forward status {st}")
    r = rk.value
    return U[:r].T.copy(), S[:r].copy(), Vt[:r].T.copy()


def build_tsan(extra=()):
    """The stand-alone driver built with ThreadSanitizer."""
    return _build_exe("adj_host_tsan" + ("_split_all" if extra else ""),
                      ["-fsanitize=thread", *extra])


def build_asan(extra=()):
    """The stand-alone driver built with AddressSanitizer and
    UndefinedBehaviorSanitizer (host code only)."""
    return _build_exe("adj_host_asan" + ("_split_all" if extra else ""),
                      ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                       "-fno-omit-frame-pointer", *extra])


_exes = {}


def _build_exe(name, flags):
    """Builds the stand-alone driver once per process and flag set."""
    if name not in _exes:
        os.makedirs(OUT, exist_ok=True)
        exe = os.path.join(OUT, name)
        cmd = ["g++", "-std=c++20", "-O1", "-g", *flags, "-pthread", "-DADJ_HOST_MAIN", SRC,
               "-o", exe]
        subprocess.run(cmd, check=True, capture_output=True, text=True)
        _exes[name] = exe
    return _exes[name]


def run_exe(exe, fs, w, ybar, nt, workdir, chunking=None):
    """Runs the stand-alone driver; returns (returncode, stderr, outputs or None)."""
    wl = fs.wl
    li, recs, ranks, dm, stride = records_from_oracle(fs)
    X = np.ascontiguousarray(np.asarray(wl["X"], dtype=np.float64).T)
    Y = np.ascontiguousarray(np.asarray(wl["Y"], dtype=np.float64).T)
    m, n, dim = wl["m"], wl["n"], X.shape[0]
    inp = os.path.join(workdir, "adj_in.bin")
    out = os.path.join(workdir, "adj_out.bin")
    with open(inp, "wb") as f:
        np.asarray([m, n, fs.L, dim, dm, stride, li.shape[0], recs.size, ranks.size],
                   dtype=np.int64).tofile(f)
        li.astype(np.int64).tofile(f)
        recs.astype(np.int32).tofile(f)
        ranks.astype(np.int32).tofile(f)
        X.tofile(f)
        Y.tofile(f)
        np.asarray([wl["h"], wl.get("gauss_c", 1.0)], dtype=np.float64).tofile(f)
        np.asarray(w, dtype=np.float64).tofile(f)
        np.asarray(ybar, dtype=np.float64).tofile(f)
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1 exitcode=66",
               ASAN_OPTIONS="detect_leaks=1 exitcode=67")
    extra = [str(chunking[0]), str(chunking[1])] if chunking else []
    p = subprocess.run([exe, inp, out, str(nt), *extra], capture_output=True, text=True,
                       env=env, timeout=900)
    if p.returncode != 0:
        return p.returncode, p.stderr, None
    v = np.fromfile(out, dtype=np.float64)
    gw, gh = v[:n], v[n]
    gX = v[n + 1:n + 1 + m * dim].reshape(m, dim)
    gY = v[n + 1 + m * dim:].reshape(n, dim)
    return 0, p.stderr, (gw, gh, gX, gY)
