"""The C-ABI library on a machine without a GPU: it loads, exports every
symbol include/hbaca.h declares, and rejects invalid arguments before any
HIP call."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1901_06101_amd", "libhbaca.so")

pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libhbaca.so not built")


def _declared():
    text = open(os.path.join(ROOT, "include", "hbaca.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hb\w+)\s*\(", text)))


def test_exports_every_declared_symbol():
    from paper_1901_06101_amd import _binding
    lib = _binding.load(LIB)
    names = _declared()
    assert "hbaca_compress" in names and "hb_result_free" in names
    missing = [n for n in names if not hasattr(lib, n)]
    assert missing == []
    assert set(names) == set(_binding.EXPORTED)


def test_status_strings():
    from paper_1901_06101_amd import _binding
    lib = _binding.load(LIB)
    for st in range(-6, 1):
        assert lib.hb_status_string(st).decode()
    assert lib.hb_status_string(-99).decode() == "unknown status"


def _call(precision=0, record_tape=0, **over):
    from paper_1901_06101_amd import _binding
    lib = _binding.load(LIB)
    p = _binding.HbParams()
    p.dim, p.h, p.gauss_c, p.wavenumber = 3, 0.5, 1.0, 20.0
    p.precision = precision
    p.record_tape = record_tape
    args = dict(entry=1, params=C.byref(p), X=C.c_void_p(16), Y=C.c_void_p(16), m=100, n=100,
                tol=1e-6, d=8, leaf=50)
    args.update(over)
    out = C.c_void_p(1234)
    st = lib.hbaca_compress(args["entry"], args["params"], args["X"], args["Y"], args["m"],
                            args["n"], args["tol"], args["d"], args["leaf"], None, C.byref(out))
    return st, out


@pytest.mark.parametrize("over,expect", [
    (dict(tol=0.0), -1), (dict(tol=1.0), -1), (dict(tol=float("nan")), -5),
    (dict(d=0), -1), (dict(d=33), -6), (dict(leaf=0), -1), (dict(m=0), -1),
    (dict(entry=9), -1), (dict(X=None), -1), (dict(params=None), -1),
])
def test_invalid_arguments_rejected_on_host(over, expect):
    st, out = _call(**over)
    assert st == expect
    assert out.value is None


@pytest.mark.parametrize("precision,entry,expect", [(2, 1, -1), (-1, 1, -1), (1, 3, -6)])
def test_precision_modes_checked_on_host(precision, entry, expect):
    """Only FP64 and mixed precision exist; mixed precision is for real
    kernels only."""
    st, out = _call(precision=precision, entry=entry)
    assert st == expect
    assert out.value is None


@pytest.mark.parametrize("record_tape,expect", [(3, -1), (-1, -1)])
def test_record_modes_checked_on_host(record_tape, expect):
    """0 (nothing), 1 (pivot tapes) and 2 (also the frozen structure of the
    adjoint) are the only recording modes."""
    st, out = _call(record_tape=record_tape)
    assert st == expect
    assert out.value is None


def test_result_accessors_reject_null():
    from paper_1901_06101_amd import _binding
    lib = _binding.load(LIB)
    assert lib.hb_result_rank(None, 0) == -1
    assert lib.hb_result_nblocks(None) == -1
    assert lib.hb_result_copy(None, 0, None, None, None, None) == -1
    assert lib.hbaca_apply(None, 0, None, None, 0, None) == -1
    assert lib.hbaca_vjp(None, None, None, None, None, None, None, None) == -1
    assert lib.hbaca_adjoint(None, None, None, None, None, None, None, None) == -1
    out = C.c_void_p(1234)
    assert lib.hbaca_recompute_frozen(None, None, None, None, None, C.byref(out)) == -1
    stride = C.c_int32(0)
    count = C.c_int64(0)
    assert lib.hb_result_leaf_frozen(None, 0, C.byref(stride), None) == -1
    assert lib.hb_result_merge_ranks(None, None, C.byref(count)) == -1
    assert out.value is None
    lib.hb_result_free(None)


def test_struct_layouts_match_the_header(tmp_path):
    """The binding's ctypes structures have the header's sizes and field
    offsets (compiled with the host C compiler)."""
    import shutil
    import subprocess
    from paper_1901_06101_amd import _binding
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "hbaca.h"', "int main(void) {"]
    for cname, cls in (("hb_params", _binding.HbParams), ("hb_stats", _binding.HbStats)):
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in cls._fields_:
            lines.append(f'printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run([cc, "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True,
                   capture_output=True, text=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(line.split()[:2]): int(line.split()[2]) for line in out if line.strip()}
    for cname, cls in (("hb_params", _binding.HbParams), ("hb_stats", _binding.HbStats)):
        assert got[(cname, "size")] == C.sizeof(cls), cname
        for f, _ in cls._fields_:
            assert got[(cname, f)] == getattr(cls, f).offset, (cname, f)
