"""The EFIE2D kernel's Bessel functions (csrc/hb_bessel.h: Miller's backward
recurrence with Neumann's series below 25, Hankel's asymptotic expansion
above) built for the host and compared with SciPy's independent routines
(Cephes j0/y0 and AMOS hankel2) over the arguments the EFIE2D workloads
reach: H_0^(2) = J_0 - i Y_0 to 1e-14 of its modulus, on both sides of the
switch between the two methods and at the zeros of J_0 and Y_0."""
import ctypes as C
import os
import subprocess

import numpy as np
import pytest
import scipy.special as sp

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "bessel_host")


@pytest.fixture(scope="module")
def j0y0():
    out = os.path.join(HERE, "_build")
    os.makedirs(out, exist_ok=True)
    lib = os.path.join(out, "libbessel_host.so")
    subprocess.run(["g++", "-O2", "-shared", "-fPIC", "-o", lib,
                    os.path.join(HERE, "bessel_host.cpp")], check=True)
    L = C.CDLL(lib)
    L.hb_host_j0y0.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_long]

    def f(x):
        x = np.ascontiguousarray(x, dtype=np.float64)
        j = np.empty_like(x)
        y = np.empty_like(x)
        L.hb_host_j0y0(x.ctypes.data, j.ctypes.data, y.ctypes.data, x.size)
        return j, y
    return f


def test_hankel2_against_scipy(j0y0):
    x = np.concatenate([np.geomspace(1e-8, 1.0, 400), np.linspace(1.0, 60.0, 20001),
                        np.linspace(24.9, 25.1, 2001), np.geomspace(60.0, 2e4, 4000)])
    j, y = j0y0(x)
    h = j - 1j * y
    ref = sp.hankel2(0, x)
    rel = np.abs(h - ref) / np.abs(ref)
    assert rel.max() <= 1e-14, (rel.max(), x[rel.argmax()])
    # Cephes separately for each part, relative to the modulus (Cephes'
    # own j0 / y0 are the less accurate routines at some large arguments:
    # they differ from AMOS by up to about 1.3e-12 there)
    assert np.max(np.abs(j - sp.j0(x)) / np.abs(ref)) <= 5e-12
    assert np.max(np.abs(y - sp.y0(x)) / np.abs(ref)) <= 5e-12


def test_zeros_and_small_arguments(j0y0):
    j, _ = j0y0(np.array([2.404825557695773, 5.520078110286311]))
    assert np.all(np.abs(j) < 1e-15)
    _, y = j0y0(np.array([0.8935769662791675, 3.957678419314858]))
    assert np.all(np.abs(y) < 1e-15)
    x = np.array([1e-12, 1e-9])
    j, y = j0y0(x)
    assert np.allclose(j, 1.0, rtol=0, atol=1e-15)
    assert np.allclose(y, (2 / np.pi) * (np.log(x / 2) + np.euler_gamma), rtol=1e-14, atol=0)
