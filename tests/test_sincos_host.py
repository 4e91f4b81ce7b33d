"""The kernels' FP64 phase factor, compiled for the host from the same header.

cis_halfturns(u) must equal exp(i pi u) to a few units in the last place for
the half-turn counts the kernels see (|u| up to ~1e6), checked against mpmath
at 50 digits on the exact binary value of u.
"""
import ctypes
import os
import subprocess

import mpmath as mp
import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1910_10391_amd", "csrc")

SHIM = r'''
#include "rad_math.h"
extern "C" void host_cis(const double *u, int n, double *c, double *s) {
    for (int i = 0; i < n; ++i) rad::cis_halfturns(u[i], c[i], s[i]);
}
'''


@pytest.fixture(scope="module")
def shim(tmp_path_factory):
    d = tmp_path_factory.mktemp("cis")
    src = d / "shim.hip"
    src.write_text(SHIM)
    so = d / "shim.so"
    subprocess.run(["/opt/rocm/bin/hipcc", "--offload-arch=gfx950", "-O2", "-fPIC", "-shared",
                    "-I", CSRC, str(src), "-o", str(so)], check=True, capture_output=True)
    lib = ctypes.CDLL(str(so))
    D = ctypes.POINTER(ctypes.c_double)
    lib.host_cis.argtypes = [D, ctypes.c_int, D, D]
    return lib


def _run(lib, u):
    u = np.ascontiguousarray(u, dtype=np.float64)
    c = np.empty_like(u)
    s = np.empty_like(u)
    D = ctypes.POINTER(ctypes.c_double)
    lib.host_cis(u.ctypes.data_as(D), u.size, c.ctypes.data_as(D), s.ctypes.data_as(D))
    return c, s


def test_cis_against_mpmath(shim):
    mp.mp.dps = 50
    rng = np.random.default_rng(1)
    u = np.concatenate([rng.uniform(-1, 1, 800), rng.uniform(-1e4, 1e4, 800),
                        rng.uniform(-1e6, 1e6, 400), np.arange(-8, 9) * 0.25,
                        np.arange(-8, 9) * 0.5 + 1e-12])
    c, s = _run(shim, u)
    err = 0.0
    for ui, ci, si in zip(u, c, s):
        x = mp.pi * mp.mpf(float(ui))
        err = max(err, abs(float(mp.cos(x)) - ci), abs(float(mp.sin(x)) - si))
    assert err < 4e-16, err


def test_cis_unit_modulus_and_symmetry(shim):
    rng = np.random.default_rng(2)
    u = rng.uniform(-1e5, 1e5, 100000)
    c, s = _run(shim, u)
    assert np.max(np.abs(c * c + s * s - 1.0)) < 1e-15
    c2, s2 = _run(shim, -u)
    assert np.array_equal(c2, c) and np.array_equal(s2, -s)
