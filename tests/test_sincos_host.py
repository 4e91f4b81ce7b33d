"""The kernels' FP64 phase factor, compiled for the host from the same header.

cis_halfturns(u) must equal exp(i pi u) to a few units in the last place for
the half-turn counts the kernels see (|u| up to ~1e6), checked against mpmath
at 50 digits on the exact binary value of u -- and stay exact far past that:
the sign (-1)^q of the nearest integer q is taken in FP64, so half-turn counts
up to 2^51 (a photon energy close to the particle energy makes k* = kE/(E - hw)
and so the phase arbitrarily large, Sec. II eq. (Lindhard_substi)) must not
pick up a wrong sign.
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


def test_cis_past_32_bit_parity(shim):
    """|u| in [2^31, 2^50]: odd and even integers, their quarter offsets and random
    values; a parity taken through a 32-bit conversion would flip the sign of about half
    of them.  At these sizes u - rint(u) is a multiple of the spacing of doubles near u,
    so the reference is evaluated on the exact binary value of u as before."""
    mp.mp.dps = 60
    rng = np.random.default_rng(4)
    ints = np.concatenate([2.0 ** np.arange(31, 51), 2.0 ** np.arange(31, 51) + 1.0,
                           2.0 ** np.arange(31, 50) + 3.0, 2.0 ** 31 * np.arange(1, 9) + 1.0])
    offs = np.concatenate([ints + 0.25, ints - 0.25, ints + 0.5])
    rnd = np.ldexp(rng.uniform(1.0, 2.0, 600), rng.integers(31, 50, 600))
    u = np.concatenate([ints, offs, rnd])
    u = np.concatenate([u, -u])
    c, s = _run(shim, u)
    err = 0.0
    for ui, ci, si in zip(u, c, s):
        x = mp.pi * mp.mpf(float(ui))
        err = max(err, abs(float(mp.cos(x)) - ci), abs(float(mp.sin(x)) - si))
    assert err < 4e-16, err
    odd = np.abs(np.fmod(u[:ints.size], 2.0)) == 1.0
    assert np.all(c[:ints.size][odd] == -1.0) and np.all(c[:ints.size][~odd] == 1.0)
