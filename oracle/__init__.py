"""Plain CPU oracle for the radiation integrals.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The product path
(the HIP library and its Python binding) never imports it, and it never imports
the product: the two share no code.  Inputs come from the seeded generators in
``paper_1910_10391_amd.synth``, which hold none of the method's arithmetic.

The heavy loop is ``rad_oracle.c`` (plain C, libm sin/cos, no fast-math, no FMA
contraction, OpenMP over integrals).  This module compiles it with gcc, loads
it with ctypes and adds the plain bookkeeping steps:

* ``spectrum``      -- one segment: classical / spin-0 / spin-1/2 cubes
                       (Sec. II eq. (integralrad1), (Lindhard_substi), (cue));
* ``batch``         -- several segments summed incoherently per output
                       (Sec. II, sections: the spectrum of a trajectory is the
                       sum of the spectra of its sections);
* ``angle_integrate`` -- dI/dhw as the midpoint sum over the angular grid
                       (Sec. IV, the host sum over the spatial integrals).

Every function is pinned by the CPU tests (closed forms, identities, brute
force); see ``tests/test_oracle_pins.py``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

__all__ = [
    "HBARC_EVM", "ALPHA", "ME_EV", "build", "amplitudes", "spectrum", "batch",
    "angle_integrate", "angle_weights", "max_threads", "KIND_CLASSICAL", "KIND_SPIN0",
    "KIND_SPINHALF",
]

# CODATA 2018 (typed here independently of the product's headers)
HBARC_EVM = 1.973269804e-7
ALPHA = 7.2973525693e-3
ME_EV = 0.51099895e6

KIND_CLASSICAL, KIND_SPIN0, KIND_SPINHALF = 1, 2, 4

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rad_oracle.c")
_LIB = os.path.join(_HERE, "_rad_oracle.so")
_lock = threading.Lock()
_libs = {}

_D = ctypes.POINTER(ctypes.c_double)


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (plain -O2, no fast-math, no contraction)."""
    if not force and os.path.exists(_LIB):
        return _LIB
    tmp = _LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-fno-fast-math", "-ffp-contract=off", "-fopenmp", "-fPIC",
           "-shared", "-std=c11", _SRC, "-o", tmp, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB)
    return _LIB


def build_variant(src: str, out: str) -> str:
    """Compile another copy of the oracle source (used by the mutation tests)."""
    cmd = ["gcc", "-O2", "-fno-fast-math", "-ffp-contract=off", "-fopenmp", "-fPIC",
           "-shared", "-std=c11", src, "-o", out, "-lm"]
    subprocess.run(cmd, check=True)
    return out


_current = [None]


class use_library:
    """Context manager: route the oracle calls to another build of its source.

    Only the mutation tests use it, to show that the pins fail on planted
    mistakes.
    """

    def __init__(self, path):
        self.path = path

    def __enter__(self):
        self.prev = _current[0]
        _current[0] = self.path
        return self

    def __exit__(self, *exc):
        _current[0] = self.prev
        return False


def _load(path=None):
    path = path or _current[0] or _LIB
    with _lock:
        if path not in _libs:
            if path == _LIB and not os.path.exists(_LIB):
                build(force=True)
            lib = ctypes.CDLL(path)
            i64, cint = ctypes.c_int64, ctypes.c_int
            lib.oracle_amplitudes.argtypes = [i64] + [_D] * 11 + [ctypes.c_double, i64, _D, i64,
                                                                  _D, _D, _D, _D, cint]
            lib.oracle_amplitudes.restype = cint
            lib.oracle_spectrum.argtypes = ([i64] + [_D] * 11 +
                                            [ctypes.c_double, ctypes.c_double, cint, _D, cint, _D,
                                             cint, _D, cint, _D, cint])
            lib.oracle_spectrum.restype = cint
            lib.oracle_max_threads.argtypes = []
            lib.oracle_max_threads.restype = cint
            # the OpenMP thread count before any call sets one
            lib.default_threads = int(lib.oracle_max_threads())
            _libs[path] = lib
    return _libs[path]


def _threads(lib, threads):
    """threads > 0 as given; 0: the host's default count (a call with threads = 1 sets
    OpenMP's count for later calls, so the default is passed explicitly)."""
    return int(threads) if threads > 0 else lib.default_threads


def max_threads() -> int:
    """OpenMP threads the oracle uses by default on this host."""
    return _threads(_load(), 0)


_COLS = ("t", "x", "y", "dz", "vx", "vy", "dvz", "ax", "ay", "az")


def _ptr(a):
    return a.ctypes.data_as(_D)


def _seg_args(seg):
    cols = [np.ascontiguousarray(seg[c], dtype=np.float64) for c in _COLS]
    n = cols[0].shape[0]
    for c in cols:
        if c.shape != (n,):
            raise ValueError("segment columns must be 1-D arrays of equal length")
    w = seg.get("w")
    w = None if w is None else np.ascontiguousarray(w, dtype=np.float64)
    if w is not None and w.shape != (n,):
        raise ValueError("weights must match the segment length")
    keep = cols + ([w] if w is not None else [])
    args = [ctypes.c_int64(n)] + [_ptr(c) for c in cols] + [_ptr(w) if w is not None else None]
    return args, keep


def amplitudes(seg, kappa, nx, ny, want_j=True, threads=0):
    """Complex amplitudes A (3 components) and J for a list of wavenumbers and directions.

    Follows Sec. II eq. (integralrad1)-(integralrad2) in the Sec. II small-angle
    expansion; J is the integral of eq. (Iterm)'s second display.  ``kappa`` is
    hw/(hbar c) in 1/m (or kappa* for the quantum integrals); ``nx``/``ny`` are
    equal-length direction lists.  Returns (A[n_kappa, n_dir, 3] complex,
    J[n_kappa, n_dir] complex or None).
    """
    lib = _load()
    args, keep = _seg_args(seg)
    kappa = np.ascontiguousarray(np.atleast_1d(kappa), dtype=np.float64)
    nx = np.ascontiguousarray(np.atleast_1d(nx), dtype=np.float64)
    ny = np.ascontiguousarray(np.atleast_1d(ny), dtype=np.float64)
    if nx.shape != ny.shape:
        raise ValueError("nx and ny must have the same length")
    A = np.zeros((kappa.size, nx.size, 6))
    J = np.zeros((kappa.size, nx.size, 2)) if want_j else None
    rc = lib.oracle_amplitudes(*args, ctypes.c_double(float(seg["gamma"])),
                               ctypes.c_int64(kappa.size), _ptr(kappa), ctypes.c_int64(nx.size),
                               _ptr(nx), _ptr(ny), _ptr(A), _ptr(J) if want_j else None,
                               ctypes.c_int(_threads(lib, threads)))
    if rc != 0:
        raise ValueError("oracle_amplitudes rejected its arguments")
    del keep
    Ac = A[..., 0::2] + 1j * A[..., 1::2]
    Jc = (J[..., 0] + 1j * J[..., 1]) if want_j else None
    return Ac, Jc


def _kinds_list(kinds):
    return [k for k in (KIND_CLASSICAL, KIND_SPIN0, KIND_SPINHALF) if kinds & k]


def spectrum(seg, hw_eV, thx, thy, kinds=KIND_CLASSICAL, threads=0):
    """d2I/(d hw dOmega) cubes [n_w][n_y][n_x] for one segment.

    classical: alpha/(4 pi^2) |A(k)|^2                     (Sec. II eq. (integralrad1))
    spin-0   : alpha/(4 pi^2) (E*/E) |A(k*)|^2             (Sec. II eq. (Lindhard_substi))
    spin-1/2 : alpha/(4 pi^2) [(E*^2+E^2)/(2E^2)|A(k*)|^2
                               + hw^2/(2E^2 gamma^2)|J(k*)|^2]   (Sec. II eq. (cue))
    with k = hw/(hbar c), k* = k E/(E - hw), E* = E - hw; 0 where hw >= E.
    Returns a dict kind -> cube.
    """
    lib = _load()
    args, keep = _seg_args(seg)
    hw = np.ascontiguousarray(hw_eV, dtype=np.float64)
    thx = np.ascontiguousarray(thx, dtype=np.float64)
    thy = np.ascontiguousarray(thy, dtype=np.float64)
    ks = _kinds_list(kinds)
    if not ks or kinds & ~7:
        raise ValueError("kinds must be a non-empty mask of 1, 2, 4")
    out = np.zeros((len(ks), hw.size, thy.size, thx.size))
    rc = lib.oracle_spectrum(*args, ctypes.c_double(float(seg["gamma"])),
                             ctypes.c_double(float(seg.get("energy_eV", np.inf))),
                             ctypes.c_int(hw.size), _ptr(hw), ctypes.c_int(thx.size), _ptr(thx),
                             ctypes.c_int(thy.size), _ptr(thy), ctypes.c_int(kinds), _ptr(out),
                             ctypes.c_int(_threads(lib, threads)))
    if rc != 0:
        raise ValueError("oracle_spectrum rejected its arguments")
    del keep
    return {k: out[i] for i, k in enumerate(ks)}


def batch(segs, out_index, n_out, hw_eV, thx, thy, kinds, threads=0):
    """Sum of per-segment spectra into n_out outputs, in segment order.

    Sec. II (sections): a trajectory is cut into sections, each with its entry
    energy fixed, and the spectrum of the trajectory is the sum of the section
    spectra.  Returns an array [n_out][n_kinds][n_w][n_y][n_x].
    """
    ks = _kinds_list(kinds)
    out = np.zeros((n_out, len(ks), len(hw_eV), len(thy), len(thx)))
    for seg, o in zip(segs, out_index):
        sp = spectrum(seg, hw_eV, thx, thy, kinds, threads)
        for i, k in enumerate(ks):
            out[o, i] += sp[k]
    return out


def angle_weights(th):
    """Cell widths of a 1-D angle grid: boundaries half-way between neighbours.

    For a cell-centred uniform grid every width equals the spacing.  A single
    point has width 1 (the integral reduces to the point value).
    """
    th = np.asarray(th, dtype=np.float64)
    n = th.size
    if n == 1:
        return np.ones(1)
    w = np.empty(n)
    w[1:-1] = 0.5 * (th[2:] - th[:-2])
    w[0] = th[1] - th[0]
    w[-1] = th[-1] - th[-2]
    return w


def angle_integrate(cube, thx, thy):
    """dI/d hw = sum_{jy,jx} cube[..., jy, jx] dthx_jx dthy_jy (midpoint rule).

    Sec. IV: the spectrum dI/dw is the sum over the spatial integrals of the cube.
    """
    cube = np.asarray(cube, dtype=np.float64)
    wx = angle_weights(thx)
    wy = angle_weights(thy)
    return np.einsum("...yx,y,x->...", cube, wy, wx)
