"""Seeded synthetic channeling trajectories (Python side of ``channeling.c``).

Inputs only: nothing here evaluates a radiation integral.  A trajectory is cut
into sections (Sec. II: the energy is fixed at its section-entry value and the
spectra of the sections are summed).  Each section is returned as a segment
dict with the columns ``t, x, y, dz, vx, vy, dvz, ax, ay, az``, ``gamma`` and
``energy_eV`` of the section entry, and ``dz``/``dvz`` re-referenced to
``beta0 = 1 - 1/(2 gamma_s^2)`` of that section (only t - z and 1 - v_z enter
the integrand, so the shift is exact).
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
import subprocess
import threading
from concurrent.futures import ThreadPoolExecutor

import numpy as np

ME_EV = 0.51099895e6

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "channeling.c")
_LIB = os.path.join(_HERE, "_libsynth.so")
_lock = threading.Lock()
_lib = None


class _Params(ctypes.Structure):
    _fields_ = [("energy_eV", ctypes.c_double), ("charge", ctypes.c_double),
                ("U0_eV", ctypes.c_double), ("d_m", ctypes.c_double), ("q", ctypes.c_double),
                ("length_m", ctypes.c_double), ("theta_sigma", ctypes.c_double),
                ("X0_m", ctypes.c_double), ("eps_s_eV", ctypes.c_double),
                ("ms_on", ctypes.c_int32), ("loss_on", ctypes.c_int32),
                ("n_min", ctypes.c_int64), ("n_max", ctypes.c_int64), ("seed", ctypes.c_uint64)]


@dataclasses.dataclass
class ChannelingConfig:
    """Planar harmonic+quartic well (depth U0, width d), Si-like scattering."""
    energy_eV: float = 10e9
    charge: float = +1.0            # +1 positron, -1 electron
    U0_eV: float = 20.0
    d_m: float = 1.92e-10
    q: float = 0.5
    length_m: float = 100e-6
    theta_sigma: float = 10e-6
    X0_m: float = 0.0937            # radiation length of Si
    eps_s_eV: float = 10.6e6        # Sec. III
    ms_on: bool = True
    loss_on: bool = True
    n_min: int = 40000
    n_max: int = 120000
    n_sections: int = 1
    seed: int = 2

    def _c(self):
        return _Params(self.energy_eV, self.charge, self.U0_eV, self.d_m, self.q, self.length_m,
                       self.theta_sigma, self.X0_m, self.eps_s_eV, int(self.ms_on),
                       int(self.loss_on), int(self.n_min), int(self.n_max),
                       int(self.seed) & 0xFFFFFFFFFFFFFFFF)


def build(force: bool = True) -> str:
    """Compile the generator with gcc."""
    if not force and os.path.exists(_LIB):
        return _LIB
    tmp = _LIB + ".tmp%d" % os.getpid()
    subprocess.run(["gcc", "-O2", "-ffp-contract=off", "-fPIC", "-shared", "-std=c11", "-fopenmp", _SRC, "-o", tmp,
                    "-lm"], check=True)
    os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB):
                build(force=True)
            lib = ctypes.CDLL(_LIB)
            P = ctypes.POINTER(_Params)
            D = ctypes.POINTER(ctypes.c_double)
            lib.chan_lengths.argtypes = [P, ctypes.c_int64, ctypes.c_int64,
                                         ctypes.POINTER(ctypes.c_int64)]
            lib.chan_lengths.restype = ctypes.c_int
            lib.chan_generate.argtypes = [P, ctypes.c_int64, ctypes.c_int64] + [D] * 11
            lib.chan_generate.restype = ctypes.c_int
            _lib = lib
    return _lib


def lengths(cfg: ChannelingConfig, n_particles: int, first: int = 0) -> np.ndarray:
    """Steps per trajectory (n steps -> n+1 samples) of particles first..first+n-1."""
    lib = _load()
    out = np.zeros(n_particles, dtype=np.int64)
    p = cfg._c()
    lib.chan_lengths(ctypes.byref(p), n_particles, first,
                     out.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
    return out


_COLS = ("t", "x", "y", "dz", "vx", "vy", "dvz", "ax", "ay", "az", "energy")


def trajectory(cfg: ChannelingConfig, particle: int) -> dict:
    """Whole trajectory of one particle: columns relative to the entry gamma."""
    lib = _load()
    n = int(lengths(cfg, 1, particle)[0])
    cols = {c: np.empty(n + 1) for c in _COLS}
    p = cfg._c()
    D = ctypes.POINTER(ctypes.c_double)
    rc = lib.chan_generate(ctypes.byref(p), particle, n,
                           *[cols[c].ctypes.data_as(D) for c in _COLS])
    if rc != 0:
        raise RuntimeError("chan_generate failed")
    return cols


def sections(cfg: ChannelingConfig, traj: dict) -> list:
    """Cut a trajectory into cfg.n_sections sections of equal step count.

    Section s holds samples k_s..k_{s+1} (both ends), its entry energy E_s and
    gamma_s = E_s/m_e, with dvz, dz re-referenced to beta0_s = 1 - 1/(2 gamma_s^2).
    """
    n = traj["t"].size - 1
    ns = max(1, int(cfg.n_sections))
    bounds = [(s * n) // ns for s in range(ns + 1)]
    g_ref = cfg.energy_eV / ME_EV
    segs = []
    for s in range(ns):
        k0, k1 = bounds[s], bounds[s + 1]
        if k1 <= k0:
            continue
        sl = slice(k0, k1 + 1)
        E_s = float(traj["energy"][k0])
        g_s = E_s / ME_EV
        shift = 0.5 / (g_s * g_s) - 0.5 / (g_ref * g_ref)   # beta_ref - beta0_s
        seg = {c: np.ascontiguousarray(traj[c][sl]) for c in _COLS if c != "energy"}
        seg["dvz"] = seg["dvz"] + shift
        seg["dz"] = seg["dz"] + shift * seg["t"]
        seg["gamma"] = g_s
        seg["energy_eV"] = E_s
        seg["w"] = None
        segs.append(seg)
    return segs


def generate(cfg: ChannelingConfig, n_particles: int, first: int = 0, threads: int = 8):
    """Sections of particles first..first+n_particles-1, grouped per particle.

    Returns a list (one entry per particle) of lists of segment dicts.
    """
    def one(i):
        return sections(cfg, trajectory(cfg, first + i))

    if n_particles <= 1 or threads <= 1:
        return [one(i) for i in range(n_particles)]
    with ThreadPoolExecutor(max_workers=threads) as ex:
        return list(ex.map(one, range(n_particles)))
