"""Binding of the GPU trajectory generator (include/rad_traj.h): planar channeling
trajectories generated on the device, ready for the radiation integrals without a
host round trip.  Argument marshalling only."""
from __future__ import annotations

import ctypes

import numpy as np

from . import rad

NCOL = 11
COLUMNS = rad.COLUMNS + ("energy",)
_bound = False


class TrajParams(ctypes.Structure):
    _fields_ = [("energy_eV", ctypes.c_double), ("charge", ctypes.c_double),
                ("U0_eV", ctypes.c_double), ("d_m", ctypes.c_double), ("q", ctypes.c_double),
                ("length_m", ctypes.c_double), ("theta_sigma", ctypes.c_double),
                ("X0_m", ctypes.c_double), ("eps_s_eV", ctypes.c_double),
                ("ms_on", ctypes.c_int32), ("loss_on", ctypes.c_int32),
                ("n_min", ctypes.c_int64), ("n_max", ctypes.c_int64), ("seed", ctypes.c_uint64)]


def _lib():
    global _bound
    L = rad.lib()
    if not _bound:
        P, I, I64, S = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_size_t
        PP = ctypes.POINTER(TrajParams)
        L.rad_traj_lengths.restype = I
        L.rad_traj_lengths.argtypes = [PP, I64, I, ctypes.POINTER(ctypes.c_int64)]
        L.rad_traj_workspace_bytes.restype = S
        L.rad_traj_workspace_bytes.argtypes = [I]
        L.rad_traj_generate.restype = I
        L.rad_traj_generate.argtypes = [PP, I64, I, P, I64, P, S, P]
        _bound = True
    return L


def params(cfg):
    """rad_traj_params of a channeling configuration (an object with the fields of
    rad_traj_params, e.g. ``synth.channeling.ChannelingConfig``)."""
    return TrajParams(float(cfg.energy_eV), float(cfg.charge), float(cfg.U0_eV), float(cfg.d_m),
                      float(cfg.q), float(cfg.length_m), float(cfg.theta_sigma), float(cfg.X0_m),
                      float(cfg.eps_s_eV), int(bool(cfg.ms_on)), int(bool(cfg.loss_on)), int(cfg.n_min),
                      int(cfg.n_max), int(cfg.seed) & (2 ** 64 - 1))


def lengths(cfg, n_particles, first=0):
    """Steps of particles first .. first+n-1 (host computation)."""
    out = np.zeros(n_particles, dtype=np.int64)
    p = params(cfg)
    rad._check(_lib().rad_traj_lengths(ctypes.byref(p), int(first), int(n_particles),
                                       out.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))), "rad_traj_lengths")
    return out


class DeviceTrajectories(rad.DeviceSegments):
    """Trajectories generated on the GPU, one segment per particle (the whole crystal,
    gamma and energy of the entry), usable wherever rad.DeviceSegments is."""

    def __init__(self, cfg, n_particles, first=0, stream=None, device="cuda"):
        import torch
        if int(getattr(cfg, "n_sections", 1)) != 1:
            raise ValueError("the GPU generator makes one section per particle")
        p = params(cfg)
        steps = lengths(cfg, n_particles, first)
        self.n = [int(s) + 1 for s in steps]
        total = int(sum(self.n))
        self.data = torch.empty((NCOL, total), dtype=torch.float64, device=device)
        ws = torch.empty(max(1, int(_lib().rad_traj_workspace_bytes(int(n_particles)))), dtype=torch.uint8,
                         device=device)
        rad._check(_lib().rad_traj_generate(ctypes.byref(p), int(first), int(n_particles), rad._dptr(self.data),
                                            total, rad._dptr(ws), ws.numel(), rad._stream(stream)),
                   "rad_traj_generate")
        self._ws = ws
        base = self.data.data_ptr()
        row = total * 8
        gamma = float(cfg.energy_eV) / (0.51099895e6)
        self.structs = (rad.Segment * n_particles)()
        off = 0
        for k, n in enumerate(self.n):
            st = self.structs[k]
            st.n = n
            for i, c in enumerate(rad.COLUMNS):
                setattr(st, c, base + i * row + off * 8)
            st.w = None
            st.gamma = gamma
            st.energy_eV = float(cfg.energy_eV)
            off += n
        self.offsets = np.concatenate([[0], np.cumsum(self.n)[:-1]]).astype(np.int64)

    def host(self, i):
        """Particle i as a dict of host arrays (the columns of the generator)."""
        o, n = int(self.offsets[i]), self.n[i]
        a = self.data[:, o:o + n].cpu().numpy()
        return {c: a[j].copy() for j, c in enumerate(COLUMNS)}
