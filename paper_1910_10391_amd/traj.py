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
        L.rad_traj_workspace_bytes.argtypes = [PP, I64, I]
        L.rad_traj_generate.restype = I
        L.rad_traj_generate.argtypes = [PP, I64, I, P, I64, P, S, P]
        L.rad_traj_sections_workspace_bytes.restype = S
        L.rad_traj_sections_workspace_bytes.argtypes = [I, I]
        L.rad_traj_sections.restype = I
        L.rad_traj_sections.argtypes = [PP, I64, I, I, P, I64, P, I64, ctypes.POINTER(ctypes.c_double), P, S, P]
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
    """Trajectories generated on the GPU, usable wherever rad.DeviceSegments is.  With
    ``cfg.n_sections`` > 1 the segments are the sections (cut on the GPU, each with its
    entry gamma and energy) and ``out_index`` gives each section's particle; otherwise
    one segment per particle."""

    def __init__(self, cfg, n_particles, first=0, stream=None, device="cuda"):
        import torch
        p = params(cfg)
        steps = lengths(cfg, n_particles, first)
        n_full = [int(s_) + 1 for s_ in steps]
        total = int(sum(n_full))
        self.traj_data = torch.empty((NCOL, total), dtype=torch.float64, device=device)
        ws = torch.empty(max(1, int(_lib().rad_traj_workspace_bytes(ctypes.byref(p), int(first),
                                                                       int(n_particles)))),
                         dtype=torch.uint8, device=device)
        rad._check(_lib().rad_traj_generate(ctypes.byref(p), int(first), int(n_particles),
                                            rad._dptr(self.traj_data), total, rad._dptr(ws), ws.numel(),
                                            rad._stream(stream)), "rad_traj_generate")
        self._ws = ws
        self.traj_n = n_full
        self.traj_offsets = np.concatenate([[0], np.cumsum(n_full)[:-1]]).astype(np.int64)
        ns = int(getattr(cfg, "n_sections", 1))
        me = 0.51099895e6
        if ns <= 1:
            self.data = self.traj_data
            self.n = list(n_full)
            gammas = [float(cfg.energy_eV) / me] * n_particles
            energies = [float(cfg.energy_eV)] * n_particles
            self.out_index = list(range(n_particles))
        else:
            sec_n = []
            for n in steps:
                n = int(n)
                sec_n += [((s_ + 1) * n) // ns - (s_ * n) // ns + 1 for s_ in range(ns)]
            sec_total = int(sum(sec_n))
            self.data = torch.empty((NCOL, sec_total), dtype=torch.float64, device=device)
            wss = torch.empty(max(1, int(_lib().rad_traj_sections_workspace_bytes(int(n_particles), ns))),
                              dtype=torch.uint8, device=device)
            entry = np.zeros(n_particles * ns)
            rad._check(_lib().rad_traj_sections(ctypes.byref(p), int(first), int(n_particles), ns,
                                                rad._dptr(self.traj_data), total, rad._dptr(self.data), sec_total,
                                                entry.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                                rad._dptr(wss), wss.numel(), rad._stream(stream)),
                       "rad_traj_sections")
            self.n = sec_n
            energies = [float(e) for e in entry]
            gammas = [e / me for e in energies]
            self.out_index = [i for i in range(n_particles) for _ in range(ns)]
        self.entry_energy = np.array(energies)
        total_seg = int(sum(self.n))
        base = self.data.data_ptr()
        row = total_seg * 8
        self.structs = (rad.Segment * len(self.n))()
        off = 0
        for k, n in enumerate(self.n):
            st = self.structs[k]
            st.n = n
            for i, c in enumerate(rad.COLUMNS):
                setattr(st, c, base + i * row + off * 8)
            st.w = None
            st.gamma = gammas[k]
            st.energy_eV = energies[k]
            off += n
        self.offsets = np.concatenate([[0], np.cumsum(self.n)[:-1]]).astype(np.int64)

    def host(self, i):
        """Particle i's whole trajectory as a dict of host arrays (the generator's columns)."""
        o, n = int(self.traj_offsets[i]), self.traj_n[i]
        a = self.traj_data[:, o:o + n].cpu().numpy()
        return {c: a[j].copy() for j, c in enumerate(COLUMNS)}

    def segment_host(self, j):
        """Segment j (a section, or a whole trajectory) as a dict of host arrays."""
        o, n = int(self.offsets[j]), self.n[j]
        a = self.data[:, o:o + n].cpu().numpy()
        d = {c: a[k].copy() for k, c in enumerate(COLUMNS)}
        d.update(gamma=float(self.structs[j].gamma), energy_eV=float(self.structs[j].energy_eV), w=None)
        return d
