"""Workload presets: trajectories plus (hw, theta_x, theta_y) grids.

Each preset names a workload by what it is.  Every free choice (grid spacing,
section count, seeds) is written out here:

* ``undulator_fp64``  -- one electron, gamma = 2e4, planar undulator with
  lambda_u = 20 um and K = 0.5 over 20 periods in 8192 uniform steps (8193
  samples, trapezoid); 128 linear hw up to 1.5x the on-axis first harmonic x
  16x16 cell-centred angles in |theta_x|, |theta_y| <= 1/gamma; classical.
* ``positron_spinhalf`` -- 256 positrons at 10 GeV in the harmonic+quartic
  planar well (depth 20 eV, width 1.92 A), 100 um, entry x uniform across the
  channel, entry angles N(0, 10 urad), Gaussian multiple scattering and
  radiative loss, 4e4..1.2e5 steps; 512 log hw in 0.5..200 MeV x 32x32 angles
  within 5/gamma; spin-1/2.
* ``pm_mixed`` -- 1024 positrons + 1024 electrons (electron well), same
  generator at 10 GeV; 256 log hw in 0.5..200 MeV x 16x16 angles within
  5/gamma; classical, spin-0 and spin-1/2.
* ``electron_50gev_sections`` -- 512 electrons at 50 GeV in 1 mm cut into 10
  sections, 1e5..3e5 steps per trajectory; 256 log hw in 1 MeV..20 GeV x
  16x16 angles within 4/gamma; spin-1/2.
"""
from __future__ import annotations

import dataclasses

from . import analytic
from .channeling import ChannelingConfig, ME_EV

KIND_CLASSICAL, KIND_SPIN0, KIND_SPINHALF = 1, 2, 4


@dataclasses.dataclass
class Grid:
    hw_eV: object
    thx: object
    thy: object

    @property
    def shape(self):
        return (len(self.hw_eV), len(self.thy), len(self.thx))


def undulator_fp64():
    gamma, K, lam, nper = 2.0e4, 0.5, 20e-6, 20
    seg = analytic.undulator(gamma, K, lam, nper, n_steps=8192)
    hw1 = analytic.undulator_fundamental_eV(gamma, K, lam)
    grid = Grid(analytic.linear_omega(128, 1.5 * hw1), analytic.cell_centred(16, 1.0 / gamma),
                analytic.cell_centred(16, 1.0 / gamma))
    return dict(name="undulator_fp64", segments=[seg], out_index=[0], n_out=1, grid=grid,
                kinds=KIND_CLASSICAL)


def channeling_grid(n_w, n_theta, lo_eV, hi_eV, gamma, half_width_over_gamma):
    th = analytic.cell_centred(n_theta, half_width_over_gamma / gamma)
    return Grid(analytic.log_omega(n_w, lo_eV, hi_eV), th, th.copy())


def positron_config(seed=2, charge=+1.0):
    return ChannelingConfig(energy_eV=10e9, charge=charge, length_m=100e-6, n_min=40000,
                            n_max=120000, n_sections=1, seed=seed)


def positron_grid(n_w=512, n_theta=32):
    return channeling_grid(n_w, n_theta, 0.5e6, 200e6, 10e9 / ME_EV, 5.0)


def electron_50gev_config(seed=5):
    return ChannelingConfig(energy_eV=50e9, charge=-1.0, length_m=1e-3, n_min=100000,
                            n_max=300000, n_sections=10, seed=seed)


def electron_50gev_grid(n_w=256, n_theta=16):
    return channeling_grid(n_w, n_theta, 1e6, 20e9, 50e9 / ME_EV, 4.0)


def pm_configs(seed=3):
    """Positron and electron generators of the mixed-precision workload."""
    return (ChannelingConfig(energy_eV=10e9, charge=+1.0, seed=seed),
            ChannelingConfig(energy_eV=10e9, charge=-1.0, seed=seed + 1000))


def pm_grid(n_w=256, n_theta=16):
    return channeling_grid(n_w, n_theta, 0.5e6, 200e6, 10e9 / ME_EV, 5.0)
