"""Analytic trajectories in the small-angle variables of Sec. II.

Every trajectory is returned as a dict of NumPy float64 columns
``t, x, y, dz, vx, vy, dvz, ax, ay, az`` (c = 1, metres) plus ``gamma`` and
``energy_eV`` and optionally quadrature weights ``w``.  ``dz = z - beta0 t``
and ``dvz = v_z - beta0`` with ``beta0 = 1 - 1/(2 gamma^2)`` exactly; ``a`` is
d(beta)/dt.  The columns are mutually consistent: x' = vx, vx' = ax,
dz' = dvz, dvz' = az.

These are inputs only: nothing here evaluates a radiation integral.
"""
from __future__ import annotations

import math

import numpy as np

ME_EV = 0.51099895e6          # electron rest energy [eV] (CODATA 2018)
C_MS = 299792458.0            # speed of light [m/s]


def _pack(t, x, y, dz, vx, vy, dvz, ax, ay, az, gamma, w=None, energy_eV=None):
    seg = {k: np.ascontiguousarray(v, dtype=np.float64) for k, v in
           dict(t=t, x=x, y=y, dz=dz, vx=vx, vy=vy, dvz=dvz, ax=ax, ay=ay, az=az).items()}
    seg["gamma"] = float(gamma)
    seg["energy_eV"] = float(energy_eV if energy_eV is not None else gamma * ME_EV)
    seg["w"] = None if w is None else np.ascontiguousarray(w, dtype=np.float64)
    return seg


def undulator_K(B0_T, lambda_m):
    """Deflection parameter K = e B0 lambda / (2 pi m_e c) of a planar undulator."""
    return B0_T * lambda_m * C_MS / (2.0 * math.pi * ME_EV)


def undulator(gamma, K, lambda_u, n_periods, samples_per_period=None, n_steps=None,
              rule="trapezoid", t0=0.0):
    """Planar undulator motion x = a sin(Omega t) in the expansion-consistent form.

    Omega = 2 pi / lambda_u, tau = Omega t:
      x = K/(gamma Omega) sin tau,  vx = K/gamma cos tau,  ax = -(K/gamma) Omega sin tau,
      dvz = -vx^2/2,  az = -vx ax,  dz = -(K^2/(4 gamma^2)) (t + sin(2 tau)/(2 Omega)).
    ``rule='trapezoid'``: n_steps intervals, n_steps+1 samples, trapezoid weights
    (w=None).  ``rule='rect'``: n_periods*samples_per_period samples over whole
    periods with equal weights dt (exact for periodic integrands).
    """
    Om = 2.0 * math.pi / lambda_u
    T = n_periods * lambda_u
    if rule == "rect":
        if samples_per_period is None:
            raise ValueError("rect rule needs samples_per_period")
        n = int(n_periods * samples_per_period)
        dt = T / n
        t = t0 + dt * np.arange(n)
        w = np.full(n, dt)
    else:
        if n_steps is None:
            n_steps = int(n_periods * samples_per_period)
        t = t0 + np.linspace(0.0, T, n_steps + 1)
        w = None
    tau = Om * t
    vx = (K / gamma) * np.cos(tau)
    x = (K / (gamma * Om)) * np.sin(tau)
    ax = -(K / gamma) * Om * np.sin(tau)
    dvz = -0.5 * vx * vx
    az = -vx * ax
    dz = -(K * K / (4.0 * gamma * gamma)) * (t + np.sin(2.0 * tau) / (2.0 * Om))
    z0 = np.zeros_like(t)
    return _pack(t, x, z0, dz, vx, z0, dvz, ax, z0, az, gamma, w)


def arc(gamma, radius, half_span_over_gamma=25.0, n_steps=20000):
    """Circular arc of radius R in the x-z plane, small-angle form, t in [-T, T].

    vx = t/R, ax = 1/R, x = t^2/(2R), dvz = -t^2/(2R^2), az = -t/R^2,
    dz = -t^3/(6R^2); the velocity turns by +-half_span_over_gamma/gamma.
    """
    T = half_span_over_gamma * radius / gamma
    t = np.linspace(-T, T, n_steps + 1)
    vx = t / radius
    x = t * t / (2.0 * radius)
    ax = np.full_like(t, 1.0 / radius)
    dvz = -t * t / (2.0 * radius * radius)
    az = -t / (radius * radius)
    dz = -t ** 3 / (6.0 * radius * radius)
    z0 = np.zeros_like(t)
    return _pack(t, x, z0, dz, vx, z0, dvz, ax, z0, az, gamma)


def uniform(gamma, vx, vy, length, n_steps=1000):
    """Straight-line motion with constant transverse velocity (no acceleration)."""
    t = np.linspace(0.0, length, n_steps + 1)
    dvz0 = -0.5 * (vx * vx + vy * vy)
    one = np.ones_like(t)
    zero = np.zeros_like(t)
    return _pack(t, vx * t, vy * t, dvz0 * t, vx * one, vy * one, dvz0 * one, zero, zero, zero,
                 gamma)


def wiggle3d(gamma, lambda_u, n_periods, n_steps, Kx=1.0, Ky=0.6, eps=0.3, seed_phase=0.4,
             t0=0.0):
    """A smooth, non-planar, non-periodic 3-D motion with every column non-trivial.

    vx = (Kx/gamma)[cos(W t) + eps sin(2.3 W t + p)], vy = (Ky/gamma) sin(1.7 W t),
    dvz = -(vx^2 + vy^2)/2 + (eps/gamma^2) cos(0.9 W t), with x, dz the exact
    integrals and a the exact derivatives.  Used for identity pins, where every
    term of the integrand must matter.
    """
    W = 2.0 * math.pi / lambda_u
    p = seed_phase
    t = t0 + np.linspace(0.0, n_periods * lambda_u, n_steps + 1)
    kx, ky = Kx / gamma, Ky / gamma
    a1, a2, a3, a4 = W, 2.3 * W, 1.7 * W, 0.9 * W
    vx = kx * (np.cos(a1 * t) + eps * np.sin(a2 * t + p))
    ax = kx * (-a1 * np.sin(a1 * t) + eps * a2 * np.cos(a2 * t + p))
    x = kx * (np.sin(a1 * t) / a1 - eps * np.cos(a2 * t + p) / a2)
    vy = ky * np.sin(a3 * t)
    ay = ky * a3 * np.cos(a3 * t)
    y = -ky * np.cos(a3 * t) / a3
    e = eps / gamma ** 2
    dvz = -0.5 * (vx * vx + vy * vy) + e * np.cos(a4 * t)
    az = -(vx * ax + vy * ay) - e * a4 * np.sin(a4 * t)
    # dz = int dvz dt, in closed form term by term
    # vx^2 = kx^2 [cos^2(a1 t) + 2 eps cos(a1 t) sin(a2 t + p) + eps^2 sin^2(a2 t + p)]
    def i_cos2(a):
        return t / 2.0 + np.sin(2.0 * a * t) / (4.0 * a)

    def i_sin2(a, ph):
        return t / 2.0 - np.sin(2.0 * (a * t + ph)) / (4.0 * a)

    # cos(a1 t) sin(a2 t + p) = [sin((a2+a1) t + p) + sin((a2-a1) t + p)] / 2
    def i_cs():
        s, d = a2 + a1, a2 - a1
        return 0.5 * (-np.cos(s * t + p) / s - np.cos(d * t + p) / d)

    ivx2 = kx * kx * (i_cos2(a1) + 2.0 * eps * i_cs() + eps * eps * i_sin2(a2, p))
    ivy2 = ky * ky * (t / 2.0 - np.sin(2.0 * a3 * t) / (4.0 * a3))
    dz = -0.5 * (ivx2 + ivy2) + e * np.sin(a4 * t) / a4
    # constant of integration: dz(t0) = 0
    dz = dz - dz[0]
    return _pack(t, x, y, dz, vx, vy, dvz, ax, ay, az, gamma)


def cell_centred(n, half_width):
    """Cell-centred grid on [-half_width, half_width]: th_j = -H + (j + 1/2) 2H/n."""
    return -half_width + (np.arange(n) + 0.5) * (2.0 * half_width / n)


def linear_omega(n, hw_max):
    """Linear photon-energy grid hw_i = (i+1) hw_max / n (excludes 0)."""
    return (np.arange(n) + 1.0) * (hw_max / n)


def log_omega(n, lo, hi):
    """Log-spaced photon-energy grid including both endpoints."""
    return np.geomspace(lo, hi, n)


def undulator_fundamental_eV(gamma, K, lambda_u, theta=0.0):
    """hbar w_1(theta) = 2 gamma^2 (2 pi hbar c / lambda_u) / (1 + K^2/2 + gamma^2 theta^2)."""
    hbarc = 1.973269804e-7
    return 2.0 * gamma ** 2 * (2.0 * math.pi * hbarc / lambda_u) / (
        1.0 + 0.5 * K * K + (gamma * theta) ** 2)
