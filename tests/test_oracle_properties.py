"""Property tests of the oracle on random smooth planar trajectories (Hypothesis): facts the
expansion of Sec. II fixes for any motion, independent of the oracle's own numbers.

* mirror symmetry: for motion in the x-z plane (y = v_y = a_y = 0) the integrand and the phase
  are even in thy except f_y, which is odd, so every spectrum is even in thy, bit for bit (the
  oracle evaluates each direction on its own, and thy enters only through thy^2 and the sign
  of f_y);
* every spectrum is >= 0 (sums of squared moduli with non-negative weights, Sec. II eq.
  (integralrad1), eq. (Lindhard_substi), eq. (cue));
* a shift of the time axis, t -> t + t0 with the same samples, multiplies each amplitude by a
  phase constant over the trajectory (psi changes by (1/(2 gamma^2) + th^2/2) t0), so the spectra
  do not change beyond rounding;
* as hw/E -> 0 both quantum spectra tend to the classical one (k* -> k, E*/E -> 1, the J term
  vanishes), Sec. II eq. (Lindhard_substi) and eq. (cue).
"""
import math

import numpy as np
import pytest

hypothesis = pytest.importorskip("hypothesis")
from hypothesis import given, settings, strategies as st  # noqa: E402

import oracle  # noqa: E402

KINDS = oracle.KIND_CLASSICAL | oracle.KIND_SPIN0 | oracle.KIND_SPINHALF
HBARC = 1.973269804e-7


def planar(gamma, modes, n, periods):
    """x(t) = sum_m a_m sin(W_m t + p_m) in the small-angle form of Sec. II: v_x = dx/dt,
    a_x = dv_x/dt, 1 - v_z = 1/(2 gamma^2) + v_x^2/2 (so dvz = -v_x^2/2 and a_z = -v_x a_x
    about beta0), dz the integral of dvz (trapezoid, from 0); y = v_y = a_y = 0."""
    W0 = min(W for _, W, _ in modes)
    t = np.linspace(0.0, periods * 2.0 * math.pi / W0, n)
    x = sum(a * np.sin(W * t + p) for a, W, p in modes)
    vx = sum(a * W * np.cos(W * t + p) for a, W, p in modes)
    ax = sum(-a * W * W * np.sin(W * t + p) for a, W, p in modes)
    dvz = -0.5 * vx * vx
    az = -vx * ax
    dz = np.concatenate([[0.0], np.cumsum(0.5 * (dvz[1:] + dvz[:-1]) * np.diff(t))])
    z = np.zeros_like(t)
    return dict(t=t, x=x, y=z.copy(), dz=dz, vx=vx, vy=z.copy(), dvz=dvz, ax=ax, ay=z.copy(), az=az,
                gamma=gamma, w=None)


@st.composite
def cases(draw):
    gamma = draw(st.floats(1e3, 1e5))
    n_modes = draw(st.integers(1, 3))
    lam = draw(st.floats(5e-6, 5e-5))                    # period of the slowest mode [m]
    W0 = 2.0 * math.pi / lam
    modes = []
    for m in range(n_modes):
        K = draw(st.floats(0.05, 2.0))                    # gamma x velocity amplitude
        W = W0 * (1.0 if m == 0 else draw(st.floats(1.0, 4.0)))
        modes.append((K / (gamma * W), W, draw(st.floats(0.0, 2.0 * math.pi))))
    n = draw(st.integers(40, 240))
    periods = draw(st.integers(1, 4))
    seg = planar(gamma, modes, n, periods)
    hw1 = 2.0 * gamma * gamma * (W0 * HBARC)              # 2 gamma^2 hbar c k_u, hw scale
    hw = np.array(sorted(draw(st.lists(st.floats(0.02, 3.0), min_size=1, max_size=3)))) * hw1
    a, b = draw(st.floats(0.05, 2.0)), draw(st.floats(0.05, 2.0))
    thy = np.array([-b, -a, 0.0, a, b]) / gamma
    thx = np.array(sorted(draw(st.lists(st.floats(-2.0, 2.0), min_size=1, max_size=3)))) / gamma
    return seg, hw, thx, thy


@settings(max_examples=30, deadline=None)
@given(cases())
def test_planar_motion_is_mirror_symmetric_and_nonnegative(c):
    seg, hw, thx, thy = c
    seg["energy_eV"] = 4.0 * float(hw.max())
    sp = oracle.spectrum(seg, hw, thx, thy, KINDS)
    for k, cube in sp.items():
        assert np.all(cube >= 0.0), k
        assert np.array_equal(cube, cube[:, ::-1, :]), k          # thy -> -thy, bit for bit


@settings(max_examples=25, deadline=None)
@given(cases(), st.floats(0.1, 3.0))
def test_time_shift_leaves_spectra_unchanged(c, shift):
    seg, hw, thx, thy = c
    seg["energy_eV"] = 4.0 * float(hw.max())
    a = oracle.spectrum(seg, hw, thx, thy, KINDS)
    moved = dict(seg)
    moved["t"] = seg["t"] + shift * (seg["t"][-1] - seg["t"][0])
    b = oracle.spectrum(moved, hw, thx, thy, KINDS)
    for k in a:
        scale = max(float(np.abs(a[k]).max()), 1e-300)
        assert float(np.abs(a[k] - b[k]).max()) <= 1e-9 * scale, k


@settings(max_examples=25, deadline=None)
@given(cases())
def test_quantum_spectra_tend_to_the_classical_one(c):
    seg, hw, thx, thy = c
    seg["energy_eV"] = 1e13 * float(hw.max())                 # hw / E <= 1e-13
    sp = oracle.spectrum(seg, hw, thx, thy, KINDS)
    cl = sp[oracle.KIND_CLASSICAL]
    scale = max(float(cl.max()), 1e-300)
    for k in (oracle.KIND_SPIN0, oracle.KIND_SPINHALF):
        assert float(np.abs(sp[k] - cl).max()) <= 1e-9 * scale, k
