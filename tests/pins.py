"""Pins of the CPU oracle against facts that do not come from the oracle itself.

Each ``pin_*`` function raises AssertionError when the oracle disagrees with a
closed form, an identity, a brute-force evaluation of the unexpanded formula,
or a value the paper prints.  They run against whatever build of the oracle is
active (``oracle.use_library``), so the mutation test can show that planted
mistakes fail at least one of them.

Independent references used here:
* textbook closed forms via SciPy Bessel functions (undulator harmonics,
  synchrotron K_{2/3}/K_{1/3}),
* the exact 3-D vector forms of Sec. II eq. (integralrad1)-(integralrad2) and
  eq. (Iterm), written with NumPy cross products on unexpanded n, beta, r,
* integration by parts (f = d/dt[n x (n x beta)/(1 - n.beta)],
  n.beta_dot/(1 - n.beta)^2 = d/dt[1/(1 - n.beta)], d/dt(t - n.r) = 1 - n.beta),
* Parseval's theorem for the frequency integral,
* the grating factor of an N-period motion,
* the paper's undulator example (Sec. IV, Fig. 2): 2 GeV, 53 mm, N = 20,
  B0 = 1 T, a peak at 380 eV (``tests/golden/paper_undulator.json``).
"""
from __future__ import annotations

import json
import math
import os

import numpy as np
from scipy.integrate import simpson
from scipy.special import jv, kv

import oracle
from paper_1910_10391_amd.synth import analytic

HBARC = 1.973269804e-7
PREF = 7.2973525693e-3 / (4.0 * math.pi ** 2)
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _rel(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))) / np.max(np.abs(b)))


def _trap(t):
    w = np.empty_like(t)
    w[1:-1] = 0.5 * (t[2:] - t[:-2])
    w[0] = 0.5 * (t[1] - t[0])
    w[-1] = 0.5 * (t[-1] - t[-2])
    return w


def exact_vectors(seg, nx, ny):
    """Unexpanded n, beta, beta_dot, r of a segment and the exact LW pieces."""
    g = seg["gamma"]
    b0 = 1.0 - 1.0 / (2.0 * g * g)
    n = np.array([nx, ny, math.sqrt(1.0 - nx * nx - ny * ny)])
    beta = np.stack([seg["vx"], seg["vy"], b0 + seg["dvz"]], 1)
    bdot = np.stack([seg["ax"], seg["ay"], seg["az"]], 1)
    r = np.stack([seg["x"], seg["y"], b0 * seg["t"] + seg["dz"]], 1)
    D = 1.0 - beta @ n
    f = np.cross(n, np.cross(n - beta, bdot)) / (D * D)[:, None]
    nnb = np.cross(n, np.cross(n, beta))
    psi = seg["t"] - r @ n
    return dict(n=n, beta=beta, bdot=bdot, D=D, f=f, nnb=nnb, psi=psi)


# ---------------------------------------------------------------- P1
def pin_uniform_motion_zero():
    """No acceleration, no radiation: every kind is exactly zero (Sec. II eq. (integralrad2))."""
    seg = analytic.uniform(1e4, 3e-5, -2e-5, 1e-4, n_steps=1000)
    seg["energy_eV"] = 5e9
    hw = np.array([1e3, 1e5, 1e6, 4e9, 6e9])
    th = np.array([-2e-4, 0.0, 1e-4])
    sp = oracle.spectrum(seg, hw, th, th, 7)
    for k, cube in sp.items():
        assert np.all(cube == 0.0), "kind %d not zero for uniform motion" % k
    A, J = oracle.amplitudes(seg, [1e12, 3e13], [1e-4, -2e-4], [5e-5, 0.0])
    assert np.all(A == 0) and np.all(J == 0)


# ---------------------------------------------------------------- P2
def pin_grating_identity():
    """N periods of a periodic motion (rectangle rule over whole periods):
    S_N = S_1 sin^2(N Phi/2) / sin^2(Phi/2), Phi = kappa lambda (1+K^2/2+g^2 th^2)/(2 g^2)."""
    g, K, lam = 2e4, 0.5, 20e-6
    nx, ny = 0.6 / g, -0.3 / g
    s1 = analytic.undulator(g, K, lam, 1, samples_per_period=64, rule="rect")
    s7 = analytic.undulator(g, K, lam, 7, samples_per_period=64, rule="rect")
    k1 = analytic.undulator_fundamental_eV(g, K, lam) / HBARC
    ks = np.array([0.37, 0.93, 1.41]) * k1
    A1, _ = oracle.amplitudes(s1, ks, [nx], [ny], want_j=False)
    A7, _ = oracle.amplitudes(s7, ks, [nx], [ny], want_j=False)
    S1 = np.sum(np.abs(A1[:, 0]) ** 2, 1)
    S7 = np.sum(np.abs(A7[:, 0]) ** 2, 1)
    Phi = ks * lam * (1 + K * K / 2 + (g * g) * (nx * nx + ny * ny)) / (2 * g * g)
    pred = S1 * np.sin(7 * Phi / 2) ** 2 / np.sin(Phi / 2) ** 2
    assert _rel(S7, pred) < 1e-10, (S7, pred)


# ---------------------------------------------------------------- P3
def pin_undulator_peak_bessel():
    """On-axis undulator harmonics (velocity form, boundary terms cancel at w_h):
    S(w_h, 0) = [2 pi N h gamma K JJ_h/(1+K^2/2)]^2, JJ_h = J_{(h-1)/2}(xi) - J_{(h+1)/2}(xi),
    xi = h K^2/(4(1+K^2/2)); even harmonics vanish on axis."""
    g, K, lam, N = 2e4, 0.5, 20e-6, 20
    seg = analytic.undulator(g, K, lam, N, samples_per_period=512, rule="rect")
    hw1 = analytic.undulator_fundamental_eV(g, K, lam)
    hw = np.array([hw1, 2 * hw1, 3 * hw1])
    S = oracle.spectrum(seg, hw, [0.0], [0.0], 1)[1][:, 0, 0] / PREF
    for i, h in ((0, 1), (2, 3)):
        xi = h * K * K / (4 * (1 + K * K / 2))
        JJ = jv((h - 1) // 2, xi) - jv((h + 1) // 2, xi)
        ref = (2 * math.pi * N * h * g * K * JJ / (1 + K * K / 2)) ** 2
        assert abs(S[i] / ref - 1) < 1e-12, (h, S[i], ref)
    assert S[1] < 1e-20 * S[0]


# ---------------------------------------------------------------- P4
def pin_harmonic_positions():
    """Peaks at w_h(theta) = h 2 g^2 w0 / (1 + K^2/2 + g^2 theta^2) within 0.25 %."""
    g, K, lam = 2e4, 0.5, 20e-6
    seg = analytic.undulator(g, K, lam, 20, n_steps=8192)
    cases = [((0.0, 0.0), 1), ((0.0, 0.0), 3), ((0.5 / g, 0.0), 2), ((0.0, 0.5 / g), 1),
             ((0.9 / g, 0.9 / g), 1), ((0.9 / g, 0.9 / g), 2), ((0.5 / g, 0.0), 3)]
    for (tx, ty), h in cases:
        hh = h * analytic.undulator_fundamental_eV(g, K, lam, math.hypot(tx, ty))
        hw = np.linspace(0.97 * hh, 1.03 * hh, 301)
        s = oracle.spectrum(seg, hw, [tx], [ty], 1)[1][:, 0, 0]
        i = int(np.argmax(s))
        assert 0 < i < hw.size - 1, "no interior peak"
        assert abs(hw[i] / hh - 1) < 2.5e-3, ((tx, ty), h, hw[i] / hh - 1)


# ---------------------------------------------------------------- P5
def pin_synchrotron_jackson():
    """Circular arc vs the single-passage synchrotron spectrum (Jackson):
    S = (4/3)(wR)^2 (1/g^2+psi^2)^2 [K_{2/3}^2(xi) + psi^2/(1/g^2+psi^2) K_{1/3}^2(xi)],
    xi = (wR/3)(1/g^2+psi^2)^{3/2}."""
    g, R = 1e4, 1.0
    seg = analytic.arc(g, R, 60.0, 60000)
    wc = 1.5 * g ** 3 / R
    for y in (0.05, 0.3, 1.0):
        for gpsi in (0.0, 0.7):
            k, psi = y * wc, gpsi / g
            A, _ = oracle.amplitudes(seg, [k], [0.0], [psi], want_j=False)
            S = float(np.sum(np.abs(A) ** 2))
            a = 1 / g ** 2 + psi ** 2
            xi = k * R / 3 * a ** 1.5
            ref = (4 / 3) * (k * R) ** 2 * a * a * (kv(2 / 3, xi) ** 2 + psi ** 2 / a * kv(1 / 3, xi) ** 2)
            assert abs(S / ref - 1) < 2e-4, (y, gpsi, S / ref - 1)


# ---------------------------------------------------------------- P6
def pin_sum_rule():
    """Parseval with u = psi(t), dpsi/dt = 1 - n.beta:
    int_0^inf S dkappa = pi sum_k w_k |f_k|^2 / (1 - n.beta_k), with f and 1 - n.beta
    from the exact vectors."""
    g, K, lam = 2e4, 0.5, 20e-6
    seg = analytic.undulator(g, K, lam, 4, n_steps=4 * 2048)
    nx, ny = 0.4 / g, 0.2 / g
    k1 = analytic.undulator_fundamental_eV(g, K, lam) / HBARC
    ks = np.linspace(0.0, 12 * k1, 6001)
    A, _ = oracle.amplitudes(seg, ks, [nx], [ny], want_j=False)
    lhs = simpson(np.sum(np.abs(A[:, 0, :]) ** 2, 1), x=ks)
    ev = exact_vectors(seg, nx, ny)
    rhs = math.pi * np.sum(_trap(seg["t"]) * np.sum(ev["f"] ** 2, 1) / ev["D"])
    assert abs(lhs / rhs - 1) < 1e-4, lhs / rhs - 1


# ---------------------------------------------------------------- P7
def pin_transversality():
    """n.A = 0: nx A_x + ny A_y + A_z vanishes (n is perpendicular to f)."""
    g = 2e4
    seg = analytic.wiggle3d(g, 20e-6, 3.0, 6000)
    nx = np.array([0.7, -1.3, 2.1]) / g
    ny = np.array([-0.45, 0.8, 1.7]) / g
    k1 = analytic.undulator_fundamental_eV(g, 1.0, 20e-6) / HBARC
    A, _ = oracle.amplitudes(seg, np.array([0.6, 1.3, 2.7]) * k1, nx, ny, want_j=False)
    for j in range(nx.size):
        res = nx[j] * A[:, j, 0] + ny[j] * A[:, j, 1] + A[:, j, 2]
        scale = np.abs(A[:, j, 2])
        assert np.all(np.abs(res) < 1e-9 * scale), (j, np.abs(res) / scale)


# ---------------------------------------------------------------- velocity form
def _wiggle_case():
    g, lam = 2e4, 20e-6
    seg = analytic.wiggle3d(g, lam, 3.0, 60000)
    k1 = analytic.undulator_fundamental_eV(g, 1.0, lam) / HBARC
    return seg, np.array([0.6, 1.3, 2.7]) * k1, [(0.7 / g, -0.45 / g), (-1.1 / g, 0.3 / g)]


def pin_velocity_form():
    """Integration by parts, f = d/dt[n x (n x beta)/(1 - n.beta)]:
    A = [n x (n x beta)/(1-n.beta) e^{i kappa psi}]_ends - i kappa int n x (n x beta) e^{i kappa psi} dt,
    per component, with the right side from the exact vectors (no acceleration used)."""
    seg, ks, dirs = _wiggle_case()
    w = _trap(seg["t"])
    for nx, ny in dirs:
        A, _ = oracle.amplitudes(seg, ks, [nx], [ny], want_j=False)
        ev = exact_vectors(seg, nx, ny)
        V = ev["nnb"] / ev["D"][:, None]
        for i, k in enumerate(ks):
            e = np.exp(1j * k * ev["psi"])
            rhs = V[-1] * e[-1] - V[0] * e[0] - 1j * k * np.sum(w[:, None] * ev["nnb"] * e[:, None], 0)
            err = np.abs(A[i, 0] - rhs) / np.abs(rhs)
            assert np.all(err < 2e-5), ((nx, ny), i, err)


def pin_j_by_parts():
    """n.beta_dot/(1-n.beta)^2 = d/dt[1/(1-n.beta)], so
    J = [e^{i kappa psi}/(1-n.beta)]_ends - i kappa int e^{i kappa psi} dt."""
    seg, ks, dirs = _wiggle_case()
    w = _trap(seg["t"])
    for nx, ny in dirs:
        _, J = oracle.amplitudes(seg, ks, [nx], [ny], want_j=True)
        ev = exact_vectors(seg, nx, ny)
        for i, k in enumerate(ks):
            e = np.exp(1j * k * ev["psi"])
            rhs = e[-1] / ev["D"][-1] - e[0] / ev["D"][0] - 1j * k * np.sum(w * e)
            assert abs(J[i, 0] - rhs) / abs(rhs) < 2e-5, ((nx, ny), i, abs(J[i, 0] - rhs) / abs(rhs))


# ---------------------------------------------------------------- P9
def pin_exact_lw_scaling():
    """Brute force of the unexpanded eq. (integralrad1)-(integralrad2) at moderate gamma:
    the expansion error in S is O(1/gamma^2) -- small, and ~4x smaller per doubling."""
    errs = []
    for g in (40.0, 80.0):
        lam = 20e-6
        seg = analytic.wiggle3d(g, lam, 2.0, 20000)
        nx, ny = 0.7 / g, -0.45 / g
        k1 = analytic.undulator_fundamental_eV(g, 1.0, lam) / HBARC
        ks = np.array([0.7, 1.0, 1.6]) * k1
        A, _ = oracle.amplitudes(seg, ks, [nx], [ny], want_j=False)
        ev = exact_vectors(seg, nx, ny)
        w = _trap(seg["t"])
        e = []
        for i, k in enumerate(ks):
            Aex = np.sum(w[:, None] * ev["f"] * np.exp(1j * k * ev["psi"])[:, None], 0)
            S, Sex = np.sum(np.abs(A[i, 0]) ** 2), np.sum(np.abs(Aex) ** 2)
            e.append(abs(S - Sex) / Sex)
        errs.append(max(e))
    assert errs[0] < 5e-3 and errs[1] < 1.3e-3, errs
    assert 3.0 < errs[0] / errs[1] < 5.5, errs


# ---------------------------------------------------------------- P8
def pin_quantum_composition():
    """Spin-0 = (E*/E) S_cl(w*) (Sec. II eq. (Lindhard_substi)); spin-1/2 = BCK weights
    (Sec. II eq. (cue)); both reduce to the classical spectrum as E -> infinity and vanish
    for hw >= E."""
    g, K, lam = 2e4, 0.5, 20e-6
    seg = analytic.undulator(g, K, lam, 5, n_steps=5 * 256)
    E = 10.22e9
    seg["energy_eV"] = E
    hw1 = analytic.undulator_fundamental_eV(g, K, lam)
    hw = np.array([0.3, 0.9, 1.7]) * hw1
    th = np.array([-0.4 / g, 0.25 / g])
    q = oracle.spectrum(seg, hw, th, th, 7)
    hws = hw * E / (E - hw)
    cl_star = oracle.spectrum(seg, hws, th, th, 1)[1]
    Es = E - hw
    assert _rel(q[2], (Es / E)[:, None, None] * cl_star) < 1e-11
    kst = hw / HBARC * E / (E - hw)
    nx = np.repeat(th[None, :], 2, 0).ravel()
    ny = np.repeat(th[:, None], 2, 1).ravel()
    _, J = oracle.amplitudes(seg, kst, nx, ny)
    SJ = (np.abs(J) ** 2).reshape(3, 2, 2)
    wI = ((Es ** 2 + E ** 2) / (2 * E ** 2))[:, None, None]
    wJ = (hw ** 2 / (2 * E ** 2 * g ** 2))[:, None, None]
    assert _rel(q[4], wI * cl_star + PREF * wJ * SJ) < 1e-11
    # J term is not negligible here, so a wrong J weight would show
    assert np.max(PREF * wJ * SJ) > 1e-6 * np.max(q[4])
    # classical limit
    seg["energy_eV"] = 1e30
    ql = oracle.spectrum(seg, hw, th, th, 7)
    assert _rel(ql[2], ql[1]) < 1e-12 and _rel(ql[4], ql[1]) < 1e-12
    # kinematically forbidden photons
    seg["energy_eV"] = 1.0 * hw1
    qf = oracle.spectrum(seg, hw, th, th, 6)
    assert np.all(qf[2][2] == 0) and np.all(qf[4][2] == 0)
    assert np.all(qf[2][:2] > 0) and np.all(qf[4][:2] > 0)


# ---------------------------------------------------------------- quadrature
def pin_trapezoid_rule():
    """Default weights are the textbook trapezoid rule from t (non-uniform t allowed)."""
    g = 2e4
    seg = analytic.wiggle3d(g, 20e-6, 1.0, 500)
    rng = np.random.default_rng(7)
    t = np.sort(seg["t"][0] + (seg["t"][-1] - seg["t"][0]) * rng.random(seg["t"].size))
    t[0], t[-1] = seg["t"][0], seg["t"][-1]
    seg = dict(seg)
    seg["t"] = t
    wt = np.zeros_like(t)
    for i in range(t.size - 1):          # interval by interval
        wt[i] += 0.5 * (t[i + 1] - t[i])
        wt[i + 1] += 0.5 * (t[i + 1] - t[i])
    k1 = analytic.undulator_fundamental_eV(g, 1.0, 20e-6) / HBARC
    A0, J0 = oracle.amplitudes(seg, [0.8 * k1], [1e-5], [-2e-5])
    seg["w"] = wt
    A1, J1 = oracle.amplitudes(seg, [0.8 * k1], [1e-5], [-2e-5])
    assert _rel(A0, A1) < 1e-13 and _rel(J0, J1) < 1e-13


def pin_angle_integrate():
    """Midpoint sum over the angular cells (Sec. IV host sum)."""
    th = analytic.cell_centred(8, 3e-4)
    cube = np.ones((2, 8, 8))
    assert np.allclose(oracle.angle_integrate(cube, th, th), (6e-4) ** 2, rtol=1e-13)
    lin = np.ones((1, 8, 1)) * th[None, None, :]
    assert abs(oracle.angle_integrate(lin, th, th)[0]) < 1e-20
    thy = np.array([0.0, 1.0, 3.0])
    wy = oracle.angle_weights(thy)
    assert np.allclose(wy, [1.0, 1.5, 2.0])


def pin_batch_sections():
    """Sections sum incoherently into their output (Sec. II, sections)."""
    g, K, lam = 2e4, 0.5, 20e-6
    s1 = analytic.undulator(g, K, lam, 2, n_steps=512)
    s2 = analytic.undulator(g, K, lam, 3, n_steps=768, t0=2 * lam)
    hw = np.array([0.5, 1.0]) * analytic.undulator_fundamental_eV(g, K, lam)
    th = np.array([0.0, 0.5 / g])
    b = oracle.batch([s1, s2, s1], [1, 0, 1], 2, hw, th, th, 1)
    a1 = oracle.spectrum(s1, hw, th, th, 1)[1]
    a2 = oracle.spectrum(s2, hw, th, th, 1)[1]
    assert _rel(b[0, 0], a2) < 1e-15 and _rel(b[1, 0], 2 * a1) < 1e-15


# ---------------------------------------------------------------- golden
def pin_paper_undulator_380():
    """Sec. IV (Fig. 2): a 2 GeV electron in a 53 mm, 20-period, 1 T undulator radiates a
    forward harmonic at about 380 eV (the 7th); odd harmonics only on axis."""
    with open(os.path.join(GOLDEN, "paper_undulator.json")) as f:
        gold = json.load(f)
    g = gold["energy_eV"] / oracle.ME_EV
    K = analytic.undulator_K(gold["B0_T"], gold["lambda_m"])
    seg = analytic.undulator(g, K, gold["lambda_m"], gold["n_periods"], samples_per_period=512,
                             rule="rect")
    hw = np.linspace(350.0, 410.0, 601)
    s = oracle.spectrum(seg, hw, [0.0], [0.0], 1)[1][:, 0, 0]
    pk = hw[int(np.argmax(s))]
    assert abs(pk / gold["peak_eV"] - 1) < gold["peak_rel_tol"], pk
    hw1 = analytic.undulator_fundamental_eV(g, K, gold["lambda_m"])
    assert abs(pk / (7 * hw1) - 1) < 1e-3
    # even harmonic 6 at 324.7 eV is suppressed on axis relative to the 7th
    s6 = oracle.spectrum(seg, [6 * hw1], [0.0], [0.0], 1)[1][0, 0, 0]
    assert s6 < 1e-6 * s.max()


ALL_PINS = [
    pin_uniform_motion_zero, pin_grating_identity, pin_undulator_peak_bessel,
    pin_harmonic_positions, pin_synchrotron_jackson, pin_sum_rule, pin_transversality,
    pin_velocity_form, pin_j_by_parts, pin_exact_lw_scaling, pin_quantum_composition,
    pin_trapezoid_rule, pin_angle_integrate, pin_batch_sections, pin_paper_undulator_380,
]
