"""The GPU trajectory generator against the CPU generator (same model, same random
streams), and the radiation integrals of GPU trajectories against the oracle."""
import dataclasses

import numpy as np
import pytest

import oracle
from paper_1910_10391_amd.synth import analytic, channeling, presets

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def T():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1910_10391_amd import traj
    return traj


def _compare(gpu, cpu, label):
    """Every column bit for bit: the GPU generator takes the CPU generator's steps in the
    same order without FMA contraction, and draws its normals with the same IEEE-only
    logarithm and cosine, so not even the side of a plane's kink a step lands on can
    differ."""
    for c in ("t", "x", "y", "dz", "vx", "vy", "dvz", "ax", "ay", "az", "energy"):
        a, b = gpu[c], cpu[c]
        assert a.shape == b.shape, (label, c)
        assert np.all(np.isfinite(a)), (label, c)
        if not np.array_equal(a, b):
            k = int(np.argmax(a != b))
            raise AssertionError("%s: column %s differs first at sample %d of %d (%r vs %r)"
                                 % (label, c, k, len(b), a[k], b[k]))


def test_generator_harmonic_closed_form(T):
    """The GPU generator against the closed form of its model directly: q = 0, no
    scattering, no loss, small amplitude, x = A sin(W t + phi), W^2 = 8 U0 / (E d^2)."""
    cfg = dataclasses.replace(presets.positron_config(seed=21), length_m=50e-6, n_min=20000, n_max=20000,
                              q=0.0, ms_on=False, loss_on=False, theta_sigma=1e-9)
    W = np.sqrt(8 * cfg.U0_eV / (cfg.energy_eV * cfg.d_m ** 2))
    dt = T.DeviceTrajectories(cfg, 4)
    for i in range(4):
        tr = dt.host(i)
        x0, v0 = tr["x"][0], tr["vx"][0]
        A = np.hypot(x0, v0 / W)
        ref = x0 * np.cos(W * tr["t"]) + v0 / W * np.sin(W * tr["t"])
        assert np.abs(tr["x"] - ref).max() < 1e-8 * A
        assert np.all(tr["energy"] == cfg.energy_eV)


def test_generator_matches_cpu(T):
    for charge, seed in ((+1.0, 4), (-1.0, 5)):
        cfg = dataclasses.replace(presets.positron_config(seed=seed, charge=charge), length_m=20e-6,
                                  n_min=3000, n_max=9000)
        dt = T.DeviceTrajectories(cfg, 6, first=17)
        assert np.array_equal(np.array(dt.n) - 1, channeling.lengths(cfg, 6, first=17))
        for i in range(6):
            _compare(dt.host(i), channeling.trajectory(cfg, 17 + i), "charge %+d particle %d" % (charge, i))


def test_generator_switches_and_edges(T):
    base = dataclasses.replace(presets.positron_config(seed=8), length_m=5e-6, n_min=1, n_max=3)
    for kw in (dict(ms_on=False), dict(loss_on=False), dict(ms_on=False, loss_on=False), dict(q=0.0),
               dict(q=1.0), dict(theta_sigma=0.0), dict(n_min=1, n_max=1)):
        cfg = dataclasses.replace(base, **kw)
        dt = T.DeviceTrajectories(cfg, 5)
        for i in range(5):
            _compare(dt.host(i), channeling.trajectory(cfg, i), str(kw))


def test_generator_full_size(T):
    """The 256-particle positron workload at full length (40 082 to 119 975 samples, through
    plane crossings, scattering and radiative loss) and 64 particles of the 50 GeV electron
    workload: every trajectory bit for bit the CPU generator's."""
    for cfg, n in ((presets.positron_config(), 256), (presets.electron_50gev_config(), 64)):
        dt = T.DeviceTrajectories(cfg, n)
        for i in range(n):
            _compare(dt.host(i), channeling.trajectory(cfg, i), "full size particle %d (n %d)" % (i, dt.n[i]))
        print("%d full-length trajectories bitwise equal (%d samples)" % (n, sum(dt.n) + n), flush=True)


def test_spectrum_of_gpu_trajectories_matches_oracle(T):
    """GPU trajectories straight into the radiation integrals (no host round trip),
    against the oracle on the same trajectories (FP64 spin-1/2), and against the
    oracle on the CPU generator's trajectories."""
    from paper_1910_10391_amd import rad
    cfg = dataclasses.replace(presets.positron_config(seed=12), length_m=10e-6, n_min=2000, n_max=4000)
    dt = T.DeviceTrajectories(cfg, 3)
    g = cfg.energy_eV / oracle.ME_EV
    hw = analytic.log_omega(37, 0.5e6, 200e6)
    th = analytic.cell_centred(7, 5.0 / g)
    grid = rad.Grid(hw, th, th)
    got = rad.batch(grid, dt, [0, 1, 2], 3, rad.SPINHALF, rad.FP64).cpu().numpy()[:, 0]
    for i in range(3):
        mine = dt.host(i)
        mine.update(gamma=g, energy_eV=cfg.energy_eV, w=None)
        ref = oracle.spectrum(mine, hw, th, th, oracle.KIND_SPINHALF)[oracle.KIND_SPINHALF]
        err = float(np.linalg.norm(got[i] - ref) / np.linalg.norm(ref))
        seg = channeling.sections(cfg, channeling.trajectory(cfg, i))[0]
        ref_cpu = oracle.spectrum(seg, hw, th, th, oracle.KIND_SPINHALF)[oracle.KIND_SPINHALF]
        err_cpu = float(np.linalg.norm(got[i] - ref_cpu) / np.linalg.norm(ref_cpu))
        print("spectrum of GPU trajectory %d: M1 %.2e (oracle on the same trajectory), %.2e (on the CPU "
              "generator's)" % (i, err, err_cpu), flush=True)
        assert err < 1e-9
        assert err_cpu == err             # the same trajectory, bit for bit


def test_sections_match_cpu_cut(T):
    """Sections cut on the GPU (entry gamma per section, dz and dvz re-referenced)
    against the CPU cut of the CPU generator's trajectories; then the incoherent
    section sum of the spectrum against the oracle on the GPU's own sections."""
    from paper_1910_10391_amd import rad
    cfg = dataclasses.replace(presets.electron_50gev_config(seed=6), length_m=40e-6, n_min=3000, n_max=7000)
    assert cfg.n_sections == 10
    dt = T.DeviceTrajectories(cfg, 3, first=2)
    assert dt.out_index == [i for i in range(3) for _ in range(10)]
    assert len(dt.n) == 30
    for i in range(3):
        cpu_secs = channeling.sections(cfg, channeling.trajectory(cfg, 2 + i))
        assert len(cpu_secs) == 10
        for s in range(10):
            g = dt.segment_host(10 * i + s)
            c = cpu_secs[s]
            assert g["t"].size == c["t"].size
            assert g["gamma"] == c["gamma"] and g["energy_eV"] == c["energy_eV"]
            c = dict(c, energy=np.zeros_like(c["t"]))
            g["energy"] = np.zeros_like(g["t"])
            _compare(g, c, "particle %d section %d" % (i, s))
    g0 = cfg.energy_eV / oracle.ME_EV
    hw = analytic.log_omega(21, 1e6, 20e9)
    th = analytic.cell_centred(5, 4.0 / g0)
    grid = rad.Grid(hw, th, th)
    got = rad.batch(grid, dt, dt.out_index, 3, rad.SPINHALF, rad.FP64).cpu().numpy()[:, 0]
    segs = [dt.segment_host(j) for j in range(30)]
    ref = oracle.batch(segs, dt.out_index, 3, hw, th, th, oracle.KIND_SPINHALF)[:, 0]
    err = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
    print("sections spectrum: M1 %.2e" % err, flush=True)
    assert err < 1e-9
