"""A seeded sweep of small configurations against the oracle: photon-energy counts from 1
to past four blocks of 64, direction grids from 1 x 1 to 13 x 13 (uniform, which takes the
phase recurrence, or irregular), one to four segments of 2 to 2500 samples summed into
one or more outputs, the trapezoid default or explicit weights, every subset of the
kinds, both precisions and the three launch forms (one block per item, the persistent
plan, its graph replay), with photon energies above the particle energy now and then
(forbidden: exact zeros of the quantum spectra).  Each case element by element within the precision's
tolerance and the pointwise bound (parity.py)."""
import dataclasses

import numpy as np
import pytest

import oracle
from parity import assert_parity
from paper_1910_10391_amd.synth import analytic, channeling, presets

pytestmark = pytest.mark.gpu

N_CASES = 24
FP64_TOL = 1e-9
MIXED_TOL = 1e-4


@pytest.fixture(scope="module")
def rad():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1910_10391_amd import rad as r
    r.lib()
    return r


def _segments(rng, n_segs):
    cfg = dataclasses.replace(presets.positron_config(seed=int(rng.integers(1 << 30))), length_m=3e-6,
                              n_min=1, n_max=2500, n_sections=1)
    segs = [tr[0] for tr in channeling.generate(cfg, n_segs, first=int(rng.integers(1000)), threads=4)]
    for s in segs:
        if rng.random() < 0.3:                    # explicit weights: a random positive rule
            s["w"] = rng.uniform(0.5, 1.5, s["t"].size) * (s["t"][-1] - s["t"][0]) / max(s["t"].size - 1, 1)
    return cfg, segs


def _axis(rng, n, half):
    if n == 1 or rng.random() < 0.6:
        return analytic.cell_centred(n, half)     # uniform: the phase recurrence
    return np.sort(rng.uniform(-half, half, n))  # irregular: the direct phase factors


def _case(rng):
    n_w = int(rng.choice([1, 7, 63, 64, 65, 129, 200, 257]))
    n_x, n_y = (int(v) for v in rng.integers(1, 14, 2))
    n_segs = int(rng.integers(1, 5))
    n_out = int(rng.integers(1, n_segs + 1))
    out_index = sorted(int(v) for v in rng.integers(0, n_out, n_segs))
    out_index[:n_out] = list(range(n_out))       # every output gets a segment
    kinds = int(rng.integers(1, 8))
    prec = int(rng.integers(0, 2))
    form = ("batch", "plan", "graph")[int(rng.integers(0, 3))]
    forbidden = n_w > 1 and rng.random() < 0.3
    return n_w, n_x, n_y, n_segs, n_out, sorted(out_index), kinds, prec, form, forbidden


def _energies(rng, n_w, E, forbidden):
    """Photon energies up to half the particle energy, or, with forbidden photons, up to
    0.9 E and a fifth of them in [1.1 E, 2 E] (the endpoint itself, where kappa* diverges,
    has its own test)."""
    if n_w == 1:
        return np.array([0.37 * E])
    if not forbidden:
        return analytic.log_omega(n_w, 1e5, float(rng.choice([5e8, 0.5 * E])))
    k = max(1, n_w // 5)
    return np.concatenate([analytic.log_omega(n_w - k, 1e5, 0.9 * E), np.geomspace(1.1 * E, 2.0 * E, k)])


@pytest.mark.parametrize("case", range(N_CASES))
def test_random_configuration(rad, case):
    import torch
    rng = np.random.default_rng(7000 + case)
    n_w, n_x, n_y, n_segs, n_out, out_index, kinds, prec, form, forbidden = _case(rng)
    cfg, segs = _segments(rng, n_segs)
    g = cfg.energy_eV / oracle.ME_EV
    hw = _energies(rng, n_w, cfg.energy_eV, forbidden)
    thx, thy = _axis(rng, n_x, 5.0 / g), _axis(rng, n_y, 5.0 / g)
    label = "case %d: w %d, %d x %d, %d segments (n %s) into %d, kinds %d, %s, %s" % (
        case, n_w, n_x, n_y, n_segs, [s["t"].size for s in segs], n_out, kinds,
        "mixed" if prec else "fp64", form)
    print(label, flush=True)
    grid = rad.Grid(hw, thx, thy)
    if form == "batch":
        out = rad.batch(grid, segs, out_index, n_out, kinds, precision=prec)
    else:
        side = torch.cuda.Stream()
        with torch.cuda.stream(side):
            plan = rad.Plan(grid, segs, out_index, n_out, kinds, precision=prec, stream=side)
            out = plan.launch(stream=side) if form == "plan" else plan.launch_graph(stream=side)
            side.synchronize()
            if form == "graph":                   # a second replay equals the first
                again = plan.launch_graph(torch.empty_like(out), stream=side)
                side.synchronize()
                assert torch.equal(again, out), label
            plan.close()
    out = out.cpu().numpy()
    ref = oracle.batch(segs, out_index, n_out, hw, thx, thy, kinds)
    tol = MIXED_TOL if prec else FP64_TOL
    for o in range(n_out):
        for i in range(ref.shape[1]):
            assert_parity(out[o, i], ref[o, i], thx, thy, tol, "%s, output %d kind %d" % (label, o, i))
    grid.close()


@pytest.mark.parametrize("prec", [0, 1])
def test_smallest_configuration(rad, prec):
    """One photon energy, one direction, a 2-sample segment beside a longer one, all
    kinds, every form."""
    import torch
    cfg = dataclasses.replace(presets.positron_config(seed=5), length_m=2e-6, n_min=1, n_max=1, n_sections=1)
    short = channeling.generate(cfg, 1, threads=1)[0][0]
    assert short["t"].size == 2
    cfg2 = dataclasses.replace(cfg, n_min=700, n_max=700)
    segs = [short, channeling.generate(cfg2, 1, first=3, threads=1)[0][0]]
    hw, th = np.array([2.5e8]), np.array([1.3e-5])
    grid = rad.Grid(hw, th, th)
    ref = oracle.batch(segs, [0, 1], 2, hw, th, th, 7)
    tol = MIXED_TOL if prec else FP64_TOL
    outs = [rad.batch(grid, segs, [0, 1], 2, 7, precision=prec).cpu().numpy()]
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        plan = rad.Plan(grid, segs, [0, 1], 2, 7, precision=prec, stream=side)
        outs.append(plan.launch(stream=side).cpu().numpy())
        outs.append(plan.launch_graph(stream=side).cpu().numpy())
        plan.close()
    for f, out in zip(("batch", "plan", "graph"), outs):
        for o in range(2):
            for i in range(3):
                assert_parity(out[o, i], ref[o, i], th, th, tol, "1 x 1 x 1, %s, output %d kind %d" % (f, o, i))
    grid.close()
