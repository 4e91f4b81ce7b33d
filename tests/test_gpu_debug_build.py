"""The index-checking debug build (librad_debug.so, -DRAD_DEBUG=1) on ordinary parity
cases: the same results as the oracle, and not one descriptor, chunk or partial-amplitude
index outside its launch's bounds (rad_debug_violations)."""
import os

import numpy as np
import pytest

import oracle
from parity import assert_parity
from paper_1910_10391_amd.synth import analytic, channeling

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
DEBUG_LIB = os.path.join(ROOT, "paper_1910_10391_amd", "librad_debug.so")


@pytest.fixture
def dbg(monkeypatch):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1910_10391_amd import rad
    D = rad.load(DEBUG_LIB)
    monkeypatch.setattr(rad, "_lib", D)          # every binding call below goes to the debug build
    assert D.rad_debug_violations(1) == 0
    yield rad, D


def test_debug_build_parity_without_index_violations(dbg):
    rad, D = dbg
    cfg = channeling.ChannelingConfig(energy_eV=50e9, charge=-1.0, length_m=30e-6, n_min=2000, n_max=7000,
                                      n_sections=3, seed=9)
    trs = channeling.generate(cfg, 3, threads=1)
    segs, idx = [], []
    for p, secs in enumerate(trs):
        for s in secs:
            segs.append(s)
            idx.append(p)
    g = segs[0]["gamma"]
    hw = analytic.log_omega(70, 1e6, 20e9)
    th = analytic.cell_centred(16, 4.0 / g)
    grid = rad.Grid(hw, th, th)
    ref = oracle.batch(segs, idx, 3, hw, th, th, 7)
    out = rad.batch(grid, segs, idx, 3, 7).cpu().numpy()
    plan = rad.Plan(grid, segs, idx, 3, 7, precision=rad.MIXED)
    outp = plan.launch().cpu().numpy()
    for o in range(3):
        for i in range(3):
            assert_parity(out[o, i], ref[o, i], th, th, 1e-9, "debug build traj %d kind %d" % (o, i))
            assert_parity(outp[o, i], ref[o, i], th, th, 1e-4, "debug build mixed plan traj %d kind %d" % (o, i))
    # the cell path of the sampler: a sparse mask over 8 x 8 cells
    mask = np.zeros((len(segs), 70, 4), dtype=np.uint8)
    mask[0, :30, 1] = 1
    mask[4, 40:, :] = 1
    cells = rad.cells(grid, segs, rad.SPINHALF, mask).cpu().numpy()
    w = oracle.angle_weights(th)
    fine = oracle.spectrum(segs[4], hw, th, th, 4)[4]
    want = np.einsum("wyx,y,x->w", fine.reshape(70, 2, 8, 2, 8)[:, 1, :, 0, :], w[8:], w[:8])
    assert np.allclose(cells[4, 40:, 2], want[40:], rtol=1e-9, atol=0)
    # the same cells with the mask on the device: the kernels read it, skipping blocks
    import torch
    cells_d = rad.cells(grid, segs, rad.SPINHALF, torch.from_numpy(mask).cuda()).cpu().numpy()
    assert np.abs(cells_d - cells).max() <= 1e-12 * np.abs(cells).max() and not cells_d[mask == 0].any()
    plan.close()
    grid.close()
    n = D.rad_debug_violations(0)
    print("debug build: %d index violations" % n)
    assert n == 0
