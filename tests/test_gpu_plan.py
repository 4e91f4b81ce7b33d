"""Persistent plans, hipGraph replay and the autotuner (GPU)."""
import os

import numpy as np
import pytest

import oracle
from parity import assert_parity
from paper_1910_10391_amd.synth import analytic, channeling

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rad():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1910_10391_amd import rad as r
    r.lib()
    return r


def _sections(n_particles=4, seed=31):
    cfg = channeling.ChannelingConfig(energy_eV=50e9, charge=-1.0, length_m=40e-6, n_min=3000,
                                      n_max=12000, n_sections=4, seed=seed)
    trs = channeling.generate(cfg, n_particles, threads=1)
    segs, idx = [], []
    for p, secs in enumerate(trs):
        for s in secs:
            segs.append(s)
            idx.append(p)
    return segs, idx


def test_plan_matches_batch_and_oracle(rad):
    segs, idx = _sections()
    g = segs[0]["gamma"]
    hw = analytic.log_omega(80, 1e6, 20e9)
    th = analytic.cell_centred(12, 4.0 / g)
    grid = rad.Grid(hw, th, th)
    ds = rad.DeviceSegments(segs)
    for prec, tol in ((rad.FP64, 1e-9), (rad.MIXED, 1e-4)):
        ref_b = rad.batch(grid, ds, idx, 5, 7, precision=prec).cpu().numpy()
        plan = rad.Plan(grid, ds, idx, 5, 7, precision=prec)
        got = plan.launch().cpu().numpy()
        assert np.all(got[4] == 0)
        for o in range(4):
            for i in range(3):
                a, b = got[o, i], ref_b[o, i]
                assert np.linalg.norm(a - b) <= 1e-13 * np.linalg.norm(b)
        ref = oracle.batch(segs, idx, 5, hw, th, th, 7)
        for o in range(4):
            for i in range(3):
                assert_parity(got[o, i], ref[o, i], th, th, tol, "plan prec %d traj %d kind %d" % (prec, o, i))


def test_graph_replays_equal_eager(rad):
    """Replay the captured graph several times with eager work and syncs in between;
    every replay must equal the eager launch bit for bit."""
    import torch
    segs, idx = _sections(3, seed=37)
    g = segs[0]["gamma"]
    hw = analytic.log_omega(64, 1e6, 20e9)
    th = analytic.cell_centred(8, 4.0 / g)
    grid = rad.Grid(hw, th, th)
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        plan = rad.Plan(grid, segs, idx, 3, rad.SPINHALF, precision=rad.MIXED, stream=side)
        eager = plan.launch(stream=side)
        torch.cuda.synchronize()
        ref = eager.clone()
        out = torch.full_like(eager, -1.0)
        for rep in range(4):
            out.fill_(-1.0)                      # eager work between replays
            plan.launch_graph(out, stream=side)
            side.synchronize()
            assert torch.equal(out, ref), "replay %d differs" % rep
            junk = rad.batch(grid, segs[:1], [0], 1, rad.CLASSICAL, stream=side)   # other eager kernels
            side.synchronize()
            del junk
        again = plan.launch(stream=side)
        side.synchronize()
        assert torch.equal(again, ref)


def test_graph_needs_created_stream(rad):
    segs, idx = _sections(1, seed=41)
    hw = np.array([1e6, 1e7])
    th = np.array([0.0, 1e-5])
    grid = rad.Grid(hw, th, th)
    plan = rad.Plan(grid, segs, idx, 1, rad.SPINHALF)
    import torch
    with pytest.raises(rad.RadError):
        plan.launch_graph(stream=torch.cuda.default_stream())


def test_autotune_picks_and_caches(rad, tmp_path, monkeypatch):
    from paper_1910_10391_amd import autotune
    monkeypatch.setenv("RAD_AUTOTUNE_CACHE", str(tmp_path / "tune.json"))
    segs, idx = _sections(3, seed=43)
    g = segs[0]["gamma"]
    hw = analytic.log_omega(128, 1e6, 20e9)
    th = analytic.cell_centred(16, 4.0 / g)
    grid = rad.Grid(hw, th, th)
    ds = rad.DeviceSegments(segs)
    keys = [(p, m, j) for p in (0, 1) for m in (0, 1) for j in (0, 1)]
    keep = {k: rad.tune_get_variant(*k) for k in keys}
    try:
        for persistent in (False, True):
            res = autotune.tune(grid, ds, 7, rad.MIXED, persistent=persistent, sample=4, min_evals=0,
                                verbose=True)
            fields = sorted(f for r in res.values() for f in ("variant", "wg", "target") if f in r)
            assert fields == ["variant", "variant"], res            # two integral sets; a sample: no shape
            for k, r in res.items():
                assert not r["cached"]
                f = [f for f in ("variant", "wg", "target") if f in r][0]
                if f == "variant":
                    assert r["ms"][str(r[f])] == min(r["ms"].values())
                else:                                     # the planner's own unless clearly beaten
                    assert r["ms"][str(r[f])] <= min(r["ms"].values()) / (1.0 - autotune.MARGIN)
            again = autotune.tune(grid, ds, 7, rad.MIXED, persistent=persistent, sample=4, min_evals=0)
            assert all(r["cached"] for r in again.values()) and len(again) == len(res)
        # a sample that is the whole workload also tunes the spread and the chunk target
        whole = autotune.tune(grid, ds, 7, rad.MIXED, persistent=True, sample=len(segs), min_evals=0,
                              use_cache=False, verbose=True)
        wg = [r for k, r in whole.items() if k.startswith("wg-")]
        tgt = [r for k, r in whole.items() if k.startswith("chunk-")]
        assert len(wg) == 1 and wg[0]["wg"] == rad.tune_get_shape(True, True)
        assert len(tgt) == 1 and tgt[0]["target"] == rad.tune_get_chunk_target()
        assert os.path.exists(tmp_path / "tune.json")
        out = rad.batch(grid, ds, idx, 3, 7, precision=rad.MIXED).cpu().numpy()
        ref = oracle.batch(segs, idx, 3, hw, th, th, 7)
        for o in range(3):
            assert_parity(out[o, 2], ref[o, 2], th, th, 1e-4, "tuned traj %d" % o)
    finally:
        for k in keys:
            rad.tune_set_variant(*k, keep[k])
        for p in (0, 1):
            for m in (0, 1):
                rad.tune_set_shape(p, m, 0)
        rad.tune_set_chunk_target(0)


def test_shape_knobs_keep_results(rad):
    """The spread over photon energies changes no bit of the spectra, in either form and
    precision; the chunk target changes them by rounding only (the chunk sums come in
    another order)."""
    segs, idx = _sections(3, seed=53)
    g = segs[0]["gamma"]
    hw = analytic.log_omega(200, 1e6, 20e9)       # 4 blocks of 64 energies at wg = 1, ragged
    th = analytic.cell_centred(12, 4.0 / g)
    grid = rad.Grid(hw, th, th)
    ds = rad.DeviceSegments(segs)
    try:
        for prec in (rad.FP64, rad.MIXED):
            mixed = prec == rad.MIXED
            ref = rad.batch(grid, ds, idx, 3, 7, precision=prec).cpu().numpy()
            for persistent in (False, True):
                for wg in (1, 2, 4):
                    rad.tune_set_shape(persistent, mixed, wg)
                    if persistent:
                        plan = rad.Plan(grid, ds, idx, 3, 7, precision=prec)
                        out = plan.launch().cpu().numpy()
                        plan.close()
                    else:
                        out = rad.batch(grid, ds, idx, 3, 7, precision=prec).cpu().numpy()
                    assert np.array_equal(out, ref), (prec, persistent, wg)
                rad.tune_set_shape(persistent, mixed, 0)
            for target in (64, 20000):
                rad.tune_set_chunk_target(target)
                out = rad.batch(grid, ds, idx, 3, 7, precision=prec).cpu().numpy()
                err = np.abs(out - ref).max() / np.abs(ref).max()
                print("prec %d chunk target %d: max diff %.2e" % (prec, target, err), flush=True)
                assert err < (1e-12 if prec == rad.FP64 else 1e-6)
            rad.tune_set_chunk_target(0)
    finally:
        for p in (0, 1):
            for m in (0, 1):
                rad.tune_set_shape(p, m, 0)
        rad.tune_set_chunk_target(0)


def test_cells_match_full_grid(rad):
    """rad_cells (masked cell integrals) equals the full-grid cube summed over each cell."""
    import torch
    segs, idx = _sections(2, seed=47)
    segs = segs[:3]
    g = segs[0]["gamma"]
    hw = analytic.log_omega(100, 1e6, 20e9)      # 2 photon-energy blocks, ragged
    th = analytic.cell_centred(16, 4.0 / g)      # 2 x 2 cells of 8 x 8
    grid = rad.Grid(hw, th, th)
    rng = np.random.default_rng(5)
    mask = (rng.random((3, 100, 4)) < 0.3).astype(np.uint8)
    mask[1] = 0                                   # a segment with nothing to do
    mask[2, :, 3] = 1
    for prec, tol in ((rad.FP64, 1e-12), (rad.MIXED, 1e-4)):
        for kind, ki in ((rad.CLASSICAL, 0), (rad.SPINHALF, 2)):
            got = rad.cells(grid, segs, kind, mask, precision=prec).cpu().numpy()
            full = rad.batch(grid, segs, [0, 1, 2], 3, 7, precision=rad.FP64).cpu().numpy()[:, ki]
            w = oracle.angle_weights(th)
            cell = np.zeros((3, 100, 4))
            for c in range(4):
                ci, cj = c % 2, c // 2
                blk = full[:, :, cj * 8:(cj + 1) * 8, ci * 8:(ci + 1) * 8]
                cell[:, :, c] = np.einsum("swyx,y,x->sw", blk, w[cj * 8:(cj + 1) * 8], w[ci * 8:(ci + 1) * 8])
            ref = np.where(mask > 0, cell, 0.0)
            assert np.all(got[mask == 0] == 0)
            err = np.abs(got - ref).max() / np.abs(ref).max()
            print("cells prec %d kind %d: max rel err %.3e" % (prec, kind, err), flush=True)
            assert err < tol
