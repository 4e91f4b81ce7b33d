"""Parity at full size: the benchmark's workload, launched exactly as bench.py launches it
(256 trajectories planned into one persistent launch, rad_plan_create + rad_plan_launch,
512 x 32 x 32 grid, spin-1/2, FP64 and mixed; rad_batch on the same batch gives the same
bits), checked on sampled outputs that the oracle computes point by point."""
import numpy as np
import pytest

import bench
import oracle

pytestmark = pytest.mark.gpu


def test_positron_spinhalf_full_size_sampled():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1910_10391_amd import rad
    cfg, segs, g = bench.build_workload(256)
    ds = rad.DeviceSegments(segs)
    grid = rad.Grid(g.hw_eV, g.thx, g.thy)
    idx = list(range(len(segs)))
    print("full-size: %d trajectories, %d..%d samples" % (len(segs), min(ds.n), max(ds.n)), flush=True)
    def planned(prec):
        plan = rad.Plan(grid, ds, idx, len(segs), rad.SPINHALF, precision=prec)
        o = plan.launch()
        plan.close()
        return o
    out_t = planned(rad.FP64)
    assert torch.equal(out_t, rad.batch(grid, ds, idx, len(segs), rad.SPINHALF))
    out = out_t[:, 0].cpu().numpy()
    del out_t
    outm = planned(rad.MIXED)[:, 0].cpu().numpy()
    assert np.all(np.isfinite(out)) and np.all(out >= 0)
    traj, iw, ix, iy = bench.sample_points(segs, g)
    # a fixed random sample of single points from every trajectory on top of the blocks
    rng = np.random.default_rng(42)
    pts = [(int(rng.integers(len(segs))), int(rng.integers(g.shape[0])),
            int(rng.integers(g.shape[1])), int(rng.integers(g.shape[2]))) for _ in range(24)]
    sel = np.ix_(iw, iy, ix)
    for p in traj:
        ref = oracle.spectrum(segs[p], g.hw_eV[iw], g.thx[ix], g.thy[iy], oracle.KIND_SPINHALF)[4]
        for name, cube, tol in (("fp64", out, 1e-9), ("mixed", outm, 1e-4)):
            m1, m2 = bench.rel_metrics(cube[p][sel], ref)
            print("traj %d (%d samples) %s: M1 %.3e M2 %.3e" % (p, ds.n[p], name, m1, m2), flush=True)
            assert m1 <= tol and m2 <= tol
    for p, i, jy, jx in pts:
        ref = oracle.spectrum(segs[p], g.hw_eV[i:i + 1], g.thx[jx:jx + 1], g.thy[jy:jy + 1],
                              oracle.KIND_SPINHALF)[4][0, 0, 0]
        got = out[p, i, jy, jx]
        # single points: relative to the row scale (cancellation makes tiny points noisy)
        scale = max(abs(ref), 1e-6 * float(np.max(out[p, i])))
        assert abs(got - ref) <= 1e-9 * scale, (p, i, jy, jx, got, ref)


def test_electron_50gev_sections_full_size_sampled():
    """512 electrons x 10 sections (1e5..3e5 samples per trajectory), spin-1/2, as a
    persistent mixed-precision plan replayed from a hipGraph and as plain FP64."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1910_10391_amd import rad
    segs, idx, g = bench.build_sections_workload(512)
    ds = rad.DeviceSegments(segs)
    grid = rad.Grid(g.hw_eV, g.thx, g.thy)
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        plan = rad.Plan(grid, ds, idx, 512, rad.SPINHALF, precision=rad.MIXED, stream=side)
        outm = plan.launch_graph(stream=side)
        side.synchronize()
        outm = outm[:, 0].cpu().numpy()
    out = rad.batch(grid, ds, idx, 512, rad.SPINHALF)[:, 0].cpu().numpy()
    iw = np.arange(0, g.shape[0], 16)
    ix = np.arange(0, g.shape[2], 4)
    iy = np.arange(0, g.shape[1], 4)
    sel = np.ix_(iw, iy, ix)
    lens = np.array([sum(ds.n[i] for i in range(len(segs)) if idx[i] == p) for p in range(512)])
    for p in (int(np.argmin(lens)), int(np.argmax(lens))):
        mine = [segs[i] for i in range(len(segs)) if idx[i] == p]
        ref = oracle.batch(mine, [0] * len(mine), 1, g.hw_eV[iw], g.thx[ix], g.thy[iy],
                           oracle.KIND_SPINHALF)[0, 0]
        for name, cube, tol in (("fp64", out, 1e-9), ("mixed plan graph", outm, 1e-4)):
            m1, m2 = bench.rel_metrics(cube[p][sel], ref)
            print("trajectory %d (%d samples, %d sections) %s: M1 %.3e M2 %.3e"
                  % (p, lens[p], len(mine), name, m1, m2), flush=True)
            assert m1 <= tol and m2 <= tol


def test_pm_mixed_full_size_sampled():
    """1024 e+ + 1024 e-, classical + spin-0 + spin-1/2 in mixed precision."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1910_10391_amd import rad
    segs, g = bench.build_pm_workload(1024)
    ds = rad.DeviceSegments(segs)
    grid = rad.Grid(g.hw_eV, g.thx, g.thy)
    idx = list(range(len(segs)))
    out = rad.batch(grid, ds, idx, len(segs), 7, precision=rad.MIXED).cpu().numpy()
    iw = np.arange(0, g.shape[0], 16)
    ix = np.arange(0, g.shape[2], 4)
    iy = np.arange(0, g.shape[1], 4)
    sel = np.ix_(iw, iy, ix)
    for p in (0, 1, 1024, 1025, int(np.argmax(ds.n))):
        ref = oracle.spectrum(segs[p], g.hw_eV[iw], g.thx[ix], g.thy[iy], 7)
        for i, k in enumerate((1, 2, 4)):
            m1, m2 = bench.rel_metrics(out[p, i][sel], ref[k])
            print("pm trajectory %d kind %d: M1 %.3e M2 %.3e" % (p, k, m1, m2), flush=True)
            assert m1 <= 1e-4 and m2 <= 1e-4
