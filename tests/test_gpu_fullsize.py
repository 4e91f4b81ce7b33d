"""Parity at full size: the benchmark's workload, launched exactly as bench.py launches it
(256 trajectories in one rad_batch call, 512 x 32 x 32 grid, spin-1/2, FP64 and mixed),
checked on sampled outputs that the oracle computes point by point."""
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
    out = rad.batch(grid, ds, idx, len(segs), rad.SPINHALF)[:, 0].cpu().numpy()
    outm = rad.batch(grid, ds, idx, len(segs), rad.SPINHALF, precision=rad.MIXED)[:, 0].cpu().numpy()
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
