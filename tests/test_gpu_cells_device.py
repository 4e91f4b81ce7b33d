"""Cell integrals with the mask in device memory (rad_cells_device) against rad_cells with
the same mask read on the host, for empty, sparse, block-shaped and full masks, a
photon-energy count that is not a multiple of 64, both precisions and the classical and
spin-1/2 kinds: zeros where the mask is 0, the same values to rounding elsewhere (the
device form plans the time chunks for every cell, so the order of the chunk sums can
differ), bitwise for the full mask (the same plan); the default grouped items against the
one-block items, bit for bit, in both mask forms; the FP64 cells against the direct-sum
oracle; and the sampler's estimate through the device-mask path against the host-mask
one."""
import ctypes
import dataclasses

import numpy as np
import pytest

import oracle
from paper_1910_10391_amd.synth import analytic, channeling, presets

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def R():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1910_10391_amd import rad
    rad.lib()
    return rad


def _positrons(n, first=0):
    cfg = dataclasses.replace(presets.positron_config(seed=21), length_m=6e-6, n_min=2000, n_max=4000)
    return cfg, [tr[0] for tr in channeling.generate(cfg, n, first=first, threads=8)]


def _masks(rng, n_segs, n_w, n_cells):
    yield "empty", np.zeros((n_segs, n_w, n_cells), dtype=np.uint8)
    yield "sparse", (rng.random((n_segs, n_w, n_cells)) < 0.03).astype(np.uint8)
    m = np.zeros((n_segs, n_w, n_cells), dtype=np.uint8)
    m[0, :64, 1] = 1                                   # one whole block of one cell
    m[2, 128:, :] = 1                                  # the ragged last block, every cell
    yield "blocks", m
    yield "full", np.ones((n_segs, n_w, n_cells), dtype=np.uint8)


def test_device_mask_matches_host_mask(R):
    import torch
    rad = R
    cfg, segs = _positrons(3)
    g = segs[0]["gamma"]
    hw = analytic.log_omega(150, 1e6, 200e6)          # 150 energies: 2 full blocks + a ragged one
    th = analytic.cell_centred(16, 5.0 / g)
    grid = rad.Grid(hw, th, th)
    ds = rad.DeviceSegments(segs)
    rng = np.random.default_rng(5)
    for name, m in _masks(rng, 3, 150, 4):
        md = torch.from_numpy(m).cuda()
        for kind in (rad.CLASSICAL, rad.SPINHALF):
            for prec in (rad.FP64, rad.MIXED):
                a = rad.cells(grid, ds, kind, m, prec).cpu().numpy()
                b = rad.cells(grid, ds, kind, md, prec).cpu().numpy()
                err = np.abs(a - b).max() / max(np.abs(a).max(), 1e-300)
                print("mask %s kind %d prec %d: %d selected, bitwise %s, max diff %.2e" % (
                    name, kind, prec, int(m.sum()), np.array_equal(a, b), err), flush=True)
                assert not b[m == 0].any() and (b[m != 0] != 0).all()
                assert err <= 1e-12, (name, kind, prec)
                if name == "full":
                    assert np.array_equal(a, b), (name, kind, prec)
    # the cell blocks' spread over photon energies: the same sums (to rounding; the time
    # chunking follows the item count), in both mask forms
    try:
        for wg in (2, 4):
            rad.tune_set_cell_spread(wg)
            for name, m in _masks(rng, 3, 150, 4):
                if name == "empty":
                    continue
                for form in (m, torch.from_numpy(m).cuda()):
                    ref = None
                    b = rad.cells(grid, ds, rad.SPINHALF, form, rad.MIXED).cpu().numpy()
                    rad.tune_set_cell_spread(1)
                    ref = rad.cells(grid, ds, rad.SPINHALF, form, rad.MIXED).cpu().numpy()
                    rad.tune_set_cell_spread(wg)
                    err = np.abs(b - ref).max() / np.abs(ref).max()
                    assert err <= 1e-12 and not b[m == 0].any(), (wg, name, err)
            print("cell spread %d: the same cells" % wg, flush=True)
    finally:
        rad.tune_set_cell_spread(0)
    # FP64 cells of the full mask against the direct-sum oracle
    b = rad.cells(grid, ds, rad.SPINHALF, torch.ones((3, 150, 4), dtype=torch.uint8, device="cuda"),
                  rad.FP64).cpu().numpy()
    w = oracle.angle_weights(th)
    for s in (0, 2):
        fine = oracle.spectrum(segs[s], hw, th, th, oracle.KIND_SPINHALF)[oracle.KIND_SPINHALF]
        cellsum = np.zeros((150, 4))
        for cj in range(2):                            # cell c = cj * 2 + ci covers rows cj, columns ci
            for ci in range(2):
                blk = fine[:, cj * 8:(cj + 1) * 8, ci * 8:(ci + 1) * 8]
                cellsum[:, cj * 2 + ci] = np.einsum("wyx,y,x->w", blk, w[cj * 8:(cj + 1) * 8], w[ci * 8:(ci + 1) * 8])
        err = np.abs(b[s] - cellsum).max() / np.abs(cellsum).max()
        print("device-mask cells vs oracle, segment %d: %.2e" % (s, err), flush=True)
        assert err < 1e-9
    grid.close()


def test_grouped_items_equal_one_block_items(R):
    """The default cell form groups a (segment, cell, time chunk)'s selected 64-energy blocks
    by four, two and one (each staged direction then serves up to 256 energies): with both
    mask forms its cells equal the one-block form's bit for bit (the same sums in the same
    order, the same chunking).  450 energies (7 full blocks and a ragged one); per (segment,
    cell) anything from no block to all eight, so that every group size and remainder
    occurs."""
    import torch
    rad = R
    cfg, segs = _positrons(3, first=7)
    g = segs[0]["gamma"]
    hw = analytic.log_omega(450, 1e6, 200e6)
    th = analytic.cell_centred(16, 5.0 / g)
    grid = rad.Grid(hw, th, th)
    ds = rad.DeviceSegments(segs)
    rng = np.random.default_rng(11)
    n_wb = 8
    masks = []
    for case in range(3):
        blocks = rng.random((3, n_wb, 4)) < (0.35, 0.6, 0.9)[case]   # (segment, block, cell)
        m = (rng.random((3, 450, 4)) < 0.3) & np.repeat(blocks, 64, axis=1)[:, :450]
        masks.append(m.astype(np.uint8))
    full = np.ones((3, 450, 4), dtype=np.uint8)
    try:
        for i, m in enumerate(masks + [full]):
            per = [[int(m[s, b * 64:(b + 1) * 64, c].any()) for b in range(n_wb)] for s in range(3) for c in range(4)]
            sizes = sorted({sum(r) for r in per})
            for form in ("host", "device"):
                mm = m if form == "host" else torch.from_numpy(m).cuda()
                for kind in (rad.CLASSICAL, rad.SPINHALF):
                    for prec in (rad.FP64, rad.MIXED):
                        rad.tune_set_cell_spread(0)
                        assert rad.tune_get_cell_spread() == 0
                        a = rad.cells(grid, ds, kind, mm, prec).cpu().numpy()
                        rad.tune_set_cell_spread(1)
                        b = rad.cells(grid, ds, kind, mm, prec).cpu().numpy()
                        assert np.array_equal(a, b), (i, form, kind, prec)
                        assert not a[m == 0].any() and (a[m != 0] != 0).all()
            print("mask %d (%d selected energies, blocks per (segment, cell) %s): grouped = one-block, bitwise"
                  % (i, int(m.sum()), sizes), flush=True)
    finally:
        rad.tune_set_cell_spread(0)
    grid.close()


def test_device_mask_errors(R):
    """A mask that is not device memory of the stated size is refused before any launch."""
    import torch
    rad = R
    _, segs = _positrons(1)
    hw = analytic.log_omega(64, 1e6, 200e6)
    th = analytic.cell_centred(16, 5.0 / segs[0]["gamma"])
    grid = rad.Grid(hw, th, th)
    ds = rad.DeviceSegments(segs)
    L = rad.lib()
    nb = L.rad_cells_device_workspace_bytes(grid.handle, ds.structs, 1, rad.SPINHALF, rad.MIXED, 8, 8)
    assert nb > 0
    ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
    out = torch.empty((1, 64, 4), dtype=torch.float64, device="cuda")
    host = np.ones((1, 64, 4), dtype=np.uint8)
    good = torch.ones((1, 64, 4), dtype=torch.uint8, device="cuda")
    P = rad._dptr
    args = [grid.handle, ds.structs, 1, rad.SPINHALF, rad.MIXED, 8, 8, P(good), P(out), P(ws), nb, None]
    assert L.rad_cells_device(*args) == rad.OK
    for i, v in ((7, ctypes.c_void_p(host.ctypes.data)), (7, None), (10, nb - 1), (5, 4)):
        bad = list(args)
        bad[i] = v
        assert L.rad_cells_device(*bad) != rad.OK, i
    torch.cuda.synchronize()
    grid.close()


def test_estimate_device_path_equals_host_path(R):
    """The error-driven selection runs with the mask on the device; the same cells
    through the host-mask call and the same combination agree to rounding."""
    import torch
    from paper_1910_10391_amd import sampler as S
    from paper_1910_10391_amd.mlp import MLP
    rad = R
    cfg, segs = _positrons(2, first=40)
    gamma = segs[0]["gamma"]
    hw = analytic.log_omega(70, 1e6, 150e6)
    grids = S.Grids(hw, gamma, n_fine=16, half_width_over_gamma=5.0)
    smp = S.Sampler(MLP(S.N_FEATURES, 3, seed=3), dict(mu=-8.0, sigma=2.0), grids, cfg.d_m,
                    coverage=0.6, cap=3, tau=float("inf"), fill="coarse", select="error", eps=1e-4)
    ds = rad.DeviceSegments(segs)
    for prec in (rad.FP64, rad.MIXED):
        res = smp.estimate(ds, precision=prec)
        coarse = smp.coarse(ds, prec)
        feat = S.features(ds, cfg.d_m)
        pred = S.predict(smp.mlp, grids, feat)
        mask, est = smp.select_error(pred, coarse)
        assert np.array_equal(mask.cpu().numpy(), res["mask"])
        cells = rad.cells(grids.fine, ds, S.KIND, mask.cpu().numpy(), prec)
        ref = smp.combine(cells, mask, coarse, est, None, None).cpu().numpy()
        got = res["dIdw"].cpu().numpy()
        err = np.abs(got - ref).max() / np.abs(ref).max()
        print("estimate device path prec %d: max diff %.2e, refined %.2f of 4 cells" % (
            prec, err, res["refined_cells_mean"]))
        assert err <= 1e-12, prec
        assert 0.5 < res["refined_cells_mean"] < 4.0     # cells refined and cells left out
