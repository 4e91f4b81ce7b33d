"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Every comparison uses the same seeded inputs on both sides and the norm
metrics of ``parity.py``; FP64 must agree to 1e-9, the mixed-precision form to
1e-4 (the tolerance derivation is in the design notes).
"""
import numpy as np
import pytest

import oracle
from parity import assert_parity, metrics
from paper_1910_10391_amd.synth import analytic, channeling, presets

pytestmark = pytest.mark.gpu

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


def _cpu(t):
    return t.detach().cpu().numpy()


def _small_channeling(n_particles=3, n_sections=1, charge=+1.0, seed=21, n=(3000, 5000),
                      energy=10e9, length=10e-6):
    cfg = channeling.ChannelingConfig(energy_eV=energy, charge=charge, length_m=length,
                                      n_min=n[0], n_max=n[1], n_sections=n_sections, seed=seed)
    return cfg, channeling.generate(cfg, n_particles, threads=1)


def test_device_is_gfx950(rad):
    import torch
    props = torch.cuda.get_device_properties(0)
    print("device:", props.name, getattr(props, "gcnArchName", "?"), flush=True)
    assert "gfx950" in getattr(props, "gcnArchName", "gfx950")


def test_undulator_fp64_full(rad):
    """The undulator workload at full size (8193 samples, 128 w x 16 x 16), classical FP64."""
    p = presets.undulator_fp64()
    g = p["grid"]
    seg = p["segments"][0]
    grid = rad.Grid(g.hw_eV, g.thx, g.thy)
    out = _cpu(rad.classical(grid, seg))
    ref = oracle.spectrum(seg, g.hw_eV, g.thx, g.thy, oracle.KIND_CLASSICAL)[1]
    assert_parity(out, ref, g.thx, g.thy, FP64_TOL, "undulator fp64")


def test_quantum_ragged_grid(rad):
    """Spin-0 and spin-1/2 on a grid whose sizes fit no tile (w 37, x 7, y 5)."""
    cfg, tr = _small_channeling(1, seed=5)
    seg = tr[0][0]
    g = seg["gamma"]
    hw = analytic.log_omega(37, 0.5e6, 5e9)       # reaches hw >= E? no: E = 10 GeV
    thx = analytic.cell_centred(7, 5.0 / g)
    thy = analytic.cell_centred(5, 5.0 / g) + 0.3 / g
    grid = rad.Grid(hw, thx, thy)
    out = _cpu(rad.quantum(grid, seg, rad.SPIN0 | rad.SPINHALF))
    ref = oracle.spectrum(seg, hw, thx, thy, oracle.KIND_SPIN0 | oracle.KIND_SPINHALF)
    assert_parity(out[0], ref[2], thx, thy, FP64_TOL, "spin0 ragged")
    assert_parity(out[1], ref[4], thx, thy, FP64_TOL, "spinhalf ragged")
    only_half = _cpu(rad.quantum(grid, seg, rad.SPINHALF))
    assert np.array_equal(only_half[0], out[1])


def test_forbidden_photons_zero(rad):
    """hw >= E gives exactly zero in the quantum kinds; classical is unaffected."""
    cfg, tr = _small_channeling(1, seed=6)
    seg = dict(tr[0][0])
    seg["energy_eV"] = 50e6
    hw = np.array([1e6, 20e6, 49e6, 50e6, 80e6, 200e6])
    th = analytic.cell_centred(4, 3.0 / seg["gamma"])
    grid = rad.Grid(hw, th, th)
    out = _cpu(rad.batch(grid, [seg], [0], 1, 7))[0]
    ref = oracle.spectrum(seg, hw, th, th, 7)
    assert np.all(out[1][3:] == 0) and np.all(out[2][3:] == 0)
    for i, k in enumerate((1, 2, 4)):
        assert_parity(out[i], ref[k], th, th, FP64_TOL, "kind %d" % k)


def test_batch_sections_uneven(rad):
    """Sections of several trajectories, uneven lengths, summed per trajectory (kinds 1|2|4)."""
    cfg, trs = _small_channeling(3, n_sections=3, charge=-1.0, seed=9, n=(2000, 7000),
                                 energy=50e9, length=30e-6)
    segs, idx = [], []
    for p, secs in enumerate(trs):
        for s in secs:
            segs.append(s)
            idx.append(p)
    g = segs[0]["gamma"]
    hw = analytic.log_omega(70, 1e6, 20e9)
    th = analytic.cell_centred(8, 4.0 / g)
    grid = rad.Grid(hw, th, th)
    out = _cpu(rad.batch(grid, segs, idx, 4, 7))
    ref = oracle.batch(segs, idx, 4, hw, th, th, 7)
    assert np.all(out[3] == 0)
    for o in range(3):
        for i, k in enumerate(("classical", "spin0", "spinhalf")):
            assert_parity(out[o, i], ref[o, i], th, th, FP64_TOL, "traj %d %s" % (o, k))


def test_explicit_weights_and_short_segment(rad):
    """Explicit quadrature weights (rectangle rule) and the shortest segment (n = 2)."""
    seg = analytic.undulator(2e4, 0.5, 20e-6, 3, samples_per_period=100, rule="rect")
    hw1 = analytic.undulator_fundamental_eV(2e4, 0.5, 20e-6)
    hw = analytic.linear_omega(65, 2.5 * hw1)
    th = analytic.cell_centred(5, 1.0 / 2e4)
    grid = rad.Grid(hw, th, th)
    out = _cpu(rad.classical(grid, seg))
    ref = oracle.spectrum(seg, hw, th, th, 1)[1]
    assert_parity(out, ref, th, th, FP64_TOL, "rect weights")
    short = {k: (v[:2] if isinstance(v, np.ndarray) else v) for k, v in seg.items()}
    out2 = _cpu(rad.classical(grid, short))
    ref2 = oracle.spectrum(short, hw, th, th, 1)[1]
    assert_parity(out2, ref2, th, th, FP64_TOL, "n=2")


def test_mixed_precision(rad):
    """FP32 integrand and sincos, FP64 phase/reduction/accumulation: <= 1e-4 per spectrum."""
    p = presets.undulator_fp64()
    g = p["grid"]
    seg = p["segments"][0]
    grid = rad.Grid(g.hw_eV, g.thx, g.thy)
    out = _cpu(rad.classical(grid, seg, precision=rad.MIXED))
    ref = oracle.spectrum(seg, g.hw_eV, g.thx, g.thy, 1)[1]
    assert_parity(out, ref, g.thx, g.thy, MIXED_TOL, "undulator mixed")
    cfg, tr = _small_channeling(2, seed=13)
    segs = [tr[0][0], tr[1][0]]
    gm = segs[0]["gamma"]
    hw = analytic.log_omega(64, 0.5e6, 200e6)
    th = analytic.cell_centred(8, 5.0 / gm)
    grid = rad.Grid(hw, th, th)
    out = _cpu(rad.batch(grid, segs, [0, 1], 2, 7, precision=rad.MIXED))
    ref = oracle.batch(segs, [0, 1], 2, hw, th, th, 7)
    for o in range(2):
        for i in range(3):
            assert_parity(out[o, i], ref[o, i], th, th, MIXED_TOL, "mixed traj %d kind %d" % (o, i))


def test_phase_recurrence_and_direct_forms(rad):
    """Uniform grids with one spacing take the FP64 phase recurrence, others the direct
    phase factors; both against the oracle, through one-block-per-item and persistent
    launches, with partial tiles."""
    cfg, tr = _small_channeling(2, seed=29)
    segs = [tr[0][0], tr[1][0]]
    gm = segs[0]["gamma"]
    hw = analytic.log_omega(70, 0.5e6, 200e6)
    u9 = analytic.cell_centred(9, 5.0 / gm)
    u7 = analytic.cell_centred(7, 5.0 / gm * 7 / 9)            # the same spacing, 7 points
    rng = np.random.default_rng(5)
    irregular = np.sort(rng.uniform(-5.0 / gm, 5.0 / gm, 6))
    cases = [(u9, u9, True), (u9, u7, True), (u9, analytic.cell_centred(7, 4.0 / gm), False),
             (irregular, u9, False), (u9[:1], u7, True), (u9[::-1].copy(), u9[::-1].copy(), True),
             (u9, u9[::-1].copy(), False)]
    for thx, thy, rec in cases:
        grid = rad.Grid(hw, thx, thy)
        assert (grid.step != 0.0) == rec, (len(thx), len(thy), grid.step)
        if rec and len(thx) > 1:
            assert abs(grid.step - (thx[1] - thx[0])) < 1e-12 * abs(thx[1] - thx[0])
        ref = oracle.batch(segs, [0, 1], 2, hw, thx, thy, 7)
        out = _cpu(rad.batch(grid, segs, [0, 1], 2, 7))
        outp = _cpu(rad.Plan(grid, segs, [0, 1], 2, 7).launch())
        for o in range(2):
            for i in range(3):
                what = "%s %dx%d out %d kind %d" % ("recurrence" if rec else "direct", len(thx), len(thy), o, i)
                assert_parity(out[o, i], ref[o, i], thx, thy, FP64_TOL, what)
                assert_parity(outp[o, i], ref[o, i], thx, thy, FP64_TOL, "persistent " + what)


def test_variants_agree(rad):
    """Every kernel variant (direction tile, occupancy), one-block-per-item and persistent,
    FP64 and mixed, on a uniform 9 x 9 grid (FP64 phase recurrence) and an irregular
    9 x 7 grid (direct phase factors), both leaving partial direction tiles.  A variant
    without room for J (the 4x6 tile) runs the classical and spin-0 set, 4x4 the J set."""
    cfg, tr = _small_channeling(1, seed=17)
    seg = tr[0][0]
    hw = analytic.log_omega(130, 0.5e6, 200e6)
    th = analytic.cell_centred(9, 5.0 / seg["gamma"])
    rng = np.random.default_rng(11)
    thy_irr = np.sort(rng.uniform(-5.0 / seg["gamma"], 5.0 / seg["gamma"], 7))
    grids = [(th, th, rad.Grid(hw, th, th)), (th, thy_irr, rad.Grid(hw, th, thy_irr))]
    assert grids[0][2].step != 0.0 and grids[1][2].step == 0.0
    refs = [oracle.spectrum(seg, hw, gx, gy, 7) for gx, gy, _ in grids]
    keys = [(p, m, j) for p in (0, 1) for m in (0, 1) for j in (0, 1)]
    keep = {k: rad.tune_get_variant(*k) for k in keys}
    try:
        for v in range(rad.tune_num_variants()):
            for k in keys:
                try:
                    rad.tune_set_variant(*k, v)
                except rad.RadError as e:
                    assert e.status == rad.EUNSUPPORTED and k[2] == 1, (v, k)
                    rad.tune_set_variant(*k, 0)
            for (gx, gy, grid), ref in zip(grids, refs):
                for prec, tol in ((rad.FP64, FP64_TOL), (rad.MIXED, MIXED_TOL)):
                    out = _cpu(rad.batch(grid, [seg], [0], 1, 7, precision=prec))[0]
                    plan = rad.Plan(grid, [seg], [0], 1, 7, precision=prec)
                    outp = _cpu(plan.launch())[0]
                    for i, k in enumerate((1, 2, 4)):
                        what = "variant %d %dx%d prec %d kind %d" % (v, len(gx), len(gy), prec, k)
                        assert_parity(out[i], ref[k], gx, gy, tol, what)
                        assert_parity(outp[i], ref[k], gx, gy, tol, "persistent " + what)
    finally:
        for k in keys:
            rad.tune_set_variant(*k, keep[k])


def _cis_reference(turns, scale):
    """cos and sin of scale * pi * turns with the exact reduction f = turns - rint(turns),
    evaluated by mpmath at 40 digits."""
    import mpmath as mp
    mp.mp.dps = 40
    c = np.empty(turns.size)
    s = np.empty(turns.size)
    for i, u in enumerate(turns):
        f = mp.mpf(float(u)) - mp.mpf(float(np.rint(u)))
        a = scale * mp.pi * f
        sign = -1.0 if (scale == 1 and int(np.rint(u)) % 2) else 1.0
        c[i] = sign * float(mp.cos(a))
        s[i] = sign * float(mp.sin(a))
    return c, s


def test_phase_factor_routines(rad):
    """The phase factor as the kernels compute it (rad_phase_factors), against mpmath:
    the FP64 routine on half turns (exact reduction, Chebyshev fits, sign by parity) for
    |u| up to 1e6, at every multiple of 1/4 and past 2^31 up to 2^50 (the sign must stay
    right where a 32-bit parity would overflow), within 3 ulp of 1 (fit error about 1 ulp,
    Horner evaluation 1.5, the final product 0.5); the mixed form's hardware FP32 sine and
    cosine of revolutions, whose error (FP32 rounding of the reduced argument, 2 pi 2^-26
    = 9.4e-8, plus the instruction's own) must stay far inside the mixed tolerance."""
    import torch
    rng = np.random.default_rng(3)
    # past 2^31 half turns (photon energies near the particle energy, Sec. II eq.
    # (Lindhard_substi)): integers of both parities, quarter offsets, random values to 2^50
    big = np.concatenate([2.0 ** np.arange(31, 51), 2.0 ** np.arange(31, 51) + 1.0])
    big = np.concatenate([big, big + 0.25, big - 0.5, np.ldexp(rng.uniform(1.0, 2.0, 500), rng.integers(31, 50, 500))])
    u = np.concatenate([rng.uniform(-0.5, 0.5, 6000), rng.uniform(-1e4, 1e4, 6000), rng.uniform(-1e6, 1e6, 3000),
                        np.arange(-8.0, 8.25, 0.25), [1e-300, -1e-300, 3.0e-9, 2.0 ** 30 + 0.375], big, -big])
    ud = torch.tensor(u, dtype=torch.float64, device="cuda")
    c, s = (t.cpu().numpy() for t in rad.phase_factors(ud, rad.FP64))
    rc, rs = _cis_reference(u, 1)
    err64 = max(np.abs(c - rc).max(), np.abs(s - rs).max())
    r = u / 2.0
    rd = torch.tensor(r, dtype=torch.float64, device="cuda")
    cm, sm = (t.cpu().numpy() for t in rad.phase_factors(rd, rad.MIXED))
    mc, ms = _cis_reference(r, 2)
    err32 = max(np.abs(cm - mc).max(), np.abs(sm - ms).max())
    print("phase factor max abs error: FP64 %.2e, mixed (hardware FP32) %.2e" % (err64, err32))
    assert err64 <= 3 * 2.0 ** -52, err64
    assert err32 <= 1e-6, err32
    assert np.all(np.abs(c[np.rint(u) == u]) == 1.0) and np.all(s[np.rint(u) == u] == 0.0)
    with pytest.raises(rad.RadError):
        rad.phase_factors(ud, 7)


def test_bitwise_reproducible(rad):
    cfg, tr = _small_channeling(2, seed=23)
    segs = [tr[0][0], tr[1][0]]
    hw = analytic.log_omega(96, 0.5e6, 200e6)
    th = analytic.cell_centred(6, 5.0 / segs[0]["gamma"])
    grid = rad.Grid(hw, th, th)
    ds = rad.DeviceSegments(segs)
    a = _cpu(rad.batch(grid, ds, [0, 0], 1, 7))
    b = _cpu(rad.batch(grid, ds, [0, 0], 1, 7))
    assert np.array_equal(a, b)


def test_angle_integrate(rad):
    import torch
    hw = np.array([1e6, 2e6, 3e6])
    thx = analytic.cell_centred(5, 1e-4)
    thy = np.array([-1e-4, 0.0, 2e-4])
    grid = rad.Grid(hw, thx, thy)
    rng = np.random.default_rng(3)
    cubes = rng.random((2, 3, 3, 5))
    got = _cpu(rad.angle_integrate(grid, torch.from_numpy(cubes).cuda()))
    ref = oracle.angle_integrate(cubes, thx, thy)
    assert np.allclose(got, ref, rtol=1e-14, atol=0)


def test_error_paths(rad):
    """Host-side validation: nothing is launched for invalid calls."""
    import torch
    seg = analytic.undulator(2e4, 0.5, 20e-6, 1, n_steps=64)
    hw = np.array([1e6, 2e6])
    th = np.array([0.0, 1e-5])
    grid = rad.Grid(hw, th, th)
    ds = rad.DeviceSegments([seg])
    out = torch.zeros(grid.shape, dtype=torch.float64, device="cuda")
    need = rad.workspace_bytes(grid, ds.n[0], rad.CLASSICAL)
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    L = rad.lib()
    import ctypes
    st = rad._stream(None)
    # workspace too small
    r = L.rad_classical(grid.handle, ctypes.byref(ds.structs[0]), 0, rad._dptr(out), rad._dptr(ws),
                        need - 1, st)
    assert r == 2
    # host pointer in place of a device column
    host = np.zeros(65)
    bad = rad.Segment.from_buffer_copy(ds.structs[0])
    bad.vx = host.ctypes.data
    r = L.rad_classical(grid.handle, ctypes.byref(bad), 0, rad._dptr(out), rad._dptr(ws), need, st)
    assert r == 1 and b"not a device allocation" in L.rad_last_error()
    # n larger than the allocation behind the columns
    bad = rad.Segment.from_buffer_copy(ds.structs[0])
    bad.n = 10 ** 7
    r = L.rad_classical(grid.handle, ctypes.byref(bad), 0, rad._dptr(out), rad._dptr(ws),
                        ws.numel(), st)
    assert r in (1, 2)
    # output too small: the binding checks tensor bounds (torch sub-allocates, so the
    # C side can only check the enclosing device allocation)
    small = torch.zeros(3, dtype=torch.float64, device="cuda")
    with pytest.raises(ValueError):
        rad.classical(grid, ds, out=small)
    # n < 2, bad gamma, bad kinds, quantum without energy
    for field, val, kinds in (("n", 1, 1), ("gamma", 0.0, 1), ("gamma", float("nan"), 1),
                              ("energy_eV", 0.0, 4)):
        bad = rad.Segment.from_buffer_copy(ds.structs[0])
        setattr(bad, field, val)
        idx = (ctypes.c_int * 1)(0)
        r = L.rad_batch(grid.handle, ctypes.byref(bad), 1, idx, 1, kinds, 0, rad._dptr(out),
                        rad._dptr(ws), need, st)
        assert r == 1, (field, val)
    idx = (ctypes.c_int * 1)(1)
    r = L.rad_batch(grid.handle, ds.structs, 1, idx, 1, 1, 0, rad._dptr(out), rad._dptr(ws), need, st)
    assert r == 1
    torch.cuda.synchronize()
    assert torch.all(out == 0)
