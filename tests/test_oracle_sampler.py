"""Pins of the sampler's CPU reference (oracle/sampler.py) by closed forms and hand-worked cases."""
import numpy as np

from oracle import sampler as osm


D = 1.92e-10   # plane spacing [m]


def _sinusoid(a, omega, periods, per_period=200, t0=0.0):
    n = periods * per_period + 1
    t = t0 + np.arange(n) * (2 * np.pi / omega / per_period)
    phase = omega * t + 0.3
    return t, a * np.sin(phase), a * omega * np.cos(phase)


def test_features_sinusoid_closed_form():
    """x = a sin(W t): every amplitude is a (to O((W dt)^2)), omega_osc = W (to 1/periods)."""
    a = 10.5 / 32 * (D / 2)              # the middle of bin 10
    W = 3.0e6                            # rad per metre of ct
    t, x, vx = _sinusoid(a, W, periods=50)
    vy = np.full_like(t, 2.5e-5)
    f = osm.features(t, x, vx, vy, gamma=2e4, plane_spacing=D)
    assert f.shape == (38,)
    assert abs(f[0] - np.log(2.0)) < 1e-15
    hist = f[1:33]
    assert hist[10] == 1.0 and hist.sum() == 1.0
    assert abs(np.exp(f[33]) * 1e5 / W - 1.0) < 1.0 / 50
    # direction moments in units of 1/gamma: a whole number of periods (plus the
    # closing sample) averages cos to ~0; the spread of a W cos is a W / sqrt(2)
    assert abs(f[34]) < 0.05 * a * W * 2e4
    assert abs(f[35] - 2e4 * 2.5e-5) < 1e-12 and abs(f[37]) < 1e-9
    assert abs(f[36] / (2e4 * a * W / np.sqrt(2)) - 1.0) < 0.01


def test_features_two_amplitudes():
    """Half the oscillations at a1, half at a2: two bins of weight 1/2."""
    a1, a2 = 3.5 / 32 * (D / 2), 20.5 / 32 * (D / 2)
    W = 1.0e6
    t1, x1, v1 = _sinusoid(a1, W, periods=20, t0=0.0)
    # continue with the second amplitude from a turning point of the first (phase 0.3 + k 2pi)
    t2, x2, v2 = _sinusoid(a2, W, periods=20, t0=t1[-1])
    t = np.concatenate([t1, t2[1:]])
    x = np.concatenate([x1, x2[1:] - x2[0] + x1[-1]])
    vx = np.concatenate([v1, v2[1:]])
    f = osm.features(t, x, vx, np.zeros_like(t), gamma=1e4, plane_spacing=D)
    hist = f[1:33]
    # one half-oscillation straddles the junction; it falls between the two bins
    assert abs(hist[3] - 0.5) < 0.05 and abs(hist[20] - 0.5) < 0.05
    assert abs(hist.sum() - 1.0) < 1e-12


def test_features_over_barrier_and_no_turning():
    """Monotonic drift across several planes: no turning point, omega_osc = 0, last bin."""
    t = np.linspace(0.0, 1e-4, 1000)
    x = 5 * D * t / t[-1]
    vx = np.full_like(t, 5 * D / t[-1])
    f = osm.features(t, x, vx, -vx, gamma=1e4, plane_spacing=D)
    assert f[32] == 1.0 and f[1:32].sum() == 0.0
    assert f[33] == np.log(1.0 / 1e5)
    assert abs(f[34] + f[35]) < 1e-15 and f[36] == 0.0 and f[37] == 0.0


def _unit_grid_select(masses, coarse_values, coverage, cap, tau):
    """1 trajectory, 1 energy, 2 x 2 fine grid with unit widths, 1 x 1 cells (each cell's
    centre value is its single fine point)."""
    pred = np.log(np.asarray(masses, dtype=np.float64)).reshape(1, 1, 2, 2)
    coarse = np.asarray(coarse_values, dtype=np.float64).reshape(1, 1, 4)
    w = np.ones(2)
    return osm.select(pred, 0.0, 1.0, coarse, w, w, 1, 1, coverage, cap, tau)


def test_select_hand_worked():
    m = [0.125, 0.5, 0.125, 0.25]                           # ranks: 1, 3, then 0 and 2 (ties by index)
    mask, fb, pm = _unit_grid_select(m, m, coverage=0.75, cap=4, tau=0.25)
    assert fb[0, 0] == 0 and np.allclose(pm[0, 0], m, rtol=1e-15)
    assert mask[0, 0].tolist() == [0, 1, 0, 1]              # mass ahead of cell 0 is 0.75: not below 0.75
    mask, _, _ = _unit_grid_select(m, m, coverage=0.8, cap=4, tau=0.25)
    assert mask[0, 0].tolist() == [1, 1, 0, 1]              # cell 0 before cell 2 (equal mass)
    mask, _, _ = _unit_grid_select(m, m, coverage=1.0, cap=2, tau=0.25)
    assert mask[0, 0].tolist() == [0, 1, 0, 1]              # the cap
    # the prediction is a shape: a uniform rescaling of the exact values passes, and the
    # predicted masses come out at the exact scale
    mask, fb, pm = _unit_grid_select(m, [2 * v for v in m], coverage=0.5, cap=1, tau=1e-9)
    assert fb[0, 0] == 0 and mask[0, 0].tolist() == [0, 1, 0, 0]
    assert np.allclose(pm[0, 0], [2 * v for v in m], rtol=1e-14)
    # shape mismatch: exact [0.5, 0.125, 0.25, 0.125] against the shape of m (same total):
    # lambda = 1, sum |P - C| = 1.0 against sum C = 1.0
    mask, fb, _ = _unit_grid_select(m, [0.5, 0.125, 0.25, 0.125], coverage=0.5, cap=1, tau=0.99)
    assert fb[0, 0] == 1 and mask.all()
    mask, fb, _ = _unit_grid_select(m, [0.5, 0.125, 0.25, 0.125], coverage=0.5, cap=1, tau=1.01)
    assert fb[0, 0] == 0
    # a partial mismatch: exact = m except cell 3 doubled (sum 1.25): lambda = 1.25,
    # deviations |1.25 m - C| = [0.03125, 0.125, 0.03125, 0.1875], sum 0.375 = 0.3 x 1.25
    c3 = list(m)
    c3[3] *= 2
    _, fb, _ = _unit_grid_select(m, c3, coverage=0.5, cap=1, tau=0.31)
    assert fb[0, 0] == 0
    _, fb, _ = _unit_grid_select(m, c3, coverage=0.5, cap=1, tau=0.29)
    assert fb[0, 0] == 1
    mask, fb, _ = _unit_grid_select(m, [0.0] * 4, coverage=0.5, cap=1, tau=10.0)
    assert fb[0, 0] == 1 and mask.all()                     # no coarse value


def test_centre_values_of_even_and_odd_cells():
    v = np.arange(36.0).reshape(6, 6)
    # 2 x 2 cells: every point is central
    assert np.allclose(osm.centre_values(v, 2, 2), osm.cell_sums(v, np.ones(6), np.ones(6), 2, 2) / 4)
    # 3 x 3 cells: the middle point
    assert osm.centre_values(v, 3, 3).tolist() == [v[1, 1], v[1, 4], v[4, 1], v[4, 4]]
    # 6 x 6: the central 2 x 2
    assert osm.centre_values(v, 6, 6).tolist() == [(v[2, 2] + v[2, 3] + v[3, 2] + v[3, 3]) / 4]


def test_select_widens_to_energy_blocks():
    n_w = 100                                               # blocks [0, 64), [64, 100)
    pred = np.full((1, n_w, 2, 2), -50.0)
    pred[0, 3, 0, 1] = 0.0                                  # energy 3: only cell 1 carries mass
    pred[0, 70, 1, 0] = 0.0                                 # energy 70: only cell 2
    coarse = np.exp(pred).reshape(1, n_w, 4)
    w = np.ones(2)
    mask, fb, _ = osm.select(pred, 0.0, 1.0, coarse, w, w, 1, 1, 0.25, 4, 0.25)
    assert not fb.any()
    assert mask[0, :64, 1].all() and not mask[0, 64:, 1].any()
    assert mask[0, 64:, 2].all() and not mask[0, :64, 2].any()
    # other energies select their own top cell (cell 0 by index among equal masses)
    assert mask[0, :, 0].all() and not mask[0, :, 3].any()


def test_combine_exact_and_coarse():
    rng = np.random.default_rng(3)
    wx, wy = rng.random(4) + 0.5, rng.random(4) + 0.5
    S = rng.random((2, 5, 4, 4))
    cells = osm.cell_sums(S, wx, wy, 2, 2)
    coarse = rng.random((2, 5, 4))
    full = np.einsum("swyx,y,x->sw", S, wy, wx)
    ones = np.ones((2, 5, 4), np.uint8)
    assert np.allclose(osm.combine(cells, ones, coarse, wx, wy, 2, 2), full, rtol=1e-14)
    # a spectrum constant over each cell: the coarse value times the area is exact
    const = np.repeat(np.repeat(coarse.reshape(2, 5, 2, 2), 2, axis=2), 2, axis=3)
    exact = np.einsum("swyx,y,x->sw", const, wy, wx)
    zeros = np.zeros_like(ones)
    assert np.allclose(osm.combine(cells, zeros, coarse, wx, wy, 2, 2), exact, rtol=1e-14)
    # a mixed mask takes each cell from its own source
    mask = (rng.random((2, 5, 4)) < 0.5).astype(np.uint8)
    got = osm.combine(cells, mask, coarse, wx, wy, 2, 2)
    area = osm.cell_areas(wx, wy, 2, 2)
    ref = sum(cells[..., c] * mask[..., c] + coarse[..., c] * area[c] * (1 - mask[..., c]) for c in range(4))
    assert np.allclose(got, ref, rtol=1e-14)
    # with predicted cell masses the unselected cells take those
    pm = rng.random((2, 5, 4))
    got = osm.combine(cells, mask, coarse, wx, wy, 2, 2, cell_pred=pm)
    ref = sum(cells[..., c] * mask[..., c] + pm[..., c] * (1 - mask[..., c]) for c in range(4))
    assert np.allclose(got, ref, rtol=1e-14)
    # an energy that fell back is the full-grid value, whatever its cells say
    fb = np.zeros((2, 5), np.uint8)
    fb[0, 1] = fb[1, 4] = 1
    got_fb = osm.combine(cells, mask, coarse, wx, wy, 2, 2, cell_pred=pm, fallback=fb, full=full)
    assert got_fb[0, 1] == full[0, 1] and got_fb[1, 4] == full[1, 4]
    assert np.array_equal(got_fb[fb == 0], got[fb == 0])


def test_cell_sums_order():
    """Cell c = cj * ncx + ci covers columns [ci cx, (ci+1) cx) and rows [cj cy, (cj+1) cy)."""
    v = np.zeros((4, 6))
    v[3, 4] = 1.0                                           # row 3, column 4 -> cj 1, ci 2
    c = osm.cell_sums(v, np.ones(6), np.ones(4), 2, 2)
    assert c.tolist() == [0, 0, 0, 0, 0, 1.0]


def _two_odd_cells(cell0, cell1):
    """1 trajectory, 1 energy, a 6 x 3 fine grid of unit widths split into two 3 x 3 cells;
    cellN gives the 3 x 3 intensities (row-major) of cell N."""
    v = np.zeros((3, 6))
    v[:, :3] = np.asarray(cell0, dtype=np.float64).reshape(3, 3)
    v[:, 3:] = np.asarray(cell1, dtype=np.float64).reshape(3, 3)
    return v.reshape(1, 1, 3, 6)


def test_select_error_hand_worked():
    """Cell 0 flat, cell 1 with its centre at 1 and the other eight directions at 2: the
    corrected estimate of cell 1 is C_1 x 17 / 1 against the midpoint C_1 x 9, an estimated
    error of 8 C_1; cell 0 has none.  With C = (1, 1), sum E = 9 + 17 = 26."""
    v = _two_odd_cells(np.ones(9), [2, 2, 2, 2, 1, 2, 2, 2, 2])
    pred = np.log(v)
    coarse = np.array([1.0, 1.0]).reshape(1, 1, 2)
    wx, wy = np.ones(6), np.ones(3)
    mask, est = osm.select_error(pred, 0.0, 1.0, coarse, wx, wy, 3, 3, eps=0.3, cap=2)
    assert np.allclose(est[0, 0], [9.0, 17.0], rtol=1e-15)
    assert mask[0, 0].tolist() == [0, 1]                    # 8 > 0.3 x 26 = 7.8
    mask, _ = osm.select_error(pred, 0.0, 1.0, coarse, wx, wy, 3, 3, eps=0.31, cap=2)
    assert mask[0, 0].tolist() == [0, 0]                    # 8 <= 0.31 x 26 = 8.06
    # the prediction is a shape: mu changes nothing; the exact centre values set the scale
    mask, est = osm.select_error(pred - 7.0, 7.0, 1.0, 3.0 * coarse, wx, wy, 3, 3, eps=0.3, cap=2)
    assert np.allclose(est[0, 0], [27.0, 51.0], rtol=1e-14) and mask[0, 0].tolist() == [0, 1]
    # sigma sharpens the shape: sigma = 2 squares it, cell 1 -> (8 x 4 + 1) / 1 = 33
    _, est = osm.select_error(pred, 0.0, 2.0, coarse, wx, wy, 3, 3, eps=0.3, cap=2)
    assert np.allclose(est[0, 0], [9.0, 33.0], rtol=1e-14)
    # a centre predicted at zero intensity: the midpoint value stands in, no estimated error
    pred0 = pred.copy()
    pred0[0, 0, 1, 4] = -np.inf
    mask, est = osm.select_error(pred0, 0.0, 1.0, coarse, wx, wy, 3, 3, eps=0.0, cap=2)
    assert est[0, 0].tolist() == [9.0, 9.0] and mask[0, 0].tolist() == [0, 0]


def test_select_error_ranking_and_cap():
    """Three odd cells with estimated errors 8, 4 and 0 (C = 1): with eps = 0 every cell with
    an error is taken, largest first, within the cap."""
    v = np.zeros((3, 9))
    v[:, 0:3] = 1.0
    v[:, 3:6] = [[2, 2, 2], [2, 1, 2], [2, 2, 2]]           # 17 vs 9: error 8
    v[:, 6:9] = [[1.5, 1.5, 1.5], [1.5, 1, 1.5], [1.5, 1.5, 1.5]]   # 13 vs 9: error 4
    pred = np.log(v).reshape(1, 1, 3, 9)
    coarse = np.ones((1, 1, 3))
    wx, wy = np.ones(9), np.ones(3)
    mask, est = osm.select_error(pred, 0.0, 1.0, coarse, wx, wy, 3, 3, eps=0.0, cap=3)
    assert np.allclose(est[0, 0], [9.0, 17.0, 13.0], rtol=1e-15)
    assert mask[0, 0].tolist() == [0, 1, 1]
    mask, _ = osm.select_error(pred, 0.0, 1.0, coarse, wx, wy, 3, 3, eps=0.0, cap=1)
    assert mask[0, 0].tolist() == [0, 1, 0]
    # left after taking cell 1: 4 > eps x 39 for eps < 4/39; before: 12 > eps x 39
    mask, _ = osm.select_error(pred, 0.0, 1.0, coarse, wx, wy, 3, 3, eps=0.1, cap=3)
    assert mask[0, 0].tolist() == [0, 1, 1]
    mask, _ = osm.select_error(pred, 0.0, 1.0, coarse, wx, wy, 3, 3, eps=0.11, cap=3)
    assert mask[0, 0].tolist() == [0, 1, 0]


def test_select_error_exact_for_a_perfect_prediction():
    """When the prediction is the true map (odd cells: the centre value is the middle
    direction), every corrected estimate is the exact cell integral, so the combination is
    exact with no cell refined."""
    rng = np.random.default_rng(3)
    n_w, cx = 5, 3
    v = rng.random((2, n_w, 9, 12)) + 0.05
    wx, wy = rng.random(12) + 0.5, rng.random(9) + 0.5
    coarse = v[:, :, 1::3, 1::3].reshape(2, n_w, 12)        # the middle direction of each cell
    mask, est = osm.select_error(np.log(v), 0.0, 1.0, coarse, wx, wy, cx, cx, eps=1.0, cap=12)
    assert not mask.any()
    exact = np.einsum("swyx,y,x->sw", v, wy, wx)
    got = osm.combine(np.zeros_like(est), mask, coarse, wx, wy, cx, cx, cell_pred=est)
    assert np.allclose(got, exact, rtol=1e-13)


def test_select_error_widens_to_energy_blocks():
    """A cell taken at one energy of a 64-energy block is taken at all of them."""
    v = np.ones((1, 70, 3, 6))
    v[0, 10, :, 3:] = [[2, 2, 2], [2, 1, 2], [2, 2, 2]]
    v[0, 66, :, :3] = [[2, 2, 2], [2, 1, 2], [2, 2, 2]]
    coarse = np.ones((1, 70, 2))
    mask, _ = osm.select_error(np.log(v), 0.0, 1.0, coarse, np.ones(6), np.ones(3), 3, 3, eps=0.01, cap=2)
    assert mask[0, :64, 1].all() and not mask[0, :64, 0].any()
    assert mask[0, 64:, 0].all() and not mask[0, 64:, 1].any()
