"""CPU reference of the learned sampler's non-network steps (test infrastructure only).

Only ``tests/`` may import this module; it shares no code with the product.
Plain NumPy loops over the definitions:

* ``features``  -- trajectory features: log(gamma/1e4); the histogram of the
                   transverse oscillation amplitudes over [0, d/2] (32 bins,
                   amplitudes at or above d/2 in the last bin), normalised to
                   sum 1; log(omega_osc / 1e5 m^-1).  A turning point is a sign
                   change of v_x between samples k and k+1 (v_x >= 0 counts as
                   positive), located at x[k+1]; an amplitude is half the
                   distance between consecutive turning points; omega_osc is pi
                   times the number of sign changes over the time span.  With
                   fewer than two turning points the single amplitude is half
                   the total excursion of x.  Only the first 4096 turning points
                   enter the histogram, stored in single precision (the
                   kernel's bounded buffer); the count for omega_osc is total.
* ``select``    -- cells in decreasing predicted mass while the predicted mass
                   ahead of a cell is below coverage x the total, at most ``cap``
                   cells; every cell when |M_pred/M_coarse - 1| > tau or
                   M_coarse is not positive; then widened to whole blocks of 64
                   photon energies.
* ``combine``   -- exact cell integrals where selected, coarse centre value x
                   cell area elsewhere.

These steps are the sampler's bookkeeping around the radiation integrals of
Sec. II (the integrals themselves are the direct-sum oracle in ``oracle``); the
network's prediction is an input here.  Pinned in ``tests/test_oracle_sampler.py``
by closed forms (a pure sinusoid's amplitude and frequency), hand-worked
selections and the exactness of the combination when every cell is selected.
"""
from __future__ import annotations

import numpy as np

HIST_BINS = 32
MAX_TURNING = 4096
WBLOCK = 64


def features(t, x, vx, gamma, plane_spacing):
    """34 features of one trajectory (FP64, as defined in the module docstring)."""
    t = np.asarray(t, dtype=np.float64)
    x = np.asarray(x, dtype=np.float64)
    vx = np.asarray(vx, dtype=np.float64)
    pos = vx >= 0.0
    turning = [x[k + 1] for k in range(len(x) - 1) if pos[k] != pos[k + 1]]
    total = len(turning)
    kept = [float(np.float32(v)) for v in turning[:MAX_TURNING]]
    half = 0.5 * plane_spacing
    amps = [0.5 * abs(kept[i + 1] - kept[i]) for i in range(len(kept) - 1)]
    if not amps:
        amps = [0.5 * (x.max() - x.min())]
    hist = np.zeros(HIST_BINS)
    for a in amps:
        b = int(a / half * HIST_BINS)
        hist[min(max(b, 0), HIST_BINS - 1)] += 1.0
    span = t[-1] - t[0]
    w_osc = np.pi * total / span if span > 0 else 0.0
    out = np.empty(2 + HIST_BINS)
    out[0] = np.log(gamma / 1e4)
    out[1:1 + HIST_BINS] = hist / len(amps)
    out[-1] = np.log(max(w_osc, 1.0) / 1e5)
    return out


def cell_sums(values, wx, wy, cx, cy):
    """Sum over each cx x cy cell of values[..., y, x] * wy[y] * wx[x] -> [..., n_cells]
    (cells in row-major order: cell c = cj * (n_x / cx) + ci)."""
    v = np.asarray(values, dtype=np.float64)
    ny, nx = v.shape[-2:]
    ncx, ncy = nx // cx, ny // cy
    out = np.zeros(v.shape[:-2] + (ncx * ncy,))
    for cj in range(ncy):
        for ci in range(ncx):
            blk = v[..., cj * cy:(cj + 1) * cy, ci * cx:(ci + 1) * cx]
            out[..., cj * ncx + ci] = np.einsum("...yx,y,x->...", blk, wy[cj * cy:(cj + 1) * cy],
                                                wx[ci * cx:(ci + 1) * cx])
    return out


def cell_areas(wx, wy, cx, cy):
    return cell_sums(np.ones((len(wy), len(wx))), wx, wy, cx, cy)


def select(pred, mu, sigma, coarse, wx, wy, cx, cy, coverage, cap, tau):
    """Selection mask [n_traj, n_w, n_cells] (uint8) and fallback flags [n_traj, n_w]."""
    pred = np.asarray(pred, dtype=np.float64)
    n_traj, n_w = pred.shape[:2]
    pm = cell_sums(np.exp(mu + sigma * pred), wx, wy, cx, cy)
    cm = np.asarray(coarse, dtype=np.float64) * cell_areas(wx, wy, cx, cy)
    n_cells = pm.shape[-1]
    mask = np.zeros((n_traj, n_w, n_cells), dtype=np.uint8)
    fb = np.zeros((n_traj, n_w), dtype=np.uint8)
    for s in range(n_traj):
        for w in range(n_w):
            Mp, Mc = pm[s, w].sum(), cm[s, w].sum()
            if not Mc > 0 or abs(Mp / Mc - 1.0) > tau:
                fb[s, w] = 1
                mask[s, w, :] = 1
                continue
            order = sorted(range(n_cells), key=lambda c: (-pm[s, w, c], c))
            ahead = 0.0
            for r, c in enumerate(order):
                if r >= cap or not ahead < coverage * Mp:
                    break
                mask[s, w, c] = 1
                ahead += pm[s, w, c]
    for b0 in range(0, n_w, WBLOCK):
        blk = mask[:, b0:b0 + WBLOCK, :]
        mask[:, b0:b0 + WBLOCK, :] = np.repeat(blk.max(axis=1, keepdims=True), blk.shape[1], axis=1)
    return mask, fb


def combine(cells, mask, coarse, wx, wy, cx, cy):
    """dI/dhw [n_traj, n_w]."""
    area = cell_areas(wx, wy, cx, cy)
    per = np.where(np.asarray(mask) > 0, cells, np.asarray(coarse) * area)
    return per.sum(axis=-1)
