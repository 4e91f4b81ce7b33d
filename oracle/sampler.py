"""CPU reference of the learned sampler's non-network steps (test infrastructure only).

Only ``tests/`` may import this module; it shares no code with the product.
Plain NumPy loops over the definitions:

* ``features``  -- trajectory features: log(gamma/1e4); the histogram of the
                   transverse oscillation amplitudes over [0, d/2] (32 bins,
                   amplitudes at or above d/2 in the last bin), normalised to
                   sum 1; log(omega_osc / 1e5 m^-1); gamma times the mean and the
                   standard deviation of v_x and of v_y over the samples.  A turning point is a sign
                   change of v_x between samples k and k+1 (v_x >= 0 counts as
                   positive), located at x[k+1]; an amplitude is half the
                   distance between consecutive turning points; omega_osc is pi
                   times the number of sign changes over the time span.  With
                   fewer than two turning points the single amplitude is half
                   the total excursion of x.  Only the first 4096 turning points
                   enter the histogram, stored in single precision (the
                   kernel's bounded buffer); the count for omega_osc is total.
* ``select``    -- the prediction gives the angular shape; its scale lambda is
                   fitted to the exact centre values (ratio of the area-weighted
                   sums of exact and predicted centre values, the predicted centre
                   value being the mean predicted intensity of the fine directions
                   nearest the centre).  Every cell is selected when the scaled
                   centre values deviate from the exact ones by more than tau in
                   area-weighted relative L1 norm (or a sum is zero); otherwise
                   cells in decreasing (scaled) predicted mass while the mass ahead
                   of a cell is below coverage x the total, at most ``cap`` cells;
                   then widened to whole blocks of 64 photon energies.
* ``select_error`` -- error-driven selection: the network's sub-cell shape corrects
                   each exact centre value, E_c = C_c M_c / P_c (M_c the predicted
                   cell mass, P_c the predicted centre value; C_c A_c where P_c is
                   0), whose distance from the plain midpoint value, e_c =
                   |E_c - C_c A_c|, estimates the error of leaving the cell out.
                   Cells are taken in decreasing e_c while the estimated error of
                   the cells not yet taken exceeds eps x sum_c E_c, at most ``cap``;
                   widened to blocks of 64 energies as in ``select``.
* ``combine``   -- exact cell integrals where selected; elsewhere the predicted
                   cell mass (or E_c), or the coarse centre value x cell area.

These steps are the sampler's bookkeeping around the radiation integrals of
Sec. II (the integrals themselves are the direct-sum oracle in ``oracle``); the
network's prediction is an input here.  Pinned in ``tests/test_oracle_sampler.py``
by closed forms (a pure sinusoid's amplitude and frequency), hand-worked
selections, the exactness of the combination when every cell is selected, and the
exactness of the error-driven estimate when the prediction is the true map.
"""
from __future__ import annotations

import numpy as np

HIST_BINS = 32
N_FEATURES = HIST_BINS + 6
MAX_TURNING = 4096
WBLOCK = 64


def features(t, x, vx, vy, gamma, plane_spacing):
    """38 features of one trajectory (FP64, as defined in the module docstring)."""
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
    vy = np.asarray(vy, dtype=np.float64)
    out = np.empty(N_FEATURES)
    out[0] = np.log(gamma / 1e4)
    out[1:1 + HIST_BINS] = hist / len(amps)
    out[1 + HIST_BINS] = np.log(max(w_osc, 1.0) / 1e5)
    out[2 + HIST_BINS] = gamma * vx.mean()
    out[3 + HIST_BINS] = gamma * vy.mean()
    out[4 + HIST_BINS] = gamma * vx.std()
    out[5 + HIST_BINS] = gamma * vy.std()
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


def centre_values(values, cx, cy):
    """Mean of values[..., y, x] over the fine directions nearest each cell centre (the
    central 2 x 2 of an even cell, the middle point of an odd one) -> [..., n_cells]."""
    v = np.asarray(values, dtype=np.float64)
    ny, nx = v.shape[-2:]
    ncx, ncy = nx // cx, ny // cy
    xs = sorted({(cx - 1) // 2, cx // 2})
    ys = sorted({(cy - 1) // 2, cy // 2})
    out = np.zeros(v.shape[:-2] + (ncx * ncy,))
    for cj in range(ncy):
        for ci in range(ncx):
            pts = [v[..., cj * cy + y, ci * cx + x] for y in ys for x in xs]
            out[..., cj * ncx + ci] = sum(pts) / len(pts)
    return out


def select(pred, mu, sigma, coarse, wx, wy, cx, cy, coverage, cap, tau):
    """Selection mask [n_traj, n_w, n_cells] (uint8), fallback flags [n_traj, n_w] and the
    scaled predicted cell masses [n_traj, n_w, n_cells]."""
    pred = np.asarray(pred, dtype=np.float64)
    n_traj, n_w = pred.shape[:2]
    intensity = np.exp(mu + sigma * pred)
    pm = cell_sums(intensity, wx, wy, cx, cy)
    pc = centre_values(intensity, cx, cy)
    area = cell_areas(wx, wy, cx, cy)
    coarse = np.asarray(coarse, dtype=np.float64)
    n_cells = pm.shape[-1]
    mask = np.zeros((n_traj, n_w, n_cells), dtype=np.uint8)
    fb = np.zeros((n_traj, n_w), dtype=np.uint8)
    for s in range(n_traj):
        for w in range(n_w):
            C = (coarse[s, w] * area).sum()
            P = (pc[s, w] * area).sum()
            lam = C / P if P > 0 else 0.0
            pm[s, w] *= lam
            D = (np.abs(lam * pc[s, w] - coarse[s, w]) * area).sum()
            if not C > 0 or not P > 0 or D > tau * C:
                fb[s, w] = 1
                mask[s, w, :] = 1
                continue
            Mp = pm[s, w].sum()
            order = sorted(range(n_cells), key=lambda c: (-pm[s, w, c], c))
            ahead = 0.0
            for r, c in enumerate(order):
                if r >= cap or not ahead < coverage * Mp:
                    break
                mask[s, w, c] = 1
                ahead += pm[s, w, c]
    return widen(mask), fb, pm


def widen(mask):
    """A cell selected for one energy of a block of 64 is selected for all of them (in place)."""
    for b0 in range(0, mask.shape[1], WBLOCK):
        blk = mask[:, b0:b0 + WBLOCK, :]
        mask[:, b0:b0 + WBLOCK, :] = np.repeat(blk.max(axis=1, keepdims=True), blk.shape[1], axis=1)
    return mask


def select_error(pred, mu, sigma, coarse, wx, wy, cx, cy, eps, cap):
    """Error-driven selection: mask [n_traj, n_w, n_cells] (uint8) and the cell estimates E_c
    [n_traj, n_w, n_cells] that stand in for the cells left out."""
    pred = np.asarray(pred, dtype=np.float64)
    n_traj, n_w = pred.shape[:2]
    intensity = np.exp(mu + sigma * pred)
    pm = cell_sums(intensity, wx, wy, cx, cy)
    pc = centre_values(intensity, cx, cy)
    area = cell_areas(wx, wy, cx, cy)
    coarse = np.asarray(coarse, dtype=np.float64)
    n_cells = pm.shape[-1]
    mask = np.zeros((n_traj, n_w, n_cells), dtype=np.uint8)
    est = np.zeros((n_traj, n_w, n_cells))
    for s in range(n_traj):
        for w in range(n_w):
            for c in range(n_cells):
                mid = coarse[s, w, c] * area[c]
                est[s, w, c] = coarse[s, w, c] * pm[s, w, c] / pc[s, w, c] if pc[s, w, c] > 0 else mid
            e = [abs(est[s, w, c] - coarse[s, w, c] * area[c]) for c in range(n_cells)]
            budget = eps * est[s, w].sum()
            order = sorted(range(n_cells), key=lambda c: (-e[c], c))
            for r, c in enumerate(order):
                left = sum(e[j] for j in order[r:])      # estimated error of the cells not yet taken
                if r >= cap or not left > budget:
                    break
                mask[s, w, c] = 1
    return widen(mask), est


def combine(cells, mask, coarse, wx, wy, cx, cy, cell_pred=None, fallback=None, full=None):
    """dI/dhw [n_traj, n_w]: exact cells where selected, else the predicted cell mass
    (``cell_pred``) or the coarse centre value x area; where ``fallback`` is set, the
    full-grid value ``full`` [n_traj, n_w] itself (the sampler falls back to the full
    grid on a mass mismatch)."""
    other = cell_pred if cell_pred is not None else np.asarray(coarse) * cell_areas(wx, wy, cx, cy)
    per = np.where(np.asarray(mask) > 0, cells, other)
    out = per.sum(axis=-1)
    if fallback is not None:
        out = np.where(np.asarray(fallback) > 0, full, out)
    return out
