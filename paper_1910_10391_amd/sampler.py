"""Learned angular sampler: where to refine the angular grid, decided by a small MLP.

For every trajectory and photon energy the sampler estimates dI/d hw on a fine
n x n grid of directions within +-H/gamma from

1. the exact spectrum at the centres of the (n/8) x (n/8) cells (``rad.batch`` on a
   coarse grid),
2. the network's predicted angular shape (log intensity up to a constant) at every
   fine direction (``rad_mlp_forward_grid``; inputs: 38 trajectory features from
   ``rad_features`` and (log hw, gamma thx, gamma thy)), scaled to the exact centre
   values,
3. exact integrals over the cells the prediction ranks highest, until 99 % of the
   predicted intensity is covered (``rad_sampler_select``, ``rad_cells``), or over
   the cells whose midpoint value the predicted sub-cell shape says is furthest off,
   until the estimated error left is small (``rad_sampler_select_error``),
4. for the remaining cells the predicted cell mass (``fill="pred"``), the coarse
   value times the area (``fill="coarse"``) or, with the error-driven rule, the
   centre value corrected by the predicted sub-cell shape (``rad_sampler_combine``).

When the scaled prediction at the cell centres deviates from the exact centre
values by more than ``tau`` (relative L1 norm) a photon energy falls back to the
full grid.  The full-grid integral
(``rad.batch`` on the fine grid) is the reference that judges the error.  The
network is trained on spectra the method itself computes (``training_set``) with
the library's BF16 forward/backward kernels and Adam (``train``).

Every compute step runs in librad's HIP kernels; this module only marshals.
"""
from __future__ import annotations

import ctypes
import math
import time

import numpy as np

from . import rad
from .mlp import MLP

N_FEATURES = 38
CELL = 8
KIND = rad.SPINHALF
_bound = False


def _lib():
    global _bound
    L = rad.lib()
    if not _bound:
        P, I, S, F, D = ctypes.c_void_p, ctypes.c_int, ctypes.c_size_t, ctypes.c_float, ctypes.c_double
        sig = {
            "rad_features": (I, [ctypes.POINTER(rad.Segment), I, D, P, P, S, P]),
            "rad_sampler_select": (I, [P, I, P, F, F, P, I, I, F, I, F, P, P, P, P]),
            "rad_sampler_select_error": (I, [P, I, P, F, F, P, I, I, F, I, P, P, P]),
            "rad_sampler_combine": (I, [P, I, I, I, P, P, P, P, P, P]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _bound = True
    return L


def cell_centred(n, half):
    return -half + (np.arange(n) + 0.5) * (2.0 * half / n)


class Grids:
    """Fine (n x n) and coarse (cell-centre) direction grids within +-H/gamma, and the
    network's point inputs (normalised log hw, gamma thx / H, gamma thy / H) for
    every fine grid point, laid out [w][thy][thx]."""

    def __init__(self, hw_eV, gamma, n_fine=64, half_width_over_gamma=5.0, logw_norm=None):
        import torch
        self.hw = np.asarray(hw_eV, dtype=np.float64)
        self.gamma, self.n, self.H = float(gamma), int(n_fine), float(half_width_over_gamma)
        if self.n % CELL:
            raise ValueError("the fine grid must be a multiple of %d" % CELL)
        th = cell_centred(self.n, self.H / self.gamma)
        thc = cell_centred(self.n // CELL, self.H / self.gamma)
        self.fine = rad.Grid(self.hw, th, th)
        self.coarse = rad.Grid(self.hw, thc, thc)
        self.n_cells = (self.n // CELL) ** 2
        lw = np.log(self.hw)
        self.logw_norm = logw_norm or (float(lw.mean()), float(max(lw.std(), 1e-12)))
        u = (lw - self.logw_norm[0]) / self.logw_norm[1]
        g = self.gamma * th / self.H
        X = np.empty((self.hw.size, self.n, self.n, 3), dtype=np.float32)
        X[..., 0] = u[:, None, None]
        X[..., 1] = g[None, None, :]
        X[..., 2] = g[None, :, None]
        self.point_x = torch.from_numpy(X.reshape(-1, 3)).cuda()

    @property
    def points_per_traj(self):
        return self.hw.size * self.n * self.n


def features(dsegs, plane_spacing_m, stream=None):
    """[n_segs, 38] float32 features (rad_features)."""
    import torch
    n = len(dsegs)
    feat = torch.empty((n, N_FEATURES), dtype=torch.float32, device="cuda")
    ws = torch.empty(max(48 * n, 256), dtype=torch.uint8, device="cuda")
    rad._check(_lib().rad_features(dsegs.structs, n, float(plane_spacing_m), rad._dptr(feat),
                                   rad._dptr(ws), ws.numel(), rad._stream(stream)), "rad_features")
    return feat


def predict(mlp, grids, feat, chunk_points=1 << 27):
    """Normalised log-intensity prediction [n_traj, n_w, n, n] for every fine point
    (rad_mlp_forward_grid: no per-point inputs are materialised)."""
    import torch
    n_traj = feat.shape[0]
    ppt = grids.points_per_traj
    out = torch.empty((n_traj, ppt), dtype=torch.float32, device="cuda")
    per_call = max(1, chunk_points // ppt)
    for t0 in range(0, n_traj, per_call):
        t1 = min(n_traj, t0 + per_call)
        mlp.forward_grid(feat[t0:t1].contiguous(), grids.point_x, y=out[t0:t1])
    return out.view(n_traj, grids.hw.size, grids.n, grids.n)


class Sampler:
    """The learned sampler for one kind of workload (fixed grids and normalisation)."""

    def __init__(self, mlp, norm, grids, plane_spacing_m, coverage=0.99, cap=16, tau=0.25, fill="pred",
                 select="mass", eps=1e-3):
        self.mlp, self.norm, self.grids = mlp, dict(norm), grids
        self.d = float(plane_spacing_m)
        self.coverage, self.cap, self.tau = float(coverage), int(cap), float(tau)
        if fill not in ("pred", "coarse"):
            raise ValueError("fill must be 'pred' or 'coarse'")
        if select not in ("mass", "error"):
            raise ValueError("select must be 'mass' or 'error'")
        self.fill, self.select_rule, self.eps = fill, select, float(eps)

    def coarse(self, dsegs, precision):
        n = len(dsegs)
        c = rad.batch(self.grids.coarse, dsegs, list(range(n)), n, KIND, precision)
        return c.view(n, self.grids.hw.size, self.grids.n_cells)

    def select(self, pred, coarse, coverage=None, cap=None, tau=None, mu=None, sigma=None):
        """mask, fallback flags and predicted cell masses (rad_sampler_select)."""
        import torch
        n = pred.shape[0]
        g = self.grids
        mask = torch.empty((n, g.hw.size, g.n_cells), dtype=torch.uint8, device="cuda")
        fb = torch.empty((n, g.hw.size), dtype=torch.uint8, device="cuda")
        pm = torch.empty((n, g.hw.size, g.n_cells), dtype=torch.float64, device="cuda")
        rad._check(_lib().rad_sampler_select(
            g.fine.handle, n, rad._dptr(pred), float(self.norm["mu"] if mu is None else mu),
            float(self.norm["sigma"] if sigma is None else sigma), rad._dptr(coarse), CELL, CELL,
            float(self.coverage if coverage is None else coverage), int(self.cap if cap is None else cap),
            float(self.tau if tau is None else tau), rad._dptr(mask), rad._dptr(fb), rad._dptr(pm),
            rad._stream(None)), "rad_sampler_select")
        return mask, fb, pm

    def select_error(self, pred, coarse, eps=None, cap=None):
        """mask and cell estimates E_c (rad_sampler_select_error)."""
        import torch
        n = pred.shape[0]
        g = self.grids
        mask = torch.empty((n, g.hw.size, g.n_cells), dtype=torch.uint8, device="cuda")
        est = torch.empty((n, g.hw.size, g.n_cells), dtype=torch.float64, device="cuda")
        rad._check(_lib().rad_sampler_select_error(
            g.fine.handle, n, rad._dptr(pred), float(self.norm["mu"]), float(self.norm["sigma"]),
            rad._dptr(coarse), CELL, CELL, float(self.eps if eps is None else eps),
            int(self.cap if cap is None else cap), rad._dptr(mask), rad._dptr(est), rad._stream(None)),
            "rad_sampler_select_error")
        return mask, est

    def combine(self, cells, mask, coarse, cell_pred=None):
        """dI/dhw: exact cells where selected, else cell_pred (if given) or centre x area."""
        import torch
        n = cells.shape[0]
        out = torch.empty((n, self.grids.hw.size), dtype=torch.float64, device="cuda")
        rad._check(_lib().rad_sampler_combine(self.grids.fine.handle, n, CELL, CELL, rad._dptr(cells),
                                              rad._dptr(mask), rad._dptr(coarse),
                                              None if cell_pred is None else rad._dptr(cell_pred), rad._dptr(out),
                                              rad._stream(None)), "rad_sampler_combine")
        return out

    def estimate(self, dsegs, precision=rad.MIXED, rule="learned"):
        """dI/d hw [n_traj, n_w] and what it cost.

        rule "learned": cells chosen with the network's prediction (the sampler): by
                        predicted mass (``select="mass"``) or by the predicted error of
                        the midpoint value (``select="error"``, cells left out at their
                        corrected estimate);
        rule "coarse":  cells ranked by the coarse centre value x area, with the same
                        coverage and cap and no fallback (refinement without a network,
                        the comparison the sampler has to beat)."""
        import torch
        phases = {}

        def mark(name, t_prev):
            torch.cuda.synchronize()
            t = time.perf_counter()
            phases[name] = t - t_prev
            return t

        t0 = time.perf_counter()
        g = self.grids
        coarse = self.coarse(dsegs, precision)
        t = mark("coarse", t0)
        if rule == "learned":
            feat = features(dsegs, self.d)
            pred = predict(self.mlp, g, feat)
            t = mark("features_predict", t)
            if self.select_rule == "error":
                mask, fill = self.select_error(pred, coarse)
                fb = torch.zeros(mask.shape[:2], dtype=torch.uint8)
            else:
                mask, fb, pm = self.select(pred, coarse)
                fill = pm if self.fill == "pred" else None
        elif rule == "coarse":
            k = g.n // CELL
            lc = torch.log(coarse.float()).view(len(dsegs), g.hw.size, k, k)
            pred = lc.repeat_interleave(CELL, dim=2).repeat_interleave(CELL, dim=3).contiguous()
            mask, fb, _ = self.select(pred, coarse, tau=float("inf"), mu=0.0, sigma=1.0)
            fill = None
        else:
            raise ValueError("rule must be 'learned' or 'coarse'")
        mask_h = mask.cpu().numpy()
        t = mark("select", t)
        cells = rad.cells(g.fine, dsegs, KIND, mask_h, precision)
        t = mark("cells", t)
        dIdw = self.combine(cells, mask, coarse, fill)
        mark("combine", t)
        dt = time.perf_counter() - t0
        n_t = np.array(dsegs.n, dtype=np.float64)
        n_w = g.hw.size
        # evaluations: coarse centres + every direction of the refined cells (the selection
        # covers whole 64-energy blocks, and rad_cells evaluates exactly those)
        evals_refine = float(np.sum(n_t * mask_h.reshape(len(dsegs), -1).sum(axis=1)) * CELL * CELL)
        evals_coarse = float(np.sum(n_t) * n_w * g.n_cells)
        return dict(dIdw=dIdw, mask=mask_h, fallback=fb.cpu().numpy(), seconds=dt, phases=phases,
                    evals=evals_coarse + evals_refine, evals_full=float(np.sum(n_t) * n_w * g.n ** 2),
                    refined_cells_mean=float(mask_h.sum(axis=2).mean()))

    def full_grid(self, dsegs, precision=rad.MIXED):
        """Reference: the exact angle integral over the whole fine grid."""
        import torch
        t0 = time.perf_counter()
        n = len(dsegs)
        cube = rad.batch(self.grids.fine, dsegs, list(range(n)), n, KIND, precision)
        dIdw = rad.angle_integrate(self.grids.fine, cube[:, 0].contiguous())
        torch.cuda.synchronize()
        return dIdw, time.perf_counter() - t0

    def save(self, path):
        theta = self.mlp.get_params()
        np.savez(path, params=theta, mu=self.norm["mu"], sigma=self.norm["sigma"],
                 logw_mean=self.grids.logw_norm[0], logw_std=self.grids.logw_norm[1],
                 n_fine=self.grids.n, half_width=self.grids.H, plane_spacing=self.d,
                 coverage=self.coverage, cap=self.cap, tau=self.tau, fill=self.fill, select=self.select_rule,
                 eps=self.eps)

    @classmethod
    def load(cls, path, hw_eV, gamma):
        with np.load(path, allow_pickle=False) as z:
            grids = Grids(hw_eV, gamma, int(z["n_fine"]), float(z["half_width"]),
                          logw_norm=(float(z["logw_mean"]), float(z["logw_std"])))
            mlp = MLP(N_FEATURES, 3)
            mlp.set_params(z["params"])
            extra = dict(select=str(z["select"]), eps=float(z["eps"])) if "select" in z.files else {}
            return cls(mlp, dict(mu=float(z["mu"]), sigma=float(z["sigma"])), grids, float(z["plane_spacing"]),
                       float(z["coverage"]), int(z["cap"]), float(z["tau"]), str(z["fill"]), **extra)


# ---------------------------------------------------------------- training
def training_set(cfg, n_traj, grids, n_w_train=64, precision=rad.MIXED, chunk=64, first=0, floor_rel=1e-3,
                 verbose=False):
    """Spectra produced by the method itself: for each trajectory, n_w_train of the grid's
    photon energies (every k-th, offset by the trajectory index so that all energies are
    covered) on the full fine grid.  Returns features [N, 38], the point-table index of each
    energy [N, n_w_train] and, as the target, the angular shape of each map,
    log(S / max S + floor_rel) with the maximum over the map's directions
    [N, n_w_train, n, n] (float32); the scale comes from the exact centre values when
    cells are selected."""
    import torch
    from .synth import channeling
    n_w = grids.hw.size
    step = max(1, n_w // n_w_train)
    feats, tw, targets = [], [], []
    grid_cache = {}
    for c0 in range(0, n_traj, chunk):
        c1 = min(n_traj, c0 + chunk)
        trs = channeling.generate(cfg, c1 - c0, first=first + c0, threads=16)
        segs = [tr[0] for tr in trs]
        ds = rad.DeviceSegments(segs)
        feats.append(features(ds, cfg.d_m))
        for off in range(step):
            members = [i for i in range(c1 - c0) if (c0 + i) % step == off]
            if not members:
                continue
            iw = np.arange(off, n_w, step)[:n_w_train]
            if off not in grid_cache:
                grid_cache[off] = rad.Grid(grids.hw[iw], grids.fine.thx, grids.fine.thy)
            sub = rad.DeviceSegments([segs[i] for i in members])
            cube = rad.batch(grid_cache[off], sub, list(range(len(members))), len(members), KIND,
                             precision)[:, 0].float()
            S = cube.clamp_min(0)
            peak = S.amax(dim=(2, 3), keepdim=True).clamp_min(1e-300)
            y = torch.log(S / peak + floor_rel)
            for j, i in enumerate(members):
                targets.append((c0 + i, y[j]))
                tw.append((c0 + i, torch.from_numpy(iw.astype(np.int64))))
        if verbose and ((c0 // chunk) % 16 == 15 or c1 == n_traj):
            print("training set: %d / %d trajectories" % (c1, n_traj), flush=True)
    targets.sort(key=lambda p: p[0])
    tw.sort(key=lambda p: p[0])
    Y = torch.stack([y for _, y in targets])
    W = torch.stack([w for _, w in tw]).cuda()
    return torch.cat(feats), W, Y


def train(mlp, grids, feat, W, Y, steps=3000, batch=65536, lr=2e-3, lr_end=2e-5, seed=0, log_every=500,
          verbose=False):
    """Adam on minibatches of (trajectory, energy, direction) points; cosine learning rate.
    Returns the normalisation (mu, sigma of the log targets) and the loss history."""
    import torch
    mu = float(Y.mean())
    sigma = float(Y.std())
    gen = torch.Generator(device="cuda")
    gen.manual_seed(int(seed))
    N, nwt = W.shape
    npix = grids.n * grids.n
    losses = []
    for it in range(steps):
        a = lr_end + 0.5 * (lr - lr_end) * (1 + math.cos(math.pi * it / max(1, steps - 1)))
        ti = torch.randint(0, N, (batch,), device="cuda", generator=gen)
        wi = torch.randint(0, nwt, (batch,), device="cuda", generator=gen)
        pi = torch.randint(0, npix, (batch,), device="cuda", generator=gen)
        gw = W[ti, wi]
        x = grids.point_x[gw * npix + pi]
        t = ((Y.view(N, nwt, npix)[ti, wi, pi] - mu) / sigma).contiguous()
        loss = mlp.train_step(feat, ti.to(torch.int32), x.contiguous(), t, a)
        if it % 50 == 0 or it == steps - 1:
            losses.append((it, float(loss.item())))
            if verbose and (it % log_every == 0 or it == steps - 1):
                print("step %d lr %.2e loss %.4f" % (it, a, losses[-1][1]), flush=True)
    return dict(mu=mu, sigma=sigma), losses
