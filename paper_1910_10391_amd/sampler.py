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
            "rad_sampler_combine": (I, [P, I, I, I, P, P, P, P, P, P, P, P]),
            "rad_sampler_coarse_pred": (I, [P, I, P, I, I, P, P]),
            "rad_sampler_targets": (I, [P, ctypes.c_int64, I, F, P, P]),
            "rad_sampler_moments_workspace_bytes": (S, []),
            "rad_sampler_moments": (I, [P, ctypes.c_int64, P, P, S, P]),
            "rad_sampler_minibatch": (I, [P, P, ctypes.c_int64, I, I, P, ctypes.c_int64, P, I, ctypes.c_uint64,
                                          ctypes.c_uint64, P, P, P, P]),
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

    def combine(self, cells, mask, coarse, cell_pred=None, fallback=None, full=None):
        """dI/dhw: exact cells where selected, else cell_pred (if given) or centre x area;
        where `fallback` is set, the full-grid value `full`."""
        import torch
        n = cells.shape[0]
        out = torch.empty((n, self.grids.hw.size), dtype=torch.float64, device="cuda")
        opt = lambda t: None if t is None else rad._dptr(t)   # noqa: E731
        rad._check(_lib().rad_sampler_combine(self.grids.fine.handle, n, CELL, CELL, rad._dptr(cells),
                                              rad._dptr(mask), rad._dptr(coarse), opt(cell_pred), opt(fallback),
                                              opt(full), rad._dptr(out), rad._stream(None)),
                   "rad_sampler_combine")
        return out

    def estimate(self, dsegs, precision=rad.MIXED, rule="learned", phases=False):
        """dI/d hw [n_traj, n_w] and what it cost.

        rule "learned": cells chosen with the network's prediction (the sampler): by
                        predicted mass (``select="mass"``) or by the predicted error of
                        the midpoint value (``select="error"``, cells left out at their
                        corrected estimate);
        rule "coarse":  cells ranked by the coarse centre value x area, with the same
                        coverage and cap and no fallback (refinement without a network,
                        the comparison the sampler has to beat).

        Where no photon energy can fall back (the error-driven selection, the coarse
        ranking, or a check tolerance tau = inf) the mask stays on the device
        (rad_cells_device) and nothing waits for the GPU between the coarse step and
        the combination; the selection by predicted mass with a finite tau copies the
        fallback flags to the host, which decides which trajectories take the full
        grid.  phases=True synchronises after every step to time it."""
        import torch
        times = {}

        def mark(name, t_prev):
            if not phases:
                return t_prev
            torch.cuda.synchronize()
            t = time.perf_counter()
            times[name] = t - t_prev
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
            pred = torch.empty((len(dsegs), g.hw.size, g.n, g.n), dtype=torch.float32, device="cuda")
            rad._check(_lib().rad_sampler_coarse_pred(g.fine.handle, len(dsegs), rad._dptr(coarse), CELL, CELL,
                                                      rad._dptr(pred), rad._stream(None)), "rad_sampler_coarse_pred")
            mask, fb, _ = self.select(pred, coarse, tau=float("inf"), mu=0.0, sigma=1.0)
            fill = None
        else:
            raise ValueError("rule must be 'learned' or 'coarse'")
        n_t = np.array(dsegs.n, dtype=np.float64)
        n_w = g.hw.size
        can_fall_back = rule == "learned" and self.select_rule != "error" and self.tau != float("inf")
        if not can_fall_back:
            t = mark("select", t)
            cells = rad.cells(g.fine, dsegs, KIND, mask, precision)
            t = mark("cells", t)
            dIdw = self.combine(cells, mask, coarse, fill, None, None)
            mark("combine", t)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            mask_h = mask.cpu().numpy()
            fb_h = np.zeros(mask_h.shape[:2], dtype=np.uint8)
            return self._result(dIdw, mask_h, fb_h, dt, times, n_t, n_w, 0.0)
        mask_h = mask.cpu().numpy()
        fb_h = fb.cpu().numpy()
        t = mark("select", t)
        # energies that fell back take the full-grid value itself: the trajectories that
        # have any run through the full-grid path (the same call as full_grid for the same
        # segments), and their cells are not integrated
        full = None
        fb_rows = np.flatnonzero(fb_h.any(axis=1))
        evals_fb = 0.0
        if fb_rows.size:
            mask_h[fb_h > 0] = 0
            sub = dsegs if fb_rows.size == len(dsegs) else dsegs.subset(fb_rows)
            full_sub, _ = self.full_grid(sub, precision, sync=False)
            if fb_rows.size == len(dsegs):
                full = full_sub
            else:
                full = torch.zeros((len(dsegs), n_w), dtype=torch.float64, device="cuda")
                full.index_copy_(0, torch.from_numpy(fb_rows).cuda(), full_sub)
            fb = fb if fb.is_cuda else fb.cuda()
            evals_fb = float(np.sum(n_t[fb_rows]) * n_w * g.n ** 2)
            t = mark("fallback", t)
        cells = rad.cells(g.fine, dsegs, KIND, mask_h, precision)
        t = mark("cells", t)
        dIdw = self.combine(cells, mask, coarse, fill, fb if full is not None else None, full)
        mark("combine", t)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        return self._result(dIdw, mask_h, fb_h, dt, times, n_t, n_w, evals_fb)

    def _result(self, dIdw, mask_h, fb_h, dt, times, n_t, n_w, evals_fb):
        # evaluations: coarse centres + every direction of the refined cells (the selection
        # covers whole 64-energy blocks, and rad_cells evaluates exactly those) + the full
        # grid of trajectories with a fallback
        g = self.grids
        evals_refine = float(np.sum(n_t * mask_h.reshape(len(n_t), -1).sum(axis=1)) * CELL * CELL)
        evals_coarse = float(np.sum(n_t) * n_w * g.n_cells)
        return dict(dIdw=dIdw, mask=mask_h, fallback=fb_h, seconds=dt, phases=times,
                    evals=evals_coarse + evals_refine + evals_fb, evals_full=float(np.sum(n_t) * n_w * g.n ** 2),
                    refined_cells_mean=float(mask_h.sum(axis=2).mean()))

    def full_grid(self, dsegs, precision=rad.MIXED, sync=True):
        """Reference: the exact angle integral over the whole fine grid."""
        import torch
        t0 = time.perf_counter()
        n = len(dsegs)
        cube = rad.batch(self.grids.fine, dsegs, list(range(n)), n, KIND, precision)
        dIdw = rad.angle_integrate(self.grids.fine, cube[:, 0].contiguous())
        if sync:
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
def _cache_key(cfg, n_traj, grids, n_w_train, precision, first, floor_rel):
    """Everything a training set depends on, as one string (stored with the cache)."""
    import dataclasses
    import hashlib
    h = hashlib.sha256()
    for a in (grids.hw, np.asarray(grids.fine.thx), np.asarray(grids.fine.thy)):
        h.update(np.ascontiguousarray(a, dtype=np.float64).tobytes())
    fields = sorted(dataclasses.asdict(cfg).items())
    return repr((fields, int(n_traj), int(n_w_train), int(precision), int(first), float(floor_rel), h.hexdigest()))


def training_set(cfg, n_traj, grids, n_w_train=64, precision=rad.MIXED, chunk=64, first=0, floor_rel=1e-3,
                 verbose=False, cache=None):
    """Spectra produced by the method itself: for each trajectory, n_w_train of the grid's
    photon energies (every k-th, offset by the trajectory index so that all energies are
    covered) on the full fine grid.  Returns features [N, 38], the point-table index of each
    energy [N, n_w_train] and, as the target, the angular shape of each map,
    log(S / max S + floor_rel) with the maximum over the map's directions
    [N, n_w_train, n, n] (float32); the scale comes from the exact centre values when
    cells are selected.

    cache: a file path (.npz).  When it holds a training set made with the same
    arguments (generator settings, trajectories, grid, precision) that set is loaded
    instead of recomputed; otherwise the new set is written there."""
    import torch
    key = _cache_key(cfg, n_traj, grids, n_w_train, precision, first, floor_rel) if cache else None
    if cache:
        import os
        if os.path.exists(cache):
            with np.load(cache, allow_pickle=False) as z:
                if str(z["key"]) == key:
                    if verbose:
                        print("training set: loaded from %s" % cache, flush=True)
                    return (torch.from_numpy(z["feat"]).cuda(), torch.from_numpy(z["W"]).cuda(),
                            torch.from_numpy(z["Y"]).cuda())
    feat, W, Y = _training_set(cfg, n_traj, grids, n_w_train, precision, chunk, first, floor_rel, verbose)
    if cache:
        import os
        tmp = cache + ".tmp%d.npz" % os.getpid()
        np.savez(tmp, key=np.array(key), feat=feat.cpu().numpy(), W=W.cpu().numpy(), Y=Y.cpu().numpy())
        os.replace(tmp, cache)
    return feat, W, Y


def _training_set(cfg, n_traj, grids, n_w_train, precision, chunk, first, floor_rel, verbose):
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
            cube = rad.batch(grid_cache[off], sub, list(range(len(members))), len(members), KIND, precision)
            y = targets_of(cube, floor_rel).view(len(members), iw.size, grids.n, grids.n)
            for j, i in enumerate(members):
                targets.append((c0 + i, y[j]))
                tw.append((c0 + i, torch.from_numpy(iw.astype(np.int32))))
        if verbose and ((c0 // chunk) % 16 == 15 or c1 == n_traj):
            print("training set: %d / %d trajectories" % (c1, n_traj), flush=True)
    targets.sort(key=lambda p: p[0])
    tw.sort(key=lambda p: p[0])
    Y = torch.stack([y for _, y in targets])
    W = torch.stack([w for _, w in tw]).cuda()
    return torch.cat(feats), W, Y


def targets_of(cube, floor_rel=1e-3):
    """log(S / max S + floor_rel) of each map of a float64 cube [..., n_y, n_x] (the maximum
    over the map's directions; rad_sampler_targets), float32 of the same shape."""
    import torch
    n_dirs = int(cube.shape[-1] * cube.shape[-2])
    n_maps = cube.numel() // n_dirs
    y = torch.empty(cube.shape, dtype=torch.float32, device=cube.device)
    rad._check(_lib().rad_sampler_targets(rad._dptr(cube), n_maps, n_dirs, float(floor_rel), rad._dptr(y),
                                          rad._stream(None)), "rad_sampler_targets")
    return y


def moments(Y):
    """(mean, standard deviation) of a float32 tensor (rad_sampler_moments, FP64)."""
    import torch
    m = torch.empty(2, dtype=torch.float64, device="cuda")
    ws = torch.empty(int(_lib().rad_sampler_moments_workspace_bytes()), dtype=torch.uint8, device="cuda")
    rad._check(_lib().rad_sampler_moments(rad._dptr(Y), Y.numel(), rad._dptr(m), rad._dptr(ws), ws.numel(),
                                          rad._stream(None)), "rad_sampler_moments")
    return m


def train(mlp, grids, feat, W, Y, steps=3000, batch=65536, lr=2e-3, lr_end=2e-5, seed=0, log_every=500,
          verbose=False):
    """Adam on minibatches of (trajectory, energy, direction) points drawn by the library
    (rad_sampler_minibatch; targets standardised by their mean and standard deviation);
    cosine learning rate.  Returns the normalisation (mu, sigma of the log targets) and the
    loss history."""
    import torch
    N, nwt = W.shape
    npix = grids.n * grids.n
    mom = moments(Y)
    mu, sigma = (float(v) for v in mom.cpu().numpy())
    traj = torch.empty(batch, dtype=torch.int32, device="cuda")
    x = torch.empty((batch, 3), dtype=torch.float32, device="cuda")
    t = torch.empty(batch, dtype=torch.float32, device="cuda")
    Wi = W.to(torch.int32).contiguous()
    losses = []
    for it in range(steps):
        a = lr_end + 0.5 * (lr - lr_end) * (1 + math.cos(math.pi * it / max(1, steps - 1)))
        rad._check(_lib().rad_sampler_minibatch(rad._dptr(Y), rad._dptr(Wi), N, nwt, npix, rad._dptr(grids.point_x),
                                                grids.point_x.shape[0], rad._dptr(mom), batch, int(seed), it,
                                                rad._dptr(traj), rad._dptr(x), rad._dptr(t), rad._stream(None)),
                   "rad_sampler_minibatch")
        loss_sum = mlp.train_step(feat, traj, x, t, a)
        if it % 50 == 0 or it == steps - 1:
            losses.append((it, float(loss_sum.item()) / batch))
            if verbose and (it % log_every == 0 or it == steps - 1):
                print("step %d lr %.2e loss %.4f" % (it, a, losses[-1][1]), flush=True)
    return dict(mu=mu, sigma=sigma), losses
