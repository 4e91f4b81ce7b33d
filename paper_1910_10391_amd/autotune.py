"""Autotuner of the amplitude kernel's launch shape.

For a workload it times, on a sample of the longest segments (they dominate a
batch) and for the form that will run (the one-block-per-item calls or the
persistent plan):

1. every variant the library offers (direction tile per lane x resident blocks),
   separately for each integral set the kinds need (with and without J);
2. when the sample is the whole workload, for the whole call: the block's spread
   over photon energies (1, 2 or 4 of its 4 waves over energies, the rest over
   further direction tiles) and the work-item target that sets the chunk length.
   Both act on the launch's schedule as a whole (how many items, how long each),
   which a sample of the longest segments does not reproduce: on the 256-trajectory
   benchmark, two energy groups timed 3 % faster than four on its 8 longest
   segments and ran the full launch 4.6 % slower.

It keeps the fastest of each, sets it in the library (``rad_tune_set_variant``,
``rad_tune_set_shape``, ``rad_tune_set_chunk_target``) and records the choices in a
JSON cache keyed by (form, precision, set or kinds, grid shape, length bucket), so
that later runs on the same shape skip the search.  Timing is the amplitude kernel
alone, from HIP events the library records on its stream.
"""
from __future__ import annotations

import json
import math
import os
import tempfile

from . import rad

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "paper_1910_10391_amd",
                             "autotune.json")


def cache_path():
    return os.environ.get("RAD_AUTOTUNE_CACHE", DEFAULT_CACHE)


def _load(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(path, data):
    d = os.path.dirname(path)
    os.makedirs(d, exist_ok=True)
    fd, tmp = tempfile.mkstemp(dir=d, prefix=".autotune")
    with os.fdopen(fd, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def _sets(kinds):
    """(with_j, kinds of that set) for every integral set a kinds mask launches."""
    out = []
    if kinds & rad.CLASSICAL:
        out.append((False, rad.CLASSICAL))
    q = kinds & (rad.SPIN0 | rad.SPINHALF)
    if q:
        out.append((bool(q & rad.SPINHALF), q))
    return out


def key(persistent, precision, with_j, grid, max_n):
    bucket = int(math.log2(max(int(max_n), 2)))
    return "%s-%s-%s-%dx%dx%d-L%d" % ("plan" if persistent else "batch",
                                      "mixed" if precision == rad.MIXED else "fp64",
                                      "j" if with_j else "noj", *grid.shape, bucket)


def shape_key(persistent, precision, kinds, grid, max_n, what):
    bucket = int(math.log2(max(int(max_n), 2)))
    return "%s-%s-%s-k%d-%dx%dx%d-L%d" % (what, "plan" if persistent else "batch",
                                          "mixed" if precision == rad.MIXED else "fp64", int(kinds),
                                          *grid.shape, bucket)


WG_CHOICES = (1, 2, 4)
TARGET_CHOICES = (512, 1024, 2048, 4096, 8192, 16384)
# A launch-shape choice other than the planner's own must beat it by this much: timing
# noise alone should not move a workload off the planner's choice.
MARGIN = 0.03


def default_wg(n_w):
    """The planner's own spread over photon energies."""
    return 4 if n_w > 128 else (2 if n_w > 64 else 1)


def _search(cache, k, set_fn, choices, time_fn, result, verbose, field, default=None):
    """Time every choice, keep and set the fastest (or the cached one); a choice other
    than ``default`` must be MARGIN faster than it."""
    if k in cache:
        set_fn(cache[k][field])
        result[k] = dict(cache[k], cached=True)
        return False
    times = {}
    for c in choices:
        set_fn(c)
        times[c] = time_fn()
        if verbose:
            print("autotune %s %s %s: %.3f ms" % (k, field, c, times[c]), flush=True)
    best = min(times, key=times.get)
    if default in times and times[best] > (1.0 - MARGIN) * times[default]:
        best = default
    set_fn(best)
    cache[k] = {field: best, "ms": {str(c): t for c, t in times.items()}}
    result[k] = dict(cache[k], cached=False)
    return True


def choices(result):
    """{cache key: the chosen variant, energy spread or chunk target} of a tune() result."""
    return {k: next(r[f] for f in ("variant", "wg", "target") if f in r) for k, r in result.items()}


def _time_variant(grid, sample, kinds, precision, persistent, reps):
    import torch
    n = len(sample)
    idx = list(range(n))
    rad.profile_enable(True)
    try:
        if persistent:
            plan = rad.Plan(grid, sample, idx, n, kinds, precision)
            out = plan.launch()                      # warm-up
            torch.cuda.synchronize()
            rad.profile_read(reset=True)
            for _ in range(reps):
                plan.launch(out)
            torch.cuda.synchronize()
            plan.close()
        else:
            out = rad.batch(grid, sample, idx, n, kinds, precision)
            torch.cuda.synchronize()
            rad.profile_read(reset=True)
            for _ in range(reps):
                rad.batch(grid, sample, idx, n, kinds, precision, out=out)
            torch.cuda.synchronize()
        ms, launches = rad.profile_read(reset=True)
    finally:
        rad.profile_enable(False)
    return ms / max(launches, 1)


def pick_sample(dsegs, grid, min_segments=8, min_evals=3e11):
    """Longest segments first until the sample has both min_segments segments and
    min_evals (t, w, n) terms (long enough to fill the GPU several times over)."""
    order = sorted(range(len(dsegs)), key=lambda i: -dsegs.n[i])
    cube = grid.shape[0] * grid.shape[1] * grid.shape[2]
    take, evals = [], 0
    for i in order:
        if len(take) >= min_segments and evals >= min_evals:
            break
        take.append(i)
        evals += dsegs.n[i] * cube
    return take


def tune(grid, dsegs, kinds, precision=rad.FP64, persistent=False, sample=8, min_evals=3e11,
         reps=1, use_cache=True, verbose=False, shape=True):
    """Pick and set the fastest variant for every integral set of ``kinds``, then (with
    ``shape``, when the sample is the whole workload) the fastest spread over photon
    energies and chunk target.

    ``dsegs`` is a ``rad.DeviceSegments``; the longest segments are timed: at least
    ``sample`` of them and at least ``min_evals`` terms.
    Returns {cache key: {"variant" | "wg" | "target": choice, "ms": {choice: ms},
    "cached": bool}}.
    """
    path = cache_path()
    cache = _load(path) if use_cache else {}
    order = pick_sample(dsegs, grid, max(1, int(sample)), min_evals)
    sub = rad.DeviceSegments.__new__(rad.DeviceSegments)
    sub.n = [dsegs.n[i] for i in order]
    sub.data = dsegs.data
    sub.structs = (rad.Segment * len(order))(*[dsegs.structs[i] for i in order])
    max_n = max(dsegs.n)
    mixed = precision == rad.MIXED
    result = {}
    changed = False
    for with_j, set_kinds in _sets(kinds):
        k = key(persistent, precision, with_j, grid, max_n)
        if k in cache:
            rad.tune_set_variant(persistent, mixed, with_j, int(cache[k]["variant"]))
            result[k] = dict(cache[k], cached=True)
            continue
        times = {}
        for v in range(rad.tune_num_variants()):
            try:
                rad.tune_set_variant(persistent, mixed, with_j, v)
            except rad.RadError as e:
                if e.status == rad.EUNSUPPORTED:
                    continue                     # a tile without room for this set's accumulators
                raise
            times[v] = _time_variant(grid, sub, set_kinds, precision, persistent, reps)
            if verbose:
                print("autotune %s variant %d: %.3f ms" % (k, v, times[v]), flush=True)
        best = min(times, key=times.get)
        rad.tune_set_variant(persistent, mixed, with_j, best)
        cache[k] = {"variant": best, "ms": {str(v): t for v, t in times.items()}}
        result[k] = dict(cache[k], cached=False)
        changed = True
    if shape and len(order) == len(dsegs):
        time_call = lambda: _time_variant(grid, sub, kinds, precision, persistent, reps)   # noqa: E731
        n_w = grid.shape[0]
        wgs = [w for w in WG_CHOICES if w == 1 or n_w > 32 * w]     # at least half the block's energies exist
        changed |= _search(cache, shape_key(persistent, precision, kinds, grid, max_n, "wg"),
                           lambda w: rad.tune_set_shape(persistent, mixed, w), wgs, time_call, result, verbose,
                           "wg", default=default_wg(n_w))
        changed |= _search(cache, shape_key(persistent, precision, kinds, grid, max_n, "chunk"),
                           rad.tune_set_chunk_target, TARGET_CHOICES, time_call, result, verbose, "target",
                           default=2048)
    if changed and use_cache:
        _store(path, cache)
    return result
