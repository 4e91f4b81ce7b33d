"""Parity metrics between a GPU cube and an oracle cube.

Oscillatory cancellation makes pointwise relative error unbounded where the
spectrum is ~0, so agreement is judged on norms:
  M1: ||dS||_2 / ||S||_2 over the whole cube,
  M2: max over photon energies of ||dS(w, .)||_2 / ||S(w, .)||_2,
  M3: max over photon energies of the relative error of dI/d hw.
Rows whose reference is exactly zero (forbidden photons) must be zero on both sides.
Beside the norms, every element must pass the pointwise bound
  |dS| <= tol S + tol 1e-3 max_w S,
with max_w S the largest value of the reference over photon energies in the same
direction: an element far below its row's peak can no longer be wrong by more than
itself while the row's norm still passes.
"""
import numpy as np

import oracle


def metrics(gpu, ref, thx, thy):
    gpu = np.asarray(gpu, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    assert gpu.shape == ref.shape, (gpu.shape, ref.shape)
    assert np.all(np.isfinite(gpu)), "non-finite GPU output"
    d = gpu - ref
    m1 = np.linalg.norm(d) / max(np.linalg.norm(ref), 1e-300)
    rows_ref = np.sqrt(np.sum(ref ** 2, axis=(-2, -1)))
    rows_d = np.sqrt(np.sum(d ** 2, axis=(-2, -1)))
    zero = rows_ref == 0
    assert np.all(rows_d[zero] == 0), "GPU nonzero where the oracle row is exactly zero"
    m2 = float(np.max(rows_d[~zero] / rows_ref[~zero])) if np.any(~zero) else 0.0
    a = oracle.angle_integrate(gpu, thx, thy)
    b = oracle.angle_integrate(ref, thx, thy)
    nz = b != 0
    m3 = float(np.max(np.abs(a[nz] - b[nz]) / np.abs(b[nz]))) if np.any(nz) else 0.0
    return float(m1), m2, m3


def pointwise(gpu, ref, tol):
    """Largest |dS| / (tol S + tol 1e-3 max_w S) over the cube (<= 1 passes); the
    photon-energy axis is the third from the end ([..., n_w, n_y, n_x])."""
    gpu = np.asarray(gpu, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    d = np.abs(gpu - ref)
    peak = np.max(np.abs(ref), axis=-3, keepdims=True)
    bound = tol * np.abs(ref) + tol * 1e-3 * peak
    zero = bound == 0
    assert np.all(d[zero] == 0), "GPU nonzero where the oracle direction is exactly zero"
    return float(np.max(d[~zero] / bound[~zero])) if np.any(~zero) else 0.0


def assert_parity(gpu, ref, thx, thy, tol, what=""):
    m = metrics(gpu, ref, thx, thy)
    pw = pointwise(gpu, ref, tol)
    print("parity %s: M1 %.3e M2 %.3e M3 %.3e pointwise %.3f (tol %.1e)" % (what, m[0], m[1], m[2], pw, tol),
          flush=True)
    assert max(m) <= tol, (what, m)
    assert pw <= 1.0, (what, "pointwise", pw)
    return m
