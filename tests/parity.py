"""Parity metrics between a GPU cube and an oracle cube.

Oscillatory cancellation makes pointwise relative error unbounded where the
spectrum is ~0, so agreement is judged on norms:
  M1: ||dS||_2 / ||S||_2 over the whole cube,
  M2: max over photon energies of ||dS(w, .)||_2 / ||S(w, .)||_2,
  M3: max over photon energies of the relative error of dI/d hw.
Rows whose reference is exactly zero (forbidden photons) must be zero on both sides.
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


def assert_parity(gpu, ref, thx, thy, tol, what=""):
    m = metrics(gpu, ref, thx, thy)
    print("parity %s: M1 %.3e M2 %.3e M3 %.3e (tol %.1e)" % (what, m[0], m[1], m[2], tol), flush=True)
    assert max(m) <= tol, (what, m)
    return m
