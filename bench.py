#!/usr/bin/env python3
"""Benchmark of the radiation-integral hot path on one MI355X.

Workload (one "step" = one pass of the whole path over one batch): 256
positrons at 10 GeV channeled in a planar harmonic+quartic well (depth 20 eV,
width 1.92 A), 100 um, with multiple scattering and radiative loss, 4e4..1.2e5
samples per trajectory; spin-1/2 (BCK) spectrum on 512 log-spaced photon
energies in 0.5..200 MeV x 32 x 32 directions within 5/gamma; FP64.  Inputs are
seeded, synthetic and resident in HBM before the timed region.

Prints one JSON line: evals/s (one eval = one (t, w, n) term), trajectories/s,
the mixed-precision form's speed-up and error on the same workload, the
roofline of the amplitude kernel (HIP events on the library's stream) and the
CPU oracle timed on a bounded sample of the same workload.
"""
import argparse
import json
import math
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

METRIC = ("(t·ω·n) integrand evals/s and trajectories/s; "
          "mixed vs FP64 at stated rel err")

# MI355X: 256 CUs x 64 FP64 lanes x 2 flops (FMA) x 2.4 GHz
FP64_PEAK_TFLOPS = 78.6
VALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12     # VALU lane-instructions per second, 1e12
# Amplitude-kernel variants: direction tile (TX, TY) per lane and resident blocks per CU.
VARIANTS = {0: (4, 4, 2), 1: (4, 3, 2), 2: (4, 4, 1), 3: (4, 2, 2), 4: (4, 6, 2)}


def flops_per_eval(variant, with_j=True, recurrence=False):
    """FP64 flops per (t, w, n) eval of the amplitude kernel (FMA = 2).  Phase factors,
    34 flops each (phase product, exact reduction, f^2, an 8-term sine and a 9-term
    cosine polynomial, f * poly); complex products 6 flops each.  The first row of a
    TX x TY direction tile is folded into the x factors, so per time step the direct
    form evaluates TX + TY - 1 factors and forms TX (TY - 1) products; on a uniform grid
    (recurrence) it evaluates 4 (the tile's first factor, the multipliers along x and y
    and the shared second-difference factor) and forms 2 TX - 3 + 2 TY - 4 more products
    for the recurrences.  Then 2 flops per real accumulator and eval (A_x, A_y and J: 12)."""
    tx, ty, _ = VARIANTS[variant]
    rows = tx * (ty - 1)
    if recurrence:
        phase = (4 * 34.0 + 6.0 * (rows + 2 * tx - 3 + 2 * ty - 4)) / (tx * ty)
    else:
        phase = (34.0 * (tx + ty - 1) + 6.0 * rows) / (tx * ty)
    return phase + (12.0 if with_j else 8.0)


# VALU instructions per eval in the compiled hot loop of the 4x4 FP64 kernels (the
# persistent and the one-block-per-item kernel compile to the same loop), counted in the
# gfx950 assembly of this build (tests/test_codegen.py): direct phase factors 308 per 16
# evals with J (276 without), recurrence on a uniform grid 275 (243).
VALU_PER_EVAL_44 = {(True, False): 308.0 / 16.0, (False, False): 276.0 / 16.0,
                    (True, True): 275.0 / 16.0, (False, True): 243.0 / 16.0}
# HBM bytes per amp_persistent launch on this workload from two rocprofv3 PMC passes
# (FETCH_SIZE x2.000, WRITE_SIZE x1.000 after calibration on a 1 GiB copy), valid only
# for the kernel sources they were measured on (sha256 prefix below; a source change
# that leaves amp_persistent's gfx950 assembly identical is carried over after checking that).
KERNEL_SOURCES = ["paper_1910_10391_amd/csrc/rad_kernels.hip", "paper_1910_10391_amd/csrc/rad_math.h",
                  "paper_1910_10391_amd/csrc/sincos_coeffs.h", "paper_1910_10391_amd/csrc/rad_internal.h"]
MEASURED_TRAFFIC = {"sources_sha256": "2478343747b288b1", "particles": 256, "kernel": "amp_persistent",
                    "bytes_per_launch": 1.5467e10}


def kernel_sources_sha():
    import hashlib
    h = hashlib.sha256()
    for s in KERNEL_SOURCES:
        with open(os.path.join(ROOT, s), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=3)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--particles", type=int, default=0, help="0: the workload's own count")
    p.add_argument("--workload", default="positron_spinhalf",
                   choices=["positron_spinhalf", "electron_50gev_sections", "pm_mixed", "sweep", "traj", "sampler", "mlp"])
    p.add_argument("--no-mixed", action="store_true")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--copy-calibration", action="store_true",
                   help="run one device copy of known size first (counter scale factor)")
    p.add_argument("--no-legs", action="store_true",
                   help="skip the secondary legs of the default line (mixed-precision, sections, "
                        "undulator, sweep and trajectory-generator workloads, learned sampler, "
                        "issue-rate ceilings)")
    return p.parse_args()


def build_workload(n_particles):
    """The positron spin-1/2 workload: one segment per trajectory."""
    from paper_1910_10391_amd.synth import channeling, presets
    cfg = presets.positron_config()
    trs = channeling.generate(cfg, n_particles, threads=min(16, os.cpu_count() or 1))
    segs = [tr[0] for tr in trs]
    grid = presets.positron_grid()
    return cfg, segs, grid


def build_sections_workload(n_particles):
    """50 GeV electrons, 1 mm in 10 sections: segments, their trajectory index, grid."""
    from paper_1910_10391_amd.synth import channeling, presets
    cfg = presets.electron_50gev_config()
    trs = channeling.generate(cfg, n_particles, threads=min(16, os.cpu_count() or 1))
    segs, idx = [], []
    for p, secs in enumerate(trs):
        for sec in secs:
            segs.append(sec)
            idx.append(p)
    return segs, idx, presets.electron_50gev_grid()


def build_pm_workload(n_each):
    """n_each positrons + n_each electrons at 10 GeV, one segment each."""
    from paper_1910_10391_amd.synth import channeling, presets
    cp, ce = presets.pm_configs()
    th = min(16, os.cpu_count() or 1)
    segs = [tr[0] for tr in channeling.generate(cp, n_each, threads=th)]
    segs += [tr[0] for tr in channeling.generate(ce, n_each, threads=th)]
    return segs, presets.pm_grid()


def timed(fn, steps, sync):
    sync()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    sync()
    return (time.perf_counter() - t0) / steps


def bench_sections(args):
    """50 GeV sections workload: the persistent, autotuned, graph-replayed mixed-precision
    launch against the plain FP64 launch on the same GPU."""
    import torch
    from paper_1910_10391_amd import autotune, rad
    n = args.particles or 512
    segs, idx, g = build_sections_workload(n)
    ds = rad.DeviceSegments(segs)
    grid = rad.Grid(g.hw_eV, g.thx, g.thy)
    evals = int(sum(ds.n)) * int(np.prod(grid.shape))
    kinds = rad.SPINHALF
    print("bench: %d trajectories, %d sections, %.3e evals/step" % (n, len(segs), evals),
          file=sys.stderr, flush=True)
    tune_p = autotune.tune(grid, ds, kinds, rad.MIXED, persistent=True, sample=16)
    side = torch.cuda.Stream()
    out = torch.empty((n, 1) + grid.shape, dtype=torch.float64, device="cuda")
    with torch.cuda.stream(side):
        plan = rad.Plan(grid, ds, idx, n, kinds, precision=rad.MIXED, stream=side)
        for _ in range(args.warmup):
            plan.launch_graph(out, stream=side)
        dt_mx = timed(lambda: plan.launch_graph(out, stream=side), args.steps, side.synchronize)
    print("bench: mixed persistent graph %.3f s/step" % dt_mx, file=sys.stderr, flush=True)
    ws = torch.empty(rad.batch_workspace_bytes(grid, ds, n, kinds, rad.FP64), dtype=torch.uint8,
                     device="cuda")
    out64 = torch.empty_like(out)
    step64 = lambda: rad.batch(grid, ds, idx, n, kinds, rad.FP64, out=out64, workspace=ws)  # noqa
    step64()
    dt_64 = timed(step64, max(1, min(args.steps, 2)), torch.cuda.synchronize)
    print("bench: plain fp64 %.3f s/step" % dt_64, file=sys.stderr, flush=True)
    a, b = out[:, 0].cpu().numpy(), out64[:, 0].cpu().numpy()
    m1 = float(np.linalg.norm(a - b) / np.linalg.norm(b))
    return {
        "metric": METRIC, "value": evals / dt_mx, "unit": "evals/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": dt_mx * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64+f32",
        "data": "synthetic",
        "config": {"workload": "electron_50gev_sections: %d e- at 50 GeV, 1 mm in 10 sections, "
                               "%d..%d samples per section; spin-1/2, 256 log hw 1 MeV-20 GeV x "
                               "16x16 within 4/gamma; mixed precision, persistent plan replayed "
                               "from a hipGraph, autotuned" % (n, min(ds.n), max(ds.n)),
                   "segments": len(segs), "grid": list(grid.shape),
                   "autotune": autotune.choices(tune_p)},
        "trajectories_per_s": n / dt_mx,
        "fp64_plain": {"value": evals / dt_64, "ms_per_step": dt_64 * 1e3},
        "speedup_vs_fp64_plain": dt_64 / dt_mx,
        "mixed_vs_fp64_rel_err_M1": m1,
    }


def bench_pm(args):
    """1024 e+ + 1024 e- at 10 GeV, classical + spin-0 + spin-1/2 (two integral sets), mixed
    precision against FP64 on the same GPU."""
    import torch
    from paper_1910_10391_amd import rad
    n_each = (args.particles or 2048) // 2
    segs, g = build_pm_workload(n_each)
    ds = rad.DeviceSegments(segs)
    grid = rad.Grid(g.hw_eV, g.thx, g.thy)
    evals = 2 * int(sum(ds.n)) * int(np.prod(grid.shape))     # two integral sets (k and k*)
    idx = list(range(len(segs)))
    out = torch.empty((len(segs), 3) + grid.shape, dtype=torch.float64, device="cuda")
    out64 = torch.empty_like(out)
    ws = torch.empty(rad.batch_workspace_bytes(grid, ds, len(segs), 7, rad.FP64), dtype=torch.uint8,
                     device="cuda")
    print("bench: %d trajectories, %.3e evals/step" % (len(segs), evals), file=sys.stderr, flush=True)
    stepm = lambda: rad.batch(grid, ds, idx, len(segs), 7, rad.MIXED, out=out, workspace=ws)  # noqa
    step64 = lambda: rad.batch(grid, ds, idx, len(segs), 7, rad.FP64, out=out64, workspace=ws)  # noqa
    for _ in range(args.warmup):
        stepm()
    dt_mx = timed(stepm, args.steps, torch.cuda.synchronize)
    step64()
    dt_64 = timed(step64, 1, torch.cuda.synchronize)
    a, b = out.cpu().numpy(), out64.cpu().numpy()
    errs = {k: float(np.linalg.norm(a[:, i] - b[:, i]) / np.linalg.norm(b[:, i]))
            for i, k in enumerate(("classical", "spin0", "spinhalf"))}
    return {
        "metric": METRIC, "value": evals / dt_mx, "unit": "evals/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": dt_mx * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64+f32",
        "data": "synthetic",
        "config": {"workload": "pm_mixed: %d e+ + %d e- at 10 GeV, 100 um, %d..%d samples; "
                               "classical + spin-0 + spin-1/2, 256 log hw 0.5-200 MeV x 16x16 "
                               "within 5/gamma; mixed precision" % (n_each, n_each, min(ds.n),
                                                                   max(ds.n)),
                   "grid": list(grid.shape)},
        "trajectories_per_s": len(segs) / dt_mx,
        "fp64": {"value": evals / dt_64, "ms_per_step": dt_64 * 1e3},
        "speedup_vs_fp64": dt_64 / dt_mx,
        "mixed_vs_fp64_rel_err_M1": errs,
    }


SWEEP_WORKLOAD = ("sweep: 3000-sample undulator trajectory (gamma 2e4, K 0.5), FP64 classical, 10x10 "
                  "directions within 1/gamma x 1..1e6 linear hw up to 1.5 x the first harmonic")


def sweep_rows(counts, cpu_max):
    """One 3000-sample trajectory, FP64 classical spectrum, N integrals (10 x 10 directions x
    N / 100 photon energies) for each N in `counts`: GPU time with the inputs resident, as a
    plan replayed from a hipGraph, and including the host copies (trajectory in, cube out);
    the CPU oracle on the host's cores up to `cpu_max` integrals, and the GPU result's error
    against it."""
    import torch
    import oracle
    from paper_1910_10391_amd import rad
    from paper_1910_10391_amd.synth import analytic
    seg = analytic.undulator(2e4, 0.5, 20e-6, 20, n_steps=2999)
    ds = rad.DeviceSegments([seg])
    th = analytic.cell_centred(10, 1.0 / 2e4)
    fund = analytic.undulator_fundamental_eV(2e4, 0.5, 20e-6)
    rows = []
    for N in counts:
        n_w = N // 100
        hw = analytic.linear_omega(n_w, 1.5 * fund)
        grid = rad.Grid(hw, th, th)
        ws = torch.empty(rad.workspace_bytes(grid, ds.n[0], rad.CLASSICAL, rad.FP64), dtype=torch.uint8,
                         device="cuda")
        out = torch.empty(grid.shape, dtype=torch.float64, device="cuda")
        host = torch.empty(grid.shape, dtype=torch.float64, pin_memory=True)
        run = lambda: rad.classical(grid, ds, out=out, workspace=ws)  # noqa
        run()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        run()
        torch.cuda.synchronize()
        one = time.perf_counter() - t0
        reps = max(3, min(1000, int(0.3 / max(one, 1e-6))))
        dt = timed(run, reps, torch.cuda.synchronize)

        def with_copies():
            d2 = rad.DeviceSegments([seg])
            rad.classical(grid, d2, out=out, workspace=ws)
            host.copy_(out)
        dtc = timed(with_copies, max(2, reps // 4), torch.cuda.synchronize)
        # the same integrals as a captured plan replayed from a hipGraph (no host-side
        # planning or descriptor upload per call)
        st = torch.cuda.Stream()
        plan = rad.Plan(grid, ds, [0], 1, rad.CLASSICAL, rad.FP64, stream=st)
        pout = torch.empty((1, 1) + grid.shape, dtype=torch.float64, device="cuda")
        plan.launch_graph(pout, stream=st)
        st.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            plan.launch_graph(pout, stream=st)
        st.synchronize()
        dtg = (time.perf_counter() - t0) / reps
        gdiff = float((pout[0, 0] - out).abs().max() / out.abs().max().clamp_min(1e-300))
        assert gdiff < 1e-12, "graph replay differs from the direct call: %.3e" % gdiff
        plan.close()
        cpu, err = None, None
        if N <= cpu_max:
            t0 = time.perf_counter()
            ref = oracle.spectrum(seg, hw, th, th, oracle.KIND_CLASSICAL)[oracle.KIND_CLASSICAL]
            cpu = time.perf_counter() - t0
            err = float(np.linalg.norm(out.cpu().numpy() - ref) / np.linalg.norm(ref))
        rows.append({"integrals": N, "gpu_s": dt, "gpu_graph_s": dtg, "gpu_with_copies_s": dtc,
                     "cpu_oracle_s": cpu, "evals_per_s": 3000.0 * N / dt, "rel_err_vs_oracle_M1": err})
        print("bench sweep: %9d integrals  gpu %.3e s  graph replay %.3e s  with copies %.3e s  cpu %s" % (
            N, dt, dtg, dtc, "%.3e s" % cpu if cpu else "-"), file=sys.stderr, flush=True)
        del ws, out, host, pout
        grid.close()
    return rows


def sweep_crossover(rows):
    """The smallest count where the GPU with its copies beats the CPU oracle."""
    return next((r["integrals"] for r in rows if r["cpu_oracle_s"] and r["gpu_with_copies_s"] < r["cpu_oracle_s"]),
                None)


def bench_sweep(args):
    """Timing against the number of integrals (the axis of the paper's Sec. V timing
    figure): 10^2 .. 10^8 integrals, the CPU oracle up to 10^6; the crossover is the
    smallest count where the GPU with copies beats the CPU."""
    import oracle
    rows = sweep_rows([10 ** e for e in range(2, 9)], 10 ** 6)
    top = rows[-1]
    return {
        "metric": METRIC, "value": top["evals_per_s"], "unit": "evals/s", "n_gpus": 1,
        "steps": 1, "warmup": 1, "ms_per_step": top["gpu_s"] * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": SWEEP_WORKLOAD + "; 1e2..1e8 integrals"},
        "sweep": rows, "crossover_integrals_vs_cpu": sweep_crossover(rows), "cpu_cores": oracle.max_threads(),
    }


def leg_sweep():
    """The sweep at 10^2, 10^3, 10^4, 10^5, 10^6 and 10^8 integrals, the CPU oracle up to
    10^5 (a few seconds in all)."""
    import oracle
    rows = sweep_rows([10 ** 2, 10 ** 3, 10 ** 4, 10 ** 5, 10 ** 6, 10 ** 8], 10 ** 5)
    return {"workload": SWEEP_WORKLOAD + "; 1e2..1e8 integrals (CPU up to 1e5)", "rows": rows,
            "crossover_integrals_vs_cpu": sweep_crossover(rows), "cpu_cores": oracle.max_threads(),
            "evals_per_s_at_1e8": rows[-1]["evals_per_s"]}


def bench_traj(args):
    """Trajectory generation for the positron workload on the GPU (one thread per
    particle) against the CPU generator on the host's cores, and the end-to-end step
    (generate on the GPU, then the FP64 spin-1/2 spectrum) with no host round trip."""
    import torch
    from paper_1910_10391_amd import rad, traj
    from paper_1910_10391_amd.synth import channeling, presets
    n = args.particles or 256
    cfg = presets.positron_config()
    threads = min(16, os.cpu_count() or 1)
    t0 = time.perf_counter()
    trs = channeling.generate(cfg, n, threads=threads)
    cpu_gen = time.perf_counter() - t0
    t0 = time.perf_counter()
    ds_host = rad.DeviceSegments([tr[0] for tr in trs])
    torch.cuda.synchronize()
    h2d = time.perf_counter() - t0
    del ds_host
    traj.DeviceTrajectories(cfg, n)          # warm-up
    torch.cuda.synchronize()
    gen = lambda: traj.DeviceTrajectories(cfg, n)  # noqa
    dt_gen = timed(gen, max(1, args.steps), torch.cuda.synchronize)
    dt = gen()
    samples = int(sum(dt.n))
    print("bench traj: %d particles, %d samples: gpu %.3f s, cpu generator %.3f s (%d threads), "
          "host->device copy %.3f s" % (n, samples, dt_gen, cpu_gen, threads, h2d), file=sys.stderr, flush=True)
    g = presets.positron_grid()
    grid = rad.Grid(g.hw_eV, g.thx, g.thy)
    ws = torch.empty(rad.batch_workspace_bytes(grid, dt, n, rad.SPINHALF, rad.FP64), dtype=torch.uint8,
                     device="cuda")
    out = torch.empty((n, 1) + grid.shape, dtype=torch.float64, device="cuda")

    def step():
        d = traj.DeviceTrajectories(cfg, n)
        rad.batch(grid, d, list(range(n)), n, rad.SPINHALF, rad.FP64, out=out, workspace=ws)
    step()
    dt_step = timed(step, 1, torch.cuda.synchronize)
    evals = samples * int(np.prod(grid.shape))
    return {
        "metric": METRIC, "value": evals / dt_step, "unit": "evals/s", "n_gpus": 1, "steps": 1,
        "warmup": 1, "ms_per_step": dt_step * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "traj: %d positrons at 10 GeV, 100 um, generated on the GPU, then FP64 "
                               "spin-1/2 on 512 log hw x 32x32" % n},
        "generation": {"gpu_s": dt_gen, "cpu_generator_s": cpu_gen, "cpu_threads": threads,
                       "host_to_device_copy_s": h2d, "samples": samples,
                       "gpu_samples_per_s": samples / dt_gen, "speedup_vs_cpu": cpu_gen / dt_gen},
        "trajectories_per_s_end_to_end": n / dt_step,
    }


def _finite(o):
    """JSON-safe copy: non-finite floats become None."""
    if isinstance(o, dict):
        return {k: _finite(v) for k, v in o.items()}
    if isinstance(o, (list, tuple)):
        return [_finite(v) for v in o]
    if isinstance(o, float) and not math.isfinite(o):
        return None
    return o


def bench_sampler(args):
    """The learned angular sampler on held-out positron trajectories: train (spectra
    computed by the library, BF16 MLP on the GPU), tune its settings on validation trajectories,
    then time the sampler against the full 64 x 64 grid (both mixed precision, spin-1/2,
    512 log hw).  value = full-grid evaluations replaced per second, i.e. the full grid's
    evals divided by the sampler's time, at the measured error."""
    import tempfile
    from paper_1910_10391_amd import train_sampler
    with tempfile.TemporaryDirectory() as d:
        rep = train_sampler.main(["--report", os.path.join(d, "r.json"), "--test", str(args.particles or 64)])
    t = rep["test"]
    L = t[rep["learned_rule"]]
    return _finite({
        "metric": METRIC, "value": L["evals_full"] / L["seconds"], "unit": "evals/s", "n_gpus": 1,
        "steps": 1, "warmup": 1, "ms_per_step": L["seconds"] * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64+f32+bf16", "data": "synthetic",
        "config": {"workload": "sampler: %d held-out positrons at 10 GeV, 100 um; spin-1/2 on 512 log hw x "
                               "64x64 within 5/gamma, 8x8 cells; network trained on %d x 64 spectra"
                               % (rep["config"]["particles_test"], rep["config"]["particles_train"])},
        "speedup_vs_full_grid": L["speedup_vs_full"], "max_rel_err": L["max_rel_err"],
        "accepted_1pct": rep["accepted"], "learned_rule": rep["learned_rule"], "settings": rep["settings"],
        "evals_frac": L["evals_frac"], "learned_mass": t["learned"], "learned_error": t["learned_error"],
        "coarse_guided": t["coarse"], "coarse_only": t["coarse_only"],
        "full_grid_s": t["full_grid_seconds"], "training_s": rep.get("training_seconds"),
    })


def bench_mlp(args):
    """The sampler's network on the GPU: fused inference over every (trajectory, point) pair
    of the sampler's grid (64 trajectories x 512 energies x 64 x 64 directions) and training
    steps of 65 536 points; random weights and inputs of the sampler's shapes."""
    import torch
    from paper_1910_10391_amd.mlp import MLP
    n_traj, n_pts = (args.particles or 64), 512 * 64 * 64
    rng = np.random.default_rng(0)
    net = MLP(38, 3, seed=1)
    feat = torch.from_numpy((0.5 * rng.normal(size=(n_traj, 38))).astype(np.float32)).cuda()
    table = torch.from_numpy(rng.uniform(-1, 1, size=(n_pts, 3)).astype(np.float32)).cuda()
    y = torch.empty((n_traj, n_pts), dtype=torch.float32, device="cuda")
    net.forward_grid(feat, table, y=y)
    dt = timed(lambda: net.forward_grid(feat, table, y=y), max(1, args.steps), torch.cuda.synchronize)
    pts = n_traj * n_pts
    # dense products per point: two 256 x 256 layers on the MFMA units, 3 -> 256 and 256 -> 1 on the VALU
    mfma_flops = 2.0 * 2 * 256 * 256
    all_flops = mfma_flops + 2.0 * (3 * 256 + 256)
    B = 65536
    traj = torch.from_numpy(rng.integers(0, n_traj, B).astype(np.int32)).cuda()
    x = torch.from_numpy(rng.uniform(-1, 1, size=(B, 3)).astype(np.float32)).cuda()
    t = torch.from_numpy(rng.normal(size=B).astype(np.float32)).cuda()
    net.train_step(feat, traj, x, t, 1e-4)
    dt_tr = timed(lambda: net.train_step(feat, traj, x, t, 1e-4), 50, torch.cuda.synchronize)
    print("bench mlp: inference %.1f ms for %d points (%.3e points/s); training step %.2f ms" % (
        dt * 1e3, pts, pts / dt, dt_tr * 1e3), file=sys.stderr, flush=True)
    tf = pts * mfma_flops / dt / 1e12
    tr_bytes = mlp_training_bytes(B, 41)
    tr_flops = mlp_training_flops(B, 41)
    return {
        "metric": "network evaluations (points) per second", "value": pts / dt, "unit": "points/s", "n_gpus": 1,
        "steps": max(1, args.steps), "warmup": 1, "ms_per_step": dt * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "bf16", "data": "synthetic",
        "config": {"workload": "mlp: 38 features + 3 point inputs -> 256 -> 256 -> 256 -> 1, fused inference over "
                               "%d trajectories x %d points; training batches of %d" % (n_traj, n_pts, B)},
        "roofline": {"bound": "mfma", "achieved": tf, "peak": 2500.0, "unit": "TFLOP/s", "frac": tf / 2500.0,
                     "traffic": None},
        "all_flops_tflops": pts * all_flops / dt / 1e12,
        "training_step_ms": dt_tr * 1e3, "training_points_per_s": B / dt_tr,
        "training_roofline": {"bound": "hbm", "achieved": tr_bytes / dt_tr / 1e9, "peak": 8000.0, "unit": "GB/s",
                              "frac": tr_bytes / dt_tr / 8e12, "bytes": tr_bytes,
                              "mfma_tflops": tr_flops / dt_tr / 1e12},
    }


def mlp_training_bytes(B, n_in):
    """Algorithmic HBM bytes of one training step of B points (B a multiple of 128): every
    activation, SiLU derivative, dz and k8 copy written once and read by its consumers,
    the split-K and per-block partials, Adam's four parameter-sized arrays."""
    a = B * 256 * 2                           # one BF16 activation-sized array
    i1 = B * 64 * 2                           # the padded layer-1 input
    P = 256 * n_in + 256 + 2 * (256 * 256 + 256) + 256 + 1
    wp = 64 * 256 * 4                         # split-K partial rows per output row
    total = B * 16 + 2 * i1                   # assemble: traj + x in, in1 + in1_k8 out
    total += i1 + 3 * a                       # layer 1: in1 in; h1, ds1, h1_k8 out
    total += a + 3 * a                        # layer 2
    total += a + 2 * a                        # layer 3 (no k8 copy)
    total += 2 * a + B * 4 + 2 * a + (B // 64) * 514 * 4      # output layer and dz3
    total += 2 * (2 * a + wp * 256)           # dW3, dW2 partials
    total += 2 * (2 * a + 2 * a + (B // 128) * 256 * 4)       # dz2, dz1 (with their k8 copies)
    total += a + i1 + wp * 64                 # dW1 partials
    total += 2 * wp * 256 + wp * 64 + (B // 64) * 514 * 4 + 2 * (B // 128) * 256 * 4   # final reductions
    total += 7 * P * 4                        # Adam: p, m1, m2, g in; p, m1, m2 out
    return float(total)


def mlp_training_flops(B, n_in):
    """Dense products of one training step: forward 41(64) -> 256 -> 256 -> 256, the two
    backward data products and the three weight-gradient products (2 flops per MAC)."""
    fwd = 2.0 * B * (64 * 256 + 2 * 256 * 256)
    bwd = 2.0 * B * (2 * 256 * 256) + 2.0 * B * (2 * 256 * 256 + 256 * 64)
    return fwd + bwd


def sample_points(segs, grid):
    """The bounded sample (about 10 s of the oracle on 16 cores): the 4 shortest and the
    4 longest trajectories, every 2nd photon energy, an 8 x 8 strided subset of directions."""
    order = np.argsort([s["t"].size for s in segs], kind="stable")
    traj = sorted(set([int(i) for i in order[:4]] + [int(i) for i in order[-4:]]))
    iw = np.arange(0, len(grid.hw_eV), 2)
    ix = np.arange(0, len(grid.thx), max(1, len(grid.thx) // 8))
    iy = np.arange(0, len(grid.thy), max(1, len(grid.thy) // 8))
    return traj, iw, ix, iy


def cpu_baseline(segs, grid, traj, iw, ix, iy):
    import oracle
    hw, thx, thy = grid.hw_eV[iw], grid.thx[ix], grid.thy[iy]
    threads = oracle.max_threads()
    evals = 0
    ref = {}
    t0 = time.perf_counter()
    for p in traj:
        ref[p] = oracle.spectrum(segs[p], hw, thx, thy, oracle.KIND_SPINHALF)[4]
        evals += segs[p]["t"].size * hw.size * thx.size * thy.size
    dt = time.perf_counter() - t0
    return ref, evals / dt, dt, threads, evals


def cpu_single_core(segs, grid, traj, iw, ix, iy):
    """The oracle on one host core: the shortest trajectory of the sample at every 4th of
    its photon energies and its directions (a few seconds); evals/s and what it was."""
    import oracle
    p = min(traj, key=lambda i: segs[i]["t"].size)
    hw, thx, thy = grid.hw_eV[iw[::4]], grid.thx[ix], grid.thy[iy]
    oracle.spectrum(segs[p], hw[:1], thx[:1], thy[:1], oracle.KIND_SPINHALF, threads=1)   # warm-up
    t0 = time.perf_counter()
    oracle.spectrum(segs[p], hw, thx, thy, oracle.KIND_SPINHALF, threads=1)
    dt = time.perf_counter() - t0
    evals = segs[p]["t"].size * hw.size * thx.size * thy.size
    return {"value": evals / dt, "unit": "evals/s", "cores": 1,
            "sample": "trajectory %d, %d photon energies x %dx%d directions, %.3e evals in %.1f s"
                      % (p, hw.size, thx.size, thy.size, evals, dt)}


def rel_metrics(got, ref):
    d = got - ref
    m1 = float(np.linalg.norm(d) / np.linalg.norm(ref))
    rows = np.sqrt(np.sum(ref ** 2, axis=(-2, -1)))
    m2 = float(np.max(np.sqrt(np.sum(d ** 2, axis=(-2, -1)))[rows > 0] / rows[rows > 0]))
    return m1, m2


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor()


# ---------------------------------------------------------------- legs of the default line
# Each leg is one further configuration of the same path, measured once or twice (not
# `--steps` times) so that the default run stays within a few minutes.

PAPER_CONTEXT = {
    "source": "Sec. V, Fig. 7 (speed-ups of classical FP64 radiation integrals of 3000 time "
              "points each, GPU saturated; other hardware, quoted as context, not as a target)",
    "titan_v_vs_i7_7820x": 205.1,
    "titan_v_vs_one_xeon_gold_6140_node": "about 100 (the Xeon node, 36 hardware threads, runs about 2x "
                                          "the i7-7820X)",
}

# gfx950 hot loop of the mixed-precision 4x4 kernel with J, per 16 evaluations (time
# step x direction tile), counted in the assembly by tests/test_codegen.py: 201 VALU
# instructions, 14 of them transcendental (7 v_sin_f32 + 7 v_cos_f32).
MIXED_VALU_PER_16 = 201
MIXED_TRANS_PER_16 = 14
VALU_LANE_PEAK_T = 256 * 64 * 2.4e9 / 1e12   # lane-instructions per second at 2.4 GHz, 1e12


def leg_peaks():
    """Issue-rate ceilings measured on this GPU (rad_peak)."""
    from paper_1910_10391_amd import rad
    res = {}
    for name, which, iters in (("fp64_fma", rad.PEAK_FMA64, 4096), ("fp32_fma", rad.PEAK_FMA32, 4096),
                               ("sincos_f32", rad.PEAK_SINCOS32, 1024), ("phase_fp64", rad.PEAK_PHASE64, 256),
                               ("phase_mixed", rad.PEAK_PHASE_MIXED, 256)):
        rate, ops, ms = rad.peak(which, iters)
        res[name] = {"per_s": rate, "ms": ms}
    res["fp64_fma"]["tflops"] = res["fp64_fma"]["per_s"] / 1e12
    res["fp64_fma"]["frac_of_78.6"] = res["fp64_fma"]["tflops"] / FP64_PEAK_TFLOPS
    res["fp32_fma"]["tflops"] = res["fp32_fma"]["per_s"] / 1e12
    # lane-instructions per second: an FMA is one instruction (2 flops), a sine one
    fma_lane = res["fp64_fma"]["per_s"] / 2.0
    res["sincos_f32"]["cost_in_fma64_slots"] = fma_lane / res["sincos_f32"]["per_s"]
    res["clock_ghz_implied_by_fp64_fma"] = fma_lane / (256 * 64) / 1e9
    return res


def mixed_roofline(evals_per_s, peaks):
    """The mixed form's issue roofline: VALU lane-instructions per evaluation of its hot
    loop, the transcendental ones weighted by their measured cost in FMA issue slots,
    against the chip's lane-instruction rate at the nominal clock."""
    w = peaks["sincos_f32"]["cost_in_fma64_slots"] if peaks else 4.0
    per_eval = ((MIXED_VALU_PER_16 - MIXED_TRANS_PER_16) + w * MIXED_TRANS_PER_16) / 16.0
    achieved = evals_per_s * per_eval / 1e12
    measured_ceiling = peaks["fp64_fma"]["per_s"] / 2.0 / 1e12 if peaks else None
    return {"bound": "alu", "achieved": achieved, "peak": VALU_LANE_PEAK_T,
            "unit": "T VALU lane-instructions/s (transcendentals weighted by measured cost)",
            "frac": achieved / VALU_LANE_PEAK_T, "traffic": None,
            "kernel": "amp_persistent<4,4,J,mixed,2>", "valu_per_eval": per_eval, "sincos_weight": w,
            "frac_of_measured_fma_issue": achieved / measured_ceiling if measured_ceiling else None}


def leg_pm_mixed():
    """The mixed-precision workload: 1024 e+ + 1024 e- at 10 GeV, classical + spin-0 +
    spin-1/2 on 256 log hw x 16 x 16; mixed against FP64 on the GPU, and the error of each
    spectrum against the FP64 oracle on a sample (2 e+ and 2 e-, every 4th energy, 8 x 8
    strided directions)."""
    import torch
    import oracle
    from paper_1910_10391_amd import rad
    t0 = time.perf_counter()
    segs, g = build_pm_workload(1024)
    ds = rad.DeviceSegments(segs)
    grid = rad.Grid(g.hw_eV, g.thx, g.thy)
    n = len(segs)
    evals = 2 * int(sum(ds.n)) * int(np.prod(grid.shape))
    idx = list(range(n))
    ws = torch.empty(rad.batch_workspace_bytes(grid, ds, n, 7, rad.FP64), dtype=torch.uint8, device="cuda")
    out = torch.empty((n, 3) + grid.shape, dtype=torch.float64, device="cuda")
    t_prep = time.perf_counter() - t0
    stepm = lambda: rad.batch(grid, ds, idx, n, 7, rad.MIXED, out=out, workspace=ws)  # noqa: E731
    stepm()
    dt_mx = timed(stepm, 1, torch.cuda.synchronize)
    sample = [0, 1, 1024, 1025]
    iw, ixy = np.arange(0, len(g.hw_eV), 4), np.arange(0, len(g.thx), 2)
    sel = np.ix_(iw, ixy, ixy)
    got_mx = {p: out[p].cpu().numpy()[(slice(None),) + sel] for p in sample}
    step64 = lambda: rad.batch(grid, ds, idx, n, 7, rad.FP64, out=out, workspace=ws)  # noqa: E731
    dt_64 = timed(step64, 1, torch.cuda.synchronize)
    got_64 = {p: out[p].cpu().numpy()[(slice(None),) + sel] for p in sample}
    del ws, out
    errs = {}
    for i, (k, name) in enumerate(((1, "classical"), (2, "spin0"), (4, "spinhalf"))):
        e_mx, e_64 = [], []
        for p in sample:
            ref = oracle.spectrum(segs[p], g.hw_eV[iw], g.thx[ixy], g.thy[ixy], k)[k]
            e_mx.append(rel_metrics(got_mx[p][i], ref))
            e_64.append(rel_metrics(got_64[p][i], ref))
        errs[name] = {"mixed_M1": max(e[0] for e in e_mx), "mixed_M2": max(e[1] for e in e_mx),
                      "fp64_M1": max(e[0] for e in e_64), "fp64_M2": max(e[1] for e in e_64)}
    print("bench leg pm_mixed: mixed %.3f s, fp64 %.3f s (x%.2f)" % (dt_mx, dt_64, dt_64 / dt_mx),
          file=sys.stderr, flush=True)
    return {"workload": "pm_mixed: 1024 e+ + 1024 e- at 10 GeV, 100 um, %d..%d samples; classical + spin-0 + "
                        "spin-1/2 (two integral sets), 256 log hw 0.5-200 MeV x 16x16 within 5/gamma"
                        % (min(ds.n), max(ds.n)),
            "evals": evals, "mixed": {"value": evals / dt_mx, "unit": "evals/s", "ms_per_step": dt_mx * 1e3,
                                      "trajectories_per_s": n / dt_mx},
            "fp64": {"value": evals / dt_64, "unit": "evals/s", "ms_per_step": dt_64 * 1e3},
            "speedup_mixed_vs_fp64": dt_64 / dt_mx,
            "rel_err_vs_oracle": errs,
            "oracle_sample": "trajectories %s (2 e+, 2 e-), every 4th of 256 energies, 8x8 strided directions"
                             % sample, "prep_s": t_prep}


def leg_sections():
    """The 50 GeV sections workload: the persistent, autotuned mixed-precision plan replayed
    from a hipGraph against the plain FP64 rad_batch on the same GPU; errors against FP64
    on the GPU (whole cubes) and against the oracle (one trajectory, every 8th energy, 4 x 4
    strided directions)."""
    import torch
    import oracle
    from paper_1910_10391_amd import autotune, rad
    n = 512
    segs, idx, g = build_sections_workload(n)
    ds = rad.DeviceSegments(segs)
    grid = rad.Grid(g.hw_eV, g.thx, g.thy)
    evals = int(sum(ds.n)) * int(np.prod(grid.shape))
    tune = autotune.tune(grid, ds, rad.SPINHALF, rad.MIXED, persistent=True, sample=16)
    side = torch.cuda.Stream()
    out = torch.empty((n, 1) + grid.shape, dtype=torch.float64, device="cuda")
    with torch.cuda.stream(side):
        plan = rad.Plan(grid, ds, idx, n, rad.SPINHALF, precision=rad.MIXED, stream=side)
        plan.launch_graph(out, stream=side)
        dt_mx = timed(lambda: plan.launch_graph(out, stream=side), 2, side.synchronize)
    plan.close()
    ws = torch.empty(rad.batch_workspace_bytes(grid, ds, n, rad.SPINHALF, rad.FP64), dtype=torch.uint8,
                     device="cuda")
    out64 = torch.empty_like(out)
    step64 = lambda: rad.batch(grid, ds, idx, n, rad.SPINHALF, rad.FP64, out=out64, workspace=ws)  # noqa: E731
    dt_64 = timed(step64, 1, torch.cuda.synchronize)
    a, b = out[:, 0].cpu().numpy(), out64[:, 0].cpu().numpy()
    del ws, out, out64
    m1 = float(np.linalg.norm(a - b) / np.linalg.norm(b))
    iw, ixy = np.arange(0, len(g.hw_eV), 8), np.arange(0, len(g.thx), 4)
    p = 0
    mine = [s for s, o in zip(segs, idx) if o == p]
    ref = oracle.batch(mine, [0] * len(mine), 1, g.hw_eV[iw], g.thx[ixy], g.thy[ixy], 4)[0, 0]
    sel = np.ix_(iw, ixy, ixy)
    e_mx, e_64 = rel_metrics(a[p][sel], ref), rel_metrics(b[p][sel], ref)
    print("bench leg sections: mixed graph %.3f s, fp64 %.3f s (x%.2f)" % (dt_mx, dt_64, dt_64 / dt_mx),
          file=sys.stderr, flush=True)
    return {"workload": "electron_50gev_sections: 512 e- at 50 GeV, 1 mm in 10 sections (%d segments, %d..%d "
                        "samples each); spin-1/2, 256 log hw 1 MeV-20 GeV x 16x16 within 4/gamma"
                        % (len(segs), min(ds.n), max(ds.n)),
            "evals": evals,
            "mixed_graph": {"value": evals / dt_mx, "unit": "evals/s", "ms_per_step": dt_mx * 1e3,
                            "trajectories_per_s": n / dt_mx, "form": "persistent plan, hipGraph replay",
                            "autotune": autotune.choices(tune)},
            "fp64_plain": {"value": evals / dt_64, "unit": "evals/s", "ms_per_step": dt_64 * 1e3,
                           "form": "rad_batch"},
            "speedup_mixed_graph_vs_fp64_plain": dt_64 / dt_mx,
            "mixed_vs_fp64_gpu_M1": m1,
            "rel_err_vs_oracle": {"mixed_M1": e_mx[0], "mixed_M2": e_mx[1], "fp64_M1": e_64[0], "fp64_M2": e_64[1],
                                  "sample": "trajectory 0 (10 sections), every 8th energy, 4x4 strided directions"}}


def leg_undulator():
    """The smallest configuration: one electron on the analytic undulator trajectory (gamma 2e4,
    K 0.5, 20 periods of 20 um in 8192 steps), FP64 classical spectrum on 128 linear hw up to
    1.5 x the first harmonic x 16 x 16 directions within 1/gamma; GPU time per call (median of
    repeated calls, inputs resident) and the whole cube against the oracle."""
    import torch
    import oracle
    from paper_1910_10391_amd import rad
    from paper_1910_10391_amd.synth import presets
    c = presets.undulator_fp64()
    g = c["grid"]
    seg = c["segments"][0]
    ds = rad.DeviceSegments([seg])
    grid = rad.Grid(g.hw_eV, g.thx, g.thy)
    ws = torch.empty(rad.workspace_bytes(grid, ds.n[0], rad.CLASSICAL, rad.FP64), dtype=torch.uint8, device="cuda")
    out = torch.empty(grid.shape, dtype=torch.float64, device="cuda")
    run = lambda: rad.classical(grid, ds, out=out, workspace=ws)  # noqa: E731
    run()
    torch.cuda.synchronize()
    times = []
    for _ in range(20):
        t0 = time.perf_counter()
        run()
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    dt = float(np.median(times))
    evals = int(seg["t"].size) * int(np.prod(grid.shape))
    t0 = time.perf_counter()
    ref = oracle.spectrum(seg, g.hw_eV, g.thx, g.thy, oracle.KIND_CLASSICAL)[oracle.KIND_CLASSICAL]
    cpu = time.perf_counter() - t0
    m1, m2 = rel_metrics(out.cpu().numpy(), ref)
    grid.close()
    print("bench leg undulator: gpu %.3f ms per call, oracle %.3f s, M1 %.2e" % (dt * 1e3, cpu, m1),
          file=sys.stderr, flush=True)
    return {"workload": "undulator_fp64: 1 e- at gamma 2e4, K 0.5, 20 periods of 20 um in 8192 steps; FP64 "
                        "classical, 128 linear hw up to 1.5 x the first harmonic x 16x16 within 1/gamma",
            "evals": evals, "gpu_ms_per_call": dt * 1e3, "evals_per_s": evals / dt,
            "cpu_oracle_s": cpu, "cpu_cores": oracle.max_threads(), "speedup_vs_oracle": cpu / dt,
            "rel_err_vs_oracle": {"M1": m1, "M2": m2, "sample": "the whole cube"}}


def leg_traj():
    """The GPU trajectory generator on the benchmark's 256 positrons against the CPU generator
    on the host's cores (and the host-to-device copy the GPU generator saves); four of the
    particles compared with the CPU generator's columns bit for bit."""
    import torch
    from paper_1910_10391_amd import rad, traj
    from paper_1910_10391_amd.synth import channeling, presets
    n = 256
    cfg = presets.positron_config()
    threads = min(16, os.cpu_count() or 1)
    t0 = time.perf_counter()
    trs = channeling.generate(cfg, n, threads=threads)
    cpu_gen = time.perf_counter() - t0
    t0 = time.perf_counter()
    ds_host = rad.DeviceSegments([tr[0] for tr in trs])
    torch.cuda.synchronize()
    h2d = time.perf_counter() - t0
    del ds_host, trs
    traj.DeviceTrajectories(cfg, n)          # warm-up
    torch.cuda.synchronize()
    dt_gen = timed(lambda: traj.DeviceTrajectories(cfg, n), 2, torch.cuda.synchronize)
    d = traj.DeviceTrajectories(cfg, n)
    cols = ("t", "x", "y", "dz", "vx", "vy", "dvz", "ax", "ay", "az", "energy")
    same = all(np.array_equal(d.host(i)[c], ref[c])
               for i in (0, 85, 170, 255) for ref in [channeling.trajectory(cfg, i)] for c in cols)
    samples = int(sum(d.n))
    print("bench leg traj: gpu %.3f s, cpu generator %.3f s (%d threads), host->device copy %.3f s, "
          "sampled particles bitwise equal: %s" % (dt_gen, cpu_gen, threads, h2d, same), file=sys.stderr, flush=True)
    return {"workload": "traj: the benchmark's %d positrons (%d samples) generated on the GPU" % (n, samples),
            "gpu_s": dt_gen, "cpu_generator_s": cpu_gen, "cpu_threads": threads, "host_to_device_copy_s": h2d,
            "speedup_vs_cpu": cpu_gen / dt_gen, "speedup_vs_cpu_plus_copy": (cpu_gen + h2d) / dt_gen,
            "gpu_samples_per_s": samples / dt_gen, "bitwise_equal_particles_0_85_170_255": bool(same)}


SAMPLER_CKPT = os.path.join(ROOT, "paper_1910_10391_amd", "weights", "positron_spinhalf_sampler.npz")


def leg_sampler(n_test=32):
    """The learned angular sampler (committed network) on held-out positrons: spin-1/2 on
    512 log hw x 64 x 64 directions within 5/gamma, 8 x 8 cells; against the full grid in
    mixed precision (the reference for its error) and in plain FP64."""
    import torch
    from paper_1910_10391_amd import rad, sampler
    from paper_1910_10391_amd.synth import channeling, presets
    from paper_1910_10391_amd.train_sampler import errors
    cfg, pg = presets.positron_config(), presets.positron_grid()
    gamma = cfg.energy_eV / channeling.ME_EV
    smp = sampler.Sampler.load(SAMPLER_CKPT, pg.hw_eV, gamma)
    trs = channeling.generate(cfg, n_test, first=70000, threads=min(16, os.cpu_count() or 1))
    ds = rad.DeviceSegments([tr[0] for tr in trs])
    smp.full_grid(ds, rad.MIXED)
    full_mx, t_mx = min((smp.full_grid(ds, rad.MIXED) for _ in range(2)), key=lambda r: r[1])
    full_64, t_64 = smp.full_grid(ds, rad.FP64)
    smp.estimate(ds, precision=rad.MIXED)
    est = min((smp.estimate(ds, precision=rad.MIXED) for _ in range(2)), key=lambda r: r["seconds"])
    steps = smp.estimate(ds, precision=rad.MIXED, phases=True)["phases"]   # a synchronised run, per step
    full = full_mx.cpu().numpy()
    rel, _ = errors(est["dIdw"].cpu().numpy(), full)
    rel64, _ = errors(full_64.cpu().numpy(), full)
    print("bench leg sampler: %.3f s (full grid mixed %.3f s, fp64 %.3f s), max rel err %.4f"
          % (est["seconds"], t_mx, t_64, rel.max()), file=sys.stderr, flush=True)
    return {"workload": "sampler: %d held-out positrons at 10 GeV, 100 um; spin-1/2 on 512 log hw x 64x64 "
                        "within 5/gamma, 8x8 cells, committed network (%s rule)" % (n_test, smp.select_rule),
            "seconds": est["seconds"], "full_grid_mixed_s": t_mx, "full_grid_fp64_s": t_64,
            "speedup_vs_full_grid_mixed": t_mx / est["seconds"],
            "speedup_vs_full_grid_fp64": t_64 / est["seconds"],
            "max_rel_err_dIdw": float(rel.max()), "accepted_1pct": bool(rel.max() <= 0.01),
            "evals_frac": est["evals"] / est["evals_full"],
            "full_evals_replaced_per_s": est["evals_full"] / est["seconds"],
            "mixed_full_grid_vs_fp64_max_rel": float(rel64.max()), "phases_s": steps}


def run_leg(name, fn):
    try:
        return fn()
    except Exception as e:  # noqa: BLE001 -- a failed leg is reported in the line, not hidden
        import traceback
        traceback.print_exc()
        return {"error": "%s: %s" % (type(e).__name__, e)}


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: this build runs on exactly one GPU (--gpus 1); multi-GPU sharding is a "
              "design note only", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_1910_10391_amd import autotune, rad

    if args.workload != "positron_spinhalf":
        fn = {"electron_50gev_sections": bench_sections, "pm_mixed": bench_pm,
              "sweep": bench_sweep, "traj": bench_traj,
              "sampler": bench_sampler, "mlp": bench_mlp}[args.workload]
        print(json.dumps(fn(args)), flush=True)
        return
    t_gen = time.perf_counter()
    cfg, segs, g = build_workload(args.particles or 256)
    t_gen = time.perf_counter() - t_gen
    torch.cuda.set_device(0)
    dev = torch.device("cuda", 0)
    ds = rad.DeviceSegments(segs, device=dev)
    grid = rad.Grid(g.hw_eV, g.thx, g.thy)
    n_w, n_y, n_x = grid.shape
    n_samples = int(sum(ds.n))
    evals = n_samples * n_w * n_x * n_y
    idx = list(range(len(segs)))
    kinds = rad.SPINHALF
    ws = torch.empty(rad.batch_workspace_bytes(grid, ds, len(segs), kinds, rad.FP64),
                     dtype=torch.uint8, device=dev)
    out = torch.empty((len(segs), 1) + grid.shape, dtype=torch.float64, device=dev)
    print("bench: %d trajectories, %d samples, grid %s, %.3e evals/step, workspace %.2f GB, "
          "inputs generated in %.1f s" % (len(segs), n_samples, grid.shape, evals, ws.numel() / 1e9,
                                          t_gen), file=sys.stderr, flush=True)

    tuned = autotune.tune(grid, ds, kinds, rad.FP64, persistent=True, sample=8)
    print("bench: autotuned %s (sample ms %s)" % (autotune.choices(tuned), {k: v["ms"] for k, v in tuned.items()}),
          file=sys.stderr, flush=True)

    if args.copy_calibration:
        a = torch.ones(1 << 27, dtype=torch.float64, device=dev)    # 1 GiB
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    def step(prec, o):
        # one pass of the batched form over the batch: plan it (longest-first work list,
        # descriptors uploaded into the workspace), then the persistent amplitude kernel and
        # the finalize; planning is inside the step, as it is inside every rad_batch call
        plan = rad.Plan(grid, ds, idx, len(segs), kinds, precision=prec, workspace=ws)
        plan.launch(o)
        plan.close()

    # ---- FP64, the headline
    for _ in range(args.warmup):
        step(rad.FP64, out)
    torch.cuda.synchronize()
    rad.profile_enable(True)
    rad.profile_read(reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(rad.FP64, out)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    kern_ms, launches = rad.profile_read(reset=True)
    rad.profile_enable(False)
    print("bench: fp64 %.3f s/step, amplitude kernel %.3f ms/launch over %d launches" %
          (dt, kern_ms / max(launches, 1), launches), file=sys.stderr, flush=True)
    kern_s = kern_ms / 1e3 / max(launches, 1)
    value = evals / dt

    # ---- mixed precision on the same workload
    mixed = None
    out_mx = None
    if not args.no_mixed:
        out_mx = torch.empty_like(out)
        step(rad.MIXED, out_mx)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        n_mx = max(1, min(args.steps, 2))
        for _ in range(n_mx):
            step(rad.MIXED, out_mx)
        torch.cuda.synchronize()
        dt_mx = (time.perf_counter() - t0) / n_mx
        mixed = {"value": evals / dt_mx, "unit": "evals/s", "ms_per_step": dt_mx * 1e3,
                 "speedup_vs_fp64": dt / dt_mx}
        print("bench: mixed %.3f s/step (x%.2f)" % (dt_mx, dt / dt_mx), file=sys.stderr, flush=True)

    # ---- CPU oracle on the bounded sample, and parity of both forms there
    cpu = None
    parity = None
    if not args.no_cpu_baseline:
        traj, iw, ix, iy = sample_points(segs, g)
        ref, rate, cpu_dt, threads, cevals = cpu_baseline(segs, g, traj, iw, ix, iy)
        cpu = {"value": rate, "unit": "evals/s", "cores": threads, "kind": "oracle",
               "sample": "%d trajectories (4 shortest, 4 longest) x every 2nd of %d photon "
                         "energies x 8x8 strided directions, spin-1/2, %.3e evals in %.1f s; "
                         "host %s, nproc %d" % (len(traj), n_w, cevals, cpu_dt, cpu_model(),
                                                os.cpu_count() or 0),
               "trajectories_per_s_extrapolated": rate / (evals / len(segs)),
               "single_core": cpu_single_core(segs, g, traj, iw, ix, iy)}
        got = out[:, 0].cpu().numpy()
        sel = np.ix_(iw, iy, ix)
        m64 = [rel_metrics(got[p][sel], ref[p]) for p in traj]
        parity = {"fp64_M1_max": max(m[0] for m in m64), "fp64_M2_max": max(m[1] for m in m64),
                  "sample_trajectories": traj}
        if out_mx is not None:
            gm = out_mx[:, 0].cpu().numpy()
            mmx = [rel_metrics(gm[p][sel], ref[p]) for p in traj]
            parity["mixed_M1_max"] = max(m[0] for m in mmx)
            parity["mixed_M2_max"] = max(m[1] for m in mmx)
            mixed["rel_err_M1"] = parity["mixed_M1_max"]
            mixed["rel_err_M2"] = parity["mixed_M2_max"]

    variant = rad.tune_get_variant(True, False, True)
    rec = grid.step != 0.0
    flops = flops_per_eval(variant, True, rec) * evals
    achieved = flops / kern_s / 1e12
    traffic = None
    if (kernel_sources_sha() == MEASURED_TRAFFIC["sources_sha256"] and variant == 0
            and len(segs) == MEASURED_TRAFFIC["particles"] and MEASURED_TRAFFIC["kernel"] == "amp_persistent"):
        traffic = MEASURED_TRAFFIC["bytes_per_launch"]
    roofline = {"bound": "alu", "achieved": achieved, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / FP64_PEAK_TFLOPS, "traffic": traffic,
                "kernel": "amp_persistent<%d,%d,J,fp64,%d%s>" % (VARIANTS[variant] + (",rec" if rec else "",)),
                "kernel_ms": kern_s * 1e3, "flops_per_eval": flops_per_eval(variant, True, rec),
                "valu_issue_frac": (VALU_PER_EVAL_44[(True, rec)] * evals / kern_s / 1e12 / VALU_PEAK_TOPS
                                    if variant == 0 else None)}
    # ---- the other configurations, the ceilings and the paper's figures as context; the
    # headline's own buffers are released first
    legs = None
    context = dict(PAPER_CONTEXT)
    if cpu is not None:
        context["this_gpu_vs_host_oracle"] = {"all_cores": value / cpu["value"], "cores": cpu["cores"],
                                              "one_core": value / cpu["single_core"]["value"]}
    if not args.no_legs:
        del ws, out
        if out_mx is not None:
            del out_mx
        torch.cuda.empty_cache()
        legs = {"peaks": run_leg("peaks", leg_peaks)}
        peaks = legs["peaks"] if "error" not in legs["peaks"] else None
        if mixed is not None:
            mixed["roofline"] = mixed_roofline(mixed["value"], peaks)
        legs["sampler"] = run_leg("sampler", leg_sampler)
        torch.cuda.empty_cache()
        legs["pm_mixed"] = run_leg("pm_mixed", leg_pm_mixed)
        torch.cuda.empty_cache()
        legs["electron_50gev_sections"] = run_leg("sections", leg_sections)
        torch.cuda.empty_cache()
        legs["undulator"] = run_leg("undulator", leg_undulator)
        legs["sweep"] = run_leg("sweep", leg_sweep)
        torch.cuda.empty_cache()
        legs["traj"] = run_leg("traj", leg_traj)
        torch.cuda.empty_cache()
    res = {
        "metric": METRIC, "value": value, "unit": "evals/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": dt * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "positron_spinhalf: %d e+ at 10 GeV, planar harmonic+quartic well "
                               "(20 eV, 1.92 A), 100 um, MS + radiative loss, %d..%d samples; "
                               "spin-1/2, 512 log hw 0.5-200 MeV x 32x32 within 5/gamma"
                               % (len(segs), min(ds.n), max(ds.n)),
                   "trajectories": len(segs), "samples": n_samples, "grid": list(grid.shape),
                   "kinds": "spin-1/2", "precision": "fp64", "form": "persistent plan (rad_plan_*)",
                   "autotune": autotune.choices(tuned)},
        "trajectories_per_s": len(segs) / dt,
        "mixed": mixed,
        "parity": parity,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "paper_context": context,
        "legs": legs,
    }
    print(json.dumps(_finite(res)), flush=True)


if __name__ == "__main__":
    main()
