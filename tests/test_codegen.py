"""The hot loops of the amplitude kernels as gfx950 assembly (hipcc -S, no GPU needed):
no scratch (register spill) access inside the per-time-step loop, and the VALU
instruction counts the benchmark's issue accounting uses.  The register file is full in
these loops, so a harmless-looking source change can make the compiler spill there; this
test makes that visible."""
import collections
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1910_10391_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# (kernel symbol, VALU instructions in the hot loop per time step: 16 evaluations for a 4x4
# tile)
HOT = {
    "_ZN3rad10amp_kernelILi4ELi4ELb1ELb0ELi2ELb1EEEvNS_9AmpLaunchE": 275,   # FP64, J, recurrence
    "_ZN3rad10amp_kernelILi4ELi4ELb1ELb0ELi2ELb0EEEvNS_9AmpLaunchE": 308,   # FP64, J, direct
    "_ZN3rad10amp_kernelILi4ELi4ELb1ELb1ELi2ELb0EEEvNS_9AmpLaunchE": 201,   # mixed, J
    "_ZN3rad14amp_persistentILi4ELi4ELb1ELb0ELi2ELb1EEEvNS_9AmpLaunchE": 275,
    "_ZN3rad14amp_persistentILi4ELi4ELb1ELb0ELi2ELb0EEEvNS_9AmpLaunchE": 308,
    "_ZN3rad14amp_persistentILi4ELi4ELb1ELb1ELi2ELb0EEEvNS_9AmpLaunchE": 201,
    # 4x6 tile without J: per 24 evaluations
    "_ZN3rad10amp_kernelILi4ELi6ELb0ELb0ELi2ELb1EEEvNS_9AmpLaunchE": 323,   # FP64, recurrence
    "_ZN3rad10amp_kernelILi4ELi6ELb0ELb0ELi2ELb0EEEvNS_9AmpLaunchE": 386,   # FP64, direct
    "_ZN3rad10amp_kernelILi4ELi6ELb0ELb1ELi2ELb0EEEvNS_9AmpLaunchE": 249,   # mixed
}


@pytest.fixture(scope="module")
def asm(tmp_path_factory):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    out = tmp_path_factory.mktemp("asm") / "rad_kernels.s"
    cmd = [HIPCC, "--offload-arch=gfx950", "-O3", "-std=c++17", "-Xclang", "-target-feature", "-Xclang",
           "-packed-fp32-ops", "-I", os.path.join(ROOT, "include"), "-I", CSRC, "--cuda-device-only", "-S",
           os.path.join(CSRC, "rad_kernels.hip"), "-o", str(out)]
    subprocess.run(cmd, check=True, capture_output=True)
    return out.read_text().split("\n")


def loops(lines, symbol):
    """(instruction counts of each backward-branch loop body) of one kernel."""
    start = next(i for i, l in enumerate(lines) if l.startswith(symbol + ":"))
    end = next(i for i in range(start + 1, len(lines)) if lines[i].startswith(".Lfunc_end"))
    body = lines[start:end]
    labels = {m.group(1): i for i, l in enumerate(body) for m in [re.match(r"^(\.LBB\S+):", l)] if m}
    out = []
    for i, l in enumerate(body):
        m = re.search(r"s_cbranch_\w+\s+(\.LBB\S+)|s_branch\s+(\.LBB\S+)", l)
        if m:
            tgt = m.group(1) or m.group(2)
            if tgt in labels and labels[tgt] < i:
                ins = [x.strip().split()[0] for x in body[labels[tgt]:i + 1]
                       if x.strip() and not x.strip().startswith((".", ";")) and not x.strip().endswith(":")]
                out.append(collections.Counter(ins))
    return out


def hot_loop(lines, symbol):
    """The per-time-step loop: the innermost loop that reads the staged integrand
    (ds_read_b128) and does the most VALU work."""
    cands = [c for c in loops(lines, symbol) if c.get("ds_read_b128", 0) >= 16]
    assert cands, symbol
    inner = min(cands, key=lambda c: sum(c.values()))
    return inner


# hardware FP32 sine and cosine in the mixed-precision hot loops (the mixed form's issue
# roofline weights them by their measured cost): 7 phase factors per 4x4 tile step,
# 9 per 4x6 step
TRANS = {
    "_ZN3rad10amp_kernelILi4ELi4ELb1ELb1ELi2ELb0EEEvNS_9AmpLaunchE": 14,
    "_ZN3rad14amp_persistentILi4ELi4ELb1ELb1ELi2ELb0EEEvNS_9AmpLaunchE": 14,
    "_ZN3rad10amp_kernelILi4ELi6ELb0ELb1ELi2ELb0EEEvNS_9AmpLaunchE": 18,
}


@pytest.mark.parametrize("symbol", sorted(HOT))
def test_hot_loop_has_no_scratch_and_known_valu(asm, symbol):
    c = hot_loop(asm, symbol)
    valu = sum(v for k, v in c.items() if k.startswith("v_"))
    scratch = sum(v for k, v in c.items() if k.startswith(("scratch_", "buffer_")))
    trans = sum(v for k, v in c.items() if k.startswith(("v_sin_", "v_cos_")))
    print("%s: VALU %d, scratch %d, sin/cos %d" % (symbol, valu, scratch, trans))
    assert scratch == 0
    assert valu == HOT[symbol]
    assert trans == TRANS.get(symbol, 0)


def _pass_loop_spill_stores(lines, symbol):
    """Scratch stores inside the time-pass loop (the loop that holds the staging loops and
    the hot loop), from the loop-depth notes of the assembly: depth 2 in the persistent
    kernel (inside the work-item loop), depth 1 in the one-item kernel."""
    start = next(i for i, l in enumerate(lines) if l.startswith(symbol + ":"))
    end = next(i for i in range(start + 1, len(lines)) if lines[i].startswith(".Lfunc_end"))
    pass_depth = 2 if "persistent" in symbol or "Li6E" in symbol else 1
    depth, n = 0, 0
    for l in lines[start:end]:
        if l.startswith((".LBB", "; %bb")):
            m = re.search(r"Depth=(\d+)", l)
            depth = int(m.group(1)) if m else 0
        if "scratch_store" in l and depth == pass_depth:
            n += 1
    return n


@pytest.mark.parametrize("symbol", sorted(HOT))
def test_no_spill_stores_per_time_pass(asm, symbol):
    """The time loop's bounds and counter are wave-uniform and stay in scalar registers, so
    nothing is written to scratch once per pass of 128 time steps (spills that remain are
    per work item)."""
    n = _pass_loop_spill_stores(asm, symbol)
    print("%s: %d scratch stores per pass" % (symbol, n))
    assert n == 0


def test_bench_uses_the_counted_mixed_loop():
    """bench.py's mixed-form issue roofline uses the counts pinned above."""
    import bench
    sym = "_ZN3rad14amp_persistentILi4ELi4ELb1ELb1ELi2ELb0EEEvNS_9AmpLaunchE"
    assert bench.MIXED_VALU_PER_16 == HOT[sym] and bench.MIXED_TRANS_PER_16 == TRANS[sym]
