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
    "_ZN3rad10amp_kernelILi4ELi4ELb1ELb0ELi2ELb1EEEvNS_9AmpLaunchE": 279,   # FP64, J, recurrence
    "_ZN3rad10amp_kernelILi4ELi4ELb1ELb0ELi2ELb0EEEvNS_9AmpLaunchE": 311,   # FP64, J, direct
    "_ZN3rad10amp_kernelILi4ELi4ELb1ELb1ELi2ELb0EEEvNS_9AmpLaunchE": 204,   # mixed, J
    "_ZN3rad14amp_persistentILi4ELi4ELb1ELb0ELi2ELb1EEEvNS_9AmpLaunchE": 279,
    "_ZN3rad14amp_persistentILi4ELi4ELb1ELb0ELi2ELb0EEEvNS_9AmpLaunchE": 311,
    "_ZN3rad14amp_persistentILi4ELi4ELb1ELb1ELi2ELb0EEEvNS_9AmpLaunchE": 204,
    # 4x6 tile without J: per 24 evaluations
    "_ZN3rad10amp_kernelILi4ELi6ELb0ELb0ELi2ELb1EEEvNS_9AmpLaunchE": 327,   # FP64, recurrence
    "_ZN3rad10amp_kernelILi4ELi6ELb0ELb0ELi2ELb0EEEvNS_9AmpLaunchE": 389,   # FP64, direct
    "_ZN3rad10amp_kernelILi4ELi6ELb0ELb1ELi2ELb0EEEvNS_9AmpLaunchE": 252,   # mixed
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


@pytest.mark.parametrize("symbol", sorted(HOT))
def test_hot_loop_has_no_scratch_and_known_valu(asm, symbol):
    c = hot_loop(asm, symbol)
    valu = sum(v for k, v in c.items() if k.startswith("v_"))
    scratch = sum(v for k, v in c.items() if k.startswith(("scratch_", "buffer_")))
    print("%s: VALU %d, scratch %d" % (symbol, valu, scratch))
    assert scratch == 0
    assert valu == HOT[symbol]
