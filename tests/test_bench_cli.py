"""bench.py's command line on the CPU: more than one GPU is refused with a message, and
the accounting helpers give the documented figures."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_flop_accounting():
    sys.path.insert(0, ROOT)
    import bench
    # 4x4 tile: 7 evaluated phase factors and 12 complex products per 16 evals
    assert bench.flops_per_eval(0, True) == (7 * 34.0 + 12 * 6.0) / 16 + 12
    assert bench.flops_per_eval(0, False) == (7 * 34.0 + 12 * 6.0) / 16 + 8
    # recurrence, 4x4: 4 evaluated factors; x: 3 products + 2 multiplier steps, y: 2 + 2,
    # rows 1..3: 12 (28.375 flops per eval)
    assert bench.flops_per_eval(0, True, True) == (4 * 34.0 + 21 * 6.0) / 16 + 12 == 28.375
    # 4x3: x 3 + 2, y 1 + 1, rows 8
    assert bench.flops_per_eval(1, True, True) == (4 * 34.0 + 15 * 6.0) / 12 + 12
    assert abs(bench.VALU_PEAK_TOPS - 39.3216) < 1e-9


def test_json_sanitiser():
    sys.path.insert(0, ROOT)
    import bench
    assert bench._finite({"a": float("inf"), "b": [1.0, float("nan")], "c": "x"}) == {"a": None, "b": [1.0, None],
                                                                                       "c": "x"}
