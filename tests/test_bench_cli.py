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
    # 8 phase factors per 16 evaluations x 34 flops, complex product 6, accumulations 12
    assert bench.flops_per_eval(0, True) == 34.0 * 8 / 16 + 6 + 12
    assert bench.flops_per_eval(0, False) == 34.0 * 8 / 16 + 6 + 8
    # uniform grid, 4 x 4 tile: 5 phase factors and 10 complex products per 16 evaluations
    assert bench.flops_per_eval(0, True, True) == (5 * 34.0 + 10 * 6.0) / 16 + 6 + 12
    assert bench.flops_per_eval(1, True, True) == (5 * 34.0 + 8 * 6.0) / 12 + 6 + 12
    assert abs(bench.VALU_PEAK_TOPS - 39.3216) < 1e-9


def test_json_sanitiser():
    sys.path.insert(0, ROOT)
    import bench
    assert bench._finite({"a": float("inf"), "b": [1.0, float("nan")], "c": "x"}) == {"a": None, "b": [1.0, None],
                                                                                       "c": "x"}
