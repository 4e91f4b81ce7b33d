"""The C-ABI library loads on the CPU and exports every function include/*.h declares.

No compute call is made here (there is no GPU in the CPU suite); only calls
that the header defines to fail validation before touching a device.
"""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = sorted(os.path.join(ROOT, "include", h) for h in os.listdir(os.path.join(ROOT, "include"))
                 if h.endswith(".h"))


def declared_functions():
    src = "".join(open(h).read() for h in HEADERS)
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(rad_[a-z_0-9]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    from paper_1910_10391_amd import rad
    if not os.path.exists(rad.LIB_PATH):
        from paper_1910_10391_amd import build
        build.build()
    return rad.lib()


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("rad_setup_grid", "rad_classical", "rad_quantum", "rad_batch",
                     "rad_workspace_bytes", "rad_batch_workspace_bytes", "rad_angle_integrate",
                     "rad_free_grid", "rad_status_string", "rad_last_error"):
        assert required in names


def test_every_declared_symbol_is_exported(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_status_strings(lib):
    for s in range(5):
        assert lib.rad_status_string(s)
    assert b"unknown" in lib.rad_status_string(99)


def test_validation_before_device(lib):
    D = ctypes.POINTER(ctypes.c_double)
    h = ctypes.c_void_p()
    arr = (ctypes.c_double * 2)(1.0, 2.0)
    # sizes < 1, NULL arrays and non-finite values are rejected before any HIP call
    assert lib.rad_setup_grid(arr, 0, arr, 1, arr, 1, None, ctypes.byref(h)) == 1
    assert lib.rad_setup_grid(None, 2, arr, 1, arr, 1, None, ctypes.byref(h)) == 1
    bad = (ctypes.c_double * 1)(float("nan"))
    assert lib.rad_setup_grid(bad, 1, arr, 1, arr, 1, None, ctypes.byref(h)) == 1
    assert b"hw_eV" in lib.rad_last_error()
    assert lib.rad_workspace_bytes(None, 100, 1, 0) == 0
    assert lib.rad_batch_workspace_bytes(None, None, 0, 1, 1, 0) == 0
    assert lib.rad_tune_set_variant(0, 0, 0, 99) == 1
    assert lib.rad_tune_num_variants() == 5
    # the 4x6 tile serves only integral sets without J
    assert lib.rad_tune_set_variant(0, 0, 1, 4) == 4
    assert b"without J" in lib.rad_last_error()
    keep = ctypes.c_int()
    assert lib.rad_tune_get_variant(1, 1, 0, ctypes.byref(keep)) == 0
    assert lib.rad_tune_set_variant(1, 1, 0, 4) == 0
    assert lib.rad_tune_set_variant(1, 1, 0, keep.value) == 0
    # rad_phase_factors: precision, size and NULL checks come before any device call;
    # nothing is launched for n = 0
    lib.rad_phase_factors.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_void_p,
                                      ctypes.c_void_p, ctypes.c_void_p]
    assert lib.rad_phase_factors(None, 4, 7, None, None, None) == 1
    assert lib.rad_phase_factors(None, -1, 0, None, None, None) == 1
    assert lib.rad_phase_factors(None, 0, 1, None, None, None) == 0
    assert lib.rad_phase_factors(None, 4, 0, None, None, None) == 1 and b"turns is NULL" in lib.rad_last_error()
    d = ctypes.c_double(5.0)
    assert lib.rad_grid_step(None, ctypes.byref(d)) == 1 and d.value == 5.0
    assert b"NULL" in lib.rad_last_error()


def test_shape_knobs(lib):
    """The launch-shape knobs: energy spread per form and precision, the chunk target."""
    from paper_1910_10391_amd import rad
    rad.lib()                                           # argument types
    assert lib.rad_tune_set_shape(0, 1, 3) == 1 and b"wg 3" in lib.rad_last_error()
    assert lib.rad_tune_set_shape(0, 1, -1) == 1
    assert lib.rad_tune_get_shape(0, 1, None) == 1
    for persistent in (0, 1):
        for mixed in (0, 1):
            assert rad.tune_get_shape(persistent, mixed) == 0          # chosen by the grid
    rad.tune_set_shape(1, 0, 2)
    assert rad.tune_get_shape(1, 0) == 2 and rad.tune_get_shape(0, 0) == 0 and rad.tune_get_shape(1, 1) == 0
    rad.tune_set_shape(1, 0, 0)
    assert rad.tune_get_chunk_target() == 2048
    assert lib.rad_tune_set_chunk_target(-1) == 1 and lib.rad_tune_set_chunk_target((1 << 24) + 1) == 1
    rad.tune_set_chunk_target(8192)
    assert rad.tune_get_chunk_target() == 8192
    rad.tune_set_chunk_target(0)
    assert rad.tune_get_chunk_target() == 2048
