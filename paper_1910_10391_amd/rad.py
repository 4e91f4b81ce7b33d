"""Python binding of librad (include/rad.h): argument marshalling only.

Every step of the computation runs in the HIP kernels of ``librad.so``;
PyTorch only owns device memory (inputs, outputs, workspaces) and supplies the
stream.  If ``librad.so`` is missing the binding raises: there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
import threading

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
# RAD_LIBRARY: another build of the same library (the host-sanitizer build in the CPU tests)
LIB_PATH = os.environ.get("RAD_LIBRARY") or os.path.join(_PKG, "librad.so")

CLASSICAL, SPIN0, SPINHALF = 1, 2, 4
FP64, MIXED = 0, 1
OK, EINVAL, ENOMEM, EDEVICE, EUNSUPPORTED = 0, 1, 2, 3, 4     # rad_status
COLUMNS = ("t", "x", "y", "dz", "vx", "vy", "dvz", "ax", "ay", "az")

_lock = threading.Lock()
_lib = None


class RadError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(msg)
        self.status = status


class Segment(ctypes.Structure):
    _fields_ = ([("n", ctypes.c_int64)] + [(c, ctypes.c_void_p) for c in COLUMNS] +
                [("w", ctypes.c_void_p), ("gamma", ctypes.c_double),
                 ("energy_eV", ctypes.c_double)])


def lib():
    """The loaded librad (raises if it has not been built)."""
    global _lib
    with _lock:
        if _lib is None:
            _lib = load(LIB_PATH)
    return _lib


def load(path):
    """A build of librad at `path` with the C signatures declared (lib() loads the default
    one; the debug build's test loads librad_debug.so beside it)."""
    if not os.path.exists(path):
        raise RuntimeError("librad is not built (%s); run __graft_entry__.build()" % path)
    L = ctypes.CDLL(path)
    P, D, I, I64, S = (ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.c_int,
                       ctypes.c_int64, ctypes.c_size_t)
    SP = ctypes.POINTER(Segment)
    sig = {
        "rad_setup_grid": (I, [D, I, D, I, D, I, P, ctypes.POINTER(P)]),
        "rad_free_grid": (None, [P]),
        "rad_grid_dims": (I, [P, ctypes.POINTER(I), ctypes.POINTER(I), ctypes.POINTER(I)]),
        "rad_grid_step": (I, [P, D]),
        "rad_workspace_bytes": (S, [P, I64, I, I]),
        "rad_batch_workspace_bytes": (S, [P, SP, I, I, I, I]),
        "rad_classical": (I, [P, SP, I, P, P, S, P]),
        "rad_quantum": (I, [P, SP, I, I, P, P, S, P]),
        "rad_batch": (I, [P, SP, I, ctypes.POINTER(I), I, I, I, P, P, S, P]),
        "rad_angle_integrate": (I, [P, P, I, P, P]),
        "rad_phase_factors": (I, [P, I64, I, P, P, P]),
        "rad_status_string": (ctypes.c_char_p, [I]),
        "rad_last_error": (ctypes.c_char_p, []),
        "rad_tune_set_variant": (I, [I, I, I, I]),
        "rad_tune_get_variant": (I, [I, I, I, ctypes.POINTER(I)]),
        "rad_tune_set_shape": (I, [I, I, I]),
        "rad_tune_get_shape": (I, [I, I, ctypes.POINTER(I)]),
        "rad_tune_set_chunk_target": (I, [I64]),
        "rad_tune_get_chunk_target": (I64, []),
        "rad_tune_set_cell_spread": (I, [I]),
        "rad_tune_get_cell_spread": (I, []),
        "rad_plan_create": (I, [P, SP, I, ctypes.POINTER(I), I, I, I, P, S, P,
                                ctypes.POINTER(P)]),
        "rad_plan_launch": (I, [P, P, P]),
        "rad_plan_launch_graph": (I, [P, P, P]),
        "rad_plan_free": (None, [P]),
        "rad_cells_workspace_bytes": (S, [P, SP, I, I, I, I, I, P]),
        "rad_cells": (I, [P, SP, I, I, I, I, I, P, P, P, S, P]),
        "rad_cells_device_workspace_bytes": (S, [P, SP, I, I, I, I, I]),
        "rad_cells_device": (I, [P, SP, I, I, I, I, I, P, P, P, S, P]),
        "rad_tune_num_variants": (I, []),
        "rad_profile_enable": (I, [I]),
        "rad_profile_read": (I, [ctypes.POINTER(ctypes.c_double), ctypes.POINTER(I64), I]),
        "rad_peak": (I, [I, I64, P, I64, D, P]),
        "rad_debug_violations": (I64, [I]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    return L


def _check(status, what):
    if status != 0:
        L = lib()
        raise RadError(status, "%s: %s: %s" % (what, L.rad_status_string(status).decode(),
                                                 L.rad_last_error().decode()))


def _stream(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _dptr(t):
    return ctypes.c_void_p(t.data_ptr())


def n_kinds(kinds):
    return bin(int(kinds) & 7).count("1")


class Grid:
    """Photon energies [eV] x directions (thx, thy) [rad]; the library copies them."""

    def __init__(self, hw_eV, thx, thy, stream=None):
        self.hw = np.ascontiguousarray(hw_eV, dtype=np.float64)
        self.thx = np.ascontiguousarray(thx, dtype=np.float64)
        self.thy = np.ascontiguousarray(thy, dtype=np.float64)
        D = ctypes.POINTER(ctypes.c_double)
        h = ctypes.c_void_p()
        _check(lib().rad_setup_grid(self.hw.ctypes.data_as(D), self.hw.size,
                                    self.thx.ctypes.data_as(D), self.thx.size,
                                    self.thy.ctypes.data_as(D), self.thy.size, _stream(stream),
                                    ctypes.byref(h)), "rad_setup_grid")
        self.handle = h

    @property
    def shape(self):
        return (self.hw.size, self.thy.size, self.thx.size)

    @property
    def step(self):
        """The common direction spacing of the FP64 phase recurrence, or 0 (rad_grid_step)."""
        d = ctypes.c_double()
        _check(lib().rad_grid_step(self.handle, ctypes.byref(d)), "rad_grid_step")
        return d.value

    def close(self):
        if getattr(self, "handle", None) and self.handle.value:
            lib().rad_free_grid(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class DeviceSegments:
    """Segments uploaded to the GPU: one FP64 tensor holds every column of every segment."""

    def __init__(self, segs, device="cuda"):
        import torch
        self.n = [int(np.asarray(s["t"]).size) for s in segs]
        total = int(sum(self.n))
        has_w = [s.get("w") is not None for s in segs]
        ncol = len(COLUMNS) + (1 if any(has_w) else 0)
        host = np.empty((ncol, total), dtype=np.float64)
        off = 0
        for s, n, hw_ in zip(segs, self.n, has_w):
            for i, c in enumerate(COLUMNS):
                host[i, off:off + n] = np.asarray(s[c], dtype=np.float64)
            if ncol > len(COLUMNS):
                host[-1, off:off + n] = np.asarray(s["w"], dtype=np.float64) if hw_ else 0.0
            off += n
        self.data = torch.from_numpy(host).to(device)
        base = self.data.data_ptr()
        row = total * 8
        self.structs = (Segment * len(segs))()
        off = 0
        for k, (s, n, hw_) in enumerate(zip(segs, self.n, has_w)):
            st = self.structs[k]
            st.n = n
            for i, c in enumerate(COLUMNS):
                setattr(st, c, base + i * row + off * 8)
            st.w = base + (ncol - 1) * row + off * 8 if hw_ else None
            st.gamma = float(s["gamma"])
            st.energy_eV = float(s.get("energy_eV", 0.0) or 0.0)
            off += n

    def __len__(self):
        return len(self.structs)

    def subset(self, rows):
        """The segments `rows` (in that order), sharing this object's device columns."""
        view = DeviceSegments.__new__(DeviceSegments)
        rows = [int(r) for r in rows]
        view.n = [self.n[r] for r in rows]
        view.data = self.data
        view.structs = (Segment * len(rows))(*[self.structs[r] for r in rows])
        return view


def _as_segments(segs):
    return segs if isinstance(segs, DeviceSegments) else DeviceSegments(segs)


def workspace_bytes(grid, max_n, kinds, precision=FP64):
    return int(lib().rad_workspace_bytes(grid.handle, int(max_n), int(kinds), int(precision)))


def batch_workspace_bytes(grid, dsegs, n_out, kinds, precision=FP64):
    return int(lib().rad_batch_workspace_bytes(grid.handle, dsegs.structs, len(dsegs), int(n_out),
                                               int(kinds), int(precision)))


def _nbytes(t):
    return t.numel() * t.element_size()


def _workspace(nbytes, workspace, device):
    """The caller's workspace if it is large enough, else a new uint8 tensor."""
    import torch
    if workspace is not None:
        if not (workspace.is_cuda and workspace.is_contiguous()):
            raise ValueError("workspace must be a contiguous CUDA tensor")
        if _nbytes(workspace) >= nbytes:
            return workspace
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


def _check_out(out, shape):
    """The C ABI can only check that a pointer lies inside a device allocation; torch
    sub-allocates, so tensor bounds are checked here."""
    import torch
    if not (out.is_cuda and out.dtype == torch.float64 and out.is_contiguous()):
        raise ValueError("out must be a contiguous float64 CUDA tensor")
    if out.numel() != int(np.prod(shape)):
        raise ValueError("out has %d elements, expected shape %s" % (out.numel(), shape))


def classical(grid, seg, precision=FP64, out=None, workspace=None, stream=None):
    """Classical cube [n_w, n_y, n_x] of one segment (rad_classical)."""
    import torch
    ds = _as_segments([seg] if isinstance(seg, dict) else seg)
    dev = ds.data.device
    if out is None:
        out = torch.empty(grid.shape, dtype=torch.float64, device=dev)
    _check_out(out, grid.shape)
    ws = _workspace(workspace_bytes(grid, ds.n[0], CLASSICAL, precision), workspace, dev)
    _check(lib().rad_classical(grid.handle, ctypes.byref(ds.structs[0]), int(precision), _dptr(out),
                               _dptr(ws), _nbytes(ws), _stream(stream)), "rad_classical")
    return out


def quantum(grid, seg, kinds=SPIN0 | SPINHALF, precision=FP64, out=None, workspace=None,
            stream=None):
    """Spin-0 / spin-1/2 cubes [n_kinds, n_w, n_y, n_x] of one segment (rad_quantum)."""
    import torch
    ds = _as_segments([seg] if isinstance(seg, dict) else seg)
    dev = ds.data.device
    if out is None:
        out = torch.empty((n_kinds(kinds),) + grid.shape, dtype=torch.float64, device=dev)
    _check_out(out, (n_kinds(kinds),) + grid.shape)
    ws = _workspace(workspace_bytes(grid, ds.n[0], kinds, precision), workspace, dev)
    _check(lib().rad_quantum(grid.handle, ctypes.byref(ds.structs[0]), int(kinds), int(precision),
                             _dptr(out), _dptr(ws), _nbytes(ws), _stream(stream)), "rad_quantum")
    return out


def batch(grid, segs, out_index, n_out, kinds, precision=FP64, out=None, workspace=None,
          stream=None):
    """Cubes [n_out, n_kinds, n_w, n_y, n_x]: segments summed per output in segment order."""
    import torch
    ds = _as_segments(segs)
    dev = ds.data.device
    if len(out_index) != len(ds):
        raise ValueError("out_index must have one entry per segment")
    idx = (ctypes.c_int * len(ds))(*[int(i) for i in out_index])
    if out is None:
        out = torch.empty((n_out, n_kinds(kinds)) + grid.shape, dtype=torch.float64, device=dev)
    _check_out(out, (n_out, n_kinds(kinds)) + grid.shape)
    ws = _workspace(batch_workspace_bytes(grid, ds, n_out, kinds, precision), workspace, dev)
    _check(lib().rad_batch(grid.handle, ds.structs, len(ds), idx, int(n_out), int(kinds),
                           int(precision), _dptr(out), _dptr(ws), _nbytes(ws), _stream(stream)),
           "rad_batch")
    return out


def phase_factors(turns, precision=FP64, stream=None):
    """(cos, sin) of a contiguous float64 CUDA tensor of half turns (FP64: cos(pi u)) or
    revolutions (MIXED: cos(2 pi r)), by the integral kernels' own routine
    (rad_phase_factors)."""
    import torch
    if turns.dtype != torch.float64 or not turns.is_cuda or not turns.is_contiguous():
        raise ValueError("turns must be a contiguous float64 CUDA tensor")
    c = torch.empty_like(turns)
    s = torch.empty_like(turns)
    _check(lib().rad_phase_factors(_dptr(turns), int(turns.numel()), int(precision), _dptr(c), _dptr(s),
                                   _stream(stream)), "rad_phase_factors")
    return c, s


def angle_integrate(grid, cubes, out=None, stream=None):
    """dI/d hw [..., n_w] of cubes [..., n_w, n_y, n_x] (rad_angle_integrate)."""
    import torch
    lead = tuple(cubes.shape[:-3])
    n_cubes = int(np.prod(lead)) if lead else 1
    if tuple(cubes.shape[-3:]) != grid.shape or not cubes.is_contiguous() or cubes.dtype != torch.float64:
        raise ValueError("cubes must be contiguous float64 [..., n_w, n_y, n_x]")
    if out is None:
        out = torch.empty(lead + (grid.shape[0],), dtype=torch.float64, device=cubes.device)
    _check_out(out, lead + (grid.shape[0],))
    _check(lib().rad_angle_integrate(grid.handle, _dptr(cubes), n_cubes, _dptr(out),
                                     _stream(stream)), "rad_angle_integrate")
    return out


def cells(grid, segs, kind, mask, precision=FP64, cx=8, cy=8, out=None, workspace=None,
          stream=None):
    """Exact cell integrals [n_segs, n_w, n_cells] where ``mask`` (uint8, same shape) is set
    (rad_cells): the ``kind`` spectrum summed over each cx x cy cell times dthx dthy.  A
    mask that is a device tensor stays on the device (rad_cells_device)."""
    import torch
    ds = _as_segments(segs)
    n_w, n_y, n_x = grid.shape
    n_cells = (n_x // cx) * (n_y // cy)
    if isinstance(mask, torch.Tensor) and mask.is_cuda:
        if mask.dtype != torch.uint8 or tuple(mask.shape) != (len(ds), n_w, n_cells) or not mask.is_contiguous():
            raise ValueError("mask must be a contiguous uint8 tensor of shape %s" % ((len(ds), n_w, n_cells),))
        nb = int(lib().rad_cells_device_workspace_bytes(grid.handle, ds.structs, len(ds), int(kind),
                                                        int(precision), cx, cy))
        if nb == 0:
            raise RadError(1, "rad_cells_device_workspace_bytes: invalid arguments: %s"
                           % lib().rad_last_error().decode())
        ws = _workspace(nb, workspace, ds.data.device)
        if out is None:
            out = torch.empty((len(ds), n_w, n_cells), dtype=torch.float64, device=ds.data.device)
        _check_out(out, (len(ds), n_w, n_cells))
        _check(lib().rad_cells_device(grid.handle, ds.structs, len(ds), int(kind), int(precision), cx, cy,
                                      _dptr(mask), _dptr(out), _dptr(ws), _nbytes(ws), _stream(stream)),
               "rad_cells_device")
        return out
    m = np.ascontiguousarray(mask, dtype=np.uint8)
    if m.shape != (len(ds), n_w, n_cells):
        raise ValueError("mask must have shape %s" % ((len(ds), n_w, n_cells),))
    mp = ctypes.c_void_p(m.ctypes.data)
    nb = int(lib().rad_cells_workspace_bytes(grid.handle, ds.structs, len(ds), int(kind),
                                             int(precision), cx, cy, mp))
    if nb == 0:
        raise RadError(1, "rad_cells_workspace_bytes: invalid arguments: %s"
                       % lib().rad_last_error().decode())
    ws = _workspace(nb, workspace, ds.data.device)
    if out is None:
        out = torch.empty((len(ds), n_w, n_cells), dtype=torch.float64, device=ds.data.device)
    _check_out(out, (len(ds), n_w, n_cells))
    _check(lib().rad_cells(grid.handle, ds.structs, len(ds), int(kind), int(precision), cx, cy, mp,
                           _dptr(out), _dptr(ws), _nbytes(ws), _stream(stream)), "rad_cells")
    return out


def tune_set_variant(persistent, mixed, with_j, variant):
    _check(lib().rad_tune_set_variant(int(bool(persistent)), int(bool(mixed)), int(bool(with_j)),
                                      int(variant)), "rad_tune_set_variant")


def tune_get_variant(persistent, mixed, with_j):
    v = ctypes.c_int()
    _check(lib().rad_tune_get_variant(int(bool(persistent)), int(bool(mixed)), int(bool(with_j)),
                                      ctypes.byref(v)), "rad_tune_get_variant")
    return v.value


def tune_set_shape(persistent, mixed, wg):
    """Waves of a block over photon energies (1, 2, 4; 0: chosen by the grid)."""
    _check(lib().rad_tune_set_shape(int(bool(persistent)), int(bool(mixed)), int(wg)), "rad_tune_set_shape")


def tune_get_shape(persistent, mixed):
    v = ctypes.c_int()
    _check(lib().rad_tune_get_shape(int(bool(persistent)), int(bool(mixed)), ctypes.byref(v)), "rad_tune_get_shape")
    return v.value


def tune_set_chunk_target(target_blocks):
    """Work items the time chunking aims for (0: the default 2048)."""
    _check(lib().rad_tune_set_chunk_target(int(target_blocks)), "rad_tune_set_chunk_target")


def tune_get_chunk_target():
    return int(lib().rad_tune_get_chunk_target())


def tune_set_cell_spread(wg):
    """Waves of a cell block over photon energies (1, 2, 4; 0: the default 1)."""
    _check(lib().rad_tune_set_cell_spread(int(wg)), "rad_tune_set_cell_spread")


def tune_get_cell_spread():
    return int(lib().rad_tune_get_cell_spread())


class Plan:
    """A replayable batch (rad_plan_*): persistent kernels over a longest-first work list.

    The plan keeps the device segments, the workspace and the grid alive.  ``launch``
    issues kernels only; ``launch_graph`` captures them into a hipGraph on first use
    (per output tensor) and replays it; it needs a created stream (not the default
    stream), e.g. ``torch.cuda.Stream()``.
    """

    def __init__(self, grid, segs, out_index, n_out, kinds, precision=FP64, workspace=None,
                 stream=None):
        ds = _as_segments(segs)
        if len(out_index) != len(ds):
            raise ValueError("out_index must have one entry per segment")
        self.grid, self.ds, self.n_out, self.kinds = grid, ds, int(n_out), int(kinds)
        self.precision = int(precision)
        self.shape = (self.n_out, n_kinds(kinds)) + grid.shape
        idx = (ctypes.c_int * len(ds))(*[int(i) for i in out_index])
        self.ws = _workspace(batch_workspace_bytes(grid, ds, n_out, kinds, precision), workspace,
                             ds.data.device)
        h = ctypes.c_void_p()
        _check(lib().rad_plan_create(grid.handle, ds.structs, len(ds), idx, self.n_out, self.kinds,
                                     self.precision, _dptr(self.ws), _nbytes(self.ws),
                                     _stream(stream), ctypes.byref(h)), "rad_plan_create")
        self.handle = h

    def _out(self, out):
        import torch
        if out is None:
            out = torch.empty(self.shape, dtype=torch.float64, device=self.ds.data.device)
        _check_out(out, self.shape)
        return out

    def launch(self, out=None, stream=None):
        out = self._out(out)
        _check(lib().rad_plan_launch(self.handle, _dptr(out), _stream(stream)), "rad_plan_launch")
        return out

    def launch_graph(self, out=None, stream=None):
        out = self._out(out)
        _check(lib().rad_plan_launch_graph(self.handle, _dptr(out), _stream(stream)),
               "rad_plan_launch_graph")
        return out

    def close(self):
        if getattr(self, "handle", None) and self.handle.value:
            lib().rad_plan_free(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def tune_num_variants():
    return int(lib().rad_tune_num_variants())


def profile_enable(on=True):
    _check(lib().rad_profile_enable(int(bool(on))), "rad_profile_enable")


def profile_read(reset=False):
    ms = ctypes.c_double()
    n = ctypes.c_int64()
    _check(lib().rad_profile_read(ctypes.byref(ms), ctypes.byref(n), int(bool(reset))),
           "rad_profile_read")
    return ms.value, n.value


PEAK_FMA64, PEAK_FMA32, PEAK_SINCOS32, PEAK_PHASE64, PEAK_PHASE_MIXED = range(5)


def peak(which, iters=4096, n_threads=256 * 256 * 8, reps=3, stream=None):
    """Issue-rate microbenchmark (rad_peak): (operations per second, operations per
    launch, ms per launch), the best of `reps` timed launches after one warm-up, timed
    with events on the launch stream."""
    import torch
    out = torch.empty(int(n_threads), dtype=torch.float64, device="cuda")
    ops = ctypes.c_double()
    st = torch.cuda.current_stream() if stream is None else stream
    best = None
    for r in range(reps + 1):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        _check(lib().rad_peak(int(which), int(iters), _dptr(out), int(n_threads), ctypes.byref(ops),
                              ctypes.c_void_p(st.cuda_stream)), "rad_peak")
        e1.record(st)
        e1.synchronize()
        ms = e0.elapsed_time(e1)
        if r > 0 and (best is None or ms < best):
            best = ms
    return ops.value / (best * 1e-3), ops.value, best
